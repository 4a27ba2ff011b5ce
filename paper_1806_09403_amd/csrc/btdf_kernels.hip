// btdf_kernels.hip -- gfx950 kernels of one BTDF-IB-LBM time step.
//
//   ib_kernel   16 lanes per marker, one per stencil node: interpolation of
//               rho and the unforced velocity u* to the markers (eqs 12, 14)
//               from the streamed populations at the stencil nodes (eqs 9-10,
//               u* including G/2) and the direct force F_l = 2 rho_l
//               (U_b - u*_l) (eq 20); the weights and drs ds F_l are left
//               for the lattice kernel.
//   lbm_kernel  one thread per node (NPT nodes per thread along x): the
//               streaming pull, moments, the spread force of the markers
//               whose stencils touch the tile (eqs 13, 15, gathered from the
//               tile's marker list in LDS -- no atomics, fixed summation
//               order), the corrected velocity (eq 11), equilibrium (eq 6),
//               Guo term (eq 7) and BGK collision (eq 5), and the channel
//               ghost columns; extra workgroups form the per-body force and
//               torque sums of eq 27 into the history ring.
//
// Populations are stored as deviations f~_q = f_q - feq_q(1, u_ref) from the
// equilibrium of the reference state the run starts from, in
// structure-of-arrays planes [q][y][pitch]; sums of deviations keep the FP32
// path free of the cancellation against the reference populations, and the
// rounding of a near-reference flow small.
#include "btdf_device.h"
#include "btdf_launch.h"

namespace btdf {

// ------------------------------------------------------------------ marker kernel

// Marker kernel: 16 lanes per marker, one per node of the (up to) 4x4
// stencil, 16 markers per workgroup, over all markers of all bodies. Each
// lane pulls its node's populations and forms rho and u* there (eqs 9-10,
// u* with G/2); the weighted sums of eqs 12/14 are reduced across the 16
// lanes by shuffles and lane 0 of the group forms F_l (eq 20). Each marker's
// delta weights, stencil origin and drs ds F_l are left for the lattice
// kernel's spread gather. The per-body sums of eq 27 are formed by extra
// workgroups of the lattice kernel, after this kernel has completed.
// one marker per 16-lane group; l = marker id, act = l is a marker of ib
template <typename T>
__device__ __forceinline__ void ib_marker(const T *__restrict__ A, const LbmParams &p, const IbParams &ib, int l,
                                          bool act) {
  const int node = (int)threadIdx.x & 15;
  const int S = stencil_size(p.kind);
  const int a = node & 3, c = node >> 2;

  double wr = 0.0, wu = 0.0, wv = 0.0, X = 0.0, Y = 0.0;
  // the marker's velocity and spreading factor, loaded with its position:
  // read after the stores below they would wait for them (the arrays may
  // alias as far as the compiler knows) and add a round trip at the end
  double Ub = 0.0, Vb = 0.0, sdl = 0.0;
  int bx = 0, by = 0;
  if (act) {
    X = ib.X[l];
    Y = ib.Y[l];
    Ub = ib.U[l];
    Vb = ib.V[l];
    sdl = ib.sdrs[l];
    bx = stencil_base(p.kind, X);
    by = stencil_base(p.kind, Y);
  }
  // this lane's stencil node and its nine populations, loaded before the
  // weights are evaluated, so that the loads are in flight meanwhile
  const bool on = act && a < S && c < S;
  int i = bx + a, j = by + c;
  if (p.xper) i = wrap_index(i, p.nx);
  if (p.yper) j = wrap_index(j, p.ny);
  T gq[9];
  if (on) {
    if (i >= 1 && i <= p.nx - 2 && j >= 1 && j <= p.ny - 2) {
      // no wrap, no wall: one 32-bit offset, the shifts fold into the plane base
      const unsigned off = ((unsigned)j * (unsigned)p.pitch + (unsigned)i) * (unsigned)sizeof(T);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const char *base = reinterpret_cast<const char *>(A + (long long)q * p.plane -
                                                          (long long)ey(q) * p.pitch - ex(q));
        gq[q] = *reinterpret_cast<const T *>(base + off);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) gq[q] = pull(A, p, q, i, j);
    }
  }
  // lanes 0-3 of the group evaluate the x weights, lanes 4-7 the y weights
  double ph = 0.0;
  if (act && node < 8) {
    const int k = node & 3;
    if (k < S) ph = node < 4 ? phi(p.kind, (double)(bx + k) - X) : phi(p.kind, (double)(by + k) - Y);
  }
  const int gl = (int)threadIdx.x & ~15 & 63;  // first lane of the group within the wave
  const double phx = __shfl(ph, gl + a, 64);
  const double phy = __shfl(ph, gl + 4 + c, 64);
  if (act && node < 8 && ib.nf > 1) ib.mdf_w[8 * (long long)l + node] = ph;
  if (act) {
    T *mw = reinterpret_cast<T *>(ib.mk_w) + 10 * (long long)l;
    if (c == 0) mw[a] = (T)phx;
    if (a == 0) mw[4 + c] = (T)phy;
    if (on) {
      const double W = phx * phy;
      double drho = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const double g = (double)gq[q];
        drho += g;
        mx += ex(q) * g;
        my += ey(q) * g;
      }
      const double rho = 1.0 + drho;
      const double inv = 1.0 / rho;
      const double usx = (mx + p.urx + 0.5 * p.Gx) * inv;  // the stored values' first moment is m - u_ref
      const double usy = (my + p.ury + 0.5 * p.Gy) * inv;
      wr = W * rho;
      wu = W * usx;
      wv = W * usy;
      if (ib.nf > 1) {  // later forcing passes start from the node's rho and u*
        double *cc = ib.mdf_cache + (16 * (long long)l + node) * 3;
        cc[0] = rho;
        cc[1] = usx;
        cc[2] = usy;
      }
    }
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    wr += __shfl_xor(wr, off, 16);
    wu += __shfl_xor(wu, off, 16);
    wv += __shfl_xor(wv, off, 16);
  }
  if (act && node == 0) {
    const double Fx = 2.0 * wr * (Ub - wu);
    const double Fy = 2.0 * wr * (Vb - wv);
    ib.Fx[l] = Fx;
    ib.Fy[l] = Fy;
    ib.rho_l[l] = wr;
    ib.ux_l[l] = wu;
    ib.uy_l[l] = wv;
    const double sd = sdl;
    T *mw = reinterpret_cast<T *>(ib.mk_w) + 10 * (long long)l;
    mw[8] = (T)(Fx * sd);
    mw[9] = (T)(Fy * sd);
    ib.mk_ixy[2 * l] = p.xper ? wrap_index(bx, p.nx) : bx;
    ib.mk_ixy[2 * l + 1] = p.yper ? wrap_index(by, p.ny) : by;
    if (ib.nf > 1) {
      ib.mdf_f[2 * (long long)l] = Fx;
      ib.mdf_f[2 * (long long)l + 1] = Fy;
    }
    if (!isfinite(Fx) || !isfinite(Fy) || !(sqrt(wu * wu + wv * wv) <= 0.3)) p.flag[0] = 1 + ib.mk_body[l];
  }
}

// Forcing pass k >= 1 (eqs 29-31): u*^k = u* + f^k / (2 rho) at the stencil
// nodes, with f^k the spread of the force accumulated over passes 0 .. k-1
// (formed from the markers covering each node with the FP64 weights the
// first pass recorded); then dF = 2 rho_l (U_b - D_I u*^k) and F += dF. The last pass
// leaves F and drs ds F for the lattice kernel. 16 lanes per marker.
template <typename T>
__global__ __launch_bounds__(256) void ib_pass_kernel(LbmParams p, IbParams ib, int k, int last) {
  const int blk = p.xcd_remap ? xcd_tile((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int l = blk * 16 + ((int)threadIdx.x >> 4);
  const int node = (int)threadIdx.x & 15;
  const bool act = l < ib.nm;
  const int S = stencil_size(p.kind);
  const int a = node & 3, c = node >> 2;
  const double *fin = ib.mdf_f + (long long)((k - 1) & 1) * 2 * ib.nm;
  double *fout = ib.mdf_f + (long long)(k & 1) * 2 * ib.nm;
  double wu = 0.0, wv = 0.0;
  if (act && a < S && c < S) {
    const double W = ib.mdf_w[8 * (long long)l + a] * ib.mdf_w[8 * (long long)l + 4 + c];
    const double *cc = ib.mdf_cache + (16 * (long long)l + node) * 3;
    double fx = 0.0, fy = 0.0;
    for (int e = ib.cover_off[16 * l + node]; e < ib.cover_off[16 * l + node + 1]; ++e) {
      const int v = ib.cover_list[e];
      const long long m = v >> 4;
      const double Wm = ib.mdf_w[8 * m + ((v >> 2) & 3)] * ib.mdf_w[8 * m + 4 + (v & 3)] * ib.sdrs[m];
      fx += Wm * fin[2 * m];
      fy += Wm * fin[2 * m + 1];
    }
    wu = W * (cc[1] + 0.5 * fx / cc[0]);
    wv = W * (cc[2] + 0.5 * fy / cc[0]);
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    wu += __shfl_xor(wu, off, 16);
    wv += __shfl_xor(wv, off, 16);
  }
  if (act && node == 0) {
    const double rl = ib.rho_l[l];
    const double Fx = fin[2 * (long long)l] + 2.0 * rl * (ib.U[l] - wu);
    const double Fy = fin[2 * (long long)l + 1] + 2.0 * rl * (ib.V[l] - wv);
    fout[2 * (long long)l] = Fx;
    fout[2 * (long long)l + 1] = Fy;
    if (!isfinite(Fx) || !isfinite(Fy)) p.flag[0] = 1 + ib.mk_body[l];
    if (last) {
      ib.Fx[l] = Fx;
      ib.Fy[l] = Fy;
      const double sd = ib.sdrs[l];
      T *mw = reinterpret_cast<T *>(ib.mk_w) + 10 * (long long)l;
      mw[8] = (T)(Fx * sd);
      mw[9] = (T)(Fy * sd);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) kSgprCap void ib_kernel(const T *__restrict__ A, LbmParams p, IbParams ib) {
  // markers of one body are contiguous and share stencil nodes: consecutive
  // workgroups go to one XCD so its L2 serves the shared population lines
  const int blk = p.xcd_remap ? xcd_tile((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int l = blk * 16 + ((int)threadIdx.x >> 4);
  if (blk == 0 && threadIdx.x == 0) ib.slot[0] = (int)(p.step_ctr[0] % ib.hist_cap);
  ib_marker<T>(A, p, ib, l, l < ib.nm);
}

// Hydrodynamic force and torque on body b (eq 27 with the body's sign): a
// workgroup of NT lanes sums its markers' F_l in a fixed order and writes
// the history ring entry of the step.
template <int NT>
__device__ void body_reduce(const IbParams &ib, int b, int tid, double (*red)[NT / 64]) {
  const int l0 = ib.body_off[b], l1 = ib.body_off[b + 1];
  const double cx = ib.cx[b], cy = ib.cy[b];
  double sfx = 0.0, sfy = 0.0, stz = 0.0;
  const bool per_marker = ib.method == 2;  // RKPM spreads with a factor per marker
  for (int l = l0 + tid; l < l1; l += NT) {
    const double Fx = ib.Fx[l], Fy = ib.Fy[l];
    if (per_marker) {
      const double w = ib.sdrs[l];
      sfx += w * Fx;
      sfy += w * Fy;
      stz += w * ((ib.X[l] - cx) * Fy - (ib.Y[l] - cy) * Fx);
    } else {
      sfx += Fx;
      sfy += Fy;
      stz += (ib.X[l] - cx) * Fy - (ib.Y[l] - cy) * Fx;
    }
  }
  sfx = wave_sum(sfx);
  sfy = wave_sum(sfy);
  stz = wave_sum(stz);
  const int lane = tid & 63, w = tid >> 6;
  if (lane == 0) {
    red[0][w] = sfx;
    red[1][w] = sfy;
    red[2][w] = stz;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < NT / 64; ++k) {
      s0 += red[0][k];
      s1 += red[1][k];
      s2 += red[2][k];
    }
    const double s = per_marker ? 1.0 : ib.body_sdrs[b];
    double *h = ib.hist + ((long long)ib.slot[0] * ib.nb + b) * 3;
    h[0] = -s * s0;
    h[1] = -s * s1;
    h[2] = -s * s2;
  }
}

// ------------------------------------------------------------------ lattice kernel
constexpr int kChunk = 64;  // markers staged in LDS per pass

template <typename T, bool NT>
__device__ __forceinline__ void store(T *ptr, T v) {
  const global_ptr<T> g = (global_ptr<T>)ptr;  // device memory: a global access
  if (NT)
    __builtin_nontemporal_store(v, g);
  else
    *g = v;
}

// A batch case's stop flag (nonzero once the case went unstable), read
// with an atomic load at the start of a workgroup: the read is in flight with
// the population loads and is not moved down to its use. Batch kernels pass
// the case's flag, or kNoStop when unstable cases are not masked, so the load
// needs no branch around it (whose join would wait for it at once). The
// address carries a per-lane zero the compiler cannot see through, so the
// value stays per lane instead of being moved to a scalar register (and
// waited for) right after the load.
__device__ const int kNoStop = 0;
template <bool STOP>
__device__ __forceinline__ int stop_flag(const int *stop) {
  if constexpr (STOP) {
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    return __hip_atomic_load((global_ptr<const int>)stop + zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return 0;
}

// one tile t of the lattice: streaming pull, spread gather, collision; with
// STOP and *stop set, nothing is stored (a stopped batch case)
template <typename T, int BX, int BY, int NPT, bool NT, bool NTL, bool STOP = false>
__device__ __forceinline__ void lbm_tile(const T *__restrict__ A, T *__restrict__ B, const LbmParams &p, int t,
                                         const int *stop = nullptr) {
  constexpr int TX = BX * NPT;
  const int halt = stop_flag<STOP>(stop);
  __shared__ int s_ix[kChunk], s_iy[kChunk];
  __shared__ T s_w[kChunk][10];  // wx[4], wy[4], drs ds F_x, drs ds F_y
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int y = tyi * BY + (int)threadIdx.y;
  const int xb = txi * TX + (int)threadIdx.x;

  // A wave whose nodes and their neighbours need no wrap and no wall takes
  // the interior path: every pull is one load from a wave-uniform base plus
  // the lane's byte offset. A wave spans WR rows of the tile (1 if BX >= 64).
  constexpr int WR = BX >= 64 ? 1 : 64 / BX;
  constexpr int WX = BX >= 64 ? 64 : BX;
  const int yw = __builtin_amdgcn_readfirstlane(y - (BX >= 64 ? 0 : ((int)threadIdx.y % WR)));
  const int xw = __builtin_amdgcn_readfirstlane(BX >= 64 ? txi * TX + ((int)threadIdx.x & ~63) : txi * TX);
  // (a wave that holds column nx-2 of a channel also writes the outlet ghost)
  const bool interior = p.interior && yw >= 1 && yw + WR <= p.ny - 1 && xw >= 1 &&
                        xw + WX + (NPT - 1) * BX <= p.nx - 1 - (p.outlet ? 1 : 0);
  const unsigned rowoff = (unsigned)(y - yw) * (unsigned)p.pitch;

  // the pulls are issued first, so they are in flight while the tile
  // gathers its markers' forces
  T g[NPT][9];
  bool live[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int x = xb + k * BX;
    live[k] = y < p.ny && (interior || (x >= p.i0 && x <= p.i1));
    if (!live[k]) continue;
    // byte offset of the node from the wave's first row: one 32-bit register
    // shared by all loads and stores of the interior path
    const unsigned xoff = (rowoff + (unsigned)x) * (unsigned)sizeof(T);
    if (interior) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const char *base = reinterpret_cast<const char *>(A + (long long)q * p.plane +
                                                          (long long)(yw - ey(q)) * p.pitch - ex(q));
        g[k][q] = load<T, NTL>(reinterpret_cast<const T *>(base + xoff));
      }
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) g[k][q] = pull<T, NTL>(A, p, q, x, y);
    }
  }

  T fib_x[NPT], fib_y[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) fib_x[k] = fib_y[k] = (T)0;

  // spread (eqs 13, 15) as a gather over the markers listed for this tile;
  // the marker kernel left each marker's weights and drs ds F_l
  const int m0 = ldg(p.tile_off, t), m1 = ldg(p.tile_off, t + 1);
  const bool forced = m1 > m0;
  if (forced) {
    const int S = stencil_size(p.kind);
    const int tid = (int)threadIdx.y * BX + (int)threadIdx.x;
    const T *mw = reinterpret_cast<const T *>(p.mk_w);
    for (int c0 = m0; c0 < m1; c0 += kChunk) {
      const int cnt = min(kChunk, m1 - c0);
      __syncthreads();
      if (tid < cnt) {
        const int l = ldg(p.tile_list, c0 + tid);
        s_ix[tid] = ldg(p.mk_ixy, 2 * l);
        s_iy[tid] = ldg(p.mk_ixy, 2 * l + 1);
#pragma unroll
        for (int k = 0; k < 10; ++k) s_w[tid][k] = ldg(mw, 10 * (long long)l + k);
      }
      __syncthreads();
      for (int e = 0; e < cnt; ++e) {
        int dy = y - s_iy[e];
        if (p.yper && dy < 0) dy += p.ny;
        if ((unsigned)dy < (unsigned)S) {
          const T wyv = s_w[e][4 + dy];
#pragma unroll
          for (int k = 0; k < NPT; ++k) {
            int dx = xb + k * BX - s_ix[e];
            if (p.xper && dx < 0) dx += p.nx;
            if ((unsigned)dx < (unsigned)S) {
              const T W = s_w[e][dx] * wyv;
              fib_x[k] += W * s_w[e][8];
              fib_y[k] += W * s_w[e][9];
            }
          }
        }
      }
    }
  }
  if (y >= p.ny || halt) return;  // (after the gather's last barrier)

  const CollK<T> &K = coll<T>(p);
  bool bad = false;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int x = xb + k * BX;
    if (!live[k]) continue;
    const unsigned xoff = (rowoff + (unsigned)x) * (unsigned)sizeof(T);
    T out[9], rho;
    if (forced) {
      const ForceK<T> F = force_terms<T>(K, (T)(p.Gx + (double)fib_x[k]), (T)(p.Gy + (double)fib_y[k]));
      collide<T>(g[k], F, K, out, rho);
    } else {
      collide<T>(g[k], gforce<T>(p), K, out, rho);
    }
    bad |= !rho_ok(rho);
    if (interior) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        char *base = reinterpret_cast<char *>(B + (long long)q * p.plane + (long long)yw * p.pitch);
        store<T, NT>(reinterpret_cast<T *>(base + xoff), out[q]);
      }
      continue;
    }
    const long long base = (long long)y * p.pitch + x;
#pragma unroll
    for (int q = 0; q < 9; ++q) store<T, NT>(&B[(long long)q * p.plane + base], out[q]);
    if (p.inlet && x == 1) {
      // inlet ghost: equilibrium at the inflow velocity, density of column 1
      const T dr = inlet_dr<T>(out);
      const long long gb = (long long)y * p.pitch;
#pragma unroll
      for (int q = 0; q < 9; ++q) B[(long long)q * p.plane + gb] = inlet_ghost_calc<T>(dr, p, q);
    }
    if (p.outlet == 1 && x == p.nx - 2) {
#pragma unroll
      for (int q = 0; q < 9; ++q) B[(long long)q * p.plane + base + 1] = out[q];
    }
  }
  if (bad) p.flag[0] = -1;
}

template <typename T, int BX, int BY, int NPT, bool NT, bool NTL>
__global__ __launch_bounds__(BX *BY) kSgprCap void lbm_kernel(const T *__restrict__ A, T *__restrict__ B,
                                                     LbmParams p, TileRange r, IbParams ib) {
  if ((int)blockIdx.x >= r.count) {  // workgroups past the tiles: one body each, then the step counter
    const int gb = (int)blockIdx.x - r.count;
    if (gb >= ib.nb) {
      if (threadIdx.x == 0 && threadIdx.y == 0) p.step_ctr[0] = p.step_ctr[0] + 1;
      return;
    }
    __shared__ double red[3][BX * BY / 64];
    body_reduce<BX * BY>(ib, gb, (int)threadIdx.y * BX + (int)threadIdx.x, red);
    return;
  }
  // this launch covers tiles map[base .. base+count) (all tiles in order if map is null)
  const int li = p.xcd_remap ? xcd_tile((int)blockIdx.x, r.count) : (int)blockIdx.x;
  const int t = r.map ? r.map[r.base + li] : li;
  lbm_tile<T, BX, BY, NPT, NT, NTL>(A, B, p, t);
}

// ---- batched cases: every tile, marker and body of all cases in one launch each
// (the per-case parameters are the single-case ones, read from a table)

template <typename T, int BX, int BY, int NPT, bool NT, bool NTL>
__global__ __launch_bounds__(BX *BY) kSgprCap void lbm_batch_kernel(const CaseDesc *__restrict__ cases, BatchMap m,
                                                           int rt) {
  if ((int)blockIdx.x >= m.ntiles) {  // one body each, then one step counter per case
    const int gb = (int)blockIdx.x - m.ntiles;
    if (gb >= m.nbodies) {
      if (threadIdx.x == 0 && threadIdx.y == 0) {
        const LbmParams &p = cases[gb - m.nbodies].p;
        // an unstable case counts no step
        if (!stop_flag<true>(m.mask_unstable ? p.flag : &kNoStop)) p.step_ctr[0] = p.step_ctr[0] + 1;
      }
      return;
    }
    const CaseDesc &cd = cases[m.body_case[gb]];
    __shared__ double red[3][BX * BY / 64];
    body_reduce<BX * BY>(cd.ib, m.body_local[gb], (int)threadIdx.y * BX + (int)threadIdx.x, red);
    return;
  }
  const int li = m.xcd_remap ? xcd_tile((int)blockIdx.x, m.ntiles) : (int)blockIdx.x;
  const int c = m.tile_case[li];
  const int t = m.tile_local[li];
  // the case's parameters are copied once into registers, as a kernel
  // argument would be, rather than re-read through the table
  const LbmParams p = cases[c].p;
  const T *A = reinterpret_cast<const T *>(cases[c].pop[route_src(rt)]);
  T *B = reinterpret_cast<T *>(cases[c].pop[route_dst(rt)]);
  // an unstable case stops (stores nothing, counts no step); the others go on
  const int *stop = m.mask_unstable ? p.flag : &kNoStop;
  lbm_tile<T, BX, BY, NPT, NT, NTL, true>(A, B, p, t, stop);
}

template <typename T>
__global__ __launch_bounds__(256) kSgprCap void ib_batch_kernel(const CaseDesc *__restrict__ cases, BatchMap m, int rt) {
  const int blk = m.xcd_remap ? xcd_tile((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int c = m.mblk_case[blk];
  const int first = m.mblk_first[blk];
  const LbmParams p = cases[c].p;
  const IbParams ib = cases[c].ib;
  const T *A = reinterpret_cast<const T *>(cases[c].pop[route_src(rt)]);
  if (m.mask_unstable && p.flag[0] != 0) return;
  if (first == 0 && threadIdx.x == 0) ib.slot[0] = (int)(p.step_ctr[0] % ib.hist_cap);
  const int l = first + ((int)threadIdx.x >> 4);
  ib_marker<T>(A, p, ib, l, l < ib.nm);
}

// ------------------------------------------------------------------ state kernels
// equilibrium (eq 6) of (rho, ux, uy) stored as deviations; fields may be
// per-node (stride 1) or uniform (stride 0)
template <typename T>
__global__ void init_eq_kernel(T *__restrict__ A, LbmParams p, const double *__restrict__ rho,
                               const double *__restrict__ ux, const double *__restrict__ uy,
                               double rho0, int per_node_rho) {
  const long long n = (long long)p.nx * p.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
    const double r = per_node_rho ? rho[k] : rho0;
    const double u = ux[k], v = uy[k];
    const double uu = u * u + v * v;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double eu = ex(q) * u + ey(q) * v;
      const double feq = wq(q) * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
      A[(long long)q * p.plane + (long long)y * p.pitch + x] = (T)(feq - ref_c(q, p.urx, p.ury));
    }
  }
}

template <typename T>
__global__ void init_uniform_kernel(T *__restrict__ A, LbmParams p, double r, double u, double v) {
  const long long n = (long long)p.nx * p.ny;
  const double uu = u * u + v * v;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double eu = ex(q) * u + ey(q) * v;
      const double feq = wq(q) * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
      A[(long long)q * p.plane + (long long)y * p.pitch + x] = (T)(feq - ref_c(q, p.urx, p.ury));
    }
  }
}

// one population plane <-> packed FP64 full values
template <typename T>
__global__ void plane_to_f64_kernel(const T *__restrict__ A, LbmParams p, int q, double *__restrict__ out) {
  const long long n = (long long)p.nx * p.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
    out[k] = (double)A[(long long)q * p.plane + (long long)y * p.pitch + x] + ref_c(q, p.urx, p.ury);
  }
}

template <typename T>
__global__ void f64_to_plane_kernel(T *__restrict__ A, LbmParams p, int q, const double *__restrict__ in) {
  const long long n = (long long)p.nx * p.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
    A[(long long)q * p.plane + (long long)y * p.pitch + x] = (T)(in[k] - ref_c(q, p.urx, p.ury));
  }
}

// macroscopic fields of the current state (see btdf_get_macroscopic)
template <typename T>
__global__ void macro_kernel(const T *__restrict__ A, LbmParams p, double *__restrict__ rho,
                             double *__restrict__ ux, double *__restrict__ uy) {
  const long long n = (long long)p.nx * p.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
    const bool fluid = x >= p.i0 && x <= p.i1;
    double dr = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double g = fluid ? (double)pull(A, p, q, x, y)
                             : (double)A[(long long)q * p.plane + (long long)y * p.pitch + x];
      dr += g;
      mx += ex(q) * g;
      my += ey(q) * g;
    }
    const double r = 1.0 + dr;
    mx += p.urx;  // the stored values' first moment is m - u_ref
    my += p.ury;
    rho[k] = r;
    ux[k] = fluid ? (mx + 0.5 * p.Gx) / r : mx / r;
    uy[k] = fluid ? (my + 0.5 * p.Gy) / r : my / r;
  }
}

// ------------------------------------------------------------------ launchers
template <typename T>
static int grid_for(const LbmParams &p) {
  long long n = (long long)p.nx * p.ny;
  long long b = (n + 255) / 256;
  return (int)(b < 65536 ? b : 65536);
}

template <typename T, int BX, int BY, int NPT, bool NT, bool NTL>
static hipError_t launch_lbm_t(const T *A, T *B, const LbmParams &p, const TileRange &r, const IbParams &ib,
                               hipStream_t s) {
  // the counting launch also reduces the bodies and advances the step
  // counter (one workgroup each past the tiles), whether or not it has tiles
  const int extra = r.count_step ? ib.nb + 1 : 0;
  if (r.count + extra <= 0) return hipSuccess;
  hipLaunchKernelGGL((lbm_kernel<T, BX, BY, NPT, NT, NTL>), dim3(r.count + extra), dim3(BX, BY), 0, s, A, B, p,
                     r, ib);
  return hipGetLastError();
}

// launch shapes: {id, BX, BY, nodes per thread, nontemporal stores, nontemporal loads}
#define BTDF_VARIANTS(X)         \
  X(0, 64, 4, 1, true, false)    \
  X(1, 64, 4, 1, false, false)   \
  X(2, 256, 1, 1, true, false)   \
  X(3, 64, 4, 2, true, false)    \
  X(4, 128, 2, 2, true, false)   \
  X(5, 256, 1, 2, true, false)   \
  X(6, 32, 8, 1, true, false)    \
  X(7, 64, 8, 1, true, false)    \
  X(8, 128, 4, 1, true, false)   \
  X(9, 64, 2, 1, true, false)    \
  X(10, 128, 1, 1, true, false)  \
  X(11, 64, 4, 1, true, true)    \
  X(12, 64, 16, 1, true, false)  \
  X(13, 32, 4, 1, true, false)   \
  X(14, 32, 16, 1, true, false)  \
  X(15, 32, 8, 2, true, false)   \
  X(16, 16, 16, 1, true, false)  \
  X(17, 32, 8, 1, true, true)    \
  X(18, 16, 8, 1, true, false)   \
  X(19, 32, 2, 1, true, false)

int num_variants() { return 20; }

void variant_tile(int v, int *tx, int *ty) {
#define X(id, bx, by, npt, nt, ntl) \
  if (v == id) {                    \
    *tx = bx * npt;                 \
    *ty = by;                       \
    return;                         \
  }
  BTDF_VARIANTS(X)
#undef X
  *tx = 64;
  *ty = 4;
}

template <typename T>
static hipError_t launch_lbm_any(int v, const T *A, T *B, const LbmParams &p, const TileRange &r,
                                 const IbParams &ib, hipStream_t s) {
#define X(id, bx, by, npt, nt, ntl) \
  if (v == id) return launch_lbm_t<T, bx, by, npt, nt, ntl>(A, B, p, r, ib, s);
  BTDF_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_lbm(int prec, int v, const void *A, void *B, const LbmParams &p, const TileRange &r,
                      const IbParams &ib, hipStream_t s) {
  if (prec == 4) return launch_lbm_any<float>(v, (const float *)A, (float *)B, p, r, ib, s);
  return launch_lbm_any<double>(v, (const double *)A, (double *)B, p, r, ib, s);
}

// ---- two steps in one pass (temporal blocking) for tiles away from every marker
//
// A tile whose nodes and their neighbours carry no immersed-boundary force
// advances two steps at once: the workgroup streams and collides step n on
// the tile grown by one node (pulls from A, state n), keeps that state in
// LDS, and streams and collides step n+1 for the tile's own nodes from LDS,
// writing state n+2 to C. Each node is read and written once for two
// updates instead of twice. Only the uniform body force acts there (the
// spread force is zero on and next to such tiles), so both collisions are
// the single-step kernel's, value for value. The host hands over only tiles
// at least two nodes from every domain edge, so no pull wraps or meets a
// wall or a ghost column's update.
// OX x OY output tile worked by BX x BY threads (each thread takes the
// output nodes ii = threadIdx.x + k BX, jj = threadIdx.y + m BY); the map
// holds the id of the tile's first lattice tile (tile_x x tile_y grid).
template <typename T, int OX, int OY, int BX, int BY, bool NT>
__global__ __launch_bounds__(BX *BY) void lbm2_kernel(const T *__restrict__ A, T *__restrict__ C, LbmParams p,
                                                     const int *__restrict__ map, int count, int tile_x,
                                                     int tile_y, T *__restrict__ X,
                                                     const unsigned char *__restrict__ near) {
  constexpr int RX = OX + 2, RY = OY + 2;  // the grown tile
  __shared__ T s_f[9][RY][RX];
  __shared__ __align__(16) unsigned char s_near[3][8];  // near flags of the lattice tiles around the group (0: none)
  const int li = p.xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  const int t = map[li];
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int x0 = txi * tile_x, y0 = tyi * tile_y;
  const int tid = (int)threadIdx.y * BX + (int)threadIdx.x;
  const int W = OX / tile_x;  // lattice tiles in the group (1, 2 or 4), one tile row tall
  // A group never touches a domain edge, so its neighbouring tile positions
  // (rows tyi-1 .. tyi+1, columns txi-1 .. txi+W) all exist; the group's own
  // tiles are not near.
  if (near && tid < 24) {
    const int r = tid >> 3, c = tid & 7;
    s_near[r][c] = (c > W + 1 || (r == 1 && c >= 1 && c <= W)) ? 0 : near[(tyi - 1 + r) * p.ntx + txi - 1 + c];
  }
  const CollK<T> &K = coll<T>(p);
  const ForceK<T> &F = gforce<T>(p);
  bool bad = false;
  // step n on the grown tile: first the OX columns of every grown row, so
  // that consecutive lanes take consecutive, line-aligned nodes of a row,
  // then the two edge columns; two nodes per round, both nodes' loads issued
  // before either collision, so more loads are in flight
  constexpr int TOT = RY * OX + 2 * RY, NTH = BX * BY;
  auto node_of = [&](int k, int &i, int &j) {
    if (k < RY * OX) {
      j = k / OX;
      i = 1 + (k - j * OX);
    } else {
      j = (k - RY * OX) >> 1;
      i = (k & 1) ? OX + 1 : 0;
    }
  };
  for (int k = tid; k < TOT; k += 2 * NTH) {
    int ia, ja, ib, jb;
    node_of(k, ia, ja);
    const bool two = k + NTH < TOT;
    node_of(two ? k + NTH : k, ib, jb);
    // byte offsets of the two nodes from the tile's grown corner (x0-1, y0-1);
    // each pull is then a uniform per-population base plus one of them
    const unsigned oa = (unsigned)(ja * p.pitch + ia) * (unsigned)sizeof(T);
    const unsigned ob = (unsigned)(jb * p.pitch + ib) * (unsigned)sizeof(T);
    T ga[9], gb[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const char *base = reinterpret_cast<const char *>(A + (long long)q * p.plane +
                                                        (long long)(y0 - 1 - ey(q)) * p.pitch + (x0 - 1 - ex(q)));
      ga[q] = load_global<T>(base, oa);
      gb[q] = load_global<T>(base, ob);
    }
    T out[9], rho;
    collide<T>(ga, F, K, out, rho);
    bad |= !rho_ok(rho);
#pragma unroll
    for (int q = 0; q < 9; ++q) s_f[q][ja][ia] = out[q];
    if (two) {
      collide<T>(gb, F, K, out, rho);
      bad |= !rho_ok(rho);
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q][jb][ib] = out[q];
    }
  }
  __syncthreads();
  // whether any neighbouring tile is near (uniform: every lane reads the same words)
  unsigned nw[sizeof s_near / 4];  // the flags as words (s_near is 16-byte aligned)
  __builtin_memcpy(nw, &s_near[0][0], sizeof nw);
  const bool ring = near && (nw[0] | nw[1] | nw[2] | nw[3] | nw[4] | nw[5]) != 0;
  const int sh = __builtin_ctz((unsigned)tile_x);  // tile widths are powers of two
  // step n+1 on the tile's own nodes, pulling from the LDS copy of state n+1
#pragma unroll
  for (int jj = (int)threadIdx.y; jj < OY; jj += BY) {
#pragma unroll
    for (int ii = (int)threadIdx.x; ii < OX; ii += BX) {
      const int i = ii + 1, j = jj + 1;
      T g[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = s_f[q][j - ey(q)][i - ex(q)];
      T out[9], rho;
      collide<T>(g, F, K, out, rho);
      bad |= !rho_ok(rho);
      const unsigned off = (unsigned)(jj * p.pitch + ii) * (unsigned)sizeof(T);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        store_uniform<T, NT>(uniform_ptr(reinterpret_cast<char *>(C + (long long)q * p.plane + (long long)y0 * p.pitch + x0)),
                             off, out[q]);
      }
      // the ring: a node of the group's edge gives X its state n+1 in each
      // direction q whose neighbour (x + e_q) lies in a near tile, the one
      // population that tile's second step pulls from it
      if (ring && (ii == 0 || ii == OX - 1 || jj == 0 || jj == OY - 1)) {
        // the neighbouring tile (row, column in s_near) in each direction
        const int cl = ii == 0 ? 0 : 1 + ((ii - 1) >> sh), cm = 1 + (ii >> sh);
        const int cr = ii == OX - 1 ? W + 1 : 1 + ((ii + 1) >> sh);
        const int rd = jj == 0 ? 0 : 1, ru = jj == OY - 1 ? 2 : 1;
#pragma unroll
        for (int q = 1; q < 9; ++q) {
          const int r = ey(q) < 0 ? rd : (ey(q) > 0 ? ru : 1);
          const int c = ex(q) < 0 ? cl : (ex(q) > 0 ? cr : cm);
          if (s_near[r][c])
            store_uniform<T, false>(
                uniform_ptr(reinterpret_cast<char *>(X + (long long)q * p.plane + (long long)y0 * p.pitch + x0)),
                off, s_f[q][jj + 1][ii + 1]);
        }
      }
    }
  }
  if (bad) p.flag[0] = -1;
}

template <typename T, int OX, int OY, int BX, int BY, bool NT>
static hipError_t launch_lbm2_t(const T *A, T *C, const LbmParams &p, const int *map, int count, int tx, int ty,
                                T *X, const unsigned char *near, hipStream_t s) {
  if constexpr (9 * (OX + 2) * (OY + 2) * sizeof(T) <= 65536) {
    if (count <= 0) return hipSuccess;
    // the group is OX / tx lattice tiles (at most 4, a power of two wide) of one tile row
    if (OX % tx != 0 || OX / tx > 4 || OY != ty || (tx & (tx - 1)) != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((lbm2_kernel<T, OX, OY, BX, BY, NT>), dim3(count), dim3(BX, BY), 0, s, A, C, p, map, count,
                       tx, ty, X, near);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_lbm2_any(int v, int width, const T *A, T *C, const LbmParams &p, const int *map, int count,
                                  T *X, const unsigned char *near, hipStream_t s) {
  int tx, ty;
  variant_tile(v, &tx, &ty);
  // width lattice tiles side by side, one thread per output node
  if (width == 4) {
    if (tx == 32 && ty == 8) return launch_lbm2_t<T, 128, 8, 128, 8, true>(A, C, p, map, count, tx, ty, X, near, s);
    if (tx == 32 && ty == 4) return launch_lbm2_t<T, 128, 4, 128, 4, true>(A, C, p, map, count, tx, ty, X, near, s);
    return hipErrorInvalidValue;
  }
  if (width == 2) {
    if (tx == 32 && ty == 8) return launch_lbm2_t<T, 64, 8, 64, 8, true>(A, C, p, map, count, tx, ty, X, near, s);
    if (tx == 32 && ty == 4) return launch_lbm2_t<T, 64, 4, 64, 4, true>(A, C, p, map, count, tx, ty, X, near, s);
    if (tx == 64 && ty == 4) return launch_lbm2_t<T, 128, 4, 128, 4, true>(A, C, p, map, count, tx, ty, X, near, s);
    return hipErrorInvalidValue;
  }
#define X(id, bx, by, npt, nt, ntl)                                                                   \
  if (v == id)                                                                                      \
    return npt == 1 && width == 1 ? launch_lbm2_t<T, bx, by, bx, by, nt>(A, C, p, map, count, tx, ty, X, near, s)    \
                                  : hipErrorInvalidValue;
  BTDF_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_lbm2(int prec, int v, int width, const void *A, void *C, const LbmParams &p, const int *map,
                       int count, void *X, const unsigned char *near, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == 4)
    return launch_lbm2_any<float>(v, width, (const float *)A, (float *)C, p, map, count, (float *)X, near, s);
  return launch_lbm2_any<double>(v, width, (const double *)A, (double *)C, p, map, count, (double *)X, near, s);
}

// whether a launch shape's two-step pass can also take width (2 or 4) of its tiles side by side
bool variant_has_wide_lbm2(int v, int prec, int width) {
  int tx, ty;
  variant_tile(v, &tx, &ty);
  bool shape = false;
  if (width == 2) shape = (tx == 32 && (ty == 8 || ty == 4)) || (tx == 64 && ty == 4);
  if (width == 4) shape = tx == 32 && (ty == 8 || ty == 4);
  return shape && 9 * (width * tx + 2) * (ty + 2) * prec <= 65536;
}

// ---- three steps per pass (deeper temporal blocking)
// Shapes whose three-step pass fits: the group grown by two in LDS (160 KB
// on gfx950) and its grown-by-one region within two nodes per thread.
template <typename T, int OX, int OY>
constexpr bool lbm3_fits() {
  return 9 * (OX + 4) * (OY + 4) * (int)sizeof(T) + 64 <= 163840 && (OX + 2) * (OY + 2) <= 2 * OX * OY;
}

// Groups of several lattice tiles with a three-step pass: (group code,
// lattice tile, group in nodes). The code is W | H << 4 for W x H tiles.
#define BTDF_LBM3_GROUPS(G) \
  G(kGroup4x1, 32, 8, 128, 8) G(kGroup2x1, 32, 8, 64, 8) G(kGroup2x1, 64, 4, 128, 4)
// groups two tiles tall, on single lattices only: those of passes of five
// steps, for the three steps left over after them
#define BTDF_LBM3_SQUARES(G) G(kGroup2x2, 32, 8, 64, 16) G(kGroup1x2, 32, 8, 32, 16)

__host__ __device__ constexpr bool lbm3_group_ok(int ox, int oy, int tx, int ty) {
  return tx > 0 && ty > 0 && (tx & (tx - 1)) == 0 && (ty & (ty - 1)) == 0 && ox % tx == 0 && oy % ty == 0 &&
         ox / tx <= 4 && (oy == ty || oy == 2 * ty);
}

// Three steps A -> C for a group of lattice tiles OX x OY (W x H tiles,
// W <= 4, H <= 2; one thread per node). Step n+1 is taken over the group grown by two nodes into LDS, step
// n+2 over the group grown by one (into registers, then back into the same
// LDS rows in place), step n+3 over the group into C. The group's edge nodes
// next to a near tile also give X1 their state n+1 and X2 their state n+2
// (only the populations the near tile pulls), where the near tiles' second
// and third steps read them.
template <typename T, int OX, int OY, int BX, int BY, bool NT, bool STOP = false>
__device__ __forceinline__ void lbm3_group(const T *__restrict__ A, T *__restrict__ C, const LbmParams &p, int t,
                                           int tile_x, int tile_y, T *__restrict__ X1, T *__restrict__ X2,
                                           const unsigned char *__restrict__ near, const int *stop) {
  constexpr int RX = OX + 4, RY = OY + 4;  // the group grown by two
  // a stopped batch case stores nothing; every thread still meets every barrier
  const bool keep = !stop_flag<STOP>(stop);
  constexpr int NTH = BX * BY;
  __shared__ T s_f[9][RY][RX];
  __shared__ __align__(16) unsigned char s_near[4][8];
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int x0 = txi * tile_x, y0 = tyi * tile_y;
  const int tid = (int)threadIdx.y * BX + (int)threadIdx.x;
  const int W = OX / tile_x, H = OY / tile_y;
  // the near flags of the tiles around the group: wave 0 issues their loads
  // ahead of its first-step loads and stores them to LDS after those, just
  // before the first barrier (the first point they are read), so no wave
  // waits on them before its own loads go out
  const int nr = tid >> 3, nc = tid & 7;
  unsigned char nflag = 0;
  if (near && tid < 64) {  // wave 0 (uniform)
    // lanes outside the window (and the group's own tiles) read the group's
    // first tile, which is never near: 0 without a select on the loaded value
    const bool nwin = tid < 32 && nc <= W + 1 && nr <= H + 1 && !(nr >= 1 && nr <= H && nc >= 1 && nc <= W);
    const unsigned idx = nwin ? (unsigned)((tyi - 1 + nr) * p.ntx + txi - 1 + nc) : (unsigned)t;
    nflag = __hip_atomic_load((global_ptr<const unsigned char>)near + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const CollK<T> &K = coll<T>(p);
  const ForceK<T> &F = gforce<T>(p);
  bool bad = false;
  // step n+1 over the grown group: the OX central columns of every row
  // first (consecutive lanes on consecutive, line-aligned nodes), then the
  // four edge columns; two nodes per round, loads of both issued first
  constexpr int TOT = RY * OX + 4 * RY;
  auto node_of = [&](int k, int &i, int &j) {
    if (k < RY * OX) {
      j = k / OX;
      i = 2 + (k - j * OX);
    } else {
      const int e = k - RY * OX;
      j = e >> 2;
      const int c = e & 3;
      i = c < 2 ? c : OX + c;
    }
  };
  for (int k = tid; k < TOT; k += 2 * NTH) {
    int ia, ja, ib, jb;
    node_of(k, ia, ja);
    const bool two = k + NTH < TOT;
    node_of(two ? k + NTH : k, ib, jb);
    const unsigned oa = (unsigned)(ja * p.pitch + ia) * (unsigned)sizeof(T);
    const unsigned ob = (unsigned)(jb * p.pitch + ib) * (unsigned)sizeof(T);
    T ga[9], gb[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const char *base = reinterpret_cast<const char *>(A + (long long)q * p.plane +
                                                        (long long)(y0 - 2 - ey(q)) * p.pitch + (x0 - 2 - ex(q)));
      ga[q] = load_global<T>(base, oa);
      gb[q] = load_global<T>(base, ob);
    }
    T out[9], rho;
    collide<T>(ga, F, K, out, rho);
    bad |= !rho_ok(rho);
#pragma unroll
    for (int q = 0; q < 9; ++q) s_f[q][ja][ia] = out[q];
    if (two) {
      collide<T>(gb, F, K, out, rho);
      bad |= !rho_ok(rho);
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q][jb][ib] = out[q];
    }
  }
  if (near && tid < 32) s_near[nr][nc] = nflag;
  __syncthreads();
  unsigned nw[sizeof s_near / 4];  // the flags as words (s_near is 16-byte aligned)
  __builtin_memcpy(nw, &s_near[0][0], sizeof nw);
  const bool ring = near && (nw[0] | nw[1] | nw[2] | nw[3] | nw[4] | nw[5] | nw[6] | nw[7]) != 0;
  const int shx = __builtin_ctz((unsigned)tile_x), shy = __builtin_ctz((unsigned)tile_y);
  // this thread's node of the group, and its ring directions
  const int ii = (int)threadIdx.x, jj = (int)threadIdx.y;
  unsigned rmask = 0;
  if (ring && (ii == 0 || ii == OX - 1 || jj == 0 || jj == OY - 1)) rmask = ring_mask<OX, OY>(s_near, ii, jj, W, H, shx, shy);
  const unsigned off = (unsigned)(jj * p.pitch + ii) * (unsigned)sizeof(T);
  if (rmask && keep) {
    // the eight LDS reads first, so they are in flight together, then the stores
    T v[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) v[q] = s_f[q][jj + 2][ii + 2];
#pragma unroll
    for (int q = 1; q < 9; ++q)
      if (rmask & (1u << q))
        store_uniform<T, false>(
            uniform_ptr(reinterpret_cast<char *>(X1 + (long long)q * p.plane + (long long)y0 * p.pitch + x0)), off,
            v[q]);
  }
  // step n+2 over the group grown by one (at most two nodes per thread)
  constexpr int R2X = OX + 2, TOT2 = R2X * (OY + 2);
  static_assert(TOT2 <= 2 * NTH, "the grown-by-one region takes at most two nodes per thread");
  T o2a[9], o2b[9];
  int pa = -1, pb = -1;  // their R1 positions (j * RX + i), -1: none
  {
    auto step2 = [&](int k2, T (&o)[9]) {
      const int j2 = k2 / R2X, i2 = k2 - j2 * R2X;
      const int i = i2 + 1, j = j2 + 1;
      T g[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = s_f[q][j - ey(q)][i - ex(q)];
      T rho;
      collide<T>(g, F, K, o, rho);
      bad |= !rho_ok(rho);
      return j * RX + i;
    };
    if (tid < TOT2) pa = step2(tid, o2a);
    if (tid + NTH < TOT2) pb = step2(tid + NTH, o2b);
  }
  __syncthreads();
  T *sf = &s_f[0][0][0];
  // (one branch per node: the nine stores of a node under one mask)
  if (pa >= 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) sf[q * RY * RX + pa] = o2a[q];
  }
  if (pb >= 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) sf[q * RY * RX + pb] = o2b[q];
  }
  __syncthreads();
  // step n+3 on the group's own nodes, pulling state n+2 from LDS
  {
    const int i = ii + 2, j = jj + 2;
    T g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = s_f[q][j - ey(q)][i - ex(q)];
    T out[9], rho;
    collide<T>(g, F, K, out, rho);
    bad |= !rho_ok(rho);
    if (!keep) return;  // (after the last barrier)
#pragma unroll
    for (int q = 0; q < 9; ++q)
      store_uniform<T, NT>(uniform_ptr(reinterpret_cast<char *>(C + (long long)q * p.plane + (long long)y0 * p.pitch + x0)),
                           off, out[q]);
    if (rmask) {
      T v[9];
#pragma unroll
      for (int q = 1; q < 9; ++q) v[q] = s_f[q][j][i];
#pragma unroll
      for (int q = 1; q < 9; ++q)
        if (rmask & (1u << q))
          store_uniform<T, false>(
              uniform_ptr(reinterpret_cast<char *>(X2 + (long long)q * p.plane + (long long)y0 * p.pitch + x0)), off,
              v[q]);
    }
  }
  if (bad) p.flag[0] = -1;
}

template <typename T, int OX, int OY, int BX, int BY, bool NT>
__global__ __launch_bounds__(BX *BY) void lbm3_kernel(const T *__restrict__ A, T *__restrict__ C, LbmParams p,
                                                     const int *__restrict__ map, int count, int tile_x,
                                                     int tile_y, T *__restrict__ X1, T *__restrict__ X2,
                                                     const unsigned char *__restrict__ near) {
  const int li = p.xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  lbm3_group<T, OX, OY, BX, BY, NT>(A, C, p, map[li], tile_x, tile_y, X1, X2, near, nullptr);
}

// batches: groups of every case in one launch (a case and its group's first
// tile per workgroup), the buffers and near flags from the case table
template <typename T, int OX, int OY, int BX, int BY, bool NT>
__global__ __launch_bounds__(BX *BY) void lbm3_batch_kernel(const CaseDesc *__restrict__ cases,
                                                           const int *__restrict__ gcase,
                                                           const int *__restrict__ gtile, int count, int rt,
                                                           int mask_unstable, int xcd_remap, int tile_x,
                                                           int tile_y) {
  const int li = xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  const int c = gcase[li];
  const LbmParams p = cases[c].p;
  // an unstable case stops: its workgroups store nothing (the flag is read
  // beside the first loads rather than ahead of them)
  lbm3_group<T, OX, OY, BX, BY, NT, true>(reinterpret_cast<const T *>(cases[c].pop[route_src(rt)]),
                                          reinterpret_cast<T *>(cases[c].pop[route_dst(rt)]), p, gtile[li], tile_x,
                                          tile_y, reinterpret_cast<T *>(cases[c].pop[2]),
                                          reinterpret_cast<T *>(cases[c].pop[3]), cases[c].near,
                                          mask_unstable ? p.flag : &kNoStop);
}

template <typename T, int OX, int OY, int BX, int BY, bool NT>
static hipError_t launch_lbm3_batch_t(const CaseDesc *cases, const int *gcase, const int *gtile, int count, int rt,
                                      int mask, int xcd, int tx, int ty, hipStream_t s) {
  if constexpr (lbm3_fits<T, OX, OY>() && BX == OX && BY == OY) {
    if (count <= 0) return hipSuccess;
    if (!lbm3_group_ok(OX, OY, tx, ty)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((lbm3_batch_kernel<T, OX, OY, BX, BY, NT>), dim3(count), dim3(BX, BY), 0, s, cases, gcase,
                       gtile, count, rt, mask, xcd, tx, ty);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_lbm3_batch_any(int v, int code, const CaseDesc *cases, const int *gcase, const int *gtile,
                                        int count, int rt, int mask, int xcd, hipStream_t s) {
  int tx, ty;
  variant_tile(v, &tx, &ty);
#define ARGS cases, gcase, gtile, count, rt, mask, xcd, tx, ty, s
  if (code != kGroup1x1) {
#define G(c, TX, TY, OX, OY) \
  if (code == c && tx == TX && ty == TY) return launch_lbm3_batch_t<T, OX, OY, OX, OY, true>(ARGS);
    BTDF_LBM3_GROUPS(G)
#undef G
    return hipErrorInvalidValue;
  }
#define X(id, bx, by, npt, nt, ntl) \
  if (v == id) return npt == 1 ? launch_lbm3_batch_t<T, bx, by, bx, by, nt>(ARGS) : hipErrorInvalidValue;
  BTDF_VARIANTS(X)
#undef X
#undef ARGS
  return hipErrorInvalidValue;
}

hipError_t launch_lbm3_batch(int prec, int v, int code, const CaseDesc *cases, const int *gcase, const int *gtile,
                             int count, int rt, int mask, int xcd, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == 4) return launch_lbm3_batch_any<float>(v, code, cases, gcase, gtile, count, rt, mask, xcd, s);
  return launch_lbm3_batch_any<double>(v, code, cases, gcase, gtile, count, rt, mask, xcd, s);
}

template <typename T, int OX, int OY, int BX, int BY, bool NT>
static hipError_t launch_lbm3_t(const T *A, T *C, const LbmParams &p, const int *map, int count, int tx, int ty,
                                T *X1, T *X2, const unsigned char *near, hipStream_t s) {
  if constexpr (lbm3_fits<T, OX, OY>() && BX == OX && BY == OY) {
    if (count <= 0) return hipSuccess;
    if (!lbm3_group_ok(OX, OY, tx, ty)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((lbm3_kernel<T, OX, OY, BX, BY, NT>), dim3(count), dim3(BX, BY), 0, s, A, C, p, map, count,
                       tx, ty, X1, X2, near);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_lbm3_any(int v, int code, const T *A, T *C, const LbmParams &p, const int *map, int count,
                                  T *X1, T *X2, const unsigned char *near, hipStream_t s) {
  int tx, ty;
  variant_tile(v, &tx, &ty);
#define ARGS A, C, p, map, count, tx, ty, X1, X2, near, s
  if (code != kGroup1x1) {
#define G(c, TX, TY, OX, OY) \
  if (code == c && tx == TX && ty == TY) return launch_lbm3_t<T, OX, OY, OX, OY, true>(ARGS);
    BTDF_LBM3_GROUPS(G)
    BTDF_LBM3_SQUARES(G)
#undef G
    return hipErrorInvalidValue;
  }
#define X(id, bx, by, npt, nt, ntl) \
  if (v == id) return npt == 1 ? launch_lbm3_t<T, bx, by, bx, by, nt>(ARGS) : hipErrorInvalidValue;
  BTDF_VARIANTS(X)
#undef X
#undef ARGS
  return hipErrorInvalidValue;
}

hipError_t launch_lbm3(int prec, int v, int code, const void *A, void *C, const LbmParams &p, const int *map,
                       int count, void *X1, void *X2, const unsigned char *near, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == 4)
    return launch_lbm3_any<float>(v, code, (const float *)A, (float *)C, p, map, count, (float *)X1, (float *)X2,
                                  near, s);
  return launch_lbm3_any<double>(v, code, (const double *)A, (double *)C, p, map, count, (double *)X1,
                                 (double *)X2, near, s);
}

// whether a launch shape has a three-step pass over groups of the given
// shape (kGroup*: W x H of its tiles)
bool variant_has_lbm3(int v, int prec, int code) {
  int tx, ty;
  variant_tile(v, &tx, &ty);
  bool fits = false;
  if (code != kGroup1x1) {
#define G(c, TX, TY, OX, OY) \
  if (code == c && tx == TX && ty == TY) fits = prec == 4 ? lbm3_fits<float, OX, OY>() : lbm3_fits<double, OX, OY>();
    BTDF_LBM3_GROUPS(G)
    BTDF_LBM3_SQUARES(G)
#undef G
    return fits;
  }
#define X(id, bx, by, npt, nt, ntl) \
  if (v == id) fits = npt == 1 && (prec == 4 ? lbm3_fits<float, bx, by>() : lbm3_fits<double, bx, by>());
  BTDF_VARIANTS(X)
#undef X
  return fits;
}

// whether a launch shape has a two-step kernel (one node per thread, LDS within 64 KB)
bool variant_has_lbm2(int v, int prec) {
  int tx, ty;
  variant_tile(v, &tx, &ty);
#define X(id, bx, by, npt, nt, ntl) \
  if (v == id) return npt == 1 && 9 * (bx + 2) * (by + 2) * prec <= 65536;
  BTDF_VARIANTS(X)
#undef X
  return false;
}

template <typename T>
static hipError_t launch_lbm_batch_any(int v, const CaseDesc *cases, const BatchMap &m, int rt, hipStream_t s) {
#define X(id, bx, by, npt, nt, ntl)                                                                          \
  if (v == id) {                                                                                           \
    hipLaunchKernelGGL((lbm_batch_kernel<T, bx, by, npt, nt, ntl>), dim3(m.ntiles + m.nbodies + m.ncases),  \
                       dim3(bx, by), 0, s, cases, m, rt);                                                  \
    return hipGetLastError();                                                                              \
  }
  BTDF_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_lbm_batch(int prec, int v, const CaseDesc *cases, const BatchMap &m, int rt, hipStream_t s) {
  if (m.ntiles + m.nbodies + m.ncases <= 0) return hipSuccess;
  if (prec == 4) return launch_lbm_batch_any<float>(v, cases, m, rt, s);
  return launch_lbm_batch_any<double>(v, cases, m, rt, s);
}

hipError_t launch_ib_batch(int prec, const CaseDesc *cases, const BatchMap &m, int rt, hipStream_t s) {
  if (m.nmblk <= 0) return hipSuccess;
  if (prec == 4)
    hipLaunchKernelGGL(ib_batch_kernel<float>, dim3(m.nmblk), dim3(256), 0, s, cases, m, rt);
  else
    hipLaunchKernelGGL(ib_batch_kernel<double>, dim3(m.nmblk), dim3(256), 0, s, cases, m, rt);
  return hipGetLastError();
}

// Convective outlet (d/dt + U d/dx = 0 on the ghost column, implicit
// upwind): after the lattice kernel has written column nx-2 of B, the ghost
// of B is (ghost of A + U column nx-2 of B) / (1 + U). The reference
// offsets of the stored deviations cancel (the weights sum to one). Kept
// out of the lattice kernel, where it cost registers on every node.
template <typename T>
__device__ __forceinline__ void conv_outlet_row(const T *__restrict__ A, T *__restrict__ B, const LbmParams &p,
                                                int y) {
  const T U = (T)p.uconv, den = (T)(1.0 + p.uconv);
  const long long base = (long long)y * p.pitch + p.nx - 2;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const long long o = (long long)q * p.plane + base;
    B[o + 1] = (A[o + 1] + U * B[o]) / den;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void conv_outlet_kernel(const T *__restrict__ A, T *__restrict__ B, LbmParams p) {
  const int y = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (y < p.ny) conv_outlet_row<T>(A, B, p, y);
}

// batches: one workgroup per case, cases without a convective outlet (or stopped) return
template <typename T>
__global__ __launch_bounds__(256) void conv_outlet_batch_kernel(const CaseDesc *__restrict__ cases, int mask_unstable,
                                                                int rt) {
  const CaseDesc &cd = cases[blockIdx.x];
  if (cd.p.outlet != 2 || (mask_unstable && cd.p.flag[0] != 0)) return;
  const T *A = reinterpret_cast<const T *>(cd.pop[route_src(rt)]);
  T *B = reinterpret_cast<T *>(cd.pop[route_dst(rt)]);
  for (int y = (int)threadIdx.x; y < cd.p.ny; y += 256) conv_outlet_row<T>(A, B, cd.p, y);
}

hipError_t launch_conv_outlet(int prec, const void *A, void *B, const LbmParams &p, hipStream_t s) {
  const int blocks = (p.ny + 255) / 256;
  if (prec == 4)
    hipLaunchKernelGGL(conv_outlet_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float *)A, (float *)B, p);
  else
    hipLaunchKernelGGL(conv_outlet_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double *)A, (double *)B, p);
  return hipGetLastError();
}

hipError_t launch_conv_outlet_batch(int prec, const CaseDesc *cases, int ncases, int mask_unstable, int rt,
                                    hipStream_t s) {
  if (prec == 4)
    hipLaunchKernelGGL(conv_outlet_batch_kernel<float>, dim3(ncases), dim3(256), 0, s, cases, mask_unstable, rt);
  else
    hipLaunchKernelGGL(conv_outlet_batch_kernel<double>, dim3(ncases), dim3(256), 0, s, cases, mask_unstable, rt);
  return hipGetLastError();
}

// Rigid motion after a step (eq 4 for a rigid body): each moving body
// advances its centre and angle by one step, and its markers are placed at
// c + R(theta) r_l with the rigid velocity V + omega x (X_l - c), which the
// next step prescribes. One workgroup per body.
__global__ __launch_bounds__(256) void rigid_move_kernel(MoveParams mp) {
#pragma clang fp contract(off)
  const int b = (int)blockIdx.x;
  if (!mp.moving[b]) return;
  double *st = mp.state + 4 * (long long)b;
  const double vx = st[1], vy = st[2], om = st[3];
  const double cx = mp.cx[b] + vx, cy = mp.cy[b] + vy, th = st[0] + om;
  __syncthreads();  // every lane has read the old state
  if (threadIdx.x == 0) {
    mp.cx[b] = cx;
    mp.cy[b] = cy;
    st[0] = th;
  }
  const double c = cos(th), s = sin(th);
  for (int l = mp.body_off[b] + (int)threadIdx.x; l < mp.body_off[b + 1]; l += 256) {
    const double rx = mp.rxy[2 * (long long)l], ry = mp.rxy[2 * (long long)l + 1];
    const double X = cx + c * rx - s * ry;
    const double Y = cy + s * rx + c * ry;
    mp.X[l] = X;
    mp.Y[l] = Y;
    mp.U[l] = vx - om * (Y - cy);
    mp.V[l] = vy + om * (X - cx);
  }
}

hipError_t launch_rigid_move(const MoveParams &mp, hipStream_t s) {
  if (mp.nb == 0) return hipSuccess;
  hipLaunchKernelGGL(rigid_move_kernel, dim3(mp.nb), dim3(256), 0, s, mp);
  return hipGetLastError();
}

// Implicit direct forcing (eq 17): one workgroup per body replaces the
// direct force of its markers (eq 20, left by the marker kernel) by
// (D_I D_E)^-1 times it, with the body's inverse kept column-major, and
// leaves drs ds F_b for the lattice kernel's spread.
template <typename T>
__global__ __launch_bounds__(256) void idf_kernel(LbmParams p, IbParams ib) {
  extern __shared__ double s_f[];  // [2][max_body]
  const int b = (int)blockIdx.x;
  const int l0 = ib.body_off[b], n = ib.body_off[b + 1] - l0;
  for (int i = (int)threadIdx.x; i < n; i += 256) {
    s_f[i] = ib.Fx[l0 + i];
    s_f[ib.max_body + i] = ib.Fy[l0 + i];
  }
  __syncthreads();
  const double *Mt = ib.minv + ib.minv_off[b];
  for (int i = (int)threadIdx.x; i < n; i += 256) {
    double fx = 0.0, fy = 0.0;
    for (int j = 0; j < n; ++j) {
      const double m = Mt[(long long)j * n + i];
      fx += m * s_f[j];
      fy += m * s_f[ib.max_body + j];
    }
    const int l = l0 + i;
    ib.Fx[l] = fx;
    ib.Fy[l] = fy;
    const double sd = ib.sdrs[l];
    T *mw = reinterpret_cast<T *>(ib.mk_w) + 10 * (long long)l;
    mw[8] = (T)(fx * sd);
    mw[9] = (T)(fy * sd);
    if (!isfinite(fx) || !isfinite(fy)) p.flag[0] = 1 + b;
  }
}

// Corrected velocity (eq 11) of the last step interpolated at every marker
// (eq 12): the u_b of the boundary error, eq 45. From the post-collision
// state: the collision leaves rho unchanged and the momentum at m + F (Guo
// forcing), so u = (m' - F/2) / rho with F = G + the spread force, which is
// rebuilt at each stencil node from the covering markers' weights and
// drs ds F_l exactly as the lattice kernel summed it.
// The corrected velocity of the last step at every marker (eqs 11, 12): 16
// lanes per marker, one per stencil node, each rebuilding its node's spread
// force from the markers that cover the node in ascending order, as the
// lattice kernel summed it. TILES = false: those markers come from covering
// lists built on the host (cover_off, cover_list; packed as in AdjParams);
// TILES = true: from the lattice tile lists already on the device (each
// marker of the node's tile tested for covering the node), which needs no
// further buffer. Results go to ux_out[l * stride], uy_out[l * stride].
template <typename T, bool TILES>
__global__ __launch_bounds__(256) void marker_velocity_kernel(const T *__restrict__ A, LbmParams p, IbParams ib,
                                                              const int *__restrict__ coff,
                                                              const int *__restrict__ clist, int tile_x, int tile_y,
                                                              double *ux_out, double *uy_out, int stride) {
  const int l = (int)blockIdx.x * 16 + ((int)threadIdx.x >> 4);
  const int node = (int)threadIdx.x & 15;
  const int a = node & 3, c = node >> 2;
  const int S = stencil_size(p.kind);
  double wu = 0.0, wv = 0.0;
  if (l < ib.nm && a < S && c < S) {
    const double X = ib.X[l], Y = ib.Y[l];
    const int bx = stencil_base(p.kind, X), by = stencil_base(p.kind, Y);
    const double W = phi(p.kind, (double)(bx + a) - X) * phi(p.kind, (double)(by + c) - Y);
    int i = bx + a, j = by + c;
    if (p.xper) i = wrap_index(i, p.nx);
    if (p.yper) j = wrap_index(j, p.ny);
    const long long base = (long long)j * p.pitch + i;
    double drho = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double g = (double)A[(long long)q * p.plane + base];
      drho += g;
      mx += ex(q) * g;
      my += ey(q) * g;
    }
    const T *mw = reinterpret_cast<const T *>(ib.mk_w);
    T fx = (T)0, fy = (T)0;
    if (TILES) {
      const int t = (j / tile_y) * p.ntx + i / tile_x;
      for (int e = p.tile_off[t]; e < p.tile_off[t + 1]; ++e) {
        const int m = p.tile_list[e];
        int dy = j - p.mk_ixy[2 * m + 1];
        if (p.yper && dy < 0) dy += p.ny;
        if ((unsigned)dy >= (unsigned)S) continue;
        int dx = i - p.mk_ixy[2 * m];
        if (p.xper && dx < 0) dx += p.nx;
        if ((unsigned)dx >= (unsigned)S) continue;
        const T *w = mw + 10 * (long long)m;
        const T Wm = w[dx] * w[4 + dy];
        fx += Wm * w[8];
        fy += Wm * w[9];
      }
    } else {
      for (int e = coff[16 * l + node]; e < coff[16 * l + node + 1]; ++e) {
        const int v = clist[e];
        const T *w = mw + 10 * (long long)(v >> 4);
        const T Wm = w[(v >> 2) & 3] * w[4 + (v & 3)];
        fx += Wm * w[8];
        fy += Wm * w[9];
      }
    }
    const double ftx = (double)(T)(p.Gx + (double)fx), fty = (double)(T)(p.Gy + (double)fy);
    const double rho = 1.0 + drho;  // stored deviations: first moment m' - u_ref
    wu = W * ((mx + p.urx - 0.5 * ftx) / rho);
    wv = W * ((my + p.ury - 0.5 * fty) / rho);
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    wu += __shfl_xor(wu, off, 16);
    wv += __shfl_xor(wv, off, 16);
  }
  if (l < ib.nm && node == 0) {
    ux_out[(long long)l * stride] = wu;
    uy_out[(long long)l * stride] = wv;
  }
}

hipError_t launch_marker_velocity(int prec, const void *A, const LbmParams &p, const IbParams &ib,
                                  const int *cover_off, const int *cover_list, double *out, hipStream_t s) {
  if (ib.nm == 0) return hipSuccess;
  const int blocks = (ib.nm + 15) / 16;
  if (prec == 4)
    hipLaunchKernelGGL((marker_velocity_kernel<float, false>), dim3(blocks), dim3(256), 0, s, (const float *)A, p,
                       ib, cover_off, cover_list, 0, 0, out, out + 1, 2);
  else
    hipLaunchKernelGGL((marker_velocity_kernel<double, false>), dim3(blocks), dim3(256), 0, s, (const double *)A,
                       p, ib, cover_off, cover_list, 0, 0, out, out + 1, 2);
  return hipGetLastError();
}

hipError_t launch_marker_velocity_tiles(int prec, const void *A, const LbmParams &p, const IbParams &ib, int tile_x,
                                        int tile_y, double *ux, double *uy, hipStream_t s) {
  if (ib.nm == 0) return hipSuccess;
  if (tile_x <= 0 || tile_y <= 0) return hipErrorInvalidValue;
  const int blocks = (ib.nm + 15) / 16;
  if (prec == 4)
    hipLaunchKernelGGL((marker_velocity_kernel<float, true>), dim3(blocks), dim3(256), 0, s, (const float *)A, p,
                       ib, nullptr, nullptr, tile_x, tile_y, ux, uy, 1);
  else
    hipLaunchKernelGGL((marker_velocity_kernel<double, true>), dim3(blocks), dim3(256), 0, s, (const double *)A, p,
                       ib, nullptr, nullptr, tile_x, tile_y, ux, uy, 1);
  return hipGetLastError();
}

hipError_t launch_ib(int prec, const void *A, const LbmParams &p, const IbParams &ib, hipStream_t s) {
  if (ib.nm == 0) return hipSuccess;
  const int blocks = (ib.nm + 15) / 16;
  if (prec == 4)
    hipLaunchKernelGGL(ib_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float *)A, p, ib);
  else
    hipLaunchKernelGGL(ib_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double *)A, p, ib);
  if (ib.method == 1 && ib.nb > 0) {  // implicit direct forcing, one workgroup per body
    const size_t lds = 2 * (size_t)ib.max_body * sizeof(double);
    if (prec == 4)
      hipLaunchKernelGGL(idf_kernel<float>, dim3(ib.nb), dim3(256), lds, s, p, ib);
    else
      hipLaunchKernelGGL(idf_kernel<double>, dim3(ib.nb), dim3(256), lds, s, p, ib);
  }
  for (int k = 1; k < ib.nf; ++k) {  // further forcing passes
    const int last = k == ib.nf - 1;
    if (prec == 4)
      hipLaunchKernelGGL(ib_pass_kernel<float>, dim3(blocks), dim3(256), 0, s, p, ib, k, last);
    else
      hipLaunchKernelGGL(ib_pass_kernel<double>, dim3(blocks), dim3(256), 0, s, p, ib, k, last);
  }
  return hipGetLastError();
}

hipError_t launch_init_uniform(int prec, void *A, const LbmParams &p, double r, double u, double v,
                               hipStream_t s) {
  if (prec == 4)
    hipLaunchKernelGGL(init_uniform_kernel<float>, dim3(grid_for<float>(p)), dim3(256), 0, s,
                       (float *)A, p, r, u, v);
  else
    hipLaunchKernelGGL(init_uniform_kernel<double>, dim3(grid_for<double>(p)), dim3(256), 0, s,
                       (double *)A, p, r, u, v);
  return hipGetLastError();
}

hipError_t launch_init_eq(int prec, void *A, const LbmParams &p, const double *rho, const double *ux,
                          const double *uy, double rho0, int per_node_rho, hipStream_t s) {
  if (prec == 4)
    hipLaunchKernelGGL(init_eq_kernel<float>, dim3(grid_for<float>(p)), dim3(256), 0, s, (float *)A, p,
                       rho, ux, uy, rho0, per_node_rho);
  else
    hipLaunchKernelGGL(init_eq_kernel<double>, dim3(grid_for<double>(p)), dim3(256), 0, s, (double *)A,
                       p, rho, ux, uy, rho0, per_node_rho);
  return hipGetLastError();
}

hipError_t launch_plane_to_f64(int prec, const void *A, const LbmParams &p, int q, double *out,
                               hipStream_t s) {
  if (prec == 4)
    hipLaunchKernelGGL(plane_to_f64_kernel<float>, dim3(grid_for<float>(p)), dim3(256), 0, s,
                       (const float *)A, p, q, out);
  else
    hipLaunchKernelGGL(plane_to_f64_kernel<double>, dim3(grid_for<double>(p)), dim3(256), 0, s,
                       (const double *)A, p, q, out);
  return hipGetLastError();
}

hipError_t launch_f64_to_plane(int prec, void *A, const LbmParams &p, int q, const double *in,
                               hipStream_t s) {
  if (prec == 4)
    hipLaunchKernelGGL(f64_to_plane_kernel<float>, dim3(grid_for<float>(p)), dim3(256), 0, s,
                       (float *)A, p, q, in);
  else
    hipLaunchKernelGGL(f64_to_plane_kernel<double>, dim3(grid_for<double>(p)), dim3(256), 0, s,
                       (double *)A, p, q, in);
  return hipGetLastError();
}

hipError_t launch_macro(int prec, const void *A, const LbmParams &p, double *rho, double *ux, double *uy,
                        hipStream_t s) {
  if (prec == 4)
    hipLaunchKernelGGL(macro_kernel<float>, dim3(grid_for<float>(p)), dim3(256), 0, s,
                       (const float *)A, p, rho, ux, uy);
  else
    hipLaunchKernelGGL(macro_kernel<double>, dim3(grid_for<double>(p)), dim3(256), 0, s,
                       (const double *)A, p, rho, ux, uy);
  return hipGetLastError();
}

}  // namespace btdf
