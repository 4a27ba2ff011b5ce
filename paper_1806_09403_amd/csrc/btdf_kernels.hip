// btdf_kernels.hip -- gfx950 kernels of one BTDF-IB-LBM time step.
//
//   ib_kernel   one workgroup per body: interpolation of rho and the
//               unforced velocity u* to the markers (eqs 12, 14) from the
//               streamed populations at the stencil nodes (eqs 9-10, u*
//               including G/2), the direct force F_l = 2 rho_l (U_b - u*_l)
//               (eq 20), and the per-body sums of eq 27 (force and torque)
//               by wavefront shuffles, written to the history ring.
//   lbm_kernel  one thread per node (NPT nodes per thread along x): the
//               streaming pull, moments, the spread force of the markers
//               whose stencils touch the tile (eqs 13, 15, gathered from the
//               tile's marker list in LDS -- no atomics, fixed summation
//               order), the corrected velocity (eq 11), equilibrium (eq 6),
//               Guo term (eq 7) and BGK collision (eq 5), and the channel
//               ghost columns.
//
// Populations are stored as deviations f~_q = f_q - w_q (rho0 = 1) in
// structure-of-arrays planes [q][y][pitch]; sums of deviations keep the
// FP32 path free of the cancellation against w_q.
#include "btdf_device.h"
#include "btdf_launch.h"

namespace btdf {

// ------------------------------------------------------------------ marker kernel
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void ib_kernel(const T *__restrict__ A, LbmParams p, IbParams ib) {
  __shared__ double red[3][4];
  const int b = blockIdx.x;
  const int l0 = ib.body_off[b], l1 = ib.body_off[b + 1];
  const double cx = ib.cx[b], cy = ib.cy[b];
  const int S = stencil_size(p.kind);
  double sfx = 0.0, sfy = 0.0, stz = 0.0;
  int bad = 0;
  for (int l = l0 + (int)threadIdx.x; l < l1; l += blockDim.x) {
    const double X = ib.X[l], Y = ib.Y[l];
    const int bx = stencil_base(p.kind, X), by = stencil_base(p.kind, Y);
    double wx[4], wy[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      wx[a] = a < S ? phi(p.kind, (double)(bx + a) - X) : 0.0;
      wy[a] = a < S ? phi(p.kind, (double)(by + a) - Y) : 0.0;
    }
    // stencil origin inside the grid; in a periodic direction a node index
    // past the end then needs one subtraction (S <= 4 < 8 <= nx, ny)
    const int bxw = p.xper ? ((bx % p.nx) + p.nx) % p.nx : bx;
    const int byw = p.yper ? ((by % p.ny) + p.ny) % p.ny : by;
    double rl = 0.0, ul = 0.0, vl = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= S) break;
      int j = byw + c;
      if (j >= p.ny) j -= p.ny;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a >= S) break;
        int i = bxw + a;
        if (i >= p.nx) i -= p.nx;
        double drho = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const double g = (double)pull(A, p, q, i, j);
          drho += g;
          mx += ex(q) * g;
          my += ey(q) * g;
        }
        const double rho = 1.0 + drho;
        const double W = wx[a] * wy[c];
        rl += W * rho;
        ul += W * ((mx + 0.5 * p.Gx) / rho);
        vl += W * ((my + 0.5 * p.Gy) / rho);
      }
    }
    const double Fx = 2.0 * rl * (ib.U[l] - ul);
    const double Fy = 2.0 * rl * (ib.V[l] - vl);
    ib.Fx[l] = Fx;
    ib.Fy[l] = Fy;
    ib.rho_l[l] = rl;
    ib.ux_l[l] = ul;
    ib.uy_l[l] = vl;
    if (!isfinite(Fx) || !isfinite(Fy) || !(sqrt(ul * ul + vl * vl) <= 0.3)) bad = 1;
    sfx += Fx;
    sfy += Fy;
    stz += (X - cx) * Fy - (Y - cy) * Fx;
  }
  if (bad) p.flag[0] = 1 + b;
  sfx = wave_sum(sfx);
  sfy = wave_sum(sfy);
  stz = wave_sum(stz);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = sfx;
    red[1][w] = sfy;
    red[2][w] = stz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nw; ++k) {
      s0 += red[0][k];
      s1 += red[1][k];
      s2 += red[2][k];
    }
    const double s = ib.body_sdrs[b];
    const long long slot = p.step_ctr[0] % ib.hist_cap;
    double *h = ib.hist + (slot * ib.nb + b) * 3;
    h[0] = -s * s0;
    h[1] = -s * s1;
    h[2] = -s * s2;
  }
}

// ------------------------------------------------------------------ lattice kernel
constexpr int kChunk = 64;  // markers staged in LDS per pass

template <typename T, int BX, int BY, int NPT, bool NT>
__global__ __launch_bounds__(BX *BY) void lbm_kernel(const T *__restrict__ A, T *__restrict__ B,
                                                     LbmParams p) {
  constexpr int TX = BX * NPT;
  __shared__ int s_ix[kChunk], s_iy[kChunk];
  __shared__ double s_wx[kChunk][4], s_wy[kChunk][4], s_fx[kChunk], s_fy[kChunk];

  const int nblk = p.ntx * p.nty;
  const int t = p.xcd_remap ? xcd_tile((int)blockIdx.x, nblk) : (int)blockIdx.x;
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int y = tyi * BY + (int)threadIdx.y;
  const int xb = txi * TX + (int)threadIdx.x;

  double fib_x[NPT], fib_y[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) fib_x[k] = fib_y[k] = 0.0;

  // spread (eqs 13, 15) as a gather over the markers listed for this tile
  const int m0 = p.tile_off[t], m1 = p.tile_off[t + 1];
  if (m1 > m0) {
    const int S = stencil_size(p.kind);
    const int tid = (int)threadIdx.y * BX + (int)threadIdx.x;
    for (int c0 = m0; c0 < m1; c0 += kChunk) {
      const int cnt = min(kChunk, m1 - c0);
      __syncthreads();
      if (tid < cnt) {
        const int l = p.tile_list[c0 + tid];
        const double X = p.X[l], Y = p.Y[l];
        int bx = stencil_base(p.kind, X), by = stencil_base(p.kind, Y);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          s_wx[tid][a] = a < S ? phi(p.kind, (double)(bx + a) - X) : 0.0;
          s_wy[tid][a] = a < S ? phi(p.kind, (double)(by + a) - Y) : 0.0;
        }
        if (p.xper) bx = ((bx % p.nx) + p.nx) % p.nx;
        if (p.yper) by = ((by % p.ny) + p.ny) % p.ny;
        s_ix[tid] = bx;
        s_iy[tid] = by;
        const double s = p.sdrs[l];
        s_fx[tid] = p.Fx[l] * s;
        s_fy[tid] = p.Fy[l] * s;
      }
      __syncthreads();
      for (int e = 0; e < cnt; ++e) {
        int dy = y - s_iy[e];
        if (p.yper && dy < 0) dy += p.ny;
        if ((unsigned)dy < (unsigned)S) {
          const double wyv = s_wy[e][dy];
#pragma unroll
          for (int k = 0; k < NPT; ++k) {
            int dx = xb + k * BX - s_ix[e];
            if (p.xper && dx < 0) dx += p.nx;
            if ((unsigned)dx < (unsigned)S) {
              const double W = s_wx[e][dx] * wyv;
              fib_x[k] += W * s_fx[e];
              fib_y[k] += W * s_fy[e];
            }
          }
        }
      }
    }
  }
  if (y >= p.ny) return;

  const T omega = (T)p.omega, guo = (T)p.guo;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int x = xb + k * BX;
    if (x < p.i0 || x > p.i1) continue;
    T g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = pull(A, p, q, x, y);
    T drho = g[0];
#pragma unroll
    for (int q = 1; q < 9; ++q) drho += g[q];
    const T rho = (T)1 + drho;
    const T mx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const T my = (g[2] - g[4]) + (g[5] - g[8]) + (g[6] - g[7]);
    const T ftx = (T)(p.Gx + fib_x[k]);
    const T fty = (T)(p.Gy + fib_y[k]);
    const T inv = (T)1 / rho;
    const T ux = (mx + (T)0.5 * ftx) * inv;
    const T uy = (my + (T)0.5 * fty) * inv;
    const T uu = ux * ux + uy * uy;
    bad |= !(rho > (T)0) || !isfinite(rho);
    const long long base = (long long)y * p.pitch + x;
    T out[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const T w = (T)wq(q);
      const T eu = (T)ex(q) * ux + (T)ey(q) * uy;
      const T P = (T)3 * eu + (T)4.5 * eu * eu - (T)1.5 * uu;
      const T feq = w * (drho + rho * P);  // deviation of eq 6 from w_q
      const T Fq = guo * w *
                   (((T)3 * ((T)ex(q) - ux) + (T)9 * eu * (T)ex(q)) * ftx +
                    ((T)3 * ((T)ey(q) - uy) + (T)9 * eu * (T)ey(q)) * fty);
      out[q] = g[q] - omega * (g[q] - feq) + Fq;
      if (NT)
        __builtin_nontemporal_store(out[q], &B[(long long)q * p.plane + base]);
      else
        B[(long long)q * p.plane + base] = out[q];
    }
    if (p.inlet && x == 1) {
      // inlet ghost: equilibrium at the inflow velocity, density of column 1
      T dr = out[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) dr += out[q];
      const T r = (T)1 + dr;
      const T ui = (T)p.uin_x, vi = (T)p.uin_y;
      const T uui = ui * ui + vi * vi;
      const long long gb = (long long)y * p.pitch;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const T eu = (T)ex(q) * ui + (T)ey(q) * vi;
        B[(long long)q * p.plane + gb] =
            (T)wq(q) * (dr + r * ((T)3 * eu + (T)4.5 * eu * eu - (T)1.5 * uui));
      }
    }
    if (p.outlet && x == p.nx - 2) {
#pragma unroll
      for (int q = 0; q < 9; ++q) B[(long long)q * p.plane + base + 1] = out[q];
    }
  }
  if (bad) p.flag[0] = -1;
  if (t == 0 && threadIdx.x == 0 && threadIdx.y == 0) p.step_ctr[0] = p.step_ctr[0] + 1;
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
      A[(long long)q * p.plane + (long long)y * p.pitch + x] = (T)(feq - wq(q));
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
      A[(long long)q * p.plane + (long long)y * p.pitch + x] = (T)(feq - wq(q));
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
    out[k] = (double)A[(long long)q * p.plane + (long long)y * p.pitch + x] + wq(q);
  }
}

template <typename T>
__global__ void f64_to_plane_kernel(T *__restrict__ A, LbmParams p, int q, const double *__restrict__ in) {
  const long long n = (long long)p.nx * p.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
    A[(long long)q * p.plane + (long long)y * p.pitch + x] = (T)(in[k] - wq(q));
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

template <typename T, int BX, int BY, int NPT, bool NT>
static hipError_t launch_lbm_t(const T *A, T *B, const LbmParams &p, hipStream_t s) {
  const int nblk = p.ntx * p.nty;
  hipLaunchKernelGGL((lbm_kernel<T, BX, BY, NPT, NT>), dim3(nblk), dim3(BX, BY), 0, s, A, B, p);
  return hipGetLastError();
}

// launch shapes: {BX, BY, NPT, nontemporal}
#define BTDF_VARIANTS(X) \
  X(0, 64, 4, 1, false)  \
  X(1, 256, 1, 1, false) \
  X(2, 64, 4, 2, false)  \
  X(3, 128, 2, 2, false) \
  X(4, 256, 1, 2, false) \
  X(5, 64, 4, 1, true)   \
  X(6, 256, 1, 1, true)  \
  X(7, 64, 4, 2, true)   \
  X(8, 128, 2, 2, true)  \
  X(9, 256, 1, 2, true)

int num_variants() { return 10; }

void variant_tile(int v, int *tx, int *ty) {
#define X(id, bx, by, npt, nt) \
  if (v == id) {               \
    *tx = bx * npt;            \
    *ty = by;                  \
    return;                    \
  }
  BTDF_VARIANTS(X)
#undef X
  *tx = 64;
  *ty = 4;
}

template <typename T>
static hipError_t launch_lbm_any(int v, const T *A, T *B, const LbmParams &p, hipStream_t s) {
#define X(id, bx, by, npt, nt) \
  if (v == id) return launch_lbm_t<T, bx, by, npt, nt>(A, B, p, s);
  BTDF_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_lbm(int prec, int v, const void *A, void *B, const LbmParams &p, hipStream_t s) {
  if (prec == 4) return launch_lbm_any<float>(v, (const float *)A, (float *)B, p, s);
  return launch_lbm_any<double>(v, (const double *)A, (double *)B, p, s);
}

hipError_t launch_ib(int prec, const void *A, const LbmParams &p, const IbParams &ib, int threads,
                     hipStream_t s) {
  if (ib.nb == 0) return hipSuccess;
  if (prec == 4)
    hipLaunchKernelGGL(ib_kernel<float>, dim3(ib.nb), dim3(threads), 0, s, (const float *)A, p, ib);
  else
    hipLaunchKernelGGL(ib_kernel<double>, dim3(ib.nb), dim3(threads), 0, s, (const double *)A, p, ib);
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
