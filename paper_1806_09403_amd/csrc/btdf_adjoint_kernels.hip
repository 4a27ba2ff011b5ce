// btdf_adjoint_kernels.hip -- gfx950 kernels of the reverse (adjoint) step.
//
// One forward step maps the post-collision populations A_t to A_{t+1} and
// emits the body forces of eq 27. Its adjoint, for a scalar J built from the
// force history, maps dJ/dA_{t+1} to dJ/dA_t and adds the step's share of
// the parameter gradients. The state of the reverse sweep is kept in the
// form of the streamed populations: G_t = dJ/dg_t, g being the populations
// after the streaming pull of step t. dJ/dA_t is never stored: it is read
// from G_t by the transpose of the pull (pull_adj), which has the same
// shifted-read pattern as the forward pull, so the lattice kernel writes its
// planes aligned, one node per thread, as the forward lattice kernel does.
//
// Per reversed step, with the step's marker values (weights, drs ds F_l,
// rho_l, u*_l) recorded by the forward marker kernel:
//   adj_marker_kernel   16 lanes per marker, one per stencil node: each lane
//                       forms at its node the forward values and dJ/df
//                       (the transposed collision, as the lattice kernel
//                       does), then the marker's transposes of spreading
//                       (eqs 13, 15) and eq 27 -> dJ/dF_l, of the direct
//                       force (eq 20) -> dJ/drho_l, dJ/du*_l, and the
//                       position (phi') and marker-velocity gradients.
//   adj_lattice_kernel  every node: dJ/dA_{t+1} by pull_adj (plus the channel
//                       ghost columns), the transposed collision (eqs 5-7,
//                       11) and, at nodes a marker stencil covers, the
//                       transposed interpolation (eqs 12, 14) of the
//                       markers' dJ/drho_l, dJ/du*_l -> G_t; per-tile sums of
//                       dJ/dG and dJ/du_in.
// After the last reversed step adj_unpull_kernel turns G_0 into dJ/dA_0.
#include <algorithm>

#include "btdf_device.h"
#include "btdf_launch.h"

namespace btdf {

constexpr int kAdjChunk = 64;  // markers staged in LDS per pass

// Transpose of the streaming pull, read as a pull: the adjoint of A_q at
// node (x, y) is G_q of the fluid node that read it -- the neighbour
// (x, y) + e_q, or next to a wall the bounce-back of (x, y) itself in the
// opposite direction -- and 0 when no fluid node reads it.
template <typename T>
__device__ __forceinline__ T pull_adj(const T *__restrict__ G, const LbmParams &p, int q, int x, int y) {
  int zx = x + ex(q), zy = y + ey(q);
  if (p.yper) {
    zy = zy < 0 ? zy + p.ny : (zy >= p.ny ? zy - p.ny : zy);
  } else if (zy < 0 || zy >= p.ny) {
    if (x < p.i0 || x > p.i1) return (T)0;
    return G[(long long)opp(q) * p.plane + (long long)y * p.pitch + x];
  }
  if (p.xper)
    zx = zx < 0 ? zx + p.nx : (zx >= p.nx ? zx - p.nx : zx);
  else if (zx < p.i0 || zx > p.i1)
    return (T)0;
  return G[(long long)q * p.plane + (long long)zy * p.pitch + zx];
}

// Forward values at fluid node (x, y) from the streamed deviations g and the
// total force f (eqs 9-11): rho, the full first moment m, u = (m + f/2)/rho.
struct NodeFwd {
  double rho, mx, my, ux, uy;
};
template <typename Gv>
__device__ __forceinline__ NodeFwd node_forward(const Gv gv[9], double ftx, double fty, const LbmParams &p) {
  NodeFwd n;
  double g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) g[q] = (double)gv[q];
  const double drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  n.rho = 1.0 + drho;
  // stored values are deviations from feq(1, u_ref): their first moment is m - u_ref
  n.mx = ((g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7])) + p.urx;
  n.my = ((g[2] - g[4]) + (g[5] - g[8]) + (g[6] - g[7])) + p.ury;
  n.ux = (n.mx + 0.5 * ftx) / n.rho;
  n.uy = (n.my + 0.5 * fty) / n.rho;
  return n;
}

// dJ/dB at fluid node (x, y): the transpose of the next step's pull, plus
// the channel ghost columns this node's collision also wrote. With sU, the
// inlet's dJ/du_in share is added there.
template <typename T, typename Gv>
__device__ __forceinline__ void node_dJdB(const T *__restrict__ Gn, const LbmParams &p, int x, int y,
                                          const Gv g[9], T bb[9], double *sUx, double *sUy) {
#pragma unroll
  for (int q = 0; q < 9; ++q) bb[q] = pull_adj<T>(Gn, p, q, x, y);
  if (p.outlet && x == p.nx - 2) {  // B(nx-1, y) = B(nx-2, y)
#pragma unroll
    for (int q = 0; q < 9; ++q) bb[q] += pull_adj<T>(Gn, p, q, x + 1, y);
  }
  if (p.inlet && x == 1) {
    // B_q(0, y) = feq_q(rho_B, u_in) - c_q with rho_B the density of column 1
    // after collision, which the collision leaves equal to rho
    double rB = 1.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) rB += (double)g[q];
    const double ui = p.uin_x, vi = p.uin_y, uui = ui * ui + vi * vi;
    double rbB = 0.0, su = 0.0, sv = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double a0 = (double)pull_adj<T>(Gn, p, q, 0, y);
      const double eu = ex(q) * ui + ey(q) * vi;
      rbB += a0 * wq(q) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uui);
      su += a0 * wq(q) * rB * (3.0 * ex(q) + 9.0 * eu * ex(q) - 3.0 * ui);
      sv += a0 * wq(q) * rB * (3.0 * ey(q) + 9.0 * eu * ey(q) - 3.0 * vi);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) bb[q] = (T)((double)bb[q] + rbB);
    if (sUx) {
      *sUx += su;
      *sUy += sv;
    }
  }
}

// Weighted moments of dJ/dB at a node: s0 = sum w b, s1 = sum w b e,
// S2 = sum w b e e (the transposed collision needs no more of dJ/dB).
struct Mom {
  double s0 = 0.0, s1x = 0.0, s1y = 0.0, Sxx = 0.0, Sxy = 0.0, Syy = 0.0;
  __device__ __forceinline__ void add(int q, double bq) {
    const double b = wq(q) * bq;
    s0 += b;
    s1x += ex(q) * b;
    s1y += ey(q) * b;
    Sxx += (ex(q) * ex(q)) * b;
    Sxy += (ex(q) * ey(q)) * b;
    Syy += (ey(q) * ey(q)) * b;
  }
  // the same shift added to every direction: sum w = 1, sum w e = 0, sum w e e = I/3
  __device__ __forceinline__ void add_uniform(double c) {
    s0 += c;
    Sxx += c / 3.0;
    Syy += c / 3.0;
  }
};

// Transpose of out_q = (1 - omega) g_q + omega feq_q(rho, u) + F_q(u, f),
// u = (m + f/2) / rho (eqs 5-7, 11), at one node, from the moments of
// dJ/dB. Gives dJ/df and the parts of dJ/dg_q = (1 - omega) b_q + drb + e_q.mb.
struct CollideAdj {
  double fbx, fby, drb, mbx, mby;
};
__device__ __forceinline__ CollideAdj collide_adjoint(const NodeFwd &n, double ftx, double fty, const Mom &m,
                                                      const LbmParams &p) {
  const double omega = p.omega, guo = p.guo, ux = n.ux, uy = n.uy, inv = 1.0 / n.rho;
  const double Sux = m.Sxx * ux + m.Sxy * uy, Suy = m.Sxy * ux + m.Syy * uy;      // S2 u
  const double Sfx = m.Sxx * ftx + m.Sxy * fty, Sfy = m.Sxy * ftx + m.Syy * fty;  // S2 f
  const double su = m.s1x * ux + m.s1y * uy, uSu = ux * Sux + uy * Suy, uu = ux * ux + uy * uy;
  const double drb = omega * (m.s0 + 3.0 * su + 4.5 * uSu - 1.5 * uu * m.s0);  // d/d rho at fixed u
  const double orho = omega * n.rho;
  const double ubx = orho * (3.0 * m.s1x + 9.0 * Sux - 3.0 * ux * m.s0) + guo * (-3.0 * ftx * m.s0 + 9.0 * Sfx);
  const double uby = orho * (3.0 * m.s1y + 9.0 * Suy - 3.0 * uy * m.s0) + guo * (-3.0 * fty * m.s0 + 9.0 * Sfy);
  const double fbx = guo * (3.0 * m.s1x - 3.0 * ux * m.s0 + 9.0 * Sux);
  const double fby = guo * (3.0 * m.s1y - 3.0 * uy * m.s0 + 9.0 * Suy);
  CollideAdj r;
  r.mbx = ubx * inv;
  r.mby = uby * inv;
  r.fbx = fbx + 0.5 * r.mbx;
  r.fby = fby + 0.5 * r.mby;
  r.drb = drb - (ubx * ux + uby * uy) * inv;
  return r;
}

// sum over the workgroup of 4 values (one per wave, then wave 0), added by
// thread 0 to dst[0..3]; every thread of the (64 x 4) workgroup calls it
__device__ __forceinline__ void block_add4(double v0, double v1, double v2, double v3, double *dst) {
  __shared__ double red[4][4];
  const int tid = (int)threadIdx.y * 64 + (int)threadIdx.x;
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  v2 = wave_sum(v2);
  v3 = wave_sum(v3);
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = v0;
    red[tid >> 6][1] = v1;
    red[tid >> 6][2] = v2;
    red[tid >> 6][3] = v3;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] += ((red[0][k] + red[1][k]) + (red[2][k] + red[3][k]));
  }
}

// The spread force at the node of marker l's stencil lane k, as the forward
// lattice kernel forms it: the recorded weights and drs ds F of the markers
// covering the node, summed in ascending marker order in the population type.
template <typename T>
__device__ __forceinline__ void node_spread_force(const LbmParams &p, const AdjParams &a, int l, int k, T *fx,
                                                  T *fy) {
  const T *mw = reinterpret_cast<const T *>(p.mk_w);
  T sx = (T)0, sy = (T)0;
  const int c0 = a.node_off[16 * l + k], c1 = a.node_off[16 * l + k + 1];
#pragma unroll 4
  for (int c = c0; c < c1; ++c) {
    const int e = a.node_list[c];
    const T *w = mw + 10 * (long long)(e >> 4);
    const T W = w[(e >> 2) & 3] * w[4 + (e & 3)];
    sx += W * w[8];
    sy += W * w[9];
  }
  *fx = sx;
  *fy = sy;
}

// 16 lanes per marker (one per node of the up to 4 x 4 stencil), 16 markers
// per workgroup; every lane runs the shuffles, inactive lanes with zeros
template <typename T>
__global__ __launch_bounds__(256) void adj_marker_kernel(const T *__restrict__ A, const T *__restrict__ Gn,
                                                         LbmParams p, IbParams ib, AdjParams a) {
  const int l = (int)blockIdx.x * 16 + ((int)threadIdx.x >> 4);
  const int lane = (int)threadIdx.x & 15;
  const bool act = l < ib.nm;
  const int S = stencil_size(p.kind);
  const int i = lane & 3, j = lane >> 2;
  double X = 0.0, Y = 0.0;
  if (act) {
    X = ib.X[l];
    Y = ib.Y[l];
  }
  const int bx = stencil_base(p.kind, X), by = stencil_base(p.kind, Y);
  const bool on = act && i < S && j < S;
  double W = 0.0, dWx = 0.0, dWy = 0.0, fbx = 0.0, fby = 0.0, rk = 1.0, usx = 0.0, usy = 0.0;
  if (on) {
    const double rx = (double)(bx + i) - X, ry = (double)(by + j) - Y;
    const double px = phi(p.kind, rx), py = phi(p.kind, ry);
    W = px * py;
    dWx = -dphi(p.kind, rx) * py;  // d W / d X
    dWy = -px * dphi(p.kind, ry);  // d W / d Y
    int xx = bx + i, yy = by + j;
    if (p.xper) xx = wrap_index(xx, p.nx);
    if (p.yper) yy = wrap_index(yy, p.ny);
    // the node's forward values and dJ/df, as the lattice kernel forms them
    // every load that does not depend on the covering markers goes first
    T g[9], bb[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = pull<T>(A, p, q, xx, yy);
    node_dJdB<T>(Gn, p, xx, yy, g, bb, nullptr, nullptr);
    T sfx, sfy;
    node_spread_force<T>(p, a, l, lane, &sfx, &sfy);
    const double ftx = (double)(T)(p.Gx + (double)sfx), fty = (double)(T)(p.Gy + (double)sfy);
    const NodeFwd nf = node_forward(g, ftx, fty, p);
    Mom mo;
#pragma unroll
    for (int q = 0; q < 9; ++q) mo.add(q, (double)bb[q]);
    const CollideAdj ca = collide_adjoint(nf, ftx, fty, mo, p);
    fbx = ca.fbx;
    fby = ca.fby;
    rk = nf.rho;
    usx = (nf.mx + 0.5 * p.Gx) / nf.rho;  // u* = (m + G/2) / rho
    usy = (nf.my + 0.5 * p.Gy) / nf.rho;
  }
  auto gsum = [](double v) {
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
    return v;
  };
  // spreading (eqs 13, 15): dJ/dF_l = drs ds sum_k W_lk dJ/df_k
  const double SX = gsum(W * fbx), SY = gsum(W * fby);
  double s = 0.0, hz = 0.0, Fx = 0.0, Fy = 0.0, rl = 0.0, Fbx = 0.0, Fby = 0.0;
  double rlb = 0.0, ulb = 0.0, vlb = 0.0;
  if (act) {
    const int b = ib.mk_body[l];
    s = ib.sdrs[l];
    const double *hb = a.hist_bar + 3 * b;
    hz = hb[2];
    Fx = a.Fx[l];
    Fy = a.Fy[l];
    rl = a.rho_l[l];
    // eq 27: F_b = -s sum F_l, T_b = -s sum (X_l - c) x F_l
    Fbx = s * SX - s * hb[0] + s * hz * (Y - ib.cy[b]);
    Fby = s * SY - s * hb[1] - s * hz * (X - ib.cx[b]);
    // eq 20: F_l = 2 rho_l (U_l - u*_l)
    rlb = 2.0 * (Fbx * (ib.U[l] - a.ux_l[l]) + Fby * (ib.V[l] - a.uy_l[l]));
    ulb = -2.0 * rl * Fbx;
    vlb = -2.0 * rl * Fby;
  }
  // positions: the weights of the spreading and of the interpolation move with X_l
  const double term = on ? s * (Fx * fbx + Fy * fby) + rlb * rk + ulb * usx + vlb * usy : 0.0;
  const double PX = gsum(dWx * term), PY = gsum(dWy * term);
  if (act && lane == 0) {
    a.xy_bar[2 * l] += PX - s * hz * Fy;
    a.xy_bar[2 * l + 1] += PY + s * hz * Fx;
    a.uv_bar[2 * l] += 2.0 * rl * Fbx;
    a.uv_bar[2 * l + 1] += 2.0 * rl * Fby;
    a.c_bar[2 * l] += s * hz * Fy;  // the body centre enters the torque only
    a.c_bar[2 * l + 1] += -s * hz * Fx;
    a.mk_adj[3 * l] = rlb;
    a.mk_adj[3 * l + 1] = ulb;
    a.mk_adj[3 * l + 2] = vlb;
  }
}

template <typename T>
__global__ __launch_bounds__(kAdjTX *kAdjTY) void adj_lattice_kernel(const T *__restrict__ A,
                                                                     const T *__restrict__ Gn, T *__restrict__ Go,
                                                                     LbmParams p, AdjParams a) {
  const int ntiles = a.ntx * a.nty;
  const int t = p.xcd_remap ? xcd_tile((int)blockIdx.x, ntiles) : (int)blockIdx.x;
  const int tyi = t / a.ntx, txi = t - tyi * a.ntx;
  const int x = txi * kAdjTX + (int)threadIdx.x, y = tyi * kAdjTY + (int)threadIdx.y;
  const int tid = (int)threadIdx.y * kAdjTX + (int)threadIdx.x;
  __shared__ int s_ix[kAdjChunk], s_iy[kAdjChunk];
  __shared__ T s_w[kAdjChunk][10];
  __shared__ double s_a[kAdjChunk][3];

  // over the markers listed for the tile, in ascending order: the spread force
  // at the node as the forward step formed it, and the interpolation weights
  // applied to the markers' dJ/drho_l, dJ/du*_l
  T fibx = (T)0, fiby = (T)0;
  double Pr = 0.0, Pu = 0.0, Pv = 0.0;
  const int m0 = a.tile_off[t], m1 = a.tile_off[t + 1];
  if (m1 > m0) {
    const int S = stencil_size(p.kind);
    const T *mw = reinterpret_cast<const T *>(p.mk_w);
    for (int c0 = m0; c0 < m1; c0 += kAdjChunk) {
      const int cnt = min(kAdjChunk, m1 - c0);
      __syncthreads();
      if (tid < cnt) {
        const int l = a.tile_list[c0 + tid];
        s_ix[tid] = p.mk_ixy[2 * l];
        s_iy[tid] = p.mk_ixy[2 * l + 1];
#pragma unroll
        for (int k = 0; k < 10; ++k) s_w[tid][k] = mw[10 * (long long)l + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) s_a[tid][k] = a.mk_adj[3 * (long long)l + k];
      }
      __syncthreads();
      for (int e = 0; e < cnt; ++e) {
        int dy = y - s_iy[e];
        if (p.yper && dy < 0) dy += p.ny;
        int dx = x - s_ix[e];
        if (p.xper && dx < 0) dx += p.nx;
        if ((unsigned)dy < (unsigned)S && (unsigned)dx < (unsigned)S) {
          const T W = s_w[e][dx] * s_w[e][4 + dy];
          fibx += W * s_w[e][8];
          fiby += W * s_w[e][9];
          const double Wd = (double)s_w[e][dx] * (double)s_w[e][4 + dy];
          Pr += Wd * s_a[e][0];
          Pu += Wd * s_a[e][1];
          Pv += Wd * s_a[e][2];
        }
      }
    }
  }

  double sGx = 0.0, sGy = 0.0, sUx = 0.0, sUy = 0.0;
  const bool fluid = y < p.ny && x < p.nx && x >= p.i0 && x <= p.i1;
  if (fluid) {
    // Loads and stores are in the population type; the arithmetic is FP64
    // whatever it is: the gradients of interest are sums of large terms that
    // cancel (the isotropic part of dJ/dB drops out of every moment), and the
    // kernel is bound by memory, not by the FP64 rate.
    const double ftx = m1 > m0 ? (double)(T)(p.Gx + (double)fibx) : (double)(T)p.Gx;
    const double fty = m1 > m0 ? (double)(T)(p.Gy + (double)fiby) : (double)(T)p.Gy;
    // A tile whose nodes and their neighbours need no wrap, no wall and no
    // ghost column (tile-uniform test) reads both fields by direct offsets;
    // the other tiles take the general pulls.
    const int x0 = txi * kAdjTX, y0 = tyi * kAdjTY;
    const bool inner = x0 - 1 >= p.i0 && x0 + kAdjTX <= p.i1 && y0 >= 1 && y0 + kAdjTY <= p.ny - 1;
    const long long node = (long long)y * p.pitch + x;
    const bool ghost_out = p.outlet && x == p.nx - 2;  // B(nx-1, y) = B(nx-2, y)
    NodeFwd nf;
    Mom mo;
    T bb[9];
    double dr = 0.0, mx = 0.0, my = 0.0;
    if (inner) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const double v = (double)A[(long long)q * p.plane + node - (long long)ey(q) * p.pitch - ex(q)];
        dr += v;
        mx += ex(q) * v;
        my += ey(q) * v;
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        bb[q] = Gn[(long long)q * p.plane + node + (long long)ey(q) * p.pitch + ex(q)];
        mo.add(q, (double)bb[q]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const double v = (double)pull<T>(A, p, q, x, y);
        dr += v;
        mx += ex(q) * v;
        my += ey(q) * v;
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        bb[q] = pull_adj<T>(Gn, p, q, x, y);
        if (ghost_out) bb[q] += pull_adj<T>(Gn, p, q, x + 1, y);
        mo.add(q, (double)bb[q]);
      }
    }
    nf.rho = 1.0 + dr;
    nf.mx = mx + p.urx;  // stored values are deviations from feq(1, u_ref)
    nf.my = my + p.ury;
    nf.ux = (nf.mx + 0.5 * ftx) / nf.rho;
    nf.uy = (nf.my + 0.5 * fty) / nf.rho;
    // the inlet ghost's density adds one shift to every direction of dJ/dB
    double shift = 0.0;
    if (!inner && p.inlet && x == 1) {
      // B_q(0, y) = feq_q(rho_B, u_in) - c_q with rho_B the density of column
      // 1 after collision, which the collision leaves equal to rho
      const double rB = nf.rho;
      const double ui = p.uin_x, vi = p.uin_y, uui = ui * ui + vi * vi;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const double a0 = (double)pull_adj<T>(Gn, p, q, 0, y);
        const double eu = ex(q) * ui + ey(q) * vi;
        shift += a0 * wq(q) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uui);
        sUx += a0 * wq(q) * rB * (3.0 * ex(q) + 9.0 * eu * ex(q) - 3.0 * ui);
        sUy += a0 * wq(q) * rB * (3.0 * ey(q) + 9.0 * eu * ey(q) - 3.0 * vi);
      }
      mo.add_uniform(shift);
    }
    const CollideAdj ca = collide_adjoint(nf, ftx, fty, mo, p);
    double drb = ca.drb, mbx = ca.mbx, mby = ca.mby;
    sGx = ca.fbx;
    sGy = ca.fby;
    if (m1 > m0) {
      // transposed interpolation (eqs 12, 14) through rho and u* = (m + G/2)/rho
      const double inv = 1.0 / nf.rho;
      const double usx = (nf.mx + 0.5 * p.Gx) * inv, usy = (nf.my + 0.5 * p.Gy) * inv;
      drb += Pr - (Pu * usx + Pv * usy) * inv;
      mbx += Pu * inv;
      mby += Pv * inv;
      sGx += 0.5 * Pu * inv;
      sGy += 0.5 * Pv * inv;
    }
    const double omc = 1.0 - p.omega;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      Go[(long long)q * p.plane + node] = (T)(omc * ((double)bb[q] + shift) + drb + ex(q) * mbx + ey(q) * mby);
  }
  block_add4(sGx, sGy, sUx, sUy, a.part + 4 * (long long)t);
}

// dJ/dA_0 from G_0, all nodes (ghost columns included), packed [9][ny][nx] in FP64
template <typename T>
__global__ void adj_unpull_kernel(const T *__restrict__ G, LbmParams p, double *__restrict__ out) {
  const long long n = (long long)p.nx * p.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
#pragma unroll
    for (int q = 0; q < 9; ++q) out[(long long)q * n + k] = (double)pull_adj<T>(G, p, q, x, y);
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_adj_lattice(int prec, const void *A, const void *Gnext, void *Gout, const LbmParams &p,
                              const AdjParams &a, hipStream_t s) {
  const int blocks = a.ntx * a.nty;
  if (blocks <= 0) return hipSuccess;
  if (prec == 4)
    hipLaunchKernelGGL(adj_lattice_kernel<float>, dim3(blocks), dim3(kAdjTX, kAdjTY), 0, s, (const float *)A,
                       (const float *)Gnext, (float *)Gout, p, a);
  else
    hipLaunchKernelGGL(adj_lattice_kernel<double>, dim3(blocks), dim3(kAdjTX, kAdjTY), 0, s, (const double *)A,
                       (const double *)Gnext, (double *)Gout, p, a);
  return hipGetLastError();
}

hipError_t launch_adj_marker(int prec, const void *A, const void *Gnext, const LbmParams &p, const IbParams &ib,
                             const AdjParams &a, hipStream_t s) {
  if (ib.nm <= 0) return hipSuccess;
  const int blocks = (ib.nm + 15) / 16;
  if (prec == 4)
    hipLaunchKernelGGL(adj_marker_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float *)A,
                       (const float *)Gnext, p, ib, a);
  else
    hipLaunchKernelGGL(adj_marker_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double *)A,
                       (const double *)Gnext, p, ib, a);
  return hipGetLastError();
}

hipError_t launch_adj_unpull(int prec, const void *G, const LbmParams &p, double *out, hipStream_t s) {
  const long long n = (long long)p.nx * p.ny;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
  if (prec == 4)
    hipLaunchKernelGGL(adj_unpull_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float *)G, p, out);
  else
    hipLaunchKernelGGL(adj_unpull_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double *)G, p, out);
  return hipGetLastError();
}

}  // namespace btdf
