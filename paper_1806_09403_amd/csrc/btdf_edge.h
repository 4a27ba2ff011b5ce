// btdf_edge.h -- the boundary readings of the temporal-blocking pass at the
// domain's edges (used by the pass kernels in btdf_kernels.hip and by the
// kernels of btdf_edge.hip).
//
// The pass of depth D takes D steps (eqs 5-7 with the uniform body force)
// per read and write of a group of tiles, which needs every node of the group
// grown by D - 1 to follow from state n alone. Groups within reach of a
// domain edge take the boundary readings in every step:
//
//  * periodic directions: the grown group is computed at the wrapped nodes;
//  * walls in y (halfway bounce-back or specular free slip): pulls that
//    would leave the grid read the node's own opposite population or the
//    mirror population of the upstream column, as in single steps;
//  * the channel's ghost columns: the thread of column 1 writes the inlet
//    ghost (eq 6 at the inflow velocity and column 1's density), and the
//    thread of column nx-2 writes the zero-gradient outlet's copy;
//  * groups that reach past the grid's last column or row store only their
//    nodes inside it.
//
// An edge node of the group whose neighbour x + e_q (or, at a free-slip
// wall, the node its reflection reaches) lies in a near tile also gives X1
// its state n+1 and, for D = 3, X2 its state n+2 in that direction: the near
// tiles' later steps pull them from there. A near tile can lie across a
// periodic edge, so the test is made node by node. The convective outlet is
// not taken here: tiles within reach of one step singly.
#pragma once

#include "btdf_device.h"
#include "btdf_launch.h"

namespace btdf {

namespace {

__device__ const int kEdgeNoStop = 0;

// a batch case's stop flag, read beside the first loads
template <bool STOP>
__device__ __forceinline__ int edge_stop(const int *stop) {
  if constexpr (STOP) return __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

// population q pulled into node (x, y) (wrapped, collided) from the previous
// state, read through get(q', dx, dy) = that state's population q' at the
// node offset (dx, dy): the readings of pull() in btdf_device.h
// (the wall shifts from the constant table, fill_konst)
template <typename T, typename Get>
__device__ __forceinline__ T pull_prev(const LbmParams &p, int q, int y, Get get) {
#pragma clang fp contract(off)
  const int sy = y - ey(q);
  if (!p.yper && (sy < 0 || sy >= p.ny)) {
    const T *k = konst<T>(p);
    if (p.slip) return get(mir_y(q), -ex(q), 0) + ldg(k, 27 + q);
    return get(opp(q), 0, 0) + ldg(k, 18 + q);
  }
  return get(q, -ex(q), -ey(q));
}

// The periodic image of i in [0, n) for -n <= i < 2n: edge groups reach at
// most three nodes past a grid edge, and take the pass only where a periodic
// extent is at least the group's width plus its margins (fused_lists).
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct EdgeNode {
  int x, y;  // lattice node (wrapped in periodic directions)
  int kind;  // 0 outside the grid, 1 ghost column (not collided), 2 collided
};

// the node at position (i, j) of the group grown by g around (x0, y0)
__device__ __forceinline__ EdgeNode edge_node(const LbmParams &p, int x0, int y0, int g, int i, int j) {
  EdgeNode n;
  n.x = x0 - g + i;
  n.y = y0 - g + j;
  n.kind = 2;
  if (p.xper)
    n.x = wrap1(n.x, p.nx);
  else if (n.x < 0 || n.x >= p.nx)
    n.kind = 0;
  if (p.yper)
    n.y = wrap1(n.y, p.ny);
  else if (n.y < 0 || n.y >= p.ny)
    n.kind = 0;
  if (n.kind && (n.x < p.i0 || n.x > p.i1)) n.kind = 1;
  return n;
}

// the populations pulled into collided node n from state n in HBM
template <typename T>
__device__ __forceinline__ void edge_pull_global(const T *__restrict__ A, const LbmParams &p, const EdgeNode &n,
                                                 T (&g)[9]) {
  if (!p.yper && (n.y == 0 || n.y == p.ny - 1)) {  // a wall row
#pragma unroll
    for (int q = 0; q < 9; ++q)
      g[q] = pull_prev<T>(p, q, n.y, [&](int qq, int dx, int dy) {
        const int xs = p.xper ? wrap1(n.x + dx, p.nx) : n.x + dx;
        return ldg(A + (long long)qq * p.plane, (unsigned)(n.y + dy) * (unsigned)p.pitch + (unsigned)xs);
      });
    return;
  }
  // the node's rows y - 1, y, y + 1 and columns x - 1, x, x + 1 (wrapped
  // where periodic; a collided node of a non-periodic x has both
  // neighbouring columns in the grid)
  const int ym = p.yper ? wrap1(n.y - 1, p.ny) : n.y - 1;
  const int yp = p.yper ? wrap1(n.y + 1, p.ny) : n.y + 1;
  const int xm = p.xper ? wrap1(n.x - 1, p.nx) : n.x - 1;
  const int xp = p.xper ? wrap1(n.x + 1, p.nx) : n.x + 1;
  // element offsets within a plane (below 2^31: the plane index fits an int)
  const unsigned rows[3] = {(unsigned)yp * (unsigned)p.pitch, (unsigned)n.y * (unsigned)p.pitch,
                            (unsigned)ym * (unsigned)p.pitch};  // y - e_y for e_y = -1, 0, 1
  const unsigned cols[3] = {(unsigned)xp, (unsigned)n.x, (unsigned)xm};  // x - e_x for e_x = -1, 0, 1
#pragma unroll
  for (int q = 0; q < 9; ++q) g[q] = ldg(A + (long long)q * p.plane, rows[ey(q) + 1] + cols[ex(q) + 1]);
}

// the populations pulled into collided node (row y) at slot k of an LDS
// copy of the previous state (rows RX slots apart, planes RN apart): one test
// for a wall row per node, plain neighbour slots elsewhere
template <typename T, int RN, int RX>
__device__ __forceinline__ void edge_pull_lds(const LbmParams &p, int y, const T *__restrict__ s_f, int k, T (&g)[9]) {
  if (!p.yper && (y == 0 || y == p.ny - 1)) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
      g[q] = pull_prev<T>(p, q, y, [&](int qq, int dx, int dy) { return s_f[qq * RN + k + dy * RX + dx]; });
    return;
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) g[q] = s_f[q * RN + k - ey(q) * RX - ex(q)];
}

// the ring directions of node (x, y) of the grid: bit q set when the node
// its population q reaches next (x + e_q, or at a free-slip wall the next
// column of the same row) lies in a near tile
// (tiles are 2^shx x 2^shy nodes)
__device__ __forceinline__ unsigned edge_ring(const LbmParams &p, const unsigned char *__restrict__ near, int shx,
                                              int shy, int x, int y) {
  unsigned m = 0;
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    int xn = x + ex(q), yn = y + ey(q);
    if (!p.yper && (yn < 0 || yn >= p.ny)) {
      // into a wall: a free-slip wall reflects it to the next column of
      // the same row; bounce-back returns it to this node
      if (!p.slip) continue;
      yn = y;
    }
    if (p.xper)
      xn = wrap1(xn, p.nx);
    else if (xn < 0 || xn >= p.nx)
      continue;
    if (p.yper) yn = wrap1(yn, p.ny);
    if (near[(yn >> shy) * p.ntx + (xn >> shx)]) m |= 1u << q;
  }
  return m;
}


}  // namespace

// Three steps A -> C for a group of W x H lattice tiles (OX x OY nodes, one
// thread per node, OX * OY threads) within reach of a domain edge: the
// interior group kernel's structure (group grown by two in LDS, step n+2 in
// registers and back in place) with the boundary readings. s_f: 9 (OX + 4)
// (OY + 4) values of LDS.
template <typename T, int OX, int OY, bool STOP>
__device__ __forceinline__ void lbm3_edge_group(const T *__restrict__ A, T *__restrict__ C, const LbmParams &p,
                                                int t, int tile_x, int tile_y, T *__restrict__ X1,
                                                T *__restrict__ X2, const unsigned char *__restrict__ near,
                                                const int *stop, T *__restrict__ s_f) {
  constexpr int RX = OX + 4, RY = OY + 4, RN = RX * RY;  // the group grown by two
  constexpr int NTH = OX * OY;
  const bool keep = !edge_stop<STOP>(stop);
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int x0 = txi * tile_x, y0 = tyi * tile_y;
  const int tid = (int)(threadIdx.y * blockDim.x + threadIdx.x);
  const CollK<T> &K = coll<T>(p);
  const ForceK<T> &F = gforce<T>(p);
  bool bad = false;
  // The near flags of the tiles around the group (wrapped where periodic),
  // loaded by wave 0 ahead of its first-step loads: most edge groups have no
  // near neighbour, and then skip the ring test of their boundary nodes.
  __shared__ int s_any;
  int nflag = 0;
  if (near && tid < 64) {  // wave 0 (uniform)
    const int gw = OX / tile_x, gh = OY / tile_y, nc = gw + 2;
    if (tid < nc * (gh + 2)) {
      int c = txi - 1 + tid % nc, r = tyi - 1 + tid / nc;
      bool ok = !(r >= tyi && r < tyi + gh && c >= txi && c < txi + gw);  // (the group's own tiles)
      if (p.xper)
        c = wrap1(c, p.ntx);
      else
        ok = ok && c >= 0 && c < p.ntx;
      if (p.yper)
        r = wrap1(r, p.nty);
      else
        ok = ok && r >= 0 && r < p.nty;
      if (ok) nflag = near[r * p.ntx + c];
    }
  }
  // one node's step n+1 from its pulled populations, into its slot; column 1
  // (nx-2) also writes the inlet (outlet) ghost slot beside it
  auto first = [&](const EdgeNode &n, T (&g)[9], int k) {
    T out[9], rho;
    collide<T>(g, F, K, out, rho);
    bad |= !rho_ok(rho);
#pragma unroll
    for (int q = 0; q < 9; ++q) s_f[q * RN + k] = out[q];
    const int i = k % RX;
    if (p.inlet && n.x == 1 && i >= 1) {
      const T dr = inlet_dr<T>(out);
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q * RN + k - 1] = inlet_ghost<T>(dr, p, q);
    }
    if (p.outlet == 1 && n.x == p.nx - 2 && i + 1 < RX) {
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q * RN + k + 1] = out[q];
    }
  };
  // step n+1 over the grown group, from state n in HBM: two nodes per round,
  // the loads of both issued before either collision
  for (int k = tid; k < RN; k += 2 * NTH) {
    const int kb = k + NTH;
    const EdgeNode na = edge_node(p, x0, y0, 2, k % RX, k / RX);
    const EdgeNode nb = kb < RN ? edge_node(p, x0, y0, 2, kb % RX, kb / RX) : EdgeNode{0, 0, 0};
    T ga[9], gb[9];
    if (na.kind == 2) edge_pull_global<T>(A, p, na, ga);
    if (nb.kind == 2) edge_pull_global<T>(A, p, nb, gb);
    if (na.kind == 2) first(na, ga, k);
    if (nb.kind == 2) first(nb, gb, kb);
  }
  if (tid < 64) {
    const unsigned long long any = __builtin_amdgcn_ballot_w64(nflag != 0);
    if (tid == 0) s_any = any != 0;
  }
  __syncthreads();
  // this thread's node of the group; the ring directions of the group's
  // edge nodes, and their states n+1
  const int ii = tid % OX, jj = tid / OX;
  const int x = x0 + ii, y = y0 + jj;
  const bool mine = x < p.nx && y < p.ny;
  const int kown = (jj + 2) * RX + ii + 2;
  const long long node = (long long)y * p.pitch + x;
  unsigned rmask = 0;
  if (s_any && keep && mine && (ii == 0 || ii == OX - 1 || jj == 0 || jj == OY - 1 || x == p.nx - 1 || y == p.ny - 1))
    rmask = edge_ring(p, near, __builtin_ctz((unsigned)tile_x), __builtin_ctz((unsigned)tile_y), x, y);
  if (rmask) {
    const global_ptr<T> Xg = (global_ptr<T>)X1;
    T v[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) v[q] = s_f[q * RN + kown];
#pragma unroll
    for (int q = 1; q < 9; ++q)
      if (rmask & (1u << q)) Xg[(long long)q * p.plane + node] = v[q];
  }
  // step n+2 over the group grown by one (at most two nodes per thread),
  // into registers
  constexpr int R2X = OX + 2, TOT2 = R2X * (OY + 2);
  static_assert(TOT2 <= 2 * NTH, "the grown-by-one region takes at most two nodes per thread");
  T o2a[9], o2b[9];
  int pa = -1, pb = -1, xa = -1, xb = -1;  // their slots and lattice columns (-1: none)
  {
    auto step2 = [&](int k2, T (&o)[9], int &xc) {
      const int j2 = k2 / R2X, i2 = k2 - j2 * R2X;
      const int i = i2 + 1, j = j2 + 1, k = j * RX + i;
      const EdgeNode n = edge_node(p, x0, y0, 2, i, j);
      if (n.kind != 2) return -1;
      T g[9], rho;
      edge_pull_lds<T, RN, RX>(p, n.y, s_f, k, g);
      collide<T>(g, F, K, o, rho);
      bad |= !rho_ok(rho);
      xc = n.x;
      return k;
    };
    if (tid < TOT2) pa = step2(tid, o2a, xa);
    if (tid + NTH < TOT2) pb = step2(tid + NTH, o2b, xb);
  }
  __syncthreads();
  // back into the same slots; column 1 (nx-2) also writes the inlet
  // (outlet) ghost beside it inside the grown-by-one region
  auto put2 = [&](int k, const T (&o)[9], int xc) {
#pragma unroll
    for (int q = 0; q < 9; ++q) s_f[q * RN + k] = o[q];
    const int i = k % RX;
    if (p.inlet && xc == 1 && i - 1 >= 1) {
      const T dr = inlet_dr<T>(o);
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q * RN + k - 1] = inlet_ghost<T>(dr, p, q);
    }
    if (p.outlet == 1 && xc == p.nx - 2 && i + 1 < RX - 1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q * RN + k + 1] = o[q];
    }
  };
  if (pa >= 0) put2(pa, o2a, xa);
  if (pb >= 0) put2(pb, o2b, xb);
  __syncthreads();
  // step n+3 on the group's own nodes, pulling state n+2 from LDS
  if (mine && keep) {
    const EdgeNode n = edge_node(p, x0, y0, 2, ii + 2, jj + 2);
    if (n.kind == 2) {
      T g[9], out[9], rho;
      edge_pull_lds<T, RN, RX>(p, n.y, s_f, kown, g);
      collide<T>(g, F, K, out, rho);
      bad |= !rho_ok(rho);
      // (global stores: the buffers come from the case table as generic
      // pointers, whose stores would otherwise be flat ones)
      const global_ptr<T> Cg = (global_ptr<T>)C;
#pragma unroll
      for (int q = 0; q < 9; ++q) Cg[(long long)q * p.plane + node] = out[q];
      if (p.inlet && x == 1) {
        const T dr = inlet_dr<T>(out);
#pragma unroll
        for (int q = 0; q < 9; ++q) Cg[(long long)q * p.plane + node - 1] = inlet_ghost<T>(dr, p, q);
      }
      if (p.outlet == 1 && x == p.nx - 2) {
#pragma unroll
        for (int q = 0; q < 9; ++q) Cg[(long long)q * p.plane + node + 1] = out[q];
      }
    }
    if (rmask) {
      const global_ptr<T> Xg = (global_ptr<T>)X2;
      T v[9];
#pragma unroll
      for (int q = 1; q < 9; ++q) v[q] = s_f[q * RN + kown];
#pragma unroll
      for (int q = 1; q < 9; ++q)
        if (rmask & (1u << q)) Xg[(long long)q * p.plane + node] = v[q];
    }
  }
  if (bad && keep) p.flag[0] = -1;
}

// the launch shapes with a three-step pass over edge groups (lattice tile,
// group of W x H tiles, group in nodes): rows of tiles, and columns of four
// for the ends of a channel
#define BTDF_EDGE3_SHAPES(S)                                                                          \
  S(32, 8, 4, 1, 128, 8) S(32, 8, 2, 1, 64, 8) S(32, 8, 1, 1, 32, 8) S(32, 8, 1, 4, 32, 32)        \
  S(64, 4, 2, 1, 128, 4) S(64, 4, 1, 1, 64, 4)


}  // namespace btdf
