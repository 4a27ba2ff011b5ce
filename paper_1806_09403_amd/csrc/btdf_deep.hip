// btdf_deep.hip -- four or five steps per pass (temporal blocking of a single
// lattice, deeper than the three-step pass of btdf_kernels.hip).
//
// A group of lattice tiles whose nodes, grown by D - 1, carry no
// immersed-boundary force takes D steps at once: step n+1 over the group
// grown by D - 1 nodes, pulled from A into LDS; the inner steps n+2 .. n+D-1
// over the group grown by D - 2 .. 1 nodes, each from the LDS copy into
// registers and back into the same LDS rows after a barrier; step n+D over
// the group's own nodes into C. Only the uniform body force acts there, so
// every collision is the single-step kernel's, value for value (eqs 5-8 with
// the Guo term of the body force). Each node is read and written once per D
// updates: 72 / D bytes per update in FP32.
//
// Near tiles step singly between the marker kernels and pull their
// neighbours' intermediate states from the ring buffers: an edge node of a
// group next to a near tile stores its states n+1 .. n+D-1 in X1 .. X(D-1),
// in each direction whose neighbour lies in the near tile (the one
// population that tile's next step pulls from it). The groups with such
// nodes run in a launch of their own, with that code; the others without.
//
// The host hands over groups of tiles at least D nodes from every domain
// edge (no wrap, wall or ghost column in reach): rows of 1, 2 or 4 lattice
// tiles, or two tiles tall.
#include "btdf_device.h"
#include "btdf_launch.h"

namespace btdf {

// register nodes per thread for the inner steps (the largest of them covers
// the group grown by D - 2)
template <int D, int OX, int OY>
constexpr int deep_regs() {
  return ((OX + 2 * (D - 2)) * (OY + 2 * (D - 2)) + OX * OY - 1) / (OX * OY);
}

// whether the group's state fits the LDS (160 KB on gfx950) and its inner
// steps three register nodes per thread
template <typename T, int D, int OX, int OY>
constexpr bool deep_fits() {
  return 9 * (OX + 2 * (D - 1)) * (OY + 2 * (D - 1)) * (int)sizeof(T) + 64 <= 163840 && deep_regs<D, OX, OY>() <= 3;
}

// Ring buffers: the near tiles' states n+1 .. n+D-1, one population buffer
// each, consecutive from ring at the population buffers' 256-byte-aligned
// stride (its address is the only one the kernel takes for them).
template <typename T>
__device__ __forceinline__ long long ring_stride(const LbmParams &p) {
  return (((long long)9 * p.plane * (long long)sizeof(T) + 255) / 256 * 256) / (long long)sizeof(T);
}

// One group of W = OX / TX lattice tiles of TX x TY nodes. RING: the group
// borders a near tile, and its edge nodes write the ring; the other groups
// run without that code (its scalar registers would halve the groups a CU
// holds at five steps).
template <typename T, int D, int OX, int OY, int TX, int TY, bool RING>
__global__ __launch_bounds__(OX *OY) void lbmd_kernel(const T *__restrict__ A, T *__restrict__ C, LbmParams p,
                                                      const int *__restrict__ map, T *__restrict__ ring,
                                                      const unsigned *__restrict__ rwin) {
  constexpr int G = D - 1;                       // growth of the first step
  constexpr int RX = OX + 2 * G, RY = OY + 2 * G;  // the grown group
  constexpr int NTH = OX * OY, NR = deep_regs<D, OX, OY>();
  // (no other LDS: the state alone sets how many groups share a CU, two
  // of 128x8 nodes at five steps)
  __shared__ T s_f[9][RY][RX];
  const int count = (int)gridDim.x;
  const int li = p.xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  const int t = map[li];
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int x0 = txi * TX, y0 = tyi * TY;
  const int tid = (int)threadIdx.y * OX + (int)threadIdx.x;
  const int ii = (int)threadIdx.x, jj = (int)threadIdx.y;
  // the near flags of the tiles around the group (bit 8 r + c: row r of
  // three from the row below, column c from the column left of the group)
  const unsigned win = RING ? rwin[li] : 0u;
  const CollK<T> &K = coll<T>(p);
  const ForceK<T> &F = gforce<T>(p);
  bool bad = false;
  // step n+1 over the grown group: the OX central columns of every row
  // first (consecutive lanes on consecutive, line-aligned nodes), then the
  // 2G edge columns; two nodes per round, the loads of both issued first
  constexpr int TOT = RY * OX + 2 * G * RY;
  auto node_of = [&](int k, int &i, int &j) {
    if (k < RY * OX) {
      j = k / OX;
      i = G + (k - j * OX);
    } else {
      const int e = k - RY * OX;
      j = e / (2 * G);
      const int c = e - j * (2 * G);
      i = c < G ? c : OX + c;
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
                                                        (long long)(y0 - G - ey(q)) * p.pitch + (x0 - G - ex(q)));
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
  // The edge node whose ring stores this thread makes: the bottom row's by
  // the first OX threads and the top row's by the last OX (their own nodes),
  // the two columns' other nodes by 2 (OY - 2) threads of the first wave past
  // the bottom row, so that only these waves run the ring code.
  int ri = 0, rj = 0;
  bool redge = false;
  if (RING) {
    constexpr int CB = (OX + 63) / 64 * 64, NC = OY - 2;
    static_assert(CB + 2 * NC <= NTH - OX, "the column threads lie between the two rows' threads");
    if (tid < OX) {
      ri = tid;
      redge = true;
    } else if (tid >= NTH - OX) {
      ri = tid - (NTH - OX);
      rj = OY - 1;
      redge = true;
    } else if (tid >= CB && tid < CB + 2 * NC) {
      const int c = tid - CB;
      ri = c < NC ? 0 : OX - 1;
      rj = 1 + (c < NC ? c : c - NC);
      redge = true;
    }
  }
  // its ring directions: bit q when x + e_q lies in a near tile (the group's
  // own tiles never are)
  unsigned rmask = 0;
  if (RING && redge) {
    constexpr int W = OX / TX, H = OY / TY;
    constexpr int shx = __builtin_ctz((unsigned)TX), shy = __builtin_ctz((unsigned)TY);
    const int cl = ri == 0 ? 0 : 1 + ((ri - 1) >> shx), cm = 1 + (ri >> shx);
    const int cr = ri == OX - 1 ? W + 1 : 1 + ((ri + 1) >> shx);
    const int rd = rj == 0 ? 0 : 1 + ((rj - 1) >> shy), rm = 1 + (rj >> shy);
    const int ru = rj == OY - 1 ? H + 1 : 1 + ((rj + 1) >> shy);
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      const int r = ey(q) < 0 ? rd : (ey(q) > 0 ? ru : rm);
      const int c = ex(q) < 0 ? cl : (ex(q) > 0 ? cr : cm);
      rmask |= ((win >> (8 * r + c)) & 1u) << q;
    }
  }
  const unsigned off = (unsigned)(jj * p.pitch + ii) * (unsigned)sizeof(T);
  // the ring: state n+s of that node, from LDS, in its ring directions
  // (a per-lane zero the compiler cannot see through keeps these rare
  // stores' addresses in vector registers, so their bases are not held in
  // scalar registers across the pass)
  auto ring_store = [&](int s) {
    if (!RING || !rmask) return;
    int vz;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
    const long long plane = p.plane + vz;
    global_ptr<T> X = (global_ptr<T>)ring + (long long)(s - 1) * ring_stride<T>(p) + vz +
                      (long long)(y0 + rj) * p.pitch + (x0 + ri);
    // the eight LDS reads first, so they are in flight together, then the stores
    T v[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) v[q] = s_f[q][rj + G][ri + G];
#pragma unroll
    for (int q = 1; q < 9; ++q)
      if (rmask & (1u << q)) X[q * plane] = v[q];
  };
  ring_store(1);
  T *sf = &s_f[0][0][0];
  // the inner steps n+2 .. n+D-1, over the group grown by D-2 .. 1 nodes
#pragma unroll
  for (int s = 2; s < D; ++s) {
    const int g = D - s;
    const int R2X = OX + 2 * g, TOT2 = R2X * (OY + 2 * g);
    T o[NR][9];
    int pos[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int k2 = tid + r * NTH;
      pos[r] = -1;
      if (k2 < TOT2) {
        const int j2 = k2 / R2X, i2 = k2 - j2 * R2X;
        const int i = i2 + G - g, j = j2 + G - g;
        T gg[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) gg[q] = s_f[q][j - ey(q)][i - ex(q)];
        T rho;
        collide<T>(gg, F, K, o[r], rho);
        bad |= !rho_ok(rho);
        pos[r] = j * RX + i;
      }
    }
    __syncthreads();
    // (one branch per node: the nine stores of a node under one mask)
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (pos[r] >= 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q) sf[q * RY * RX + pos[r]] = o[r][q];
      }
    __syncthreads();
    ring_store(s);
  }
  // step n+D on the group's own nodes, pulling state n+D-1 from LDS
  {
    const int i = ii + G, j = jj + G;
    T gg[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gg[q] = s_f[q][j - ey(q)][i - ex(q)];
    T out[9], rho;
    collide<T>(gg, F, K, out, rho);
    bad |= !rho_ok(rho);
#pragma unroll
    for (int q = 0; q < 9; ++q)
      store_uniform<T, true>(uniform_ptr(reinterpret_cast<char *>(C + (long long)q * p.plane + (long long)y0 * p.pitch + x0)),
                           off, out[q]);
  }
  if (bad) p.flag[0] = -1;
}

// The shapes of the deep passes: (depth, group code, lattice tile, group in
// nodes). Four steps take rows of two tiles (four 512-thread groups per CU
// hide more latency than two of 1024 threads) and single tiles; five take
// squares of two by two tiles (64x16: 1.34 collisions per update against
// 1.55 for 128x8), columns of two, rows of four and two, and single tiles.
#define BTDF_DEEP_SHAPES(S)                                                                         \
  S(4, kGroup2x1, 32, 8, 64, 8) S(4, kGroup1x1, 32, 8, 32, 8) S(5, kGroup2x2, 32, 8, 64, 16)     \
  S(5, kGroup1x2, 32, 8, 32, 16) S(5, kGroup4x1, 32, 8, 128, 8) S(5, kGroup2x1, 32, 8, 64, 8)     \
  S(5, kGroup1x1, 32, 8, 32, 8)

template <typename T, int D, int OX, int OY, int TX, int TY>
static hipError_t launch_deep_t(const T *A, T *C, const LbmParams &p, const int *map, int count, int ring_groups,
                                void *ring, const unsigned *rwin, hipStream_t s) {
  static_assert(OX / TX <= 6 && OY / TY <= 2, "the window of tiles around a group within a 32-bit word");
  if constexpr (deep_fits<T, D, OX, OY>()) {
    // the groups that border a near tile (the first ring_groups of the map), then the others
    if (ring_groups > 0)
      hipLaunchKernelGGL((lbmd_kernel<T, D, OX, OY, TX, TY, true>), dim3(ring_groups), dim3(OX, OY), 0, s, A, C, p,
                         map, (T *)ring, rwin);
    if (count > ring_groups)
      hipLaunchKernelGGL((lbmd_kernel<T, D, OX, OY, TX, TY, false>), dim3(count - ring_groups), dim3(OX, OY), 0, s,
                         A, C, p, map + ring_groups, (T *)nullptr, (const unsigned *)nullptr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

bool variant_has_deep(int variant, int prec, int depth, int code) {
  int tx, ty;
  variant_tile(variant, &tx, &ty);
#define S(DD, CODE, TX, TY, OX, OY)                                                                \
  if (depth == DD && code == CODE && tx == TX && ty == TY)                                         \
    return prec == 4 ? deep_fits<float, DD, OX, OY>() : deep_fits<double, DD, OX, OY>();
  BTDF_DEEP_SHAPES(S)
#undef S
  return false;
}

hipError_t launch_lbm_deep(int prec, int variant, int depth, int code, const void *A, void *C, const LbmParams &p,
                           const int *map, int count, int ring_groups, void *ring, const unsigned *rwin,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!variant_has_deep(variant, prec, depth, code) || ring_groups < 0 || ring_groups > count ||
      (ring_groups > 0 && (!ring || !rwin)))
    return hipErrorInvalidValue;
  int tx, ty;
  variant_tile(variant, &tx, &ty);
#define S(DD, CODE, TX, TY, OX, OY)                                                                           \
  if (depth == DD && code == CODE && tx == TX && ty == TY)                                                    \
    return prec == 4 ? launch_deep_t<float, DD, OX, OY, TX, TY>((const float *)A, (float *)C, p, map, count,   \
                                                                ring_groups, ring, rwin, s)                   \
                     : launch_deep_t<double, DD, OX, OY, TX, TY>((const double *)A, (double *)C, p, map, count, \
                                                                 ring_groups, ring, rwin, s);
  BTDF_DEEP_SHAPES(S)
#undef S
  return hipErrorInvalidValue;
}

}  // namespace btdf
