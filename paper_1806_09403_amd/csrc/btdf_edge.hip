// btdf_edge.hip -- the blocked pass over groups of tiles within reach of a
// domain edge, and which launch shapes have it.
//
// Each level of a pass launches its edge groups apart from its interior
// groups: three steps with lbm3_edge_group (btdf_edge.h) for the launch
// shapes of 32 x 8 and 64 x 4 tiles; two steps (steps left over after
// three-step passes, or blocking of depth 2) with 256 threads over a group
// of any row of tiles, the group grown by one in LDS.
#include "btdf_edge.h"
#include "btdf_launch.h"

namespace btdf {

template <typename T>
__device__ void edge2_group(const T *__restrict__ A, T *__restrict__ C, const LbmParams &p, int t, int gw, int gh,
                            int tx, int ty, T *__restrict__ X, const unsigned char *__restrict__ near, T *s_f) {
  const int ox = gw * tx, oy = gh * ty;  // the group: gw x gh tiles
  const int RX = ox + 2, RY = oy + 2, RN = RX * RY;
  const int tyi = t / p.ntx;
  const int txi = t - tyi * p.ntx;
  const int x0 = txi * tx, y0 = tyi * ty;
  const int tid = (int)threadIdx.x, nth = (int)blockDim.x;
  const CollK<T> &K = coll<T>(p);
  const ForceK<T> &F = gforce<T>(p);
  bool bad = false;
  // step n+1 over the group grown by one, from state n in HBM; column 1
  // (nx-2) also writes the inlet (outlet) ghost slot beside it
  for (int k = tid; k < RN; k += nth) {
    const int j = k / RX, i = k - j * RX;
    const EdgeNode n = edge_node(p, x0, y0, 1, i, j);
    if (n.kind != 2) continue;
    T g[9], out[9], rho;
    edge_pull_global<T>(A, p, n, g);
    collide<T>(g, F, K, out, rho);
    bad |= !rho_ok(rho);
#pragma unroll
    for (int q = 0; q < 9; ++q) s_f[q * RN + k] = out[q];
    if (p.inlet && n.x == 1 && i >= 1) {
      const T dr = inlet_dr<T>(out);
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q * RN + k - 1] = inlet_ghost<T>(dr, p, q);
    }
    if (p.outlet == 1 && n.x == p.nx - 2 && i + 1 < RX) {
#pragma unroll
      for (int q = 0; q < 9; ++q) s_f[q * RN + k + 1] = out[q];
    }
  }
  __syncthreads();
  // step n+2 on the group's own nodes, into C; the ring of state n+1
  for (int k0 = tid; k0 < ox * oy; k0 += nth) {
    const int jj = k0 / ox, ii = k0 - jj * ox;
    const int x = x0 + ii, y = y0 + jj;
    if (x >= p.nx || y >= p.ny) continue;  // past the grid's last column or row
    const int k = (jj + 1) * RX + ii + 1;
    const long long node = (long long)y * p.pitch + x;
    const EdgeNode n = edge_node(p, x0, y0, 1, ii + 1, jj + 1);
    if (n.kind == 2) {
      T g[9], out[9], rho;
#pragma unroll
      for (int q = 0; q < 9; ++q)
        g[q] = pull_prev<T>(p, q, n.y, [&](int qq, int dx, int dy) { return s_f[qq * RN + k + dy * RX + dx]; });
      collide<T>(g, F, K, out, rho);
      bad |= !rho_ok(rho);
#pragma unroll
      for (int q = 0; q < 9; ++q) C[(long long)q * p.plane + node] = out[q];
      if (p.inlet && x == 1) {
        const T dr = inlet_dr<T>(out);
#pragma unroll
        for (int q = 0; q < 9; ++q) C[(long long)q * p.plane + node - 1] = inlet_ghost<T>(dr, p, q);
      }
      if (p.outlet == 1 && x == p.nx - 2) {
#pragma unroll
        for (int q = 0; q < 9; ++q) C[(long long)q * p.plane + node + 1] = out[q];
      }
    }
    if (near && (ii == 0 || ii == ox - 1 || jj == 0 || jj == oy - 1 || x == p.nx - 1 || y == p.ny - 1)) {
      const unsigned rm = edge_ring(p, near, __builtin_ctz((unsigned)tx), __builtin_ctz((unsigned)ty), x, y);
#pragma unroll
      for (int q = 1; q < 9; ++q)
        if (rm & (1u << q)) X[(long long)q * p.plane + node] = s_f[q * RN + k];
    }
  }
  if (bad) p.flag[0] = -1;
}

template <typename T>
__global__ __launch_bounds__(256) void lbm_edge2_kernel(const T *__restrict__ A, T *__restrict__ C, LbmParams p,
                                                        const int *__restrict__ map, int count, int gw, int gh,
                                                        int tile_x, int tile_y, T *__restrict__ X,
                                                        const unsigned char *__restrict__ near) {
  extern __shared__ __align__(16) unsigned char edge_lds[];
  const int li = p.xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  edge2_group<T>(A, C, p, map[li] & ~kEdgeFlag, gw, gh, tile_x, tile_y, X, near, reinterpret_cast<T *>(edge_lds));
}

// three steps over the listed edge groups of W x H tiles (OX x OY nodes, one
// thread per node); FP32: eight waves per SIMD, two workgroups of 1024 threads per CU
template <typename T, int OX, int OY>
__global__ __launch_bounds__(OX *OY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1, 8))) void lbm3_edge_kernel(
    const T *__restrict__ A, T *__restrict__ C, LbmParams p, const int *__restrict__ map, int count, int tile_x,
    int tile_y, T *__restrict__ X1, T *__restrict__ X2, const unsigned char *__restrict__ near) {
  __shared__ T s_f[9 * (OX + 4) * (OY + 4)];
  const int li = p.xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  lbm3_edge_group<T, OX, OY, false>(A, C, p, map[li] & ~kEdgeFlag, tile_x, tile_y, X1, X2, near, nullptr, s_f);
}

// batches: the edge groups of every case in one launch (case and first tile
// per workgroup), the buffers and near flags from the case table
template <typename T, int OX, int OY>
__global__ __launch_bounds__(OX *OY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1, 8))) void lbm3_edge_batch_kernel(
    const CaseDesc *__restrict__ cases, const int *__restrict__ gcase, const int *__restrict__ gtile, int count,
    int rt, int mask_unstable, int xcd_remap, int tile_x, int tile_y) {
  __shared__ T s_f[9 * (OX + 4) * (OY + 4)];
  const int li = xcd_remap ? xcd_tile((int)blockIdx.x, count) : (int)blockIdx.x;
  const int c = gcase[li];
  const LbmParams p = cases[c].p;
  lbm3_edge_group<T, OX, OY, true>(reinterpret_cast<const T *>(cases[c].pop[route_src(rt)]),
                                   reinterpret_cast<T *>(cases[c].pop[route_dst(rt)]), p, gtile[li] & ~kEdgeFlag,
                                   tile_x, tile_y, reinterpret_cast<T *>(cases[c].pop[2]),
                                   reinterpret_cast<T *>(cases[c].pop[3]), cases[c].near,
                                   mask_unstable ? p.flag : &kEdgeNoStop, s_f);
}

namespace {

size_t edge2_lds_bytes(int prec, int ox, int oy) { return 9 * ((size_t)ox + 2) * ((size_t)oy + 2) * (size_t)prec; }

bool has_edge3(int tx, int ty, int w, int h) {
#define S(TX, TY, W, H, OX, OY) \
  if (tx == TX && ty == TY && w == W && h == H) return true;
  BTDF_EDGE3_SHAPES(S)
#undef S
  return false;
}

}  // namespace

bool variant_has_edge(int variant, int prec, int depth, int code) {
  int tx, ty;
  variant_tile(variant, &tx, &ty);
  const int w = code & 15, h = (code >> 4) & 15;
  if (!is_edge(code) || !((h == 1 && (w == 1 || w == 2 || w == 4)) || (w == 1 && h == 4))) return false;
  // three steps: the shapes listed, where the launch shape has the interior
  // pass of its tile (the same LDS per node)
  if (depth == 3) return has_edge3(tx, ty, w, h) && variant_has_lbm3(variant, prec, kGroup1x1);
  return depth == 2 && tx >= 2 && edge2_lds_bytes(prec, w * tx, h * ty) <= 65536;
}

hipError_t launch_lbm_edge2(int prec, int variant, int code, const void *A, void *C, const LbmParams &p,
                            const int *map, int count, void *X, const unsigned char *near, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!variant_has_edge(variant, prec, 2, code)) return hipErrorInvalidValue;
  int tx, ty;
  variant_tile(variant, &tx, &ty);
  const int w = code & 15, h = (code >> 4) & 15;
  const size_t lds = edge2_lds_bytes(prec, w * tx, h * ty);
  if (prec == 4)
    hipLaunchKernelGGL(lbm_edge2_kernel<float>, dim3(count), dim3(256), lds, s, (const float *)A, (float *)C, p, map,
                       count, w, h, tx, ty, (float *)X, near);
  else
    hipLaunchKernelGGL(lbm_edge2_kernel<double>, dim3(count), dim3(256), lds, s, (const double *)A, (double *)C, p,
                       map, count, w, h, tx, ty, (double *)X, near);
  return hipGetLastError();
}

hipError_t launch_lbm_edge3(int prec, int variant, int code, const void *A, void *C, const LbmParams &p,
                            const int *map, int count, void *X1, void *X2, const unsigned char *near, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!variant_has_edge(variant, prec, 3, code)) return hipErrorInvalidValue;
  int tx, ty;
  variant_tile(variant, &tx, &ty);
  const int w = code & 15, h = (code >> 4) & 15;
#define S(TX, TY, W, H, OX, OY)                                                                                  \
  if (tx == TX && ty == TY && w == W && h == H) {                                                                \
    if (prec == 4)                                                                                               \
      hipLaunchKernelGGL((lbm3_edge_kernel<float, OX, OY>), dim3(count), dim3(OX, OY), 0, s, (const float *)A,   \
                         (float *)C, p, map, count, tx, ty, (float *)X1, (float *)X2, near);                     \
    else                                                                                                         \
      hipLaunchKernelGGL((lbm3_edge_kernel<double, OX, OY>), dim3(count), dim3(OX, OY), 0, s, (const double *)A, \
                         (double *)C, p, map, count, tx, ty, (double *)X1, (double *)X2, near);                  \
    return hipGetLastError();                                                                                    \
  }
  BTDF_EDGE3_SHAPES(S)
#undef S
  return hipErrorInvalidValue;
}

hipError_t launch_lbm_edge3_batch(int prec, int variant, int code, const CaseDesc *cases, const int *gcase,
                                  const int *gtile, int count, int rt, int mask, int xcd, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!variant_has_edge(variant, prec, 3, code)) return hipErrorInvalidValue;
  int tx, ty;
  variant_tile(variant, &tx, &ty);
  const int w = code & 15, h = (code >> 4) & 15;
#define S(TX, TY, W, H, OX, OY)                                                                                   \
  if (tx == TX && ty == TY && w == W && h == H) {                                                                 \
    if (prec == 4)                                                                                                \
      hipLaunchKernelGGL((lbm3_edge_batch_kernel<float, OX, OY>), dim3(count), dim3(OX, OY), 0, s, cases, gcase,  \
                         gtile, count, rt, mask, xcd, tx, ty);                                                    \
    else                                                                                                          \
      hipLaunchKernelGGL((lbm3_edge_batch_kernel<double, OX, OY>), dim3(count), dim3(OX, OY), 0, s, cases, gcase, \
                         gtile, count, rt, mask, xcd, tx, ty);                                                    \
    return hipGetLastError();                                                                                     \
  }
  BTDF_EDGE3_SHAPES(S)
#undef S
  return hipErrorInvalidValue;
}

}  // namespace btdf
