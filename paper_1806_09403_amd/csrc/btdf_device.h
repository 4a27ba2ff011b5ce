// btdf_device.h -- device-side building blocks of the BTDF-IB-LBM kernels:
// D2Q9 tables (eq 8 and the weights stated after eq 7), the regularised
// delta functions of Section 4.3 with their stencils, the streaming pull
// with the boundary handling, and the parameter blocks the kernels take.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btdf {

// ---- D2Q9, eq 8: e_0 .. e_8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)
__host__ __device__ __forceinline__ constexpr int ex(int q) {
  return (q == 1 || q == 5 || q == 8) ? 1 : ((q == 3 || q == 6 || q == 7) ? -1 : 0);
}
__host__ __device__ __forceinline__ constexpr int ey(int q) {
  return (q == 2 || q == 5 || q == 6) ? 1 : ((q == 4 || q == 7 || q == 8) ? -1 : 0);
}
__host__ __device__ __forceinline__ constexpr double wq(int q) {
  return q == 0 ? 4.0 / 9.0 : (q < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// direction with e_opp = -e_q
__host__ __device__ __forceinline__ constexpr int opp(int q) {
  return q == 0 ? 0 : (q < 5 ? ((q + 1) % 4) + 1 : ((q - 3) % 4) + 5);
}

// ---- delta kinds (same codes as the public header)
enum : int { kLinear2 = 2, kRoma3 = 3, kPeskin4 = 4, kCos4 = 5 };

// phi(r): eq 37, eq 38, eq 39, and the cosine 4-point kernel
__device__ __forceinline__ double phi(int kind, double r) {
  double a = fabs(r);
  if (kind == kLinear2) return a <= 1.0 ? 1.0 - a : 0.0;
  if (kind == kRoma3) {
    if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) * (1.0 / 3.0);
    if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(fmax(0.0, 1.0 - 3.0 * (1.0 - a) * (1.0 - a)))) * (1.0 / 6.0);
    return 0.0;
  }
  if (kind == kPeskin4) {
    if (a < 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(fmax(0.0, -7.0 + 12.0 * a - 4.0 * a * a))) * 0.125;
    return 0.0;
  }
  // kCos4
  return a <= 2.0 ? 0.25 * (1.0 + cospi(0.5 * a)) : 0.0;
}

// stencil nodes per direction: floor(X) .. +1 (2-point), floor(X+1/2)-1 .. +1
// (3-point), floor(X)-1 .. floor(X)+2 (4-point kernels)
__host__ __device__ __forceinline__ int stencil_size(int kind) {
  return kind == kLinear2 ? 2 : (kind == kRoma3 ? 3 : 4);
}
__host__ __device__ __forceinline__ int stencil_base(int kind, double X) {
  if (kind == kLinear2) return (int)floor(X);
  if (kind == kRoma3) return (int)floor(X + 0.5) - 1;
  return (int)floor(X) - 1;
}

// ---- parameters of one simulation, passed by value to every kernel
struct LbmParams {
  int nx, ny;       // nodes (ghost columns included)
  int pitch;        // elements between rows
  long long plane;  // elements between population planes
  int xper, yper;   // periodic flags
  int inlet, outlet;
  int i0, i1;       // fluid columns (inclusive)
  double omega;     // 1 / tau
  double guo;       // 1 - 1 / (2 tau)
  double Gx, Gy;    // uniform body-force density
  double uin_x, uin_y;
  // tiles of the lattice kernel
  int ntx, nty;
  int xcd_remap;
  int interior;          // 1: waves away from every edge take the uniform-base path
  // marker lists per tile (spread gather)
  const int *tile_off;   // [ntx*nty + 1]
  const int *tile_list;  // marker ids, ascending within a tile
  const void *mk_w;      // per marker, in the population type: wx[4], wy[4], drs ds F_x, drs ds F_y
  const int *mk_ixy;     // per marker: stencil origin (wrapped in periodic directions)
  int kind;
  long long *step_ctr;   // steps completed on the device
  int *flag;             // instability flag: 0 fine, 1 + body, -1 node
};

// tiles handled by one launch of the lattice kernel
struct TileRange {
  const int *map;  // tile ids; null = identity over all tiles
  int base, count; // launch covers map[base .. base+count)
  int count_step;  // this launch advances the device step counter
};

struct IbParams {
  int nb, nm;
  const int *body_off;  // [nb + 1]
  const int *mk_body;   // body of each marker
  const double *X, *Y, *U, *V;
  const double *cx, *cy;
  const double *body_sdrs;  // drs * ds per body
  const double *sdrs;       // drs * ds per marker
  double *Fx, *Fy, *rho_l, *ux_l, *uy_l;
  void *mk_w;               // spread weights and scaled forces for the lattice kernel
  int *mk_ixy;
  double *hist;  // [cap][nb][3]
  int hist_cap;
  int *slot;     // ring entry of the current step (written by the marker kernel)
};

// one case of a batch: its parameters and its two population buffers
struct CaseDesc {
  LbmParams p;
  IbParams ib;
  void *pop[2];
};

// where the workgroups of the batched launches go
struct BatchMap {
  const int *tile_case, *tile_local;  // per lattice workgroup: case and tile within the case
  const int *body_case, *body_local;  // per body-reduction workgroup
  const int *mblk_case, *mblk_first;  // per marker workgroup: case and its first marker
  int ntiles, nbodies, nmblk;
  int xcd_remap;
  int mask_unstable;  // skip the work of cases whose instability flag is set
};

// Streaming pull g_q(x, y) = f_q(x - e_q, y - e_q) with the boundary readings:
// periodic directions wrap, halfway bounce-back walls in y return the
// opposite population of the same node; channel ends read the ghost columns.
template <typename T, bool NTL = false>
__device__ __forceinline__ T load(const T *ptr) {
  if (NTL) return __builtin_nontemporal_load(ptr);
  return *ptr;
}

template <typename T, bool NTL = false>
__device__ __forceinline__ T pull(const T *__restrict__ A, const LbmParams &p, int q, int x, int y) {
  int sx = x - ex(q);
  int sy = y - ey(q);
  if (p.yper) {
    sy = sy < 0 ? sy + p.ny : (sy >= p.ny ? sy - p.ny : sy);
  } else if (sy < 0 || sy >= p.ny) {
    return load<T, NTL>(&A[(long long)opp(q) * p.plane + (long long)y * p.pitch + x]);
  }
  if (p.xper) sx = sx < 0 ? sx + p.nx : (sx >= p.nx ? sx - p.nx : sx);
  return load<T, NTL>(&A[(long long)q * p.plane + (long long)sy * p.pitch + sx]);
}

// Consecutive tiles go to the same XCD: hardware dispatches block b to XCD
// b % 8, so block b takes logical tile number (b % 8) * share + b / 8.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  int q = n >> 3, r = n & 7;
  int xcd = b & 7, j = b >> 3;
  return xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
}

}  // namespace btdf
