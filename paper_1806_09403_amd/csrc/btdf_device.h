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
// direction with (e_x, -e_y): the image of e_q in a wall parallel to x
__host__ __device__ __forceinline__ constexpr int mir_y(int q) {
  return q == 2 ? 4 : q == 4 ? 2 : q == 5 ? 8 : q == 8 ? 5 : q == 6 ? 7 : q == 7 ? 6 : q;
}
// direction with e_opp = -e_q
__host__ __device__ __forceinline__ constexpr int opp(int q) {
  return q == 0 ? 0 : (q < 5 ? ((q + 1) % 4) + 1 : ((q - 3) % 4) + 5);
}

// Populations are stored as deviations f_q - c_q from the equilibrium of a
// reference state, c_q = feq_q(1, u_ref) (eq 6), with u_ref the velocity the
// run starts from. sum_q c_q = 1 and sum_q e_q c_q = u_ref, so the stored
// values sum to rho - 1 and their first moment is m - u_ref: in a flow near
// its reference state every stored value, and every rounding error, is small.
__host__ __device__ __forceinline__ double ref_c(int q, double urx, double ury) {
#pragma clang fp contract(off)  // (the same bits on the host and the device)
  const double eu = ex(q) * urx + ey(q) * ury;
  return wq(q) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (urx * urx + ury * ury));
}

// ---- delta kinds (same codes as the public header)
enum : int { kLinear2 = 2, kRoma3 = 3, kPeskin4 = 4, kCos4 = 5 };

// sin(y) for |y| <= pi/2 by its Taylor series through y^21 (Horner in y^2;
// the first omitted term is below 1.2e-18 there), coefficients
// (-1)^k / (2k+1)!
__device__ __forceinline__ double sin_halfpi(double y) {
  constexpr double c[11] = {1.0,
                            -1.0 / 6.0,
                            1.0 / 120.0,
                            -1.0 / 5040.0,
                            1.0 / 362880.0,
                            -1.0 / 39916800.0,
                            1.0 / 6227020800.0,
                            -1.0 / 1307674368000.0,
                            1.0 / 355687428096000.0,
                            -1.0 / 121645100408832000.0,
                            1.0 / 51090942171709440000.0};
  const double y2 = y * y;
  double s = c[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) s = fma(s, y2, c[k]);
  return y * s;
}

// phi(r): eq 37, eq 38, eq 39, and the cosine 4-point kernel; the cosine
// kernel's cos(pi a / 2) for a in [0, 2] is -sin(pi (a - 1) / 2)
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
  return a <= 2.0 ? 0.25 * (1.0 - sin_halfpi(M_PI_2 * (a - 1.0))) : 0.0;
}

// d phi / d r of the same kernels (the adjoint's position derivatives; LINEAR2
// takes -sign(r) away from its kink at r = 0)
__device__ __forceinline__ double dphi(int kind, double r) {
  const double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
  if (kind == kLinear2) return a < 1.0 ? -sg : 0.0;
  if (kind == kRoma3) {
    if (a <= 0.5) return sg * (-a / sqrt(1.0 - 3.0 * a * a));
    if (a < 1.5) {
      const double b = 1.0 - a;
      return sg * (-3.0 - 3.0 * b / sqrt(fmax(1e-300, 1.0 - 3.0 * b * b))) * (1.0 / 6.0);
    }
    return 0.0;
  }
  if (kind == kPeskin4) {
    if (a < 1.0) return sg * (-2.0 + (2.0 - 4.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a < 2.0) return sg * (-2.0 - (6.0 - 4.0 * a) / sqrt(fmax(1e-300, -7.0 + 12.0 * a - 4.0 * a * a))) * 0.125;
    return 0.0;
  }
  return a <= 2.0 ? -sg * (0.125 * M_PI) * sinpi(0.5 * a) : 0.0;
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

// ---- per-launch constants of the collision (eqs 5-7, 11), in the population
// type; formed once on the host so the kernels read them from scalar registers

template <typename T>
struct CollK {
  T omega, omc;  // omega, 1 - omega
  T a9, a36;     // 4.5 omega w, for w = 1/9 (axes) and w = 1/36 (diagonals)
  T b9, b36;     // 3 omega w
  T c9, c36;     // 9 guo w
  T d9, d36;     // 3 guo w
  T m3g;         // -3 guo
  T urx, ury;    // reference velocity
  T cu5, cu6;    // e.u_ref of the diagonal pairs: urx + ury, ury - urx
};

// The factors of the Guo term that depend on the force density f only, per
// direction pair (1,3), (2,4), (5,7), (6,8) with e.f = f_x, f_y, f_x + f_y,
// f_y - f_x: ev = 9 guo w e.f (even part), od = 3 guo w e.f (odd part);
// g = -3 guo f (isotropic part, taken times u). Plain products and sums, so
// the host and the device form the same bits from the same f.
template <typename T>
struct ForceK {
  T fx, fy, gx, gy;
  T ev[4], od[4];
};

template <typename T>
__host__ __device__ inline ForceK<T> force_terms(const CollK<T> &k, T fx, T fy) {
#pragma clang fp contract(off)
  ForceK<T> f;
  const T e[4] = {fx, fy, fx + fy, fy - fx};
  f.fx = fx;
  f.fy = fy;
  f.gx = k.m3g * fx;
  f.gy = k.m3g * fy;
  for (int i = 0; i < 4; ++i) {
    f.ev[i] = (i < 2 ? k.c9 : k.c36) * e[i];
    f.od[i] = (i < 2 ? k.d9 : k.d36) * e[i];
  }
  return f;
}

// ---- parameters of one simulation, passed by value to every kernel
struct LbmParams {
  int nx, ny;       // nodes (ghost columns included)
  int pitch;        // elements between rows
  long long plane;  // elements between population planes
  int xper, yper;   // periodic flags
  int inlet, outlet;  // outlet: 1 zero-gradient, 2 convective (speed uconv)
  int slip;           // south/north walls: 0 bounce-back, 1 free-slip (specular)
  double uconv;
  int i0, i1;       // fluid columns (inclusive)
  double omega;     // 1 / tau
  double guo;       // 1 - 1 / (2 tau)
  double Gx, Gy;    // uniform body-force density
  double uin_x, uin_y;
  double urx, ury;  // reference velocity: populations are stored as f_q - feq_q(1, u_ref)
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
  const void *konst;     // device copy of the per-direction constants (fill_konst)
  // collision constants and the uniform body force's Guo factors, per precision
  CollK<float> kf;
  CollK<double> kd;
  ForceK<float> gf;
  ForceK<double> gd;
};

// the collision constants of tau-derived omega and guo and of u_ref, rounded
// once from FP64
template <typename T>
inline CollK<T> make_coll(double omega, double guo, double urx, double ury) {
  CollK<T> k;
  k.omega = (T)omega;
  k.omc = (T)(1.0 - omega);
  k.a9 = (T)(0.5 * omega);
  k.a36 = (T)(0.125 * omega);
  k.b9 = (T)(omega / 3.0);
  k.b36 = (T)(omega / 12.0);
  k.c9 = (T)guo;
  k.c36 = (T)(0.25 * guo);
  k.d9 = (T)(guo / 3.0);
  k.d36 = (T)(guo / 12.0);
  k.m3g = (T)(-3.0 * guo);
  k.urx = (T)urx;
  k.ury = (T)ury;
  k.cu5 = (T)(urx + ury);
  k.cu6 = (T)(ury - urx);
  return k;
}

// fill the constants of p from its omega, guo, reference velocity and body force
inline void fill_collision(LbmParams &p) {
  p.kf = make_coll<float>(p.omega, p.guo, p.urx, p.ury);
  p.kd = make_coll<double>(p.omega, p.guo, p.urx, p.ury);
  p.gf = force_terms<float>(p.kf, (float)p.Gx, (float)p.Gy);
  p.gd = force_terms<double>(p.kd, p.Gx, p.Gy);
}

template <typename T>
__device__ __forceinline__ const CollK<T> &coll(const LbmParams &p);
template <>
__device__ __forceinline__ const CollK<float> &coll<float>(const LbmParams &p) { return p.kf; }
template <>
__device__ __forceinline__ const CollK<double> &coll<double>(const LbmParams &p) { return p.kd; }
template <typename T>
__device__ __forceinline__ const ForceK<T> &gforce(const LbmParams &p);
template <>
__device__ __forceinline__ const ForceK<float> &gforce<float>(const LbmParams &p) { return p.gf; }
template <>
__device__ __forceinline__ const ForceK<double> &gforce<double>(const LbmParams &p) { return p.gd; }

// tiles handled by one launch of the lattice kernel
struct TileRange {
  const int *map;  // tile ids; null = identity over all tiles
  int base, count; // launch covers map[base .. base+count)
  int count_step;  // this launch advances the device step counter
};

// rigid body motion, one workgroup per body after each step
struct MoveParams {
  int nb;
  const int *body_off;
  const int *moving;   // [nb]
  double *state;       // [nb][4]: theta, vx, vy, omega
  double *cx, *cy;     // body centres
  double *X, *Y, *U, *V;
  const double *rxy;   // [nm][2]: offset from the centre at angle 0
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
  // forcing passes per step (Algorithm 1 step 3; eqs 29-31 when nf > 1)
  int nf;
  const int *cover_off, *cover_list;  // per marker and stencil lane: covering markers (see AdjParams)
  double *mdf_cache;                  // [nm][16][3]: rho, u*_x, u*_y at each stencil node
  double *mdf_w;                      // [nm][8]: x then y delta weights in FP64
  // comparison forcing methods (Section 3)
  int method;                         // 0 direct, 1 implicit (eq 17), 2 RKPM (eq B54)
  int max_body;                       // markers of the largest body
  const double *minv;                 // implicit: (D_I D_E)^-1 of each body, column-major
  const long long *minv_off;          // implicit: start of body b's matrix
  double *mdf_f;                      // [2][nm][2]: accumulated force after the previous / this pass
};

// one case of a batch: its parameters and its two population buffers
struct CaseDesc {
  LbmParams p;
  IbParams ib;
  void *pop[4];                // the two ping-pong buffers, then the near tiles' states n+1 and n+2 (blocking)
  const unsigned char *near;   // per lattice tile: 1 if it steps singly (blocking)
};

// a batch launch's source and destination buffers (indices into CaseDesc::pop)
__host__ __device__ inline int route(int src, int dst) { return src | (dst << 2); }
__host__ __device__ inline int route_src(int r) { return r & 3; }
__host__ __device__ inline int route_dst(int r) { return r >> 2; }

// the adjoint (reverse) step: its own 64 x 4 tiling of the lattice with the
// markers binned per tile
constexpr int kAdjTX = 64, kAdjTY = 4;
struct AdjParams {
  int ntx, nty;                     // adjoint tiles
  const int *tile_off, *tile_list;  // markers whose stencil touches each tile, ascending
  // for each marker l and stencil lane k (16 per marker), the markers whose
  // stencil covers that node, ascending, packed as (marker << 4) | (dx << 2) | dy
  const int *node_off, *node_list;
  double *part;  // [tiles][4]: dJ/dG (x, y), dJ/du_in (x, y), summed over steps per tile
  // marker side (one entry per marker)
  const double *Fx, *Fy, *rho_l, *ux_l, *uy_l;  // forward values of the step being reversed
  double *mk_adj;                                // [nm][3]: dJ/d rho_l, dJ/d u*_l (x, y)
  double *xy_bar, *uv_bar;                       // [nm][2] each, summed over steps
  double *c_bar;                                 // [nm][2]: each marker's share of dJ/d(body centre)
  const double *hist_bar;                        // [nb][3]: weights of this step's body forces
};

// where the workgroups of the batched launches go
struct BatchMap {
  const int *tile_case, *tile_local;  // per lattice workgroup: case and tile within the case
  const int *body_case, *body_local;  // per body-reduction workgroup
  const int *mblk_case, *mblk_first;  // per marker workgroup: case and its first marker
  int ntiles, nbodies, nmblk;
  int ncases;  // lattice launches: one step-counter workgroup per case past the bodies
  int xcd_remap;
  int mask_unstable;  // skip the work of cases whose instability flag is set
};

// ---- arithmetic shared by the forward and adjoint kernels
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T recip(T x);
// FP32: the hardware reciprocal refined by one Newton step. The bare
// reciprocal is within an ulp but not unbiased; used for u = (m + f/2) / rho
// every step, its bias acts like a small body force and shifts long runs.
template <>
__device__ __forceinline__ float recip<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
template <>
__device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }

// On gfx950 a wave holding more than 80 scalar registers (96 once rounded
// up) leaves room for fewer waves per SIMD than the vector registers allow:
// a 1024-thread workgroup of such waves fits once per CU instead of twice,
// and 256-thread workgroups fit six or seven per SIMD instead of eight.
// Kernels that would exceed it take this cap (the few values beyond it go
// to vector register lanes).
#define kSgprCap __attribute__((amdgpu_num_sgpr(80)))

// A wave-uniform pointer pinned to scalar registers, so that an access
// through it plus a 32-bit lane offset is one load or store with a scalar
// base (the compiler may otherwise fold the uniform part into a 64-bit
// per-lane address and spend vector instructions on every access).
// (The result is a global-memory pointer, so accesses stay global ones.)
template <typename P>
using global_ptr = __attribute__((address_space(1))) P *;
template <typename P>
__device__ __forceinline__ global_ptr<P> uniform_ptr(P *ptr) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(ptr);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (global_ptr<P>)(((unsigned long long)hi << 32) | lo);
}
// A load through a pointer into device memory, as a global access: pointers
// read from memory (a batch's case table) are otherwise taken as flat, whose
// accesses need a 64-bit address per lane and wait on the LDS counter too.
template <typename T>
__device__ __forceinline__ T load_global(const char *base, unsigned off) {
  return *(global_ptr<const T>)((global_ptr<const char>)base + off);
}
// element i of an array in device memory, as a global access
template <typename T>
__device__ __forceinline__ T ldg(const T *ptr, long long i) {
  return *((global_ptr<const T>)ptr + i);
}

// store v at byte offset off from a uniform global base (nontemporal if NT)
template <typename T, bool NT>
__device__ __forceinline__ void store_uniform(global_ptr<char> base, unsigned off, T v) {
  global_ptr<T> ptr = (global_ptr<T>)(base + off);
  if (NT)
    __builtin_nontemporal_store(v, ptr);
  else
    *ptr = v;
}

// fused multiply-add, spelled out: a * b + c rounded once
__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Corrected velocity (eq 11), equilibrium (eq 6), Guo term (eq 7) and BGK
// relaxation (eq 5) on the stored deviations g~_q = g_q - c_q of one node:
//   out~_q = (1 - omega) g~_q + omega (feq_q - c_q) + F_q.
// With drho = rho - 1, du = u - u_ref (both formed from small terms only),
// eu = e.u, ea = e.du, cu = e.u_ref and ef = e.f, opposite directions share
// the even part and differ in the sign of the odd part:
//   s    = drho eu + ea            (= rho eu - cu)
//   even = w C + 4.5 omega w (s eu + cu ea) + eu (9 guo w ef)
//   odd  = 3 omega w s + 3 guo w ef
//   C    = omega (drho (1 - 1.5 |u|^2) - 1.5 du.(u + u_ref)) - 3 guo u.f
// (s eu + cu ea = drho eu^2 + ea (eu + cu): the quadratic term of feq less
// that of c_q, written in small terms; with u_ref = 0 this is omega feq~ + F
// of the plain deviations f - w). The products of constants (and of
// constants and f) come in through k and f, so a kernel whose force is
// uniform takes them from scalar registers.
template <typename T>
__device__ __forceinline__ void collide(const T g[9], const ForceK<T> &f, const CollK<T> &k, T out[9], T &rho) {
  // Every multiply-add is written out and nothing else is fused, so the same
  // inputs give the same bits whichever kernel the collision is inlined into
  // (left to itself the compiler fuses differently once it hoists common
  // terms, as in the two-step kernel).
#pragma clang fp contract(off)
  const T drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  rho = (T)1 + drho;
  const T d57 = g[5] - g[7], d86 = g[8] - g[6];  // the diagonals' shares of m - u_ref
  const T mx = (g[1] - g[3]) + (d57 + d86);
  const T my = (g[2] - g[4]) + (d57 - d86);
  const T inv = recip<T>(rho);
  const T dux = fmx(-drho, k.urx, fmx((T)0.5, f.fx, mx)) * inv;
  const T duy = fmx(-drho, k.ury, fmx((T)0.5, f.fy, my)) * inv;
  const T ux = k.urx + dux, uy = k.ury + duy;
  const T sx = ux + k.urx, sy = uy + k.ury;
  const T a = fmx((T)-1.5, fmx(ux, ux, uy * uy), (T)1);
  const T c1 = fmx(drho, a, (T)-1.5 * fmx(dux, sx, duy * sy));
  const T C = fmx(k.omega, c1, fmx(ux, f.gx, uy * f.gy));
  const T C9 = C * (T)(1.0 / 9.0), C36 = C * (T)(1.0 / 36.0);
  out[0] = fmx(k.omc, g[0], (T)(4.0 / 9.0) * C);
  auto pair = [&](int qp, int qm, T eu, T ea, T cu, T ev, T od, T ka, T kb, T wC) {
    const T sq = fmx(drho, eu, ea);
    const T t = fmx(sq, eu, cu * ea);
    const T even = fmx(ka, t, fmx(eu, ev, wC));
    const T odd = fmx(kb, sq, od);
    out[qp] = fmx(k.omc, g[qp], even) + odd;
    out[qm] = fmx(k.omc, g[qm], even) - odd;
  };
  pair(1, 3, ux, dux, k.urx, f.ev[0], f.od[0], k.a9, k.b9, C9);
  pair(2, 4, uy, duy, k.ury, f.ev[1], f.od[1], k.a9, k.b9, C9);
  pair(5, 7, ux + uy, dux + duy, k.cu5, f.ev[2], f.od[2], k.a36, k.b36, C36);
  pair(6, 8, uy - ux, duy - dux, k.cu6, f.ev[3], f.od[3], k.a36, k.b36, C36);
}

// the density of a collision is positive and finite: one class test
// (+subnormal or +normal), the same set as rho > 0 && isfinite(rho)
template <typename T>
__device__ __forceinline__ bool rho_ok(T rho) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_classf(rho, 0x180);  // (the FP32 test: no conversion to FP64)
  else
    return __builtin_amdgcn_class(rho, 0x180);
}
// a wave's lanes whose density is not: one mask for the whole wave, kept
// in scalar registers
template <typename T>
__device__ __forceinline__ unsigned long long bad_lanes(T rho) {
  return __builtin_amdgcn_ballot_w64(!rho_ok(rho));
}

// The inlet ghost column after a step: eq 6 at the inflow velocity and
// column 1's density. As stored deviations, feq_q(1 + dr, u_in) - c_q =
// w (dr a_q + b_q) with a_q = 1 + P(u_in), b_q = P(u_in) - P(u_ref), P(u) =
// 3 e.u + 4.5 (e.u)^2 - 1.5 |u|^2, and dr the sum of column 1's
// post-collision deviations (inlet_dr). The single-step kernels form a and b
// in FP64 as they go (inlet_ghost_calc); the edge kernels of the blocked
// pass read them, and the wall shifts of pull(), from a table the host
// fills once (fill_konst, kernel parameter konst). Both take the same FP64
// operations in the same order without contraction, so they agree bit for
// bit.
template <typename T>
__device__ __forceinline__ T inlet_dr(const T (&out)[9]) {
  T dr = out[0];
#pragma unroll
  for (int q = 1; q < 9; ++q) dr += out[q];
  return dr;
}

__host__ __device__ __forceinline__ double inlet_a(const LbmParams &p, int q) {
#pragma clang fp contract(off)
  const double ein = ex(q) * p.uin_x + ey(q) * p.uin_y;
  return 1.0 + (3.0 * ein + 4.5 * ein * ein - 1.5 * (p.uin_x * p.uin_x + p.uin_y * p.uin_y));
}

__host__ __device__ __forceinline__ double inlet_b(const LbmParams &p, int q) {
#pragma clang fp contract(off)
  const double ein = ex(q) * p.uin_x + ey(q) * p.uin_y;
  const double pin = 3.0 * ein + 4.5 * ein * ein - 1.5 * (p.uin_x * p.uin_x + p.uin_y * p.uin_y);
  return pin - (ref_c(q, p.urx, p.ury) / wq(q) - 1.0);
}

template <typename T>
__device__ __forceinline__ T inlet_ghost_calc(T dr, const LbmParams &p, int q) {
#pragma clang fp contract(off)
  return (T)wq(q) * (dr * (T)inlet_a(p, q) + (T)inlet_b(p, q));
}

// the shift of a population pulled from beyond a halfway bounce-back wall
// (the stored opposite population moved from its offset c_opp to c_q) and
// from beyond a free-slip wall (the mirror population moved from c_mir)
__host__ __device__ __forceinline__ double wall_bb(const LbmParams &p, int q) {
#pragma clang fp contract(off)
  return -6.0 * wq(q) * (ex(q) * p.urx + ey(q) * p.ury);
}

__host__ __device__ __forceinline__ double wall_slip(const LbmParams &p, int q) {
#pragma clang fp contract(off)
  return -6.0 * wq(q) * ey(q) * p.ury * (1.0 + 3.0 * ex(q) * p.urx);
}

// the table: per precision (FP32, then FP64) a[9], b[9], bounce-back[9], slip[9]
constexpr int kKonstBytes = 36 * 4 + 36 * 8;

inline void fill_konst(const LbmParams &p, unsigned char (&out)[kKonstBytes]) {
  float f[36];
  double d[36];
  for (int q = 0; q < 9; ++q) {
    d[q] = inlet_a(p, q);
    d[9 + q] = inlet_b(p, q);
    d[18 + q] = wall_bb(p, q);
    d[27 + q] = wall_slip(p, q);
  }
  for (int k = 0; k < 36; ++k) f[k] = (float)d[k];
  __builtin_memcpy(out, f, sizeof f);
  __builtin_memcpy(out + sizeof f, d, sizeof d);
}

// the table's entries of precision T: k[q] = a, k[9 + q] = b, k[18 + q] =
// bounce-back shift, k[27 + q] = slip shift
template <typename T>
__device__ __forceinline__ const T *konst(const LbmParams &p) {
  return reinterpret_cast<const T *>(static_cast<const char *>(p.konst) + (sizeof(T) == 4 ? 0 : 36 * 4));
}

template <typename T>
__device__ __forceinline__ T inlet_ghost(T dr, const LbmParams &p, int q) {
#pragma clang fp contract(off)
  const T *k = konst<T>(p);
  return (T)wq(q) * (dr * ldg(k, q) + ldg(k, 9 + q));
}

// Streaming pull g_q(x, y) = f_q(x - e_q, y - e_q), as a stored deviation,
// with the boundary readings: periodic directions wrap, halfway bounce-back
// walls in y return the opposite population of the same node; channel ends
// read the ghost columns.
template <typename T, bool NTL = false>
__device__ __forceinline__ T load(const T *ptr) {
  const global_ptr<const T> g = (global_ptr<const T>)ptr;  // device memory: a global access
  if (NTL) return __builtin_nontemporal_load(g);
  return *g;
}

template <typename T, bool NTL = false>
__device__ __forceinline__ T pull(const T *__restrict__ A, const LbmParams &p, int q, int x, int y) {
  // the wall shifts are added as written (no fused multiply-add with the
  // load), so every kernel that pulls a wall population rounds it alike
#pragma clang fp contract(off)
  int sx = x - ex(q);
  int sy = y - ey(q);
  if (p.yper) {
    sy = sy < 0 ? sy + p.ny : (sy >= p.ny ? sy - p.ny : sy);
  } else if (sy < 0 || sy >= p.ny) {
    if (p.slip) {
      // specular: the mirror population of the upstream column, moved from
      // its offset c_mir to c_q (feq difference of (e_x, -e_y) and e_q)
      if (p.xper) sx = sx < 0 ? sx + p.nx : (sx >= p.nx ? sx - p.nx : sx);
      return load<T, NTL>(&A[(long long)mir_y(q) * p.plane + (long long)y * p.pitch + sx]) + (T)wall_slip(p, q);
    }
    // the stored opposite population, moved from its offset c_opp to c_q
    return load<T, NTL>(&A[(long long)opp(q) * p.plane + (long long)y * p.pitch + x]) + (T)wall_bb(p, q);
  }
  if (p.xper) sx = sx < 0 ? sx + p.nx : (sx >= p.nx ? sx - p.nx : sx);
  return load<T, NTL>(&A[(long long)q * p.plane + (long long)sy * p.pitch + sx]);
}

// The periodic image of a node index in [0, n): ((i mod n) + n) mod n,
// with one unsigned compare for an index already in range (the usual case:
// stencils reach at most a few nodes past an edge).
__host__ __device__ __forceinline__ int wrap_index(int i, int n) {
  if ((unsigned)i < (unsigned)n) return i;
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Consecutive tiles go to the same XCD: hardware dispatches block b to XCD
// b % 8, so block b takes logical tile number (b % 8) * share + b / 8.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  int q = n >> 3, r = n & 7;
  int xcd = b & 7, j = b >> 3;
  return xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
}

// The ring directions of an edge node of a group of W x H lattice tiles:
// bit q set when the neighbour x + e_q lies in a near tile. s_near holds the
// near flags of the tiles around the group (row 0 below it, column 0 left of
// it; the group's own tiles read 0).
template <int OX, int OY, int NR>
__device__ __forceinline__ unsigned ring_mask(const unsigned char (&s_near)[NR][8], int ii, int jj, int W, int H,
                                              int shx, int shy) {
  const int cl = ii == 0 ? 0 : 1 + ((ii - 1) >> shx), cm = 1 + (ii >> shx);
  const int cr = ii == OX - 1 ? W + 1 : 1 + ((ii + 1) >> shx);
  const int rd = jj == 0 ? 0 : 1 + ((jj - 1) >> shy), rm = 1 + (jj >> shy);
  const int ru = jj == OY - 1 ? H + 1 : 1 + ((jj + 1) >> shy);
  unsigned m = 0;
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    const int r = ey(q) < 0 ? rd : (ey(q) > 0 ? ru : rm);
    const int c = ex(q) < 0 ? cl : (ex(q) > 0 ? cr : cm);
    m |= s_near[r][c] ? 1u << q : 0u;
  }
  return m;
}

}  // namespace btdf
