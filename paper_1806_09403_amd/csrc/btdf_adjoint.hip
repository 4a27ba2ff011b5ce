// btdf_adjoint.hip -- reverse mode over a horizon of n steps.
//
// btdf_adjoint runs n forward steps from the handle's state (exactly as
// btdf_step would: same kernels, same history ring, same final state), then
// sweeps back through them with the adjoint kernels. States of the forward
// run are kept either all (a tape: no recomputation, n states of memory) or
// every K-th as a checkpoint (K defaults to ceil(sqrt(n))); the sweep then
// takes the segments from last to first, recomputes each segment's states
// from its checkpoint, and reverses the segment's steps. The recomputation
// runs the same deterministic kernels on the same inputs, so both modes give
// bit-identical gradients.
//
// Workspace (one region, 256-byte-aligned parts):
//   [ checkpoints or tape states | segment states | G x 2 | marker scratch |
//     adjoint tile bins | node records | tile sums | weights of the history |
//     control + one history slot | dJ/dA_0 in FP64 ]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "btdf_internal.h"

using namespace btdf;
using namespace btdf::host;

namespace {

struct AdjLayout {
  int64_t n = 0, K = 0;
  bool tape = false;
  int64_t n_store = 0;  // tape states (tape) or checkpoints (segments)
  int64_t n_seg = 0;    // segment states (checkpoint mode)
  size_t state = 0;     // bytes of one population state
  size_t off_store = 0, off_seg = 0, off_g[2] = {0, 0};
  size_t off_mk = 0, off_mkw = 0, off_mkixy = 0, off_mkadj = 0, off_xyb = 0, off_uvb = 0, off_cb = 0;
  size_t off_toff = 0, off_tlist = 0, off_tslot = 0, off_forced = 0, off_rec = 0, off_part = 0;
  size_t off_hbar = 0, off_ctl = 0, off_hist1 = 0, off_out = 0, total = 0;
  // adjoint tiles and their markers
  int ntx = 0, nty = 0, nforced = 0;
  std::vector<int> toff, tlist, tslot, forced;
};

int64_t default_K(int64_t n) {
  int64_t K = (int64_t)std::ceil(std::sqrt((double)n));
  return std::max<int64_t>(1, K);
}

void adj_layout(const btdf_t *h, int64_t n, int64_t K, AdjLayout *L) {
  L->n = n;
  L->K = K > 0 ? K : default_K(n);
  L->tape = L->K >= n;
  L->state = align256(9 * (size_t)h->plane * (size_t)h->prec);
  if (L->tape) {
    L->n_store = std::max<int64_t>(0, n - 1);  // states 1 .. n-1 (state 0 stays in the handle)
    L->n_seg = 0;
  } else {
    L->n_store = (n + L->K - 1) / L->K;  // checkpoints at t = 0, K, 2K, ...
    L->n_seg = L->K - 1;                 // states t0+1 .. t0+K-1 of one segment
  }
  L->ntx = (h->nx + kAdjTX - 1) / kAdjTX;
  L->nty = (h->ny + kAdjTY - 1) / kAdjTY;
  const int ntiles = L->ntx * L->nty;
  bin_markers(h, kAdjTX, kAdjTY, L->ntx, L->nty, L->toff, L->tlist);
  L->tslot.assign(ntiles, -1);
  L->forced.clear();
  for (int t = 0; t < ntiles; ++t)
    if (L->toff[t + 1] > L->toff[t]) {
      L->tslot[t] = (int)L->forced.size();
      L->forced.push_back(t);
    }
  L->nforced = (int)L->forced.size();

  const size_t M = (size_t)std::max(h->nm(), 1), B = (size_t)std::max(h->nb(), 1), d = sizeof(double);
  size_t o = 0;
  L->off_store = o;
  o += (size_t)L->n_store * L->state;
  L->off_seg = o;
  o += (size_t)L->n_seg * L->state;
  L->off_g[0] = o;
  o += L->state;
  L->off_g[1] = o;
  o += L->state;
  L->off_mk = o;  // Fx Fy rho_l ux_l uy_l
  o = align256(o + 5 * M * d);
  L->off_mkw = o;
  o = align256(o + 10 * M * (size_t)h->prec);
  L->off_mkixy = o;
  o = align256(o + 2 * M * sizeof(int));
  L->off_mkadj = o;
  o = align256(o + 3 * M * d);
  L->off_xyb = o;
  o = align256(o + 2 * M * d);
  L->off_uvb = o;
  o = align256(o + 2 * M * d);
  L->off_cb = o;
  o = align256(o + 2 * M * d);
  L->off_toff = o;
  o = align256(o + (size_t)(ntiles + 1) * sizeof(int));
  L->off_tlist = o;
  o = align256(o + L->tlist.size() * sizeof(int));
  L->off_tslot = o;
  o = align256(o + (size_t)ntiles * sizeof(int));
  L->off_forced = o;
  o = align256(o + (size_t)std::max(L->nforced, 1) * sizeof(int));
  L->off_rec = o;
  o = align256(o + (size_t)std::max(L->nforced, 1) * kAdjTX * kAdjTY * kAdjRec * d);
  L->off_part = o;
  o = align256(o + (size_t)ntiles * 4 * d);
  L->off_hbar = o;
  o = align256(o + (size_t)std::max<int64_t>(n, 1) * B * 3 * d);
  L->off_ctl = o;
  o = align256(o + 256);
  L->off_hist1 = o;
  o = align256(o + B * 3 * d);
  L->off_out = o;
  o = align256(o + 9 * (size_t)h->nx * h->ny * d);
  L->total = o;
}

int put(hipStream_t s, char *base, size_t off, const void *src, size_t bytes) {
  if (bytes) HIPCHK(hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s));
  return ok();
}

int adjoint_impl(btdf_t *h, int64_t n, int64_t K, const double *hist_bar, btdf_gradients *gr, char *w,
                 size_t wbytes, double *ms) {
  AdjLayout L;
  adj_layout(h, n, K, &L);
  char *own = nullptr;
  if (w == nullptr) {
    hipError_t e = hipMalloc((void **)&own, L.total);
    if (e != hipSuccess) return fail(BTDF_ENOMEM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
    w = own;
  } else if (wbytes < L.total) {
    return fail(BTDF_ENOMEM, "adjoint workspace has %zu bytes, %zu needed", wbytes, L.total);
  } else if ((uintptr_t)w & 255) {
    return fail(BTDF_EINVAL, "adjoint workspace must be 256-byte aligned");
  }
  struct Free {
    char *p;
    ~Free() {
      if (p) (void)hipFree(p);
    }
  } guard{own};

  hipStream_t s = h->stream;
  const int nb = h->nb(), nm = h->nm();
  const int ntiles = L.ntx * L.nty;
  const size_t M = (size_t)std::max(nm, 1), d = sizeof(double);
  int rc;
  // bins, history weights, zeroed sums
  if ((rc = put(s, w, L.off_toff, L.toff.data(), L.toff.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_tlist, L.tlist.data(), L.tlist.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_tslot, L.tslot.data(), L.tslot.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_forced, L.forced.data(), L.forced.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_hbar, hist_bar, (size_t)n * nb * 3 * d)))
    return rc;
  HIPCHK(hipMemsetAsync(w + L.off_xyb, 0, 2 * M * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_uvb, 0, 2 * M * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_cb, 0, 2 * M * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_part, 0, (size_t)ntiles * 4 * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_ctl, 0, 256, s));
  HIPCHK(hipMemsetAsync(w + L.off_g[0], 0, L.state, s));  // dJ/dA_n = 0: J reads the history only

  // the handle's parameters (forward run: its ring, counter and flag), and a
  // copy whose marker outputs, counter, flag and ring go to the scratch (the
  // recomputation and the sweep leave the handle's view untouched)
  const LbmParams p = make_params(h);
  const IbParams ib = make_ib(h);
  LbmParams pa = p;
  IbParams iba = ib;
  double *mk = reinterpret_cast<double *>(w + L.off_mk);
  iba.Fx = mk;
  iba.Fy = mk + M;
  iba.rho_l = mk + 2 * M;
  iba.ux_l = mk + 3 * M;
  iba.uy_l = mk + 4 * M;
  iba.mk_w = w + L.off_mkw;
  iba.mk_ixy = reinterpret_cast<int *>(w + L.off_mkixy);
  iba.hist = reinterpret_cast<double *>(w + L.off_hist1);
  iba.hist_cap = 1;
  iba.slot = reinterpret_cast<int *>(w + L.off_ctl + 16);
  pa.mk_w = iba.mk_w;
  pa.mk_ixy = iba.mk_ixy;
  pa.step_ctr = reinterpret_cast<long long *>(w + L.off_ctl);
  pa.flag = reinterpret_cast<int *>(w + L.off_ctl + 8);

  AdjParams a{};
  a.ntx = L.ntx;
  a.nty = L.nty;
  a.tile_off = reinterpret_cast<const int *>(w + L.off_toff);
  a.tile_list = reinterpret_cast<const int *>(w + L.off_tlist);
  a.tile_slot = reinterpret_cast<const int *>(w + L.off_tslot);
  a.forced = reinterpret_cast<const int *>(w + L.off_forced);
  a.nforced = L.nforced;
  a.rec = reinterpret_cast<double *>(w + L.off_rec);
  a.part = reinterpret_cast<double *>(w + L.off_part);
  a.Fx = iba.Fx;
  a.Fy = iba.Fy;
  a.rho_l = iba.rho_l;
  a.ux_l = iba.ux_l;
  a.uy_l = iba.uy_l;
  a.mk_adj = reinterpret_cast<double *>(w + L.off_mkadj);
  a.xy_bar = reinterpret_cast<double *>(w + L.off_xyb);
  a.uv_bar = reinterpret_cast<double *>(w + L.off_uvb);
  a.c_bar = reinterpret_cast<double *>(w + L.off_cb);
  const double *hbar_dev = reinterpret_cast<const double *>(w + L.off_hbar);

  std::vector<hipEvent_t> ev;
  auto mark = [&](hipEvent_t *e) -> int {
    HIPCHK(hipEventCreate(e));
    HIPCHK(hipEventRecord(*e, s));
    return ok();
  };
  struct Events {
    std::vector<hipEvent_t> *v;
    ~Events() {
      for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    }
  } evguard{&ev};
  ev.reserve(4 + 2 * (size_t)L.n_store);
  hipEvent_t e;
  if ((rc = mark(&e))) return rc;
  ev.push_back(e);

  // ---- forward run
  const int nt = h->ntx * h->nty;
  const int cur0 = h->cur;
  char *state0 = h->ws + h->off_pop[cur0];
  auto store_state = [&](int64_t i) { return w + L.off_store + (size_t)i * L.state; };
  auto seg_state = [&](int64_t i) { return w + L.off_seg + (size_t)i * L.state; };
  const size_t copy_bytes = 9 * (size_t)h->plane * (size_t)h->prec;
  if (L.tape) {
    // state t of the run: t = 0 in the handle's buffer, 1 .. n-1 in the tape,
    // n in the handle's other buffer
    for (int64_t t = 0; t < n; ++t) {
      const void *A = t == 0 ? (const void *)state0 : (const void *)store_state(t - 1);
      void *B = t == n - 1 ? (void *)(h->ws + h->off_pop[1 - cur0]) : (void *)store_state(t);
      HIPCHK(launch_ib(h->prec, A, p, ib, s));
      HIPCHK(launch_lbm(h->prec, h->variant, A, B, p, TileRange{nullptr, 0, nt, 1}, ib, s));
    }
    h->cur = 1 - cur0;
    h->steps += n;
  } else {
    for (int64_t t = 0; t < n; ++t) {
      if (t % L.K == 0)
        HIPCHK(hipMemcpyAsync(store_state(t / L.K), h->ws + h->off_pop[h->cur], copy_bytes,
                              hipMemcpyDeviceToDevice, s));
      if ((rc = enqueue_step(h, p, ib, h->cur, s, nullptr))) return rc;
      h->cur ^= 1;
      h->steps++;
    }
  }
  if ((rc = mark(&e))) return rc;
  ev.push_back(e);
  if ((rc = check_flag(h))) return rc;  // synchronises; an unstable run has no gradient

  // ---- reverse sweep, segment by segment from the last
  double t_recompute = 0.0, t_reverse = 0.0;
  int gi = 0;  // G[gi] holds dJ/dg of the step after the one being reversed
  const int64_t nseg = L.tape ? 1 : L.n_store;
  for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
    const int64_t t0 = L.tape ? 0 : sgi * L.K;
    const int64_t t1 = L.tape ? n : std::min<int64_t>(n, t0 + L.K);
    auto A_of = [&](int64_t t) -> char * {
      if (L.tape) return t == 0 ? state0 : store_state(t - 1);
      return t == t0 ? store_state(sgi) : seg_state(t - t0 - 1);
    };
    hipEvent_t r0, r1, r2;
    if ((rc = mark(&r0))) return rc;
    ev.push_back(r0);
    if (!L.tape)
      for (int64_t t = t0; t + 1 < t1; ++t) {
        HIPCHK(launch_ib(h->prec, A_of(t), pa, iba, s));
        HIPCHK(launch_lbm(h->prec, h->variant, A_of(t), A_of(t + 1), pa, TileRange{nullptr, 0, nt, 0}, iba, s));
      }
    if ((rc = mark(&r1))) return rc;
    ev.push_back(r1);
    for (int64_t t = t1 - 1; t >= t0; --t) {
      const char *A = A_of(t);
      void *Gn = w + L.off_g[gi];
      void *Go = w + L.off_g[gi ^ 1];
      a.hist_bar = hbar_dev + (size_t)t * nb * 3;
      HIPCHK(launch_ib(h->prec, A, pa, iba, s));  // the step's marker values
      HIPCHK(launch_adj_lattice(h->prec, A, Gn, Go, pa, a, s));
      HIPCHK(launch_adj_marker(pa, iba, a, s));
      HIPCHK(launch_adj_spread(h->prec, Go, pa, a, s));
      gi ^= 1;
    }
    if ((rc = mark(&r2))) return rc;
    ev.push_back(r2);
  }

  // ---- results
  double *out64 = reinterpret_cast<double *>(w + L.off_out);
  HIPCHK(launch_adj_unpull(h->prec, w + L.off_g[gi], p, out64, s));
  HIPCHK(hipStreamSynchronize(s));
  {
    long long ctr;
    int flag;
    unsigned char buf[16];
    HIPCHK(hipMemcpy(buf, w + L.off_ctl, 16, hipMemcpyDeviceToHost));
    std::memcpy(&ctr, buf, 8);
    std::memcpy(&flag, buf + 8, 4);
    if (flag != 0) return fail(BTDF_EUNSTABLE, "the recomputed steps went unstable");
  }
  if (gr->populations)
    HIPCHK(hipMemcpy(gr->populations, out64, 9 * (size_t)h->nx * h->ny * d, hipMemcpyDeviceToHost));
  std::vector<double> part((size_t)ntiles * 4);
  HIPCHK(hipMemcpy(part.data(), w + L.off_part, part.size() * d, hipMemcpyDeviceToHost));
  double sg[4] = {0, 0, 0, 0};
  for (int t = 0; t < ntiles; ++t)
    for (int k = 0; k < 4; ++k) sg[k] += part[4 * (size_t)t + k];
  if (gr->body_force) {
    gr->body_force[0] = sg[0];
    gr->body_force[1] = sg[1];
  }
  if (gr->inflow) {
    gr->inflow[0] = sg[2];
    gr->inflow[1] = sg[3];
  }
  if (gr->marker_xy && nm) HIPCHK(hipMemcpy(gr->marker_xy, a.xy_bar, 2 * (size_t)nm * d, hipMemcpyDeviceToHost));
  if (gr->marker_uv && nm) HIPCHK(hipMemcpy(gr->marker_uv, a.uv_bar, 2 * (size_t)nm * d, hipMemcpyDeviceToHost));
  if (gr->centres && nb) {
    std::vector<double> cb(2 * (size_t)nm);
    if (nm) HIPCHK(hipMemcpy(cb.data(), a.c_bar, cb.size() * d, hipMemcpyDeviceToHost));
    for (int b = 0; b < nb; ++b) {
      double sx = 0.0, sy = 0.0;
      for (int l = h->off[b]; l < h->off[b + 1]; ++l) {
        sx += cb[2 * (size_t)l];
        sy += cb[2 * (size_t)l + 1];
      }
      gr->centres[2 * b] = sx;
      gr->centres[2 * b + 1] = sy;
    }
  }
  if (ms) {  // events: start, end of the forward run, then (start, recomputed, reversed) per segment
    float f = 0.f;
    (void)hipEventElapsedTime(&f, ev[0], ev[1]);
    ms[0] = f;
    for (size_t k = 2; k + 2 < ev.size(); k += 3) {
      float a1 = 0.f, a2 = 0.f;
      (void)hipEventElapsedTime(&a1, ev[k], ev[k + 1]);
      (void)hipEventElapsedTime(&a2, ev[k + 1], ev[k + 2]);
      t_recompute += a1;
      t_reverse += a2;
    }
    ms[1] = t_recompute;
    ms[2] = t_reverse;
  }
  return ok();
}

}  // namespace

extern "C" {

size_t btdf_adjoint_workspace_bytes(btdf_t *h, int64_t n_steps, int64_t checkpoint_every) {
  if (!h || n_steps < 1 || checkpoint_every < 0) return 0;
  if (!h->layout_ok) compute_layout(h);
  AdjLayout L;
  adj_layout(h, n_steps, checkpoint_every, &L);
  return L.total;
}

int btdf_adjoint(btdf_t *h, int64_t n_steps, int64_t checkpoint_every, const double *hist_bar,
                 btdf_gradients *grads, void *work, size_t work_bytes, double *ms) {
  if (!h || !grads) return fail(BTDF_EINVAL, "NULL argument");
  if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch");
  if (n_steps < 1) return fail(BTDF_EINVAL, "n_steps must be >= 1");
  if (checkpoint_every < 0) return fail(BTDF_EINVAL, "checkpoint_every must be >= 0");
  if (h->nb() > 0 && !hist_bar) return fail(BTDF_EINVAL, "hist_bar is NULL");
  int rc = ensure_device(h);
  if (rc) return rc;
  if ((rc = check_flag(h))) return rc;
  return adjoint_impl(h, n_steps, checkpoint_every, hist_bar, grads, (char *)work, work_bytes, ms);
}

}  // extern "C"
