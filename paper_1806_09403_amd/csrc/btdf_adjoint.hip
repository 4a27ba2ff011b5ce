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
//   [ checkpoints or tape states | segment states | G x 2 | per-step marker
//     records | marker adjoints and gradients | adjoint tile bins | tile sums |
//     weights of the history (all, and one segment's) | control + one
//     history slot | dJ/dA_0 in FP64 ]
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
  int64_t n_store = 0;  // tape states 1 .. n-1, or checkpoints at t = 0, K, 2K, ...
  int64_t n_seg = 0;    // segment states (checkpoint mode: two sets of K)
  int64_t n_slot = 0;   // per-step marker records (tape: n, checkpoints: two sets of K)
  size_t state = 0;     // bytes of one population state
  size_t slot = 0;      // bytes of one marker record
  size_t off_store = 0, off_seg = 0, off_g[2] = {0, 0}, off_slots = 0;
  size_t off_mkadj = 0, off_xyb = 0, off_uvb = 0, off_cb = 0;
  size_t off_toff = 0, off_tlist = 0, off_noff = 0, off_nlist = 0, off_part = 0;
  size_t off_hbar = 0, off_hseg = 0, off_ctl = 0, off_hist1 = 0, off_out = 0, total = 0;
  // adjoint tiles and their markers; markers covering each stencil node
  int ntx = 0, nty = 0;
  std::vector<int> toff, tlist, noff, nlist;
};

int64_t default_K(int64_t n) {
  int64_t K = (int64_t)std::ceil(std::sqrt((double)n));
  return std::max<int64_t>(1, K);
}

// one marker record: Fx Fy rho_l ux_l uy_l (FP64), spread weights (10 per
// marker, population type), stencil origins (2 ints)
size_t slot_bytes(const btdf_t *h) {
  const size_t M = (size_t)std::max(h->nm(), 1);
  return align256(5 * M * sizeof(double)) + align256(10 * M * (size_t)h->prec) + align256(2 * M * sizeof(int));
}

void adj_layout(const btdf_t *h, int64_t n, int64_t K, AdjLayout *L) {
  L->n = n;
  L->K = K > 0 ? K : default_K(n);
  L->tape = L->K >= n;
  L->state = align256(9 * (size_t)h->plane * (size_t)h->prec);
  L->slot = slot_bytes(h);
  if (L->tape) {
    L->n_store = std::max<int64_t>(0, n - 1);
    L->n_seg = 0;
    L->n_slot = n;
  } else {
    L->n_store = (n + L->K - 1) / L->K;
    L->n_seg = 2 * L->K;
    L->n_slot = 2 * L->K;
  }
  L->ntx = (h->nx + kAdjTX - 1) / kAdjTX;
  L->nty = (h->ny + kAdjTY - 1) / kAdjTY;
  const int ntiles = L->ntx * L->nty;
  bin_markers(h, kAdjTX, kAdjTY, L->ntx, L->nty, L->toff, L->tlist);
  cover_lists(h, L->noff, L->nlist);

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
  L->off_slots = o;
  o += (size_t)L->n_slot * L->slot;
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
  L->off_noff = o;
  o = align256(o + L->noff.size() * sizeof(int));
  L->off_nlist = o;
  o = align256(o + L->nlist.size() * sizeof(int));
  L->off_part = o;
  o = align256(o + (size_t)ntiles * 4 * d);
  L->off_hbar = o;
  o = align256(o + (size_t)n * B * 3 * d);
  L->off_hseg = o;
  o = align256(o + (size_t)(L->tape ? 1 : 2 * L->K) * B * 3 * d);
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

// everything one adjoint call launches with
struct Adj {
  btdf_t *h = nullptr;
  const AdjLayout *L = nullptr;
  char *w = nullptr;
  LbmParams p{}, pa{};  // the handle's, and the copy whose flag and counter are the scratch's
  IbParams ib{}, iba{};
  AdjParams a{};
  int nt = 0;

  char *store(int64_t i) const { return w + L->off_store + (size_t)i * L->state; }
  // segment buffers: two sets of K states (and of K marker records), so one
  // segment can be recomputed while the next one up is reversed
  char *seg(int set, int64_t i) const { return w + L->off_seg + ((size_t)set * L->K + i) * L->state; }
  const double *hseg(int set) const {
    return reinterpret_cast<const double *>(w + L->off_hseg) + (size_t)set * L->K * std::max(h->nb(), 1) * 3;
  }
  char *gbuf(int i) const { return w + L->off_g[i]; }
  // marker record k: the marker kernel's outputs of one step
  void slot_params(int64_t k, const LbmParams &pb, const IbParams &ibb, LbmParams *po, IbParams *io) const {
    const size_t M = (size_t)std::max(h->nm(), 1);
    char *r = w + L->off_slots + (size_t)k * L->slot;
    double *mk = reinterpret_cast<double *>(r);
    *po = pb;
    *io = ibb;
    io->Fx = mk;
    io->Fy = mk + M;
    io->rho_l = mk + 2 * M;
    io->ux_l = mk + 3 * M;
    io->uy_l = mk + 4 * M;
    io->mk_w = r + align256(5 * M * sizeof(double));
    io->mk_ixy = reinterpret_cast<int *>(r + align256(5 * M * sizeof(double)) + align256(10 * M * (size_t)h->prec));
    po->mk_w = io->mk_w;
    po->mk_ixy = io->mk_ixy;
  }
  AdjParams adj_params(const IbParams &io, const double *hbar) const {
    AdjParams x = a;
    x.Fx = io.Fx;
    x.Fy = io.Fy;
    x.rho_l = io.rho_l;
    x.ux_l = io.ux_l;
    x.uy_l = io.uy_l;
    x.hist_bar = hbar;
    return x;
  }
};

// one reversed step: state A (its marker record k already holds the step's
// marker values), dJ/dg of the next step in G[gi] -> dJ/dg of this step in G[gi ^ 1]
int reverse_step(const Adj &X, const void *A, int64_t k, const double *hbar, int gi, hipStream_t s) {
  LbmParams pk;
  IbParams ik;
  X.slot_params(k, X.pa, X.iba, &pk, &ik);
  const AdjParams ak = X.adj_params(ik, hbar);
  const int prec = X.h->prec;
  HIPCHK(launch_adj_marker(prec, A, X.gbuf(gi), pk, ik, ak, s));
  HIPCHK(launch_adj_lattice(prec, A, X.gbuf(gi), X.gbuf(gi ^ 1), pk, ak, s));
  return ok();
}

// checkpoint mode, one segment of len steps whose first state is in
// seg(set, 0): recompute the states seg(set, 1 .. len-1) and every step's
// marker record (records set * K + k)
int recompute_segment(const Adj &X, int set, int64_t len, hipStream_t s) {
  const int prec = X.h->prec;
  for (int64_t k = 0; k < len; ++k) {
    LbmParams pk;
    IbParams ik;
    X.slot_params(set * X.L->K + k, X.pa, X.iba, &pk, &ik);
    HIPCHK(launch_ib(prec, X.seg(set, k), pk, ik, s));
    if (k + 1 < len)
      HIPCHK(launch_lbm(prec, X.h->variant, X.seg(set, k), X.seg(set, k + 1), pk, TileRange{nullptr, 0, X.nt, 0},
                        ik, s));
  }
  return ok();
}

// reverse the len steps of seg(set, 0 .. len-1); the weights of their forces
// are in the set's slice of hist_bar, G[gi] holds dJ/dg of the step after them
int reverse_segment(const Adj &X, int set, int64_t len, int gi, hipStream_t s) {
  const double *hseg = X.hseg(set);
  const int nb = X.h->nb();
  for (int64_t k = len - 1; k >= 0; --k) {
    int rc = reverse_step(X, X.seg(set, k), set * X.L->K + k, hseg + (size_t)k * nb * 3, gi, s);
    if (rc) return rc;
    gi ^= 1;
  }
  return ok();
}

// K forward steps of the handle from its buffer c, on stream s
int forward_steps(const Adj &X, int64_t len, int c, hipStream_t s) {
  for (int64_t k = 0; k < len; ++k) {
    int rc = enqueue_step(X.h, X.p, X.ib, c, s, nullptr);
    if (rc) return rc;
    c ^= 1;
  }
  return ok();
}

// capture what fn enqueues into an executable graph
template <typename F>
int capture(hipStream_t cap, hipGraphExec_t *out, F fn) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int rc = fn(cap);
  hipError_t e = hipStreamEndCapture(cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(BTDF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(BTDF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return ok();
}

struct Owned {
  char *mem = nullptr;
  hipStream_t cap = nullptr, side = nullptr;
  std::vector<hipEvent_t> ev;
  // forward from buffer 0 / 1; recompute into set 0 / 1; reverse of set 0 / 1
  // starting from G[0] / G[1]
  hipGraphExec_t fwd[2] = {nullptr, nullptr}, rec[2] = {nullptr, nullptr}, rev[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  ~Owned() {
    for (hipGraphExec_t g : {fwd[0], fwd[1], rec[0], rec[1], rev[0][0], rev[0][1], rev[1][0], rev[1][1]})
      if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
    if (cap) (void)hipStreamDestroy(cap);
    if (mem) (void)hipFree(mem);
  }
};

int adjoint_impl(btdf_t *h, int64_t n, int64_t K, const double *hist_bar, btdf_gradients *gr, char *w,
                 size_t wbytes, double *ms) {
  AdjLayout L;
  adj_layout(h, n, K, &L);
  Owned own;
  if (w == nullptr) {
    hipError_t e = hipMalloc((void **)&own.mem, L.total);
    if (e != hipSuccess) return fail(BTDF_ENOMEM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
    w = own.mem;
  } else if (wbytes < L.total) {
    return fail(BTDF_ENOMEM, "adjoint workspace has %zu bytes, %zu needed", wbytes, L.total);
  } else if ((uintptr_t)w & 255) {
    return fail(BTDF_EINVAL, "adjoint workspace must be 256-byte aligned");
  }

  hipStream_t s = h->stream;
  const int nb = h->nb(), nm = h->nm();
  const int ntiles = L.ntx * L.nty;
  const size_t M = (size_t)std::max(nm, 1), d = sizeof(double);
  int rc;
  if ((rc = put(s, w, L.off_toff, L.toff.data(), L.toff.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_tlist, L.tlist.data(), L.tlist.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_noff, L.noff.data(), L.noff.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_nlist, L.nlist.data(), L.nlist.size() * sizeof(int))) ||
      (rc = put(s, w, L.off_hbar, hist_bar, (size_t)n * nb * 3 * d)))
    return rc;
  HIPCHK(hipMemsetAsync(w + L.off_xyb, 0, 2 * M * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_uvb, 0, 2 * M * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_cb, 0, 2 * M * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_part, 0, (size_t)ntiles * 4 * d, s));
  HIPCHK(hipMemsetAsync(w + L.off_ctl, 0, 256, s));
  HIPCHK(hipMemsetAsync(w + L.off_g[0], 0, L.state, s));  // dJ/dA_n = 0: J reads the history only

  Adj X;
  X.h = h;
  X.L = &L;
  X.w = w;
  X.nt = h->ntx * h->nty;
  X.p = make_params(h);
  X.ib = make_ib(h);
  // the recomputation and the sweep count, flag and record history into the
  // scratch: the handle's view of its run stays the forward run's
  X.pa = X.p;
  X.iba = X.ib;
  X.iba.hist = reinterpret_cast<double *>(w + L.off_hist1);
  X.iba.hist_cap = 1;
  X.iba.slot = reinterpret_cast<int *>(w + L.off_ctl + 16);
  X.pa.step_ctr = reinterpret_cast<long long *>(w + L.off_ctl);
  X.pa.flag = reinterpret_cast<int *>(w + L.off_ctl + 8);
  AdjParams &a = X.a;
  a.ntx = L.ntx;
  a.nty = L.nty;
  a.tile_off = reinterpret_cast<const int *>(w + L.off_toff);
  a.tile_list = reinterpret_cast<const int *>(w + L.off_tlist);
  a.node_off = reinterpret_cast<const int *>(w + L.off_noff);
  a.node_list = reinterpret_cast<const int *>(w + L.off_nlist);
  a.part = reinterpret_cast<double *>(w + L.off_part);
  a.mk_adj = reinterpret_cast<double *>(w + L.off_mkadj);
  a.xy_bar = reinterpret_cast<double *>(w + L.off_xyb);
  a.uv_bar = reinterpret_cast<double *>(w + L.off_uvb);
  a.c_bar = reinterpret_cast<double *>(w + L.off_cb);
  const double *hbar_dev = reinterpret_cast<const double *>(w + L.off_hbar);

  auto mark = [&]() -> int {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    own.ev.push_back(e);
    HIPCHK(hipEventRecord(e, s));
    return ok();
  };
  if ((rc = mark())) return rc;

  const int prec = h->prec;
  const size_t copy_bytes = 9 * (size_t)h->plane * (size_t)prec;
  int gi = 0;  // G[gi] holds dJ/dg of the step after the one being reversed
  double rec_ms = 0.0, sweep_ms = 0.0;
  if (L.tape) {
    // ---- forward: state t in the handle's buffer (t = 0), the tape (1 .. n-1)
    // and the handle's other buffer (t = n); each step's marker values kept
    const int cur0 = h->cur;
    char *state0 = h->ws + h->off_pop[cur0];
    auto A_of = [&](int64_t t) -> char * { return t == 0 ? state0 : X.store(t - 1); };
    for (int64_t t = 0; t < n; ++t) {
      LbmParams pt;
      IbParams it;
      X.slot_params(t, X.p, X.ib, &pt, &it);
      void *B = t == n - 1 ? (void *)(h->ws + h->off_pop[1 - cur0]) : (void *)X.store(t);
      HIPCHK(launch_ib(prec, A_of(t), pt, it, s));
      HIPCHK(launch_lbm(prec, h->variant, A_of(t), B, pt, TileRange{nullptr, 0, X.nt, 1}, it, s));
    }
    h->cur = 1 - cur0;
    h->steps += n;
    {  // the handle's marker arrays show the last step, as after btdf_step
      LbmParams pt;
      IbParams it;
      X.slot_params(n - 1, X.p, X.ib, &pt, &it);
      HIPCHK(hipMemcpyAsync(X.ib.Fx, it.Fx, 5 * M * d, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(X.ib.mk_w, it.mk_w, 10 * M * (size_t)prec, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(X.ib.mk_ixy, it.mk_ixy, 2 * M * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    if ((rc = mark())) return rc;
    if ((rc = check_flag(h))) return rc;  // synchronises; an unstable run has no gradient
    if ((rc = mark())) return rc;
    for (int64_t t = n - 1; t >= 0; --t) {
      if ((rc = reverse_step(X, A_of(t), t, hbar_dev + (size_t)t * nb * 3, gi, s))) return rc;
      gi ^= 1;
    }
    if ((rc = mark())) return rc;
    HIPCHK(hipStreamSynchronize(s));
    float f = 0.f;
    (void)hipEventElapsedTime(&f, own.ev[2], own.ev[3]);
    sweep_ms = f;
  } else {
    // ---- forward, checkpoint at the start of every segment; whole segments
    // replay one captured graph per starting buffer
    const int64_t S = L.n_store;
    const bool graphs = S >= 3;
    if (graphs) HIPCHK(hipStreamCreateWithFlags(&own.cap, hipStreamNonBlocking));
    for (int64_t sg = 0; sg < S; ++sg) {
      const int64_t len = std::min<int64_t>(L.K, n - sg * L.K);
      HIPCHK(hipMemcpyAsync(X.store(sg), h->ws + h->off_pop[h->cur], copy_bytes, hipMemcpyDeviceToDevice, s));
      if (graphs && len == L.K) {
        hipGraphExec_t &g = own.fwd[h->cur];
        const int c = h->cur;
        if (!g && (rc = capture(own.cap, &g, [&](hipStream_t cs) { return forward_steps(X, len, c, cs); }))) return rc;
        HIPCHK(hipGraphLaunch(g, s));
      } else if ((rc = forward_steps(X, len, h->cur, s))) {
        return rc;
      }
      if (len & 1) h->cur ^= 1;
      h->steps += len;
    }
    if ((rc = mark())) return rc;
    if ((rc = check_flag(h))) return rc;

    // ---- reverse, segment by segment from the last. Segment sg uses buffer
    // set sg & 1. A side stream restores the checkpoint and recomputes the
    // segment below while this stream reverses the current one; events order
    // each recomputation after the reversal that last used its set, and each
    // reversal after its own recomputation.
    HIPCHK(hipStreamCreateWithFlags(&own.side, hipStreamNonBlocking));
    hipStream_t s2 = own.side;
    hipEvent_t evRec[2], evRev[2], e0, eEnd;
    for (int k = 0; k < 2; ++k) {
      HIPCHK(hipEventCreateWithFlags(&evRec[k], hipEventDisableTiming));
      own.ev.push_back(evRec[k]);
      HIPCHK(hipEventCreateWithFlags(&evRev[k], hipEventDisableTiming));
      own.ev.push_back(evRev[k]);
    }
    HIPCHK(hipEventCreate(&e0));
    own.ev.push_back(e0);
    HIPCHK(hipEventCreate(&eEnd));
    own.ev.push_back(eEnd);
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec_ev;  // timing of each recomputation
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(hipStreamWaitEvent(s2, e0, 0));  // the side stream starts after the forward run
    auto prep = [&](int64_t sg) -> int {
      const int set = (int)(sg & 1);
      const int64_t t0 = sg * L.K, len = std::min<int64_t>(L.K, n - t0);
      HIPCHK(hipMemcpyAsync(X.seg(set, 0), X.store(sg), copy_bytes, hipMemcpyDeviceToDevice, s2));
      HIPCHK(hipMemcpyAsync(const_cast<double *>(X.hseg(set)), hbar_dev + (size_t)t0 * nb * 3,
                            (size_t)len * nb * 3 * d, hipMemcpyDeviceToDevice, s2));
      hipEvent_t a0, a1;
      HIPCHK(hipEventCreate(&a0));
      own.ev.push_back(a0);
      HIPCHK(hipEventCreate(&a1));
      own.ev.push_back(a1);
      HIPCHK(hipEventRecord(a0, s2));
      int r;
      if (graphs && len == L.K) {
        hipGraphExec_t &g = own.rec[set];
        if (!g && (r = capture(own.cap, &g, [&](hipStream_t cs) { return recompute_segment(X, set, len, cs); })))
          return r;
        HIPCHK(hipGraphLaunch(g, s2));
      } else if ((r = recompute_segment(X, set, len, s2))) {
        return r;
      }
      HIPCHK(hipEventRecord(a1, s2));
      rec_ev.push_back({a0, a1});
      HIPCHK(hipEventRecord(evRec[set], s2));
      return ok();
    };
    if ((rc = prep(S - 1))) return rc;
    for (int64_t sg = S - 1; sg >= 0; --sg) {
      const int set = (int)(sg & 1);
      const int64_t len = std::min<int64_t>(L.K, n - sg * L.K);
      if (sg >= 1) {
        // the set of segment sg - 1 was last reversed as segment sg + 1
        if (sg + 1 < S) HIPCHK(hipStreamWaitEvent(s2, evRev[(sg + 1) & 1], 0));
        if ((rc = prep(sg - 1))) return rc;
      }
      HIPCHK(hipStreamWaitEvent(s, evRec[set], 0));
      if (graphs && len == L.K) {
        hipGraphExec_t &g = own.rev[set][gi];
        const int g0 = gi;
        if (!g && (rc = capture(own.cap, &g, [&](hipStream_t cs) { return reverse_segment(X, set, len, g0, cs); })))
          return rc;
        HIPCHK(hipGraphLaunch(g, s));
      } else if ((rc = reverse_segment(X, set, len, gi, s))) {
        return rc;
      }
      HIPCHK(hipEventRecord(evRev[set], s));
      if (len & 1) gi ^= 1;
    }
    HIPCHK(hipEventRecord(eEnd, s));
    HIPCHK(hipStreamSynchronize(s));
    float f = 0.f;
    double trec = 0.0;
    for (auto &pr : rec_ev) {
      (void)hipEventElapsedTime(&f, pr.first, pr.second);
      trec += f;
    }
    (void)hipEventElapsedTime(&f, e0, eEnd);
    sweep_ms = f;
    rec_ms = trec;
  }

  // ---- results
  double *out64 = reinterpret_cast<double *>(w + L.off_out);
  HIPCHK(launch_adj_unpull(prec, X.gbuf(gi), X.p, out64, s));
  HIPCHK(hipStreamSynchronize(s));
  {
    int flag;
    HIPCHK(hipMemcpy(&flag, w + L.off_ctl + 8, 4, hipMemcpyDeviceToHost));
    if (flag != 0) return fail(BTDF_EUNSTABLE, "the recomputed steps went unstable");
  }
  if (gr->populations)
    HIPCHK(hipMemcpy(gr->populations, out64, 9 * (size_t)h->nx * h->ny * d, hipMemcpyDeviceToHost));
  std::vector<double> part((size_t)ntiles * 4);
  HIPCHK(hipMemcpy(part.data(), w + L.off_part, part.size() * d, hipMemcpyDeviceToHost));
  double sg4[4] = {0, 0, 0, 0};
  for (int t = 0; t < ntiles; ++t)
    for (int k = 0; k < 4; ++k) sg4[k] += part[4 * (size_t)t + k];
  if (gr->body_force) {
    gr->body_force[0] = sg4[0];
    gr->body_force[1] = sg4[1];
  }
  if (gr->inflow) {
    gr->inflow[0] = sg4[2];
    gr->inflow[1] = sg4[3];
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
  if (ms) {
    float f = 0.f;
    (void)hipEventElapsedTime(&f, own.ev[0], own.ev[1]);
    ms[0] = f;         // the forward run
    ms[1] = rec_ms;    // recomputation, summed (it runs under the reverse steps)
    ms[2] = sweep_ms;  // the whole reverse sweep, recomputation included
  }
  return ok();
}

}  // namespace

extern "C" {

size_t btdf_adjoint_workspace_bytes(btdf_t *h, int64_t n_steps, int64_t checkpoint_every) {
  return guard_size([&]() -> size_t {
    if (!h || n_steps < 1 || checkpoint_every < 0) return 0;
    if (!h->layout_ok) compute_layout(h);
    AdjLayout L;
    adj_layout(h, n_steps, checkpoint_every, &L);
    return L.total;
  });
}

int btdf_adjoint(btdf_t *h, int64_t n_steps, int64_t checkpoint_every, const double *hist_bar,
                 btdf_gradients *grads, void *work, size_t work_bytes, double *ms) {
  return guard([&]() -> int {
    if (!h || !grads) return fail(BTDF_EINVAL, "NULL argument");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch");
    if (h->nf != 1) return fail(BTDF_ESTATE, "the reverse sweep needs one forcing pass per step (NF = 1)");
    if (h->method != BTDF_FORCING_DIRECT) return fail(BTDF_ESTATE, "the reverse sweep covers the direct forcing only");
    if (h->any_moving()) return fail(BTDF_ESTATE, "the reverse sweep covers fixed bodies only");
    h->stepped = false;
    if (h->bc[1] == BTDF_CONVECTIVE_OUTLET || h->bc[2] == BTDF_FREE_SLIP_WALL)
      return fail(BTDF_EINVAL, "the reverse sweep covers periodic, bounce-back and zero-gradient boundaries only");
    if (n_steps < 1) return fail(BTDF_EINVAL, "n_steps must be >= 1");
    if (checkpoint_every < 0) return fail(BTDF_EINVAL, "checkpoint_every must be >= 0");
    if (h->nb() > 0 && !hist_bar) return fail(BTDF_EINVAL, "hist_bar is NULL");
    int rc = ensure_device(h);
    if (rc) return rc;
    if ((rc = check_flag(h))) return rc;
    return adjoint_impl(h, n_steps, checkpoint_every, hist_bar, grads, (char *)work, work_bytes, ms);
  });
}

}  // extern "C"
