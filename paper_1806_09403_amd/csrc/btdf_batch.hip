// btdf_batch.hip -- many independent cases stepped together.
//
// Every case is an ordinary simulation handle (same state, same layout, same
// state I/O) whose device memory is one slice of the batch workspace. A batch
// step is two launches for all cases together: the marker kernel over the
// markers of every case and the lattice kernel over the tiles of every case
// (plus one body-reduction workgroup per body), each workgroup reading its
// case's parameters from a table. Cases of very different sizes therefore
// fill the GPU together instead of one small launch after another.
//
// Workspace: [ case table | workgroup maps | case 0 | case 1 | ... ].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "btdf_internal.h"

using namespace btdf;
using namespace btdf::host;

struct btdf_batch {
  std::vector<btdf_t *> cases;
  int prec = 4;
  hipStream_t stream = nullptr;
  // device memory
  char *ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  // layout
  std::vector<size_t> case_off;
  size_t off_desc = 0, off_maps = 0, total = 0;
  int ntiles = 0, nbodies = 0, nmblk = 0;
  BatchMap map{};
  btdf_event_pool tev;  // events of the timed stepping calls
  bool layout_ok = false, device_ok = false;
  // launch options
  int variant = 6, xcd_remap = 1, mask = 1, graph_chunk = 0, interior = 0, row_align = 128;
  int tblock = 1;        // option: three steps per pass for the cases' tiles away from their bodies
  bool blocked = false;  // it is on (the launch shape has the three-step pass)
  BatchMap map_near{};   // the near tiles of every case (and the body reductions)
  const int *g_case[kLevels] = {}, *g_tile[kLevels] = {};
  int g_count[kLevels] = {};  // interior groups of every case, level by level
  const int *ge_case[kLevels] = {}, *ge_tile[kLevels] = {};
  int ge_count[kLevels] = {};  // edge groups of every case, level by level
  int edge_tiles = 1;          // option: tiles within reach of a case's edges take the pass
  int gkind[kLevels] = {};  // the shape of each level's launch
  hipGraphExec_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
  // the blocked pass's smaller launches run on a second stream beside the
  // largest (fork and join events)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // time
  int cur = 0;
  int64_t steps = 0;
};

namespace {

void batch_drop_graph(btdf_batch_t *b) {
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
}

// sizes of the case table, the workgroup maps and every case slice
void batch_layout(btdf_batch_t *b) {
  const int K = (int)b->cases.size();
  long long max_tiles = 0, bodies = 0, mblk = 0;
  b->blocked = b->tblock && variant_has_lbm3(b->variant, b->prec, kGroup1x1);
  group_kinds(b->variant, b->prec, 3, b->gkind);
  for (btdf_t *h : b->cases) {
    h->variant = b->variant;
    h->xcd_remap = b->xcd_remap;
    h->interior = b->interior;
    h->row_align = b->row_align;
    h->tblock = b->blocked ? 3 : 0;  // each case's near tiles, groups and extra buffers
    h->edge_tiles = b->edge_tiles;
    h->reserve_pass = b->tblock != 0;  // slices keep their size across launch shapes
    compute_layout(h);
    long long mt = 0;
    for (int v = 0; v < num_variants(); ++v) {
      int tx, ty;
      variant_tile(v, &tx, &ty);
      mt = std::max(mt, (long long)((h->nx + tx - 1) / tx) * ((h->ny + ty - 1) / ty));
    }
    max_tiles += mt;
    bodies += h->nb();
    mblk += (h->nm() + 15) / 16;
  }
  size_t o = 0;
  b->off_desc = o;
  o = align256(o + (size_t)K * sizeof(CaseDesc));
  b->off_maps = o;
  // tile maps, near-tile maps and group maps (each at most two ints per tile), body and marker maps
  // (plus one int after each of the 8 + 4 kLevels lists)
  o = align256(o + (size_t)(6 * max_tiles + 2 * bodies + 2 * mblk + 8 + 4 * kLevels + 16) * sizeof(int));
  b->case_off.assign(K, 0);
  for (int c = 0; c < K; ++c) {
    b->case_off[c] = o;
    o = align256(o + b->cases[c]->total);
  }
  b->total = o;
  b->layout_ok = true;
  b->device_ok = false;
  batch_drop_graph(b);
}

// give every case its slice (moving any existing state), make each case's
// device part current, and upload the case table and workgroup maps
int batch_ensure(btdf_batch_t *b) {
  if (!b->layout_ok) batch_layout(b);
  char *old = nullptr;
  bool old_owned = false;
  // a case whose state sits in this workspace but not at its new slice would
  // have to move inside the same buffer, where slices can overlap
  bool shifted = false;
  if (b->ws)
    for (size_t c = 0; c < b->cases.size(); ++c) {
      const btdf_t *h = b->cases[c];
      if (h->state_ok && h->ws >= b->ws && h->ws < b->ws + b->ws_bytes && h->ws != b->ws + b->case_off[c])
        shifted = true;
    }
  if (shifted && !b->ws_owned)
    return fail(BTDF_ESTATE, "case slices moved (bodies were added): bind a fresh batch workspace");
  if (b->ws == nullptr || b->ws_bytes < b->total || shifted) {
    if (b->ws != nullptr && !b->ws_owned)
      return fail(BTDF_ENOMEM, "bound batch workspace has %zu bytes, %zu needed", b->ws_bytes, b->total);
    char *nw = nullptr;
    hipError_t e = hipMalloc((void **)&nw, b->total);
    if (e != hipSuccess) return fail(BTDF_ENOMEM, "hipMalloc(%zu): %s", b->total, hipGetErrorString(e));
    old = b->ws;
    old_owned = b->ws_owned;
    b->ws = nw;
    b->ws_bytes = b->total;
    b->ws_owned = true;
    b->device_ok = false;
  }
  if (!b->device_ok) {
    const int K = (int)b->cases.size();
    for (int c = 0; c < K; ++c) {
      btdf_t *h = b->cases[c];
      char *slice = b->ws + b->case_off[c];
      if (h->ws != slice) {
        int rc = bind_impl(h, slice, h->total);  // moves the case's state if it has one
        if (rc) return rc;
      }
      int rc = ensure_device(h);
      if (rc) return rc;
    }
    if (old && old_owned) HIPCHK(hipFree(old));
    // case table
    std::vector<CaseDesc> desc(K);
    std::vector<int> tile_case, tile_local, body_case, body_local, mblk_case, mblk_first;
    std::vector<int> near_case, near_local, gc[kLevels], gt[kLevels], gce[kLevels], gte[kLevels];
    for (int c = 0; c < K; ++c) {
      btdf_t *h = b->cases[c];
      desc[c].p = make_params(h);
      desc[c].ib = make_ib(h);
      desc[c].pop[0] = h->ws + h->off_pop[0];
      desc[c].pop[1] = h->ws + h->off_pop[1];
      desc[c].pop[2] = h->ws + h->off_pop3;
      desc[c].pop[3] = h->ws + h->off_pop4;
      desc[c].near = h->at<unsigned char>(h->off_near);
      const int nt = h->ntx * h->nty;
      for (int t = 0; t < nt; ++t) {
        tile_case.push_back(c);
        tile_local.push_back(t);
      }
      if (b->blocked) {
        // the case's map: its groups level by level (edge groups first in a
        // level), then near tiles
        int k = 0;
        for (int w = 0; w < kLevels; ++w)
          for (int i = 0; i < h->n_grp[w]; ++i, ++k) {
            const bool e = i < h->n_edge[w];
            (e ? gce : gc)[w].push_back(c);
            (e ? gte : gt)[w].push_back(h->fmap[k]);
          }
        for (int i = 0; i < h->n_near; ++i, ++k) {
          near_case.push_back(c);
          near_local.push_back(h->fmap[k]);
        }
      }
      for (int bb = 0; bb < h->nb(); ++bb) {
        body_case.push_back(c);
        body_local.push_back(bb);
      }
      for (int l = 0; l < h->nm(); l += 16) {
        mblk_case.push_back(c);
        mblk_first.push_back(l);
      }
    }
    b->ntiles = (int)tile_case.size();
    b->nbodies = (int)body_case.size();
    b->nmblk = (int)mblk_case.size();
    HIPCHK(hipMemcpyAsync(b->ws + b->off_desc, desc.data(), desc.size() * sizeof(CaseDesc), hipMemcpyHostToDevice,
                          b->stream));
    int *maps = reinterpret_cast<int *>(b->ws + b->off_maps);
    size_t at = 0;
    auto put = [&](const std::vector<int> &v, const int **dst) -> int {
      *dst = maps + at;
      if (!v.empty())
        HIPCHK(hipMemcpyAsync(maps + at, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
      at += v.size() + 1;
      return ok();
    };
    int rc;
    if ((rc = put(tile_case, &b->map.tile_case)) || (rc = put(tile_local, &b->map.tile_local)) ||
        (rc = put(body_case, &b->map.body_case)) || (rc = put(body_local, &b->map.body_local)) ||
        (rc = put(mblk_case, &b->map.mblk_case)) || (rc = put(mblk_first, &b->map.mblk_first)) ||
        (rc = put(near_case, &b->map_near.tile_case)) || (rc = put(near_local, &b->map_near.tile_local)))
      return rc;
    for (int w = 0; w < kLevels; ++w) {
      if ((rc = put(gc[w], &b->g_case[w])) || (rc = put(gt[w], &b->g_tile[w])) || (rc = put(gce[w], &b->ge_case[w])) ||
          (rc = put(gte[w], &b->ge_tile[w])))
        return rc;
      b->g_count[w] = (int)gc[w].size();
      b->ge_count[w] = (int)gce[w].size();
    }
    HIPCHK(hipStreamSynchronize(b->stream));  // the host vectors go out of scope
    b->map.ntiles = b->ntiles;
    b->map.nbodies = b->nbodies;
    b->map.nmblk = b->nmblk;
    b->map.ncases = K;
    b->map.xcd_remap = b->xcd_remap;
    b->map.mask_unstable = b->mask;
    // the near tiles' steps: their own tile maps, the same body and marker maps
    const BatchMap full = b->map;
    b->map_near.body_case = full.body_case;
    b->map_near.body_local = full.body_local;
    b->map_near.mblk_case = full.mblk_case;
    b->map_near.mblk_first = full.mblk_first;
    b->map_near.ntiles = (int)near_case.size();
    b->map_near.nbodies = full.nbodies;
    b->map_near.nmblk = full.nmblk;
    b->map_near.ncases = full.ncases;
    b->map_near.xcd_remap = full.xcd_remap;
    b->map_near.mask_unstable = full.mask_unstable;
    b->device_ok = true;
    batch_drop_graph(b);
  }
  return ok();
}

struct BatchEvents {
  hipEvent_t e0, e1, e2;
};

bool batch_has_conv(const btdf_batch_t *b) {
  bool conv = false;
  for (const btdf_t *c : b->cases) conv |= c->bc[1] == BTDF_CONVECTIVE_OUTLET;
  return conv;
}

int batch_enqueue(btdf_batch_t *b, int parity, hipStream_t s, const BatchEvents *te) {
  const CaseDesc *desc = reinterpret_cast<const CaseDesc *>(b->ws + b->off_desc);
  const int rt = route(parity, parity ^ 1);
  if (te) HIPCHK(hipEventRecord(te->e0, s));
  HIPCHK(launch_ib_batch(b->prec, desc, b->map, rt, s));
  if (te) HIPCHK(hipEventRecord(te->e1, s));
  HIPCHK(launch_lbm_batch(b->prec, b->variant, desc, b->map, rt, s));
  if (te) HIPCHK(hipEventRecord(te->e2, s));
  if (batch_has_conv(b)) HIPCHK(launch_conv_outlet_batch(b->prec, desc, (int)b->cases.size(), b->mask, rt, s));
  return ok();
}

// Three steps of every case (temporal blocking), from buffer parity into the
// other: each case's near tiles step singly through its buffers 2 and 3 with
// the marker kernel before each step, and the three-step pass over every
// case's other tiles runs after their first step and before their second
// (it writes the states they pull from just outside). ev: 8 events or null,
// around the marker kernels (e0-e1, e4-e5, e6-e7 with e3-e4 the pass) and the
// near steps (e1-e2, e5-e6, e7-e8 in the pairs listed).
int batch_enqueue_triple(btdf_batch_t *b, int parity, hipStream_t s, hipEvent_t *ev) {
  const CaseDesc *desc = reinterpret_cast<const CaseDesc *>(b->ws + b->off_desc);
  const int A = parity, B = parity ^ 1, K = (int)b->cases.size();
  const bool conv = batch_has_conv(b);
  auto rec = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
  auto near_step = [&](int src, int dst) -> int {
    HIPCHK(launch_lbm_batch(b->prec, b->variant, desc, b->map_near, route(src, dst), s));
    if (conv) HIPCHK(launch_conv_outlet_batch(b->prec, desc, K, b->mask, route(src, dst), s));
    return ok();
  };
  int rc;
  HIPCHK(rec(0));
  HIPCHK(launch_ib_batch(b->prec, desc, b->map, route(A, A), s));
  HIPCHK(rec(1));
  if ((rc = near_step(A, 2))) return rc;
  HIPCHK(rec(2));
  // the pass: every launch but the largest groups' on a second stream beside
  // it (the smaller ones are a few waves of workgroups long, and alone their
  // tails would leave the GPU partly idle); the smallest groups first
  bool small = false;
  for (int w = 0; w < kLevels; ++w) small = small || b->ge_count[w] > 0 || (w > 0 && b->g_count[w] > 0);
  const bool fork = small && b->g_count[0] > 0;
  if (fork) {
    if (!b->side) HIPCHK(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    if (!b->fork_ev) HIPCHK(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    if (!b->join_ev) HIPCHK(hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(b->fork_ev, s));
    HIPCHK(hipStreamWaitEvent(b->side, b->fork_ev, 0));
  }
  const hipStream_t ss = fork ? b->side : s;
  for (int w = kLevels - 1; w >= 0; --w) {
    if (b->ge_count[w])
      HIPCHK(launch_lbm_edge3_batch(b->prec, b->variant, kEdge | b->gkind[w], desc, b->ge_case[w], b->ge_tile[w],
                                    b->ge_count[w], route(A, B), b->mask, b->xcd_remap, ss));
    if (b->g_count[w] && w > 0)
      HIPCHK(launch_lbm3_batch(b->prec, b->variant, b->gkind[w], desc, b->g_case[w], b->g_tile[w], b->g_count[w],
                               route(A, B), b->mask, b->xcd_remap, ss));
  }
  if (fork) HIPCHK(hipEventRecord(b->join_ev, b->side));
  if (b->g_count[0])
    HIPCHK(launch_lbm3_batch(b->prec, b->variant, b->gkind[0], desc, b->g_case[0], b->g_tile[0], b->g_count[0],
                             route(A, B), b->mask, b->xcd_remap, s));
  if (fork) HIPCHK(hipStreamWaitEvent(s, b->join_ev, 0));
  HIPCHK(rec(3));
  HIPCHK(launch_ib_batch(b->prec, desc, b->map, route(2, 2), s));
  HIPCHK(rec(4));
  if ((rc = near_step(2, 3))) return rc;
  HIPCHK(rec(5));
  HIPCHK(launch_ib_batch(b->prec, desc, b->map, route(3, 3), s));
  HIPCHK(rec(6));
  if ((rc = near_step(3, B))) return rc;
  HIPCHK(rec(7));
  return ok();
}

// one unit of the batch's stepping: a step, or three with temporal blocking
int batch_unit(btdf_batch_t *b, int parity, hipStream_t s) {
  return b->blocked ? batch_enqueue_triple(b, parity, s, nullptr) : batch_enqueue(b, parity, s, nullptr);
}

// keep every case's host view (buffer parity, step count) in step with the batch
void batch_advance(btdf_batch_t *b, int64_t n) {
  if (n & 1) b->cur ^= 1;
  b->steps += n;
  for (btdf_t *h : b->cases) {
    h->cur = b->cur;
    h->steps += n;
  }
}

int batch_build_graph(btdf_batch_t *b) {
  batch_drop_graph(b);
  if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  const int units = b->graph_chunk / (b->blocked ? 3 : 1);
  for (int k = 0; k < units && rc == 0; ++k) rc = batch_unit(b, k & 1, b->cap_stream);
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(BTDF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return fail(BTDF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return ok();
}

int batch_step_timed_impl(btdf_batch_t *b, int64_t n, double *ms_ib, double *ms_lbm) {
  int rc = batch_ensure(b);
  if (rc) return rc;
  const int chunk = 256, NE = 8;  // events per entry
  HIPCHK(b->tev.reserve((size_t)NE * chunk));
  hipEvent_t *ev = b->tev.ev.data();
  double tib = 0.0, tlbm = 0.0;
  int64_t done = 0;
  while (done < n && rc == 0) {
    const bool tri = b->blocked && n - done >= 3;  // triples while three steps are left
    const int m = (int)std::min<int64_t>(chunk, tri ? (n - done) / 3 : n - done);
    for (int k = 0; k < m && rc == 0; ++k) {
      if (tri) {
        rc = batch_enqueue_triple(b, b->cur, b->stream, &ev[NE * k]);
        if (rc == 0) batch_advance(b, 3);
        continue;
      }
      const BatchEvents te{ev[NE * k], ev[NE * k + 1], ev[NE * k + 2]};
      rc = batch_enqueue(b, b->cur, b->stream, &te);
      if (rc == 0) batch_advance(b, 1);
    }
    if (rc) break;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
      rc = fail(BTDF_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
      break;
    }
    for (int k = 0; k < m; ++k) {
      hipEvent_t *E = &ev[NE * k];
      auto dt = [&](int i, int j) {
        float x = 0.f;
        (void)hipEventElapsedTime(&x, E[i], E[j]);
        return (double)x;
      };
      if (tri) {  // marker kernels; near steps and the pass
        tib += dt(0, 1) + dt(3, 4) + dt(5, 6);
        tlbm += dt(1, 2) + dt(2, 3) + dt(4, 5) + dt(6, 7);
      } else {
        tib += dt(0, 1);
        tlbm += dt(1, 2);
      }
    }
    done += tri ? 3 * (int64_t)m : m;
  }
  if (rc) return rc;
  if (ms_ib) *ms_ib = tib / (double)n;
  if (ms_lbm) *ms_lbm = tlbm / (double)n;
  return ok();
}

}  // namespace

extern "C" {

int btdf_batch_create(int n_cases, const btdf_grid *grids, const double *taus, const int *delta_kinds,
                      const double *thickenings, btdf_batch_t **out) {
  return guard([&]() -> int {
    if (!grids || !taus || !delta_kinds || !thickenings || !out) return fail(BTDF_EINVAL, "NULL argument");
    *out = nullptr;
    if (n_cases < 1) return fail(BTDF_EINVAL, "a batch needs at least one case");
    for (int c = 1; c < n_cases; ++c)
      if (grids[c].precision != grids[0].precision) return fail(BTDF_EINVAL, "all cases of a batch share one precision");
    btdf_batch_t *b = new (std::nothrow) btdf_batch();
    if (!b) return fail(BTDF_ENOMEM, "out of host memory");
    for (int c = 0; c < n_cases; ++c) {
      btdf_t *h = nullptr;
      int rc = btdf_create(&grids[c], taus[c], delta_kinds[c], thickenings[c], &h);
      if (rc) {
        const std::string msg = std::string("case ") + std::to_string(c) + ": " + btdf_last_error();
        for (btdf_t *x : b->cases) (void)destroy_impl(x);
        delete b;
        return fail(rc, "%s", msg.c_str());
      }
      h->owner = b;
      h->tblock = 0;  // the batch steps its cases itself, one step at a time
      h->stream = (hipStream_t)grids[0].hip_stream;
      b->cases.push_back(h);
    }
    b->prec = grids[0].precision;
    b->stream = (hipStream_t)grids[0].hip_stream;
    *out = b;
    return ok();
  });
}

int btdf_batch_destroy(btdf_batch_t *b) {
  return guard([&]() -> int {
    if (!b) return ok();
    int rc = ok();
    if (b->ws && hipStreamSynchronize(b->stream) != hipSuccess) rc = fail(BTDF_EDEVICE, "stream sync failed");
    batch_drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->side) {
      (void)hipStreamSynchronize(b->side);
      (void)hipStreamDestroy(b->side);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->join_ev) (void)hipEventDestroy(b->join_ev);
    for (btdf_t *h : b->cases) {
      h->owner = nullptr;
      h->ws = nullptr;  // slices of the batch workspace are not the case's to free
      h->ws_owned = false;
      (void)destroy_impl(h);
    }
    b->tev.release();
    if (b->ws && b->ws_owned) (void)hipFree(b->ws);
    delete b;
    return rc;
  });
}

int btdf_batch_case(btdf_batch_t *b, int i, btdf_t **h) {
  return guard([&]() -> int {
    if (!b || !h) return fail(BTDF_EINVAL, "NULL argument");
    if (i < 0 || i >= (int)b->cases.size()) return fail(BTDF_EINVAL, "no case %d", i);
    *h = b->cases[i];
    return ok();
  });
}

int btdf_batch_add_body(btdf_batch_t *b, int case_id, int n, const double *xy, const double *uv, double cx,
                        double cy, double ds, int *body_id) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    if (case_id < 0 || case_id >= (int)b->cases.size()) return fail(BTDF_EINVAL, "no case %d", case_id);
    int rc = add_body_impl(b->cases[case_id], n, xy, uv, cx, cy, ds, body_id);
    if (rc) return rc;
    b->layout_ok = false;
    return ok();
  });
}

size_t btdf_batch_workspace_bytes(const btdf_batch_t *b) {
  return guard_size([&]() -> size_t {
    if (!b) return 0;
    if (!b->layout_ok) batch_layout(const_cast<btdf_batch_t *>(b));
    return b->total;
  });
}

int btdf_batch_bind_workspace(btdf_batch_t *b, void *dev, size_t bytes) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    if (dev && ((uintptr_t)dev & 255)) return fail(BTDF_EINVAL, "workspace must be 256-byte aligned");
    if (!b->layout_ok) batch_layout(b);
    if (dev && bytes < b->total) return fail(BTDF_ENOMEM, "workspace has %zu bytes, %zu needed", bytes, b->total);
    if (dev == (void *)b->ws && dev) {
      b->ws_bytes = bytes;
      return ok();
    }
    // cases move their state into their new slices inside batch_ensure
    char *old = b->ws;
    const bool old_owned = b->ws_owned;
    if (dev) {
      b->ws = (char *)dev;
      b->ws_bytes = bytes;
      b->ws_owned = false;
    } else {
      b->ws = nullptr;
      b->ws_bytes = 0;
      b->ws_owned = false;
    }
    b->device_ok = false;
    batch_drop_graph(b);
    int rc = ok();
    if (b->ws) rc = batch_ensure(b);
    else if (old) {
      // back to library-owned memory: allocate now so the states can move out of the old slices
      rc = batch_ensure(b);
    }
    if (old && old_owned) HIPCHK(hipFree(old));
    return rc;
  });
}

int btdf_batch_set_stream(btdf_batch_t *b, void *hip_stream) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    if (b->ws && (hipStream_t)hip_stream != b->stream) HIPCHK(hipStreamSynchronize(b->stream));
    b->stream = (hipStream_t)hip_stream;
    for (btdf_t *h : b->cases) h->stream = b->stream;
    return ok();
  });
}

int btdf_batch_step(btdf_batch_t *b, int64_t n) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    if (n < 0) return fail(BTDF_EINVAL, "negative step count");
    if (n == 0) return ok();
    int rc = batch_ensure(b);
    if (rc) return rc;
    int64_t left = n;
    const int d = b->blocked ? 3 : 1;       // steps per unit
    const int64_t g = (int64_t)(b->graph_chunk / d) * d;  // steps per graph: whole units
    if (g > 0 && left >= g + (b->cur ? 1 : 0)) {
      if (b->cur) {  // graphs start from buffer 0
        if ((rc = batch_enqueue(b, b->cur, b->stream, nullptr))) return rc;
        batch_advance(b, 1);
        left--;
      }
      if (!b->graph && (rc = batch_build_graph(b))) return rc;
      while (left >= g) {
        HIPCHK(hipGraphLaunch(b->graph, b->stream));
        left -= g;
        batch_advance(b, g);  // each unit swaps the buffers once, as g steps of an odd unit do
        if (b->cur) break;
      }
    }
    for (; d > 1 && left >= d; left -= d) {
      if ((rc = batch_enqueue_triple(b, b->cur, b->stream, nullptr))) return rc;
      batch_advance(b, d);
    }
    for (; left > 0; --left) {
      if ((rc = batch_enqueue(b, b->cur, b->stream, nullptr))) return rc;
      batch_advance(b, 1);
    }
    return ok();
  });
}

int btdf_batch_step_timed(btdf_batch_t *b, int64_t n, double *ms_ib, double *ms_lbm) {
  return guard([&]() -> int {
    if (!b || !ms_ib || !ms_lbm) return fail(BTDF_EINVAL, "NULL argument");
    if (n <= 0) return fail(BTDF_EINVAL, "step count must be > 0");
    return batch_step_timed_impl(b, n, ms_ib, ms_lbm);
  });
}

int btdf_batch_status(btdf_batch_t *b, int *unstable, int64_t *n_steps) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    if (n_steps) *n_steps = b->steps;
    if (!unstable) return ok();
    if (!b->ws) {
      for (size_t c = 0; c < b->cases.size(); ++c) unstable[c] = 0;
      return ok();
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    for (size_t c = 0; c < b->cases.size(); ++c) {
      long long ctr;
      int flag;
      int rc = read_ctl(b->cases[c], &ctr, &flag);
      if (rc) return rc;
      unstable[c] = flag != 0;
    }
    return ok();
  });
}

int btdf_batch_set_option(btdf_batch_t *b, int key, int64_t value) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    switch (key) {
      case BTDF_OPT_LBM_VARIANT:
        if (value < 0 || value >= num_variants()) return fail(BTDF_EINVAL, "variant %lld out of range", (long long)value);
        if (value != b->variant) {
          b->variant = (int)value;
          b->layout_ok = false;  // the tile lists change, and with blocking the slice sizes
        }
        return ok();
      case BTDF_OPT_GRAPH_CHUNK:
        if (value < 0 || value > 4096) return fail(BTDF_EINVAL, "graph chunk must be in 0 .. 4096");
        b->graph_chunk = (int)value;
        batch_drop_graph(b);
        return ok();
      case BTDF_OPT_XCD_REMAP:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "xcd remap must be 0 or 1");
        b->xcd_remap = (int)value;
        b->layout_ok = false;
        return ok();
      case BTDF_OPT_INTERIOR_PATH:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "interior path flag must be 0 or 1");
        b->interior = (int)value;
        b->layout_ok = false;
        return ok();
      case BTDF_OPT_ROW_ALIGN:
        if (value != 0 && (value < 4 || value > 4096 || (value & (value - 1))))
          return fail(BTDF_EINVAL, "row alignment must be 0 or a power of two in 4 .. 4096 bytes");
        for (const btdf_t *h : b->cases)
          if (h->state_ok) return fail(BTDF_ESTATE, "layout options must be set before the first device use");
        b->row_align = (int)value;
        b->layout_ok = false;
        return ok();
      case BTDF_OPT_MASK_UNSTABLE:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "mask flag must be 0 or 1");
        b->mask = (int)value;
        b->device_ok = false;
        return ok();
      case BTDF_OPT_TEMPORAL_BLOCKING:
        if (value < 0 || value > 3) return fail(BTDF_EINVAL, "temporal blocking must be 0 (off), 1 (deepest), 2 or 3");
        if ((value != 0) != (b->tblock != 0)) {
          b->tblock = value != 0;  // batches block three steps per pass or not at all
          b->layout_ok = false;    // every case's lists and slice size
        }
        return ok();
      case BTDF_OPT_EDGE_TILES:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "edge tiles must be 0 (step singly) or 1 (blocked)");
        if (value != b->edge_tiles) {
          b->edge_tiles = (int)value;
          b->layout_ok = false;  // every case's lists
        }
        return ok();
      default: return fail(BTDF_EINVAL, "unknown or read-only batch option %d", key);
    }
  });
}

int btdf_batch_get_option(const btdf_batch_t *b, int key, int64_t *value) {
  return guard([&]() -> int {
    if (!b || !value) return fail(BTDF_EINVAL, "NULL argument");
    switch (key) {
      case BTDF_OPT_LBM_VARIANT: *value = b->variant; return ok();
      case BTDF_OPT_NUM_VARIANTS: *value = num_variants(); return ok();
      case BTDF_OPT_GRAPH_CHUNK: *value = b->graph_chunk; return ok();
      case BTDF_OPT_XCD_REMAP: *value = b->xcd_remap; return ok();
      case BTDF_OPT_INTERIOR_PATH: *value = b->interior; return ok();
      case BTDF_OPT_MASK_UNSTABLE: *value = b->mask; return ok();
      case BTDF_OPT_ROW_ALIGN: *value = b->row_align; return ok();
      case BTDF_OPT_TEMPORAL_BLOCKING: *value = b->tblock; return ok();
      case BTDF_OPT_EDGE_TILES: *value = b->edge_tiles; return ok();
      case BTDF_OPT_FUSED_NODES:  // grid nodes of all cases in the blocked pass
        if (!b->layout_ok) batch_layout(const_cast<btdf_batch_t *>(b));
        *value = 0;
        if (b->blocked)
          for (const btdf_t *h : b->cases) *value += h->pass_nodes;
        return ok();
      case BTDF_OPT_TILE_X:
      case BTDF_OPT_TILE_Y: {
        int tx, ty;
        variant_tile(b->variant, &tx, &ty);
        *value = key == BTDF_OPT_TILE_X ? tx : ty;
        return ok();
      }
      case BTDF_OPT_FUSED_TILES:  // lattice tiles of all cases in the blocked pass
        if (!b->layout_ok) batch_layout(const_cast<btdf_batch_t *>(b));
        *value = 0;
        if (b->blocked)
          for (const btdf_t *h : b->cases)
            *value += h->pass_tiles();
        return ok();
      case BTDF_OPT_STEPS_PER_PASS:
        if (!b->layout_ok) batch_layout(const_cast<btdf_batch_t *>(b));
        *value = b->blocked ? 3 : 1;
        return ok();
      default: return fail(BTDF_EINVAL, "unknown batch option %d", key);
    }
  });
}

int btdf_batch_autotune(btdf_batch_t *b, int64_t steps_per_trial, int *best_variant) {
  return guard([&]() -> int {
    if (!b) return fail(BTDF_EINVAL, "NULL batch");
    if (steps_per_trial < 1) return fail(BTDF_EINVAL, "steps_per_trial must be >= 1");
    double best = 1e300;
    int bv = b->variant, bi = b->interior;
    for (int v = 0; v < num_variants(); ++v) {
      for (int in = 0; in < 2; ++in) {
        b->variant = v;
        b->interior = in;
        b->layout_ok = false;
        double a = 0.0, l = 0.0;
        int rc = batch_step_timed_impl(b, steps_per_trial, &a, &l);
        if (rc) return rc;
        if (a + l < best) {
          best = a + l;
          bv = v;
          bi = in;
        }
      }
    }
    b->variant = bv;
    b->interior = bi;
    b->layout_ok = false;
    if (best_variant) *best_variant = bv;
    return ok();
  });
}

}  // extern "C"
