// btdf_internal.h -- host-side state of a simulation handle and the helpers
// shared by the single-case API (btdf_api.hip) and the batch API
// (btdf_batch.hip). Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "btdf.h"
#include "btdf_launch.h"

#define HIPCHK(call)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return btdf::host::fail(BTDF_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// HIP events of the timed stepping calls: created on first use and kept
// until the handle is destroyed, so timing a run neither creates nor
// destroys events while its steps are in flight
struct btdf_event_pool {
  std::vector<hipEvent_t> ev;
  hipError_t reserve(size_t n) {
    while (ev.size() < n) {
      hipEvent_t e = nullptr;
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    return hipSuccess;
  }
  void release() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }
};

struct btdf_sim {
  void *owner = nullptr;  // the batch this handle is a case of (null: stand-alone)
  // configuration
  int nx = 0, ny = 0;
  int bc[4] = {0, 0, 0, 0};
  int prec = 8;
  int hist_cap = 4096;
  int kind = btdf::kCos4;
  double tau = 1.0, drs = 1.0;
  double G[2] = {0, 0}, uin[2] = {0, 0};
  double rho0 = 1.0, u0[2] = {0, 0};
  hipStream_t stream = nullptr;
  // bodies (host copies)
  std::vector<double> X, Y, U, V, sdrs;
  std::vector<int> off{0};
  std::vector<double> cx, cy, bsdrs;
  std::vector<char> stage;  // host image of the body part, sent in one copy
  // lattice kernel launch shape and tiles
  // launch defaults measured fastest on the 8192^2 particle-laden workload:
  // 32x8 tiles, general pull, marker kernel before the lattice kernel
  int variant = 6, xcd_remap = 1, graph_chunk = 0, interior = 1;
  int row_pad = 0, plane_pad = 0;
  int row_align = 128;  // bytes; rows start on this boundary (0: packed rows)
  int tile_x = 64, tile_y = 4, ntx = 0, nty = 0;
  std::vector<int> tile_off, tile_list;
  std::vector<int> tile_map;  // tiles no marker touches first, then the forced tiles
  int n_free = 0, n_forced = 0;
  int nf = 1;                 // forcing passes per step
  std::vector<int> cover_off, cover_list;  // covering markers per stencil node (nf > 1)
  int method = BTDF_FORCING_DIRECT;        // how the marker force is formed and spread
  std::vector<double> minv;                // implicit: (D_I D_E)^-1 per body, column-major
  std::vector<long long> minv_off;         // implicit: start of each body's matrix in minv
  std::vector<double> s_rkpm;              // RKPM: spreading factor ds epsilon_l per marker
  std::vector<double> bds;                 // arc length per marker of each body
  int max_body = 0;                        // markers of the largest body
  std::string method_err;                  // set-up failure of the implicit / RKPM matrices
  // rigid motion (host mirror of the device integration): per body a moving
  // flag, angle, velocity and angular velocity, per marker its offset from
  // the centre at angle 0; tile lists carry a margin and are rebuilt before
  // any marker can have moved by more than it
  std::vector<int> bmoving;
  std::vector<double> theta, bvx, bvy, bom, brad;
  std::vector<double> rx, ry;
  int margin = 0;
  int64_t steps_to_rebin = 0;
  // temporal blocking: tiles taking two steps at once, then the singly stepped regions
  int tblock = 1;  // option: 0 off, 1 the default depth, 2 to 5 steps per pass
  int edge_tiles = 0;  // option: tiles within reach of a domain edge take the blocked pass
  int depth = 1;   // steps per pass of the tiles away from the bodies (set with the layout)
  bool reserve_pass = false;  // keep the blocked pass's buffers whatever the launch shape (batch cases)
  // the tile map of the pass: its groups level by level (first tile of each
  // group), then the near tiles
  std::vector<int> fmap;
  std::vector<unsigned char> near;  // per lattice tile: 1 if it steps singly
  std::vector<unsigned> rwin;       // per fmap entry of a ring group (deeper passes): the near flags around it
  int gkind[btdf::kLevels] = {};  // shape per level (set with the lists)
  int n_grp[btdf::kLevels] = {};  // groups per level
  int n_edge[btdf::kLevels] = {};  // of those, edge groups (first in the level's list)
  int n_ring[btdf::kLevels] = {};  // passes of four or five steps: groups bordering a near tile (listed first)
  long long pass_nodes = 0;        // grid nodes in the blocked pass (partial tiles counted by their nodes)
  int n_near = 0;
  int n_groups() const {
    int k = 0;
    for (int i = 0; i < btdf::kLevels; ++i) k += n_grp[i];
    return k;
  }
  int grp_start(int g) const {  // index of level g's first group in fmap
    int k = 0;
    for (int i = 0; i < g; ++i) k += n_grp[i];
    return k;
  }
  int pass_tiles() const {  // lattice tiles in the pass
    int k = 0;
    for (int i = 0; i < btdf::kLevels; ++i) k += btdf::group_tiles(gkind[i]) * n_grp[i];
    return k;
  }
  // device memory
  char *ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  // layout
  int pitch = 0;
  long long plane = 0;
  size_t off_pop[2] = {0, 0}, off_ctl = 0, grid_bytes = 0;
  size_t off_hist = 0, off_mk = 0, off_mkw = 0, off_mkixy = 0, off_mkbody = 0, off_body = 0, off_boff = 0,
         off_toff = 0, off_tlist = 0, off_tmap = 0, off_coff = 0, off_clist = 0, off_mdfc = 0, off_mdff = 0,
         off_moff = 0, off_minv = 0, off_motion = 0, off_rxy = 0, off_fmap = 0, off_rwin = 0, off_near = 0, off_pop3 = 0, off_pop4 = 0, off_pop5 = 0, off_pop6 = 0, total = 0;
  bool layout_ok = false;  // host layout current for bodies and tiles
  bool device_ok = false;  // body part uploaded into the workspace
  bool state_ok = false;   // populations hold a state
  bool stepped = false;    // a step ran after the state and the body part last changed
  int cur = 0;             // which population buffer holds the state
  int64_t steps = 0, hist_read = 0;
  int64_t forces_from = 0;   // first step whose ring entry matches the body set
  bool bodies_dirty = true;  // ring layout on the device predates the body set
  // graph of graph_chunk steps starting from buffer 0
  hipGraphExec_t graph = nullptr;
  int graph_depth = 0;  // steps per pass the graph was captured with (1: single steps)
  hipStream_t cap_stream = nullptr;
  // passes of four or five steps: the small groups' launches run on a second
  // stream beside the largest groups' (fork and join events)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  btdf_event_pool tev;  // events of the timed stepping calls

  int nb() const { return (int)cx.size(); }
  bool any_moving() const {
    for (int m : bmoving)
      if (m) return true;
    return false;
  }
  int nm() const { return (int)X.size(); }
  bool xper() const { return bc[0] == BTDF_PERIODIC; }
  bool yper() const { return bc[2] == BTDF_PERIODIC; }
  int i0() const { return xper() ? 0 : 1; }
  int i1() const { return xper() ? nx - 1 : nx - 2; }
  template <typename P>
  P *at(size_t o) const { return reinterpret_cast<P *>(ws + o); }
};


namespace btdf {
namespace host {

int fail(int code, const char *fmt, ...) noexcept;
inline int ok() { return BTDF_OK; }

// Every extern "C" entry runs its body through guard (guard_size for the
// size queries, which report 0): an exception thrown inside, such as a
// failed host allocation in a std::vector, becomes a status code and a
// message instead of crossing the C ABI.
template <typename F>
inline int guard(F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail(BTDF_ENOMEM, "out of host memory");
  } catch (const std::exception &e) {
    return fail(BTDF_EDEVICE, "internal error: %s", e.what());
  } catch (...) {
    return fail(BTDF_EDEVICE, "internal error");
  }
}
template <typename F>
inline size_t guard_size(F &&body) noexcept {
  size_t v = 0;
  if (guard([&]() -> int {
        v = body();
        return BTDF_OK;
      }) != BTDF_OK)
    return 0;
  return v;
}
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
bool valid_kind(int k);
void drop_graph(btdf_t *h);
void compute_layout(btdf_t *h);
void group_kinds(int variant, int prec, int d, int kind[kLevels]);
void bin_markers(const btdf_t *h, int tx, int ty, int ntx, int nty, std::vector<int> &off, std::vector<int> &list);
void cover_lists(const btdf_t *h, std::vector<int> &off, std::vector<int> &list);
// implicit / RKPM matrices of the current bodies ("" or the reason they cannot be formed)
constexpr int kMaxImplicitBody = 2048;
constexpr int kMoveMargin = 2;  // nodes a moving marker may travel between tile-list rebuilds
// smallest lattice that blocks by default: the 256-channel set (8 k to 520 k
// nodes per case) ran at 11.4 GLUPS case by case unblocked, 8.2 blocked
constexpr long long kBlockMinNodes = 1ll << 20;
// steps per pass by default on a single lattice, where the launch shape has them
constexpr int kDefaultDepth = 5;
// width in tile columns of the bands down which groups two tiles tall are launched
constexpr int kSquareBand = 32;
std::string forcing_setup(btdf_t *h);
LbmParams make_params(const btdf_t *h);
IbParams make_ib(const btdf_t *h);
int ensure_device(btdf_t *h);
int check_flag(btdf_t *h);
int read_ctl(btdf_t *h, long long *ctr, int *flag);
int bind_impl(btdf_t *h, void *dev, size_t bytes);
int add_body_impl(btdf_t *h, int n, const double *xy, const double *uv, double cx, double cy, double ds,
                  int *body_id);
int destroy_impl(btdf_t *h);
// HIP events around the kernels of one step (timed stepping)
struct StepEvents {
  hipEvent_t ib0, ib1, a0, a1, b0, b1;
};
// one step from population buffer src into the other, on stream s
int enqueue_step(btdf_t *h, const LbmParams &p, const IbParams &ib, int src, hipStream_t s,
                 const StepEvents *te);

}  // namespace host
}  // namespace btdf
