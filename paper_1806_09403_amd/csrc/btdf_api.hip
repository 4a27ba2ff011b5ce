// btdf_api.hip -- host side of the C ABI declared in include/btdf.h.
//
// Device memory of a handle is one workspace (caller-owned or allocated
// here) laid out as
//   [ populations A | populations B | control (step counter, flag) ]   grid part
//   [ force history ring | marker arrays | body arrays | tile lists ]  body part
// The grid part has a fixed size for the handle, so rebinding or growing
// the workspace moves it with one device copy and rebuilds the body part
// from the host copies of the bodies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "btdf_internal.h"

using namespace btdf;

namespace btdf {
namespace host {

// the last failure's message on this thread: a fixed buffer, so reporting
// an error (an allocation failure included) allocates nothing
thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) noexcept {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}


// host value of the delta functions (calibration and validation only)
double phi_host(int kind, double r) {
  double a = std::fabs(r);
  switch (kind) {
    case kLinear2: return a <= 1.0 ? 1.0 - a : 0.0;
    case kRoma3:
      if (a <= 0.5) return (1.0 + std::sqrt(1.0 - 3.0 * a * a)) / 3.0;
      if (a <= 1.5) return (5.0 - 3.0 * a - std::sqrt(std::fmax(0.0, 1.0 - 3.0 * (1.0 - a) * (1.0 - a)))) / 6.0;
      return 0.0;
    case kPeskin4:
      if (a < 1.0) return (3.0 - 2.0 * a + std::sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
      if (a < 2.0) return (5.0 - 2.0 * a - std::sqrt(std::fmax(0.0, -7.0 + 12.0 * a - 4.0 * a * a))) / 8.0;
      return 0.0;
    default: return a <= 2.0 ? 0.25 * (1.0 + std::cos(M_PI * 0.5 * a)) : 0.0;
  }
}

bool valid_kind(int k) { return k == kLinear2 || k == kRoma3 || k == kPeskin4 || k == kCos4; }


void drop_graph(btdf_t *h) {
  if (h->graph) {
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
}

// stencil-node range of a marker coordinate (all kernels are inside [floor-1, floor+2])
void marker_range(int kind, double X, int *lo, int *hi) {
  int b = stencil_base(kind, X);
  *lo = b;
  *hi = b + stencil_size(kind) - 1;
}

int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// bin every marker into each tile (tx x ty nodes, ntx x nty tiles) its
// stencil touches: off[t] .. off[t+1] index ascending marker ids in list
void bin_markers(const btdf_t *h, int tx, int ty, int ntx, int nty, std::vector<int> &off,
                 std::vector<int> &list) {
  const int ntiles = ntx * nty;
  std::vector<int> cnt(ntiles + 1, 0);
  std::vector<int> touched;
  touched.reserve(16);
  auto tiles_of = [&](int l) {
    touched.clear();
    int xlo, xhi, ylo, yhi;
    marker_range(h->kind, h->X[l], &xlo, &xhi);
    marker_range(h->kind, h->Y[l], &ylo, &yhi);
    xlo -= h->margin;  // moving bodies: every tile the stencil can reach before the next rebuild
    xhi += h->margin;
    ylo -= h->margin;
    yhi += h->margin;
    for (int j = ylo; j <= yhi; ++j) {
      int jj = h->yper() ? ((j % h->ny) + h->ny) % h->ny : j;
      if (jj < 0 || jj >= h->ny) continue;
      for (int i = xlo; i <= xhi; ++i) {
        int ii = h->xper() ? ((i % h->nx) + h->nx) % h->nx : i;
        if (ii < 0 || ii >= h->nx) continue;
        int t = floordiv(jj, ty) * ntx + floordiv(ii, tx);
        if (std::find(touched.begin(), touched.end(), t) == touched.end()) touched.push_back(t);
      }
    }
  };
  for (int l = 0; l < h->nm(); ++l) {
    tiles_of(l);
    for (int t : touched) cnt[t + 1]++;
  }
  off.assign(ntiles + 1, 0);
  for (int t = 0; t < ntiles; ++t) off[t + 1] = off[t] + cnt[t + 1];
  list.assign(std::max(1, off[ntiles]), 0);
  std::vector<int> fill(off.begin(), off.end() - 1);
  for (int l = 0; l < h->nm(); ++l) {
    tiles_of(l);
    for (int t : touched) list[fill[t]++] = l;
  }
}

// For every marker l and stencil lane k = 4 j + i (i, j < stencil size), the
// markers whose stencil covers that node, ascending, packed as
// (marker << 4) | (dx << 2) | dy with (dx, dy) the node's place in the
// covering marker's stencil.
void cover_lists(const btdf_t *h, std::vector<int> &off, std::vector<int> &list) {
  const int nm = h->nm(), S = stencil_size(h->kind);
  struct Hit {
    long long node;
    int marker, lane;
  };
  std::vector<Hit> hits;
  hits.reserve((size_t)nm * S * S);
  auto origin = [&](int l, int *ox, int *oy) {
    *ox = stencil_base(h->kind, h->X[l]);
    *oy = stencil_base(h->kind, h->Y[l]);
  };
  auto key = [&](int x, int y) -> long long {
    if (h->xper()) x = ((x % h->nx) + h->nx) % h->nx;
    if (h->yper()) y = ((y % h->ny) + h->ny) % h->ny;
    return (long long)y * h->nx + x;
  };
  for (int l = 0; l < nm; ++l) {
    int ox, oy;
    origin(l, &ox, &oy);
    for (int j = 0; j < S; ++j)
      for (int i = 0; i < S; ++i) hits.push_back({key(ox + i, oy + j), l, (i << 2) | j});
  }
  std::sort(hits.begin(), hits.end(), [](const Hit &a, const Hit &b) {
    return a.node != b.node ? a.node < b.node : a.marker < b.marker;
  });
  off.assign((size_t)nm * 16 + 1, 0);
  list.clear();
  for (int l = 0; l < nm; ++l) {
    int ox, oy;
    origin(l, &ox, &oy);
    for (int k = 0; k < 16; ++k) {
      off[(size_t)l * 16 + k] = (int)list.size();
      const int i = k & 3, j = k >> 2;
      if (i >= S || j >= S) continue;
      const long long nk = key(ox + i, oy + j);
      auto lo = std::lower_bound(hits.begin(), hits.end(), nk,
                                 [](const Hit &a, long long v) { return a.node < v; });
      for (auto it = lo; it != hits.end() && it->node == nk; ++it) list.push_back((it->marker << 4) | it->lane);
    }
  }
  off[(size_t)nm * 16] = (int)list.size();
  if (list.empty()) list.push_back(0);
}

// steps per pass of the tiles away from the bodies for the options and the
// launch shape: the depth asked for (by default kDefaultDepth on an FP32
// single lattice, 3 in FP64 and in a batch), or the deepest below it that
// the shape has (4 and 5 on single lattices only), else 1 (no blocking)
int pass_depth(const btdf_t *h) {
  if (!h->tblock) return 1;
  // by default only lattices large enough that the saved bytes outweigh the
  // extra launches of a blocked pass (single handles; a batch shares them)
  if (h->tblock == 1 && !h->owner && (long long)h->nx * h->ny < kBlockMinNodes) return 1;
  int want = h->tblock == 1 ? (h->owner || h->prec != 4 ? 3 : kDefaultDepth) : h->tblock;
  if (h->owner) want = std::min(want, 3);
  for (int d = want; d >= 4; --d)
    if (variant_has_deep(h->variant, h->prec, d, kGroup1x1)) return d;
  if (want >= 3 && variant_has_lbm3(h->variant, h->prec, kGroup1x1)) return 3;
  if (variant_has_lbm2(h->variant, h->prec)) return 2;
  return 1;
}

// whether the pass of depth d has a launch over groups of the given shape
// (two-step pass: one row of 1, 2 or 4 tiles)
static bool has_group(const btdf_t *h, int d, int code) {
  if (is_edge(code)) return variant_has_edge(h->variant, h->prec, d, code);
  if (d >= 4) return variant_has_deep(h->variant, h->prec, d, code);
  if (d == 3) return variant_has_lbm3(h->variant, h->prec, code);
  const int w = code & 15;
  if (((code >> 4) & 15) != 1) return false;
  return w == 1 ? variant_has_lbm2(h->variant, h->prec) : variant_has_wide_lbm2(h->variant, h->prec, w);
}

// The shapes of the launches of a pass of depth d, level by level (tiles
// are packed into the first level's groups, the rest into the next
// level's): groups of four tiles along rows, then two, then single tiles.
// (The launch shape decides which of them have a pass; d is kept for
// shapes that only one depth has.)
void group_kinds(int variant, int prec, int d, int kind[kLevels]) {
  (void)variant;
  (void)prec;
  // five steps: squares of two by two tiles first (the fewest recomputed
  // halo nodes per node), then columns of two, rows of two, single tiles
  static const int rows[kLevels] = {kGroup4x1, kGroup1x4, kGroup2x1, kGroup1x1};
  static const int squares[kLevels] = {kGroup2x2, kGroup1x2, kGroup2x1, kGroup1x1};
  for (int i = 0; i < kLevels; ++i) kind[i] = d >= 5 ? squares[i] : rows[i];
}

// Tiles for temporal blocking of depth d = h->depth on the current launch
// shape: a tile is "near" if a marker stencil grown by d - 1 nodes reaches
// it (a pass takes its first step over its tiles grown by d - 1 nodes, which
// must hold no forced node). Near tiles step singly, with the marker kernel
// between; the pass gives them the intermediate states of the nodes just
// outside. Of the other tiles, those within d nodes of a domain edge (or
// reaching past the grid) take the pass one by one with the boundary
// readings in every step (the edge level), unless an edge in reach is a
// convective outlet, or the zero-gradient outlet's ghost column and column
// nx-2 fall in different tiles: those tiles are near too.
void fused_lists(btdf_t *h) {
  h->fmap.clear();
  for (int g = 0; g < kLevels; ++g) h->n_grp[g] = h->n_edge[g] = h->n_ring[g] = 0;
  h->pass_nodes = 0;
  h->n_near = 0;
  h->near.clear();
  h->rwin.clear();
  const int d = h->depth;
  if (d < 2) return;
  const int tx = h->tile_x, ty = h->tile_y, ntx = h->ntx, nty = h->nty, ntiles = ntx * nty;
  // (edge groups wrap a node index by one period at most: a periodic extent
  // must hold the widest or tallest group, four tiles, and the margins)
  const bool edge_pass = h->edge_tiles && has_group(h, d, kEdge1x1) && (!h->xper() || h->nx >= 4 * tx + 8) &&
                         (!h->yper() || h->ny >= 4 * ty + 8);
  const bool conv = h->bc[1] == BTDF_CONVECTIVE_OUTLET;
  // the zero-gradient outlet's ghost (nx-1) alone in the last tile column
  const bool split_ghost = h->bc[1] == BTDF_ZERO_GRADIENT_OUTLET && (h->nx - 1) % tx == 0;
  std::vector<char> near(ntiles, 0), edge(ntiles, 0);
  for (int t = 0; t < ntiles; ++t) {
    const int x0 = (t % ntx) * tx, y0 = (t / ntx) * ty;
    const bool xr = x0 + tx + d > h->nx;  // within reach of the east edge
    if (!(x0 < d || xr || y0 < d || y0 + ty + d > h->ny)) continue;
    bool ok = edge_pass;
    if (!h->xper() && xr && conv) ok = false;
    if (!h->xper() && split_ghost && (x0 == h->nx - 1 || x0 + tx == h->nx - 1)) ok = false;
    (ok ? edge : near)[t] = 1;
  }
  for (int l = 0; l < h->nm(); ++l) {
    int xlo, xhi, ylo, yhi;
    marker_range(h->kind, h->X[l], &xlo, &xhi);
    marker_range(h->kind, h->Y[l], &ylo, &yhi);
    xlo -= d - 1 + h->margin;
    xhi += d - 1 + h->margin;
    ylo -= d - 1 + h->margin;
    yhi += d - 1 + h->margin;
    for (int j = ylo; j <= yhi; ++j) {
      const int jj = h->yper() ? ((j % h->ny) + h->ny) % h->ny : j;
      if (jj < 0 || jj >= h->ny) continue;
      for (int i = xlo; i <= xhi; ++i) {
        const int ii = h->xper() ? ((i % h->nx) + h->nx) % h->nx : i;
        if (ii < 0 || ii >= h->nx) continue;
        near[(jj / ty) * ntx + ii / tx] = 1;
      }
    }
  }
  for (int t = 0; t < ntiles; ++t)
    if (near[t]) edge[t] = 0;
  // Blocked tiles, level by level (the map lists the levels in order, each
  // group by its lower-left tile): rows of four tiles where the launch shape
  // has such a pass, then rows of two, then single tiles. A level lists its
  // edge groups first (flagged with kEdgeFlag), then its interior groups.
  // Groups are packed greedily, row by row of tiles, from any tile column, so
  // a run of L tiles of one kind in a row leaves only L mod 4 of them outside
  // groups of four.
  group_kinds(h->variant, h->prec, d, h->gkind);
  // taken[k][t]: tile t is not free for groups of kind k (0 interior, 1 edge)
  std::vector<char> taken[2] = {std::vector<char>(ntiles), std::vector<char>(ntiles)};
  for (int t = 0; t < ntiles; ++t) {
    taken[0][t] = near[t] || edge[t];
    taken[1][t] = near[t] || !edge[t];
  }
  for (int g = 0; g < kLevels; ++g) {
    const int code = h->gkind[g], w = code & 15, gh = (code >> 4) & 15;
    const size_t start = h->fmap.size();
    for (int kind = 1; kind >= 0; --kind) {
      if (code == kNoGroup || !has_group(h, d, kind ? (kEdge | code) : code)) continue;
      std::vector<char> &tk = taken[kind];
      for (int b = 0; b + gh - 1 < nty; ++b)
        for (int a = 0; a + w - 1 < ntx;) {
          const int t = b * ntx + a;
          bool ok = true;
          for (int r = 0; r < gh; ++r)
            for (int k = 0; k < w; ++k) ok = ok && !tk[t + r * ntx + k];
          if (!ok) {
            ++a;
            continue;
          }
          h->fmap.push_back(kind ? (t | kEdgeFlag) : t);
          for (int r = 0; r < gh; ++r)
            for (int k = 0; k < w; ++k) tk[t + r * ntx + k] = 1;
          a += w;
        }
      if (kind) h->n_edge[g] = (int)(h->fmap.size() - start);
    }
    h->n_grp[g] = (int)(h->fmap.size() - start);
    if (d >= 4) {
      // the groups with a near tile among the tiles around them first (they
      // write the ring), the others after them, each in packing order
      auto ring = [&](int t) {
        const int a = t % ntx, b = t / ntx;
        for (int r = b - 1; r <= b + gh; ++r)
          for (int c = a - 1; c <= a + w; ++c)
            if (r >= 0 && r < nty && c >= 0 && c < ntx && near[r * ntx + c]) return true;
        return false;
      };
      const auto mid = std::stable_partition(h->fmap.begin() + start, h->fmap.end(), ring);
      h->n_ring[g] = (int)(mid - (h->fmap.begin() + start));
      // Groups two tiles tall are launched down bands of kSquareBand tile
      // columns, row by row within a band: the groups above and below one
      // are then a band's width of launch slots away instead of a whole
      // row's, and the halo rows they share are still in the XCD's L2.
      if (gh == 2) {
        auto key = [&](int t) { return std::make_tuple((t % ntx) / kSquareBand, t / ntx, t % ntx); };
        auto cmp = [&](int a, int b) { return key(a) < key(b); };
        std::stable_sort(h->fmap.begin() + start, mid, cmp);
        std::stable_sort(mid, h->fmap.end(), cmp);
      }
      // each ring group's window of near flags (bit 8 r + c, r from the row
      // below, c from the column left of the group)
      h->rwin.resize(h->fmap.size(), 0u);
      for (size_t k = start; k < start + (size_t)h->n_ring[g]; ++k) {
        const int t = h->fmap[k], a = t % ntx, b = t / ntx;
        unsigned m = 0;
        for (int r = 0; r < gh + 2; ++r)
          for (int c = 0; c < w + 2; ++c) m |= near[(b - 1 + r) * ntx + a - 1 + c] ? 1u << (8 * r + c) : 0u;
        h->rwin[k] = m;
      }
    }
  }
  h->rwin.resize(h->fmap.size(), 0u);
  for (int t = 0; t < ntiles; ++t)
    if (!near[t]) {
      const int x0 = (t % ntx) * tx, y0 = (t / ntx) * ty;
      h->pass_nodes += (long long)std::min(tx, h->nx - x0) * std::min(ty, h->ny - y0);
    }
  const size_t start_near = h->fmap.size();
  for (int t = 0; t < ntiles; ++t)
    if (near[t]) h->fmap.push_back(t);
  h->n_near = (int)(h->fmap.size() - start_near);
  h->near.assign(near.begin(), near.end());
}

// the most tiles one marker's (margin-widened) stencil can touch, over every launch shape
int tiles_per_marker(const btdf_t *h) {
  const int L = stencil_size(h->kind) + 2 * h->margin;
  int best = 0;
  for (int v = 0; v < num_variants(); ++v) {
    int tx, ty;
    variant_tile(v, &tx, &ty);
    best = std::max(best, ((L - 1) / tx + 2) * ((L - 1) / ty + 2));
  }
  return best;
}

// Host copies of the moving bodies' markers from the mirrored centre and
// angle, with the arithmetic of the device's rigid_move_kernel.
void mirror_positions(btdf_t *h) {
  for (int b = 0; b < h->nb(); ++b) {
    if (!h->bmoving[b]) continue;
    const double c = std::cos(h->theta[b]), s = std::sin(h->theta[b]);
    const double cx = h->cx[b], cy = h->cy[b], vx = h->bvx[b], vy = h->bvy[b], om = h->bom[b];
    for (int l = h->off[b]; l < h->off[b + 1]; ++l) {
      const double X = cx + c * h->rx[l] - s * h->ry[l];
      const double Y = cy + s * h->rx[l] + c * h->ry[l];
      h->X[l] = X;
      h->Y[l] = Y;
      h->U[l] = vx - om * (Y - cy);
      h->V[l] = vy + om * (X - cx);
    }
  }
}

// advance the mirrored centres and angles by k steps, one step at a time as the device does
void mirror_advance(btdf_t *h, int64_t k) {
  for (int b = 0; b < h->nb(); ++b) {
    if (!h->bmoving[b]) continue;
    for (int64_t t = 0; t < k; ++t) {
      h->cx[b] += h->bvx[b];
      h->cy[b] += h->bvy[b];
      h->theta[b] += h->bom[b];
    }
  }
}

// per-step displacement bound of the fastest marker of a moving body
double max_marker_speed(const btdf_t *h) {
  double v = 0.0;
  for (int b = 0; b < h->nb(); ++b)
    if (h->bmoving[b]) v = std::max(v, std::hypot(h->bvx[b], h->bvy[b]) + std::fabs(h->bom[b]) * h->brad[b]);
  return v;
}

MoveParams make_move(const btdf_t *h) {
  MoveParams mp{};
  const size_t M = (size_t)std::max(h->nm(), 1), B = (size_t)std::max(h->nb(), 1);
  double *mk = h->at<double>(h->off_mk);
  double *bd = h->at<double>(h->off_body);
  mp.nb = h->nb();
  mp.body_off = h->at<int>(h->off_boff);
  mp.state = h->at<double>(h->off_motion);
  mp.moving = reinterpret_cast<const int *>(h->ws + h->off_motion + 4 * B * sizeof(double));
  mp.cx = bd;
  mp.cy = bd + B;
  mp.X = mk;
  mp.Y = mk + M;
  mp.U = mk + 2 * M;
  mp.V = mk + 3 * M;
  mp.rxy = h->at<double>(h->off_rxy);
  return mp;
}

void compute_layout(btdf_t *h) {
  const size_t elt = (size_t)h->prec;
  const int a = h->row_align > 0 ? std::max(1, h->row_align / (int)elt) : 1;
  h->pitch = (h->nx + a - 1) / a * a + h->row_pad;
  h->plane = (((long long)h->pitch * h->ny + 63) / 64) * 64 + h->plane_pad;
  const size_t pop_bytes = align256(9 * (size_t)h->plane * elt);
  h->off_pop[0] = 0;
  h->off_pop[1] = pop_bytes;
  h->off_ctl = 2 * pop_bytes;  // 256 B of counters and flags, then 512 B of constants (kKonstBytes)
  h->grid_bytes = h->off_ctl + 768;

  variant_tile(h->variant, &h->tile_x, &h->tile_y);
  h->ntx = (h->nx + h->tile_x - 1) / h->tile_x;
  h->nty = (h->ny + h->tile_y - 1) / h->tile_y;
  const int ntiles = h->ntx * h->nty;

  mirror_positions(h);
  // one node beyond the travel allowance: a device position within rounding of
  // the host's may floor to the neighbouring stencil origin
  h->margin = h->any_moving() ? kMoveMargin + 1 : 0;
  h->steps_to_rebin = 0;
  bin_markers(h, h->tile_x, h->tile_y, h->ntx, h->nty, h->tile_off, h->tile_list);
  h->tile_map.clear();
  h->tile_map.reserve(ntiles);
  for (int t = 0; t < ntiles; ++t)
    if (h->tile_off[t + 1] == h->tile_off[t]) h->tile_map.push_back(t);
  h->n_free = (int)h->tile_map.size();
  for (int t = 0; t < ntiles; ++t)
    if (h->tile_off[t + 1] != h->tile_off[t]) h->tile_map.push_back(t);
  h->n_forced = ntiles - h->n_free;

  const int nb = h->nb(), nm = h->nm();
  size_t o = h->grid_bytes;
  h->off_hist = o;
  o = align256(o + (size_t)h->hist_cap * std::max(nb, 1) * 3 * sizeof(double));
  h->off_mk = o;  // X Y U V sdrs Fx Fy rho ux uy
  o = align256(o + 10 * (size_t)std::max(nm, 1) * sizeof(double));
  h->off_mkw = o;  // 10 values per marker in the population type
  o = align256(o + 10 * (size_t)std::max(nm, 1) * elt);
  h->off_mkixy = o;
  o = align256(o + 2 * (size_t)std::max(nm, 1) * sizeof(int));
  h->off_mkbody = o;
  o = align256(o + (size_t)std::max(nm, 1) * sizeof(int));
  h->off_body = o;  // cx cy bsdrs
  o = align256(o + 3 * (size_t)std::max(nb, 1) * sizeof(double));
  h->off_boff = o;
  o = align256(o + (size_t)(nb + 1) * sizeof(int));
  // the tile region is sized for the launch shape with the most tiles and for
  // the most tiles one marker stencil can touch (2 x 5), so a change of launch
  // shape never changes the workspace size
  long long max_tiles = 0;
  for (int v = 0; v < num_variants(); ++v) {
    int tx, ty;
    variant_tile(v, &tx, &ty);
    max_tiles = std::max(max_tiles, (long long)((h->nx + tx - 1) / tx) * ((h->ny + ty - 1) / ty));
  }
  const size_t list_cap = (size_t)tiles_per_marker(h) * nm + 1;
  h->off_toff = o;
  o = align256(o + (size_t)(max_tiles + 1) * sizeof(int));
  h->off_tlist = o;
  o = align256(o + list_cap * sizeof(int));
  h->off_tmap = o;
  o = align256(o + (size_t)max_tiles * sizeof(int));
  // forcing passes beyond the first: covering-marker lists, each stencil
  // node's rho and u*, and the accumulated marker forces (two copies)
  h->cover_off.clear();
  h->cover_list.clear();
  if (h->nf > 1) cover_lists(h, h->cover_off, h->cover_list);
  h->off_coff = o;
  o = align256(o + h->cover_off.size() * sizeof(int));
  h->off_clist = o;
  o = align256(o + h->cover_list.size() * sizeof(int));
  h->off_mdfc = o;
  o = align256(o + (h->nf > 1 ? 56 * (size_t)std::max(nm, 1) * sizeof(double) : 0));
  h->off_mdff = o;
  o = align256(o + (h->nf > 1 ? 4 * (size_t)std::max(nm, 1) * sizeof(double) : 0));
  // implicit forcing: one inverse matrix per body; RKPM: nothing beyond the marker factors
  h->method_err = forcing_setup(h);
  h->off_moff = o;
  o = align256(o + h->minv_off.size() * sizeof(long long));
  h->off_minv = o;
  o = align256(o + h->minv.size() * sizeof(double));
  // temporal blocking: the tiles that take two steps at once, then the tiles
  // stepped singly (those next to the bodies and the edges, grown by their
  // neighbours), then those next to the bodies and the edges; and a third
  // population buffer for the singly stepped tiles' intermediate state
  h->depth = pass_depth(h);
  fused_lists(h);
  h->off_fmap = o;
  o = align256(o + 2 * (size_t)max_tiles * sizeof(int));
  h->off_rwin = o;  // per map entry
  o = align256(o + 2 * (size_t)max_tiles * sizeof(unsigned));
  h->off_near = o;  // one flag per tile
  o = align256(o + (size_t)max_tiles);
  h->off_pop3 = o;  // the near tiles' intermediate states n+1 .. n+depth-1
  o = align256(o + (h->depth >= 2 || h->reserve_pass ? pop_bytes : 0));
  h->off_pop4 = o;
  o = align256(o + (h->depth >= 3 || h->reserve_pass ? pop_bytes : 0));
  h->off_pop5 = o;
  o = align256(o + (h->depth >= 4 ? pop_bytes : 0));
  h->off_pop6 = o;
  o = align256(o + (h->depth >= 5 ? pop_bytes : 0));
  // (pop_bytes is a multiple of 256, so X1 .. X4 are consecutive buffers,
  // which the passes of four and five steps address from X1)
  // rigid motion: [nb][4] theta vx vy omega, then [nb] moving flags; [nm][2] offsets
  h->off_motion = o;
  o = align256(o + 4 * (size_t)std::max(nb, 1) * sizeof(double) + (size_t)std::max(nb, 1) * sizeof(int));
  h->off_rxy = o;
  o = align256(o + 2 * (size_t)std::max(nm, 1) * sizeof(double));
  h->total = o;

  h->layout_ok = true;
  h->device_ok = false;
  drop_graph(h);
}

LbmParams make_params(const btdf_t *h) {
  LbmParams p{};
  p.nx = h->nx;
  p.ny = h->ny;
  p.pitch = h->pitch;
  p.plane = h->plane;
  p.xper = h->xper();
  p.yper = h->yper();
  p.inlet = h->bc[0] == BTDF_VELOCITY_INLET;
  p.outlet = h->bc[1] == BTDF_ZERO_GRADIENT_OUTLET ? 1 : (h->bc[1] == BTDF_CONVECTIVE_OUTLET ? 2 : 0);
  p.slip = h->bc[2] == BTDF_FREE_SLIP_WALL;
  p.uconv = h->uin[0];
  p.i0 = h->i0();
  p.i1 = h->i1();
  p.omega = 1.0 / h->tau;
  p.guo = 1.0 - 1.0 / (2.0 * h->tau);
  p.Gx = h->G[0];
  p.Gy = h->G[1];
  p.uin_x = h->uin[0];
  p.uin_y = h->uin[1];
  p.urx = h->u0[0];  // the stored deviations are taken from feq(1, initial velocity)
  p.ury = h->u0[1];
  p.ntx = h->ntx;
  p.nty = h->nty;
  p.xcd_remap = h->xcd_remap;
  p.interior = h->interior;
  p.tile_off = h->at<int>(h->off_toff);
  p.tile_list = h->at<int>(h->off_tlist);
  p.mk_w = h->ws + h->off_mkw;
  p.mk_ixy = h->at<int>(h->off_mkixy);
  p.kind = h->kind;
  p.step_ctr = h->at<long long>(h->off_ctl);
  p.flag = h->at<int>(h->off_ctl + 8);
  p.konst = h->ws + h->off_ctl + 256;
  fill_collision(p);
  return p;
}

IbParams make_ib(const btdf_t *h) {
  IbParams ib{};
  const size_t M = (size_t)std::max(h->nm(), 1), B = (size_t)std::max(h->nb(), 1);
  double *mk = h->at<double>(h->off_mk);
  double *bd = h->at<double>(h->off_body);
  ib.nb = h->nb();
  ib.nm = h->nm();
  ib.body_off = h->at<int>(h->off_boff);
  ib.mk_body = h->at<int>(h->off_mkbody);
  ib.slot = h->at<int>(h->off_ctl + 16);
  ib.X = mk;
  ib.Y = mk + M;
  ib.U = mk + 2 * M;
  ib.V = mk + 3 * M;
  ib.Fx = mk + 5 * M;
  ib.Fy = mk + 6 * M;
  ib.rho_l = mk + 7 * M;
  ib.ux_l = mk + 8 * M;
  ib.uy_l = mk + 9 * M;
  ib.sdrs = mk + 4 * M;
  ib.mk_w = h->ws + h->off_mkw;
  ib.mk_ixy = h->at<int>(h->off_mkixy);
  ib.cx = bd;
  ib.cy = bd + B;
  ib.body_sdrs = bd + 2 * B;
  ib.hist = h->at<double>(h->off_hist);
  ib.hist_cap = h->hist_cap;
  ib.nf = h->nf;
  ib.cover_off = h->at<int>(h->off_coff);
  ib.cover_list = h->at<int>(h->off_clist);
  ib.mdf_cache = h->at<double>(h->off_mdfc);
  ib.mdf_w = ib.mdf_cache + 48 * M;
  ib.method = h->method;
  ib.max_body = h->max_body;
  ib.minv = h->at<double>(h->off_minv);
  ib.minv_off = h->at<long long>(h->off_moff);
  ib.mdf_f = h->at<double>(h->off_mdff);
  return ib;
}

int upload(btdf_t *h, size_t off, const void *src, size_t bytes) {
  if (bytes == 0) return ok();
  HIPCHK(hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, h->stream));
  return ok();
}

int upload_bodies(btdf_t *h) {
  // the whole body part [off_mk, total) is staged on the host and sent in one
  // copy; arrays the kernels fill (marker forces, weights, stencil origins)
  // start at zero
  const size_t M = (size_t)std::max(h->nm(), 1), B = (size_t)std::max(h->nb(), 1);
  const size_t nm = (size_t)h->nm(), nb = (size_t)h->nb();
  const size_t d = sizeof(double);
  mirror_positions(h);  // moving bodies: the markers where the mirrored motion has taken them
  std::vector<char> &st = h->stage;
  st.assign(h->total - h->off_mk, 0);
  auto st_base = [&](const btdf_t *, size_t off) { return st.data() + (off - h->off_mk); };
  auto put = [&](size_t off, const void *src, size_t bytes) {
    if (bytes) std::memcpy(st.data() + (off - h->off_mk), src, bytes);
  };
  put(h->off_mk + 0 * M * d, h->X.data(), nm * d);
  put(h->off_mk + 1 * M * d, h->Y.data(), nm * d);
  put(h->off_mk + 2 * M * d, h->U.data(), nm * d);
  put(h->off_mk + 3 * M * d, h->V.data(), nm * d);
  // the spreading factor of each marker: drs ds, or ds epsilon_l under RKPM
  const bool rk = h->method == BTDF_FORCING_RKPM && h->s_rkpm.size() == nm;
  put(h->off_mk + 4 * M * d, rk ? h->s_rkpm.data() : h->sdrs.data(), nm * d);
  put(h->off_body + 0 * B * d, h->cx.data(), nb * d);
  put(h->off_body + 1 * B * d, h->cy.data(), nb * d);
  put(h->off_body + 2 * B * d, h->bsdrs.data(), nb * d);
  put(h->off_boff, h->off.data(), (nb + 1) * sizeof(int));
  int *body_of = reinterpret_cast<int *>(st.data() + (h->off_mkbody - h->off_mk));
  for (int b = 0; b < h->nb(); ++b)
    for (int l = h->off[b]; l < h->off[b + 1]; ++l) body_of[l] = b;
  put(h->off_toff, h->tile_off.data(), h->tile_off.size() * sizeof(int));
  put(h->off_tlist, h->tile_list.data(), h->tile_list.size() * sizeof(int));
  put(h->off_tmap, h->tile_map.data(), h->tile_map.size() * sizeof(int));
  {
    double *ms = reinterpret_cast<double *>(st_base(h, h->off_motion));
    int *mv = reinterpret_cast<int *>(st_base(h, h->off_motion) + 4 * B * d);
    double *r = reinterpret_cast<double *>(st_base(h, h->off_rxy));
    for (int b = 0; b < h->nb(); ++b) {
      ms[4 * b] = h->theta[b];
      ms[4 * b + 1] = h->bvx[b];
      ms[4 * b + 2] = h->bvy[b];
      ms[4 * b + 3] = h->bom[b];
      mv[b] = h->bmoving[b];
    }
    for (size_t l = 0; l < nm; ++l) {
      r[2 * l] = h->rx[l];
      r[2 * l + 1] = h->ry[l];
    }
  }
  put(h->off_fmap, h->fmap.data(), h->fmap.size() * sizeof(int));
  put(h->off_rwin, h->rwin.data(), h->rwin.size() * sizeof(unsigned));
  put(h->off_near, h->near.data(), h->near.size());
  put(h->off_moff, h->minv_off.data(), h->minv_off.size() * sizeof(long long));
  put(h->off_minv, h->minv.data(), h->minv.size() * sizeof(double));
  put(h->off_coff, h->cover_off.data(), h->cover_off.size() * sizeof(int));
  put(h->off_clist, h->cover_list.data(), h->cover_list.size() * sizeof(int));
  HIPCHK(hipMemcpyAsync(h->ws + h->off_mk, st.data(), st.size(), hipMemcpyHostToDevice, h->stream));
  if (h->bodies_dirty)
    HIPCHK(hipMemsetAsync(h->ws + h->off_hist, 0,
                          (size_t)h->hist_cap * std::max(h->nb(), 1) * 3 * sizeof(double), h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));  // the staging buffer may change after return
  h->device_ok = true;
  h->bodies_dirty = false;
  h->stepped = false;  // the marker arrays start at zero again
  return ok();
}

int init_state(btdf_t *h) {
  LbmParams p = make_params(h);
  HIPCHK(launch_init_uniform(h->prec, h->ws + h->off_pop[0], p, h->rho0, h->u0[0], h->u0[1], h->stream));
  HIPCHK(hipMemsetAsync(h->ws + h->off_ctl, 0, 256, h->stream));
  unsigned char konst[kKonstBytes];
  fill_konst(p, konst);
  HIPCHK(hipMemcpyAsync(h->ws + h->off_ctl + 256, konst, kKonstBytes, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));  // (konst is on this stack)
  h->cur = 0;
  h->steps = 0;
  h->hist_read = 0;
  h->state_ok = true;
  h->stepped = false;
  return ok();
}

// bytes of live state to carry into a new workspace: the grid part, plus the
// force ring when it still matches the body set
size_t moved_bytes(const btdf_t *h) { return h->bodies_dirty ? h->grid_bytes : h->off_mk; }

// make the workspace hold a valid state and the current body part
int ensure_device(btdf_t *h) {
  if (!h->layout_ok) compute_layout(h);
  if (!h->method_err.empty()) return fail(BTDF_EINVAL, "%s", h->method_err.c_str());
  if (h->ws == nullptr || h->ws_bytes < h->total) {
    if (h->ws != nullptr && !h->ws_owned)
      return fail(BTDF_ENOMEM, "bound workspace has %zu bytes, %zu needed (rebind a larger one)",
                  h->ws_bytes, h->total);
    char *nw = nullptr;
    hipError_t e = hipMalloc((void **)&nw, h->total);
    if (e != hipSuccess)
      return fail(BTDF_ENOMEM, "hipMalloc(%zu): %s", h->total, hipGetErrorString(e));
    if (h->ws && h->state_ok) {
      HIPCHK(hipMemcpyAsync(nw, h->ws, moved_bytes(h), hipMemcpyDeviceToDevice, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (h->ws && h->ws_owned) HIPCHK(hipFree(h->ws));
    h->ws = nw;
    h->ws_bytes = h->total;
    h->ws_owned = true;
    h->device_ok = false;
    drop_graph(h);
  }
  if (!h->state_ok) {
    int rc = init_state(h);
    if (rc) return rc;
  }
  if (!h->device_ok) {
    int rc = upload_bodies(h);
    if (rc) return rc;
  }
  return ok();
}

int read_ctl(btdf_t *h, long long *ctr, int *flag) {
  unsigned char buf[16];
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(buf, h->ws + h->off_ctl, 16, hipMemcpyDeviceToHost));
  std::memcpy(ctr, buf, 8);
  std::memcpy(flag, buf + 8, 4);
  return ok();
}

int check_flag(btdf_t *h) {
  long long ctr;
  int flag;
  int rc = read_ctl(h, &ctr, &flag);
  if (rc) return rc;
  if (flag > 0) return fail(BTDF_EUNSTABLE, "unstable: marker of body %d (non-finite force or |u*| > 0.3)", flag - 1);
  if (flag < 0) return fail(BTDF_EUNSTABLE, "unstable: non-positive or non-finite density at a node");
  return ok();
}

int clear_flag(btdf_t *h) {
  HIPCHK(hipMemsetAsync(h->ws + h->off_ctl + 8, 0, 4, h->stream));
  return ok();
}

// One time step on the given buffers: the marker kernel (interpolation,
// direct force, spread weights), then the lattice kernel over every tile
// (and the body reductions), then the outlet and rigid motion.
int enqueue_step(btdf_t *h, const LbmParams &p, const IbParams &ib, int src, hipStream_t s,
                 const StepEvents *te) {
  const void *A = h->ws + h->off_pop[src];
  void *B = h->ws + h->off_pop[1 - src];
  if (te) HIPCHK(hipEventRecord(te->ib0, s));
  HIPCHK(launch_ib(h->prec, A, p, ib, s));
  if (te) HIPCHK(hipEventRecord(te->ib1, s));
  HIPCHK(launch_lbm(h->prec, h->variant, A, B, p, TileRange{nullptr, 0, h->ntx * h->nty, 1}, ib, s));
  if (te) HIPCHK(hipEventRecord(te->a1, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, A, B, p, s));
  // moving bodies advance after the step that used their positions (the body
  // reduction in the lattice launch reads the centres)
  if (h->any_moving()) HIPCHK(launch_rigid_move(make_move(h), s));
  return ok();
}

int build_graph(btdf_t *h, const LbmParams &p, const IbParams &ib) {
  drop_graph(h);
  if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  for (int k = 0; k < h->graph_chunk && rc == 0; ++k) rc = enqueue_step(h, p, ib, k & 1, h->cap_stream, nullptr);
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  h->graph_depth = 1;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(BTDF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph = nullptr;
    return fail(BTDF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return ok();
}

// move the handle's device memory to dev[0 .. bytes) (null: library-owned)
int bind_impl(btdf_t *h, void *dev, size_t bytes) {
  if (dev && ((uintptr_t)dev & 255)) return fail(BTDF_EINVAL, "workspace must be 256-byte aligned");
  if (!h->layout_ok) compute_layout(h);
  if (dev && bytes < h->total)
    return fail(BTDF_ENOMEM, "workspace has %zu bytes, %zu needed", bytes, h->total);
  if (dev == (void *)h->ws && dev) {
    h->ws_bytes = bytes;
    return ok();
  }
  if (!dev) {
    // back to library-owned memory on the next device call
    if (h->ws && !h->ws_owned) {
      char *nw = nullptr;
      hipError_t e = hipMalloc((void **)&nw, h->total);
      if (e != hipSuccess) return fail(BTDF_ENOMEM, "hipMalloc(%zu): %s", h->total, hipGetErrorString(e));
      if (h->state_ok) {
        HIPCHK(hipMemcpyAsync(nw, h->ws, moved_bytes(h), hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
      }
      h->ws = nw;
      h->ws_bytes = h->total;
      h->ws_owned = true;
      h->device_ok = false;
      drop_graph(h);
    }
    return ok();
  }
  if (h->ws && h->state_ok) {
    HIPCHK(hipMemcpyAsync(dev, h->ws, moved_bytes(h), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  if (h->ws && h->ws_owned) HIPCHK(hipFree(h->ws));
  h->ws = (char *)dev;
  h->ws_bytes = bytes;
  h->ws_owned = false;
  h->device_ok = false;
  drop_graph(h);
  return ok();
}

int add_body_impl(btdf_t *h, int n, const double *xy, const double *uv, double cx, double cy, double ds,
                  int *body_id) {
  if (n < 3) return fail(BTDF_EINVAL, "a body needs at least 3 markers (got %d)", n);
  if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(ds)) return fail(BTDF_EINVAL, "non-finite body parameter");
  for (int l = 0; l < n; ++l) {
    const double X = xy[2 * l], Y = xy[2 * l + 1];
    if (!std::isfinite(X) || !std::isfinite(Y)) return fail(BTDF_EINVAL, "non-finite marker %d", l);
    if (uv && (!std::isfinite(uv[2 * l]) || !std::isfinite(uv[2 * l + 1])))
      return fail(BTDF_EINVAL, "non-finite marker velocity %d", l);
    if (std::fabs(X) > 1e8 || std::fabs(Y) > 1e8) return fail(BTDF_EINVAL, "marker %d too far from the grid", l);
    int lo, hi;
    marker_range(h->kind, X, &lo, &hi);
    if (!h->xper() && (lo < h->i0() || hi > h->i1()))
      return fail(BTDF_EINVAL, "marker %d: stencil x range [%d, %d] leaves the fluid columns [%d, %d]", l, lo,
                  hi, h->i0(), h->i1());
    marker_range(h->kind, Y, &lo, &hi);
    if (!h->yper() && (lo < 0 || hi > h->ny - 1))
      return fail(BTDF_EINVAL, "marker %d: stencil y range [%d, %d] leaves the grid", l, lo, hi);
  }
  if (!(ds > 0.0)) {
    double per = 0.0;
    for (int l = 0; l < n; ++l) {
      int m = (l + 1) % n;
      per += std::hypot(xy[2 * m] - xy[2 * l], xy[2 * m + 1] - xy[2 * l + 1]);
    }
    ds = per / n;
    if (!(ds > 0.0)) return fail(BTDF_EINVAL, "degenerate body (zero perimeter)");
  }
  if ((long long)h->nm() + n > (1LL << 30)) return fail(BTDF_EINVAL, "too many markers");
  try {
    const double s = h->drs * ds;
    double rad = 0.0;
    for (int l = 0; l < n; ++l) {
      h->X.push_back(xy[2 * l]);
      h->Y.push_back(xy[2 * l + 1]);
      h->U.push_back(uv ? uv[2 * l] : 0.0);
      h->V.push_back(uv ? uv[2 * l + 1] : 0.0);
      h->sdrs.push_back(s);
      h->rx.push_back(xy[2 * l] - cx);
      h->ry.push_back(xy[2 * l + 1] - cy);
      rad = std::max(rad, std::hypot(xy[2 * l] - cx, xy[2 * l + 1] - cy));
    }
    h->bmoving.push_back(0);
    h->theta.push_back(0.0);
    h->bvx.push_back(0.0);
    h->bvy.push_back(0.0);
    h->bom.push_back(0.0);
    h->brad.push_back(rad);
    h->off.push_back(h->nm());
    h->cx.push_back(cx);
    h->cy.push_back(cy);
    h->bsdrs.push_back(s);
    h->bds.push_back(ds);
  } catch (...) {
    return fail(BTDF_ENOMEM, "out of host memory");
  }
  h->stepped = false;
  h->layout_ok = false;
  h->device_ok = false;
  h->bodies_dirty = true;
  h->hist_read = h->steps;
  h->forces_from = h->steps;
  drop_graph(h);
  if (body_id) *body_id = h->nb() - 1;
  return ok();
}

int destroy_impl(btdf_t *h) {
  int rc = ok();
  if (h->ws) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) rc = fail(BTDF_EDEVICE, "stream sync failed");
  }
  drop_graph(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  h->tev.release();
  if (h->ws && h->ws_owned) (void)hipFree(h->ws);
  delete h;
  return rc;
}

}  // namespace host
}  // namespace btdf

using namespace btdf::host;

extern "C" {

const char *btdf_last_error(void) { return g_err; }

int btdf_create(const btdf_grid *g, double tau, int delta_kind, double thickening, btdf_t **out) {
  return guard([&]() -> int {
    if (!g || !out) return fail(BTDF_EINVAL, "NULL argument");
    *out = nullptr;
    if (g->nx < 8 || g->ny < 8) return fail(BTDF_EINVAL, "nx and ny must be >= 8 (got %d, %d)", g->nx, g->ny);
    if ((long long)g->nx * g->ny > (1LL << 31) - 1) return fail(BTDF_EINVAL, "grid too large");
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(BTDF_EINVAL, "tau must be > 1/2 (got %g)", tau);
    if (!valid_kind(delta_kind)) return fail(BTDF_EINVAL, "unknown delta kind %d", delta_kind);
    if (!(thickening > 0.0) || !std::isfinite(thickening))
      return fail(BTDF_EINVAL, "thickening must be > 0 (got %g)", thickening);
    const bool xp = g->bc_west == BTDF_PERIODIC && g->bc_east == BTDF_PERIODIC;
    const bool xc = g->bc_west == BTDF_VELOCITY_INLET &&
                    (g->bc_east == BTDF_ZERO_GRADIENT_OUTLET || g->bc_east == BTDF_CONVECTIVE_OUTLET);
    const bool yp = g->bc_south == BTDF_PERIODIC && g->bc_north == BTDF_PERIODIC;
    const bool yw = g->bc_south == g->bc_north &&
                    (g->bc_south == BTDF_BOUNCEBACK_WALL || g->bc_south == BTDF_FREE_SLIP_WALL);
    if (!(xp || xc)) return fail(BTDF_EINVAL, "x ends must be a periodic pair or inlet (west) + outlet (east)");
    if (!(yp || yw)) return fail(BTDF_EINVAL, "y ends must be a periodic pair or a pair of walls of one kind");
    if (g->bc_east == BTDF_CONVECTIVE_OUTLET && !(g->inflow_ux >= 0.0))
      return fail(BTDF_EINVAL, "a convective outlet needs an inflow speed >= 0 (got %g)", g->inflow_ux);
    if (g->precision != 4 && g->precision != 8) return fail(BTDF_EINVAL, "precision must be 4 or 8");
    if (g->history_capacity < 0) return fail(BTDF_EINVAL, "history_capacity must be >= 0");
    if (g->flags != 0) return fail(BTDF_EINVAL, "flags must be 0");
    const double vals[] = {g->inflow_ux, g->inflow_uy, g->body_force_x, g->body_force_y, g->rho0, g->ux0, g->uy0};
    for (double v : vals)
      if (!std::isfinite(v)) return fail(BTDF_EINVAL, "non-finite grid parameter");
    if (!(g->rho0 > 0.0)) return fail(BTDF_EINVAL, "rho0 must be > 0");

    btdf_t *h = new (std::nothrow) btdf_sim();
    if (!h) return fail(BTDF_ENOMEM, "out of host memory");
    h->nx = g->nx;
    h->ny = g->ny;
    h->bc[0] = g->bc_west;
    h->bc[1] = g->bc_east;
    h->bc[2] = g->bc_south;
    h->bc[3] = g->bc_north;
    h->prec = g->precision;
    h->hist_cap = g->history_capacity ? g->history_capacity : 4096;
    h->kind = delta_kind;
    h->tau = tau;
    h->drs = thickening;
    h->G[0] = g->body_force_x;
    h->G[1] = g->body_force_y;
    h->uin[0] = g->inflow_ux;
    h->uin[1] = g->inflow_uy;
    h->rho0 = g->rho0;
    h->u0[0] = g->ux0;
    h->u0[1] = g->uy0;
    h->stream = (hipStream_t)g->hip_stream;
    *out = h;
    return ok();
  });
}

int btdf_destroy(btdf_t *h) {
  return guard([&]() -> int {
    if (!h) return ok();
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; destroy the batch");
    return destroy_impl(h);
  });
}

size_t btdf_workspace_bytes(const btdf_t *h) {
  return guard_size([&]() -> size_t {
    if (!h) return 0;
    if (!h->layout_ok) compute_layout(const_cast<btdf_t *>(h));
    return h->total;
  });
}

int btdf_bind_workspace(btdf_t *h, void *dev, size_t bytes) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; bind the batch's workspace");
    return bind_impl(h, dev, bytes);
  });
}

int btdf_set_stream(btdf_t *h, void *hip_stream) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; set the batch's stream");
    if (h->ws && (hipStream_t)hip_stream != h->stream) {
      // order the new stream after the work already on the old one
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->stream = (hipStream_t)hip_stream;
    return ok();
  });
}

int btdf_add_body(btdf_t *h, int n, const double *xy, const double *uv, double cx, double cy, double ds,
                  int *body_id) {
  return guard([&]() -> int {
    if (!h || !xy) return fail(BTDF_EINVAL, "NULL argument");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; use btdf_batch_add_body");
    return add_body_impl(h, n, xy, uv, cx, cy, ds, body_id);
  });
}

int btdf_set_body_motion(btdf_t *h, int body, double vx, double vy, double omega) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch");
    if (body < 0 || body >= h->nb()) return fail(BTDF_EINVAL, "no body %d", body);
    if (!std::isfinite(vx) || !std::isfinite(vy) || !std::isfinite(omega)) return fail(BTDF_EINVAL, "non-finite motion");
    if (h->method != BTDF_FORCING_DIRECT || h->nf != 1)
      return fail(BTDF_ESTATE, "moving bodies need the direct forcing method with one pass");
    const double v = std::hypot(vx, vy) + std::fabs(omega) * h->brad[body];
    if (!(v < kMoveMargin)) return fail(BTDF_EINVAL, "markers would travel %g nodes per step (at most %d)", v, kMoveMargin);
    const bool first = !h->any_moving();
    mirror_positions(h);  // where a body already moving is now
    h->bmoving[body] = 1;
    h->bvx[body] = vx;
    h->bvy[body] = vy;
    h->bom[body] = omega;
    mirror_positions(h);  // and the rigid velocity field at those positions
    if (first) h->layout_ok = false;  // tile lists gain their margin
    h->device_ok = false;
    h->steps_to_rebin = 0;
    drop_graph(h);
    return ok();
  });
}

int btdf_get_body_state(const btdf_t *h, int body, double *state) {
  return guard([&]() -> int {
    if (!h || !state) return fail(BTDF_EINVAL, "NULL argument");
    if (body < 0 || body >= h->nb()) return fail(BTDF_EINVAL, "no body %d", body);
    state[0] = h->cx[body];
    state[1] = h->cy[body];
    state[2] = h->theta[body];
    state[3] = h->bvx[body];
    state[4] = h->bvy[body];
    state[5] = h->bom[body];
    return ok();
  });
}

int btdf_get_marker_positions(btdf_t *h, double *xy) {
  return guard([&]() -> int {
    if (!h || !xy) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    const size_t nm = (size_t)h->nm(), d = sizeof(double);
    if (nm == 0) return ok();
    std::vector<double> x(nm), y(nm);
    HIPCHK(hipMemcpy(x.data(), h->ws + h->off_mk, nm * d, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(y.data(), h->ws + h->off_mk + (size_t)std::max(h->nm(), 1) * d, nm * d, hipMemcpyDeviceToHost));
    for (size_t l = 0; l < nm; ++l) {
      xy[2 * l] = x[l];
      xy[2 * l + 1] = y[l];
    }
    return ok();
  });
}

int btdf_set_marker_velocity(btdf_t *h, int body, const double *uv) {
  return guard([&]() -> int {
    if (!h || !uv) return fail(BTDF_EINVAL, "NULL argument");
    if (body < 0 || body >= h->nb()) return fail(BTDF_EINVAL, "no body %d", body);
    if (h->bmoving[body]) return fail(BTDF_ESTATE, "body %d moves rigidly; its marker velocities follow the motion", body);
    const int l0 = h->off[body], l1 = h->off[body + 1];
    for (int l = l0; l < l1; ++l)
      if (!std::isfinite(uv[2 * (l - l0)]) || !std::isfinite(uv[2 * (l - l0) + 1]))
        return fail(BTDF_EINVAL, "non-finite velocity");
    for (int l = l0; l < l1; ++l) {
      h->U[l] = uv[2 * (l - l0)];
      h->V[l] = uv[2 * (l - l0) + 1];
    }
    if (h->ws && h->device_ok) {
      const size_t M = (size_t)std::max(h->nm(), 1), d = sizeof(double);
      int rc;
      if ((rc = upload(h, h->off_mk + 2 * M * d + l0 * d, h->U.data() + l0, (l1 - l0) * d))) return rc;
      if ((rc = upload(h, h->off_mk + 3 * M * d + l0 * d, h->V.data() + l0, (l1 - l0) * d))) return rc;
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    return ok();
  });
}

static int enqueue_pass(btdf_t *h, const LbmParams &p, const IbParams &ib, hipStream_t s, hipEvent_t *ev);
static int run_blocked(btdf_t *h, const LbmParams &p, const IbParams &ib, int64_t n);
static bool blocking_active(const btdf_t *h);
static bool remainder_pair(const btdf_t *h);
static bool remainder_triple(const btdf_t *h);

// n steps from the current buffer: graphs of graph_chunk steps where they fit
static int run_steps(btdf_t *h, const LbmParams &p, const IbParams &ib, int64_t n) {
  int rc;
  int64_t left = n;
  if (h->graph_chunk > 0 && left >= h->graph_chunk + (h->cur ? 1 : 0)) {
    if (h->cur) {  // graphs start from buffer 0
      if ((rc = enqueue_step(h, p, ib, h->cur, h->stream, nullptr))) return rc;
      h->cur ^= 1;
      h->steps++;
      left--;
    }
    if ((!h->graph || h->graph_depth != 1) && (rc = build_graph(h, p, ib))) return rc;
    while (left >= h->graph_chunk) {
      HIPCHK(hipGraphLaunch(h->graph, h->stream));
      left -= h->graph_chunk;
      h->steps += h->graph_chunk;
      // an even chunk returns the state to buffer 0
      h->cur = (h->graph_chunk & 1) ? 1 : 0;
      if (h->cur) break;
    }
  }
  for (; left > 0; --left) {
    if ((rc = enqueue_step(h, p, ib, h->cur, h->stream, nullptr))) return rc;
    h->cur ^= 1;
    h->steps++;
  }
  return ok();
}

// Moving bodies: place the host markers at the mirrored motion, check that
// no stencil can leave the fluid region before the next rebuild, rebuild the
// tile lists with the margin and send them. Synchronises the stream first,
// so the host lists are not changed under a copy in flight.
static int rebin(btdf_t *h) {
  HIPCHK(hipStreamSynchronize(h->stream));
  mirror_positions(h);
  const int m = h->margin;
  for (int b = 0; b < h->nb(); ++b) {
    if (!h->bmoving[b]) continue;
    for (int l = h->off[b]; l < h->off[b + 1]; ++l) {
      int lo, hi;
      marker_range(h->kind, h->X[l], &lo, &hi);
      if (!h->xper() && (lo - m < h->i0() || hi + m > h->i1()))
        return fail(BTDF_EINVAL, "moving body %d would leave the fluid columns (step %lld)", b, (long long)h->steps);
      marker_range(h->kind, h->Y[l], &lo, &hi);
      if (!h->yper() && (lo - m < 0 || hi + m > h->ny - 1))
        return fail(BTDF_EINVAL, "moving body %d would leave the grid (step %lld)", b, (long long)h->steps);
    }
  }
  bin_markers(h, h->tile_x, h->tile_y, h->ntx, h->nty, h->tile_off, h->tile_list);
  if (h->tile_list.size() > (size_t)tiles_per_marker(h) * h->nm() + 1)
    return fail(BTDF_EDEVICE, "tile lists overflow their region");
  const int ntiles = h->ntx * h->nty;
  h->tile_map.clear();
  for (int t = 0; t < ntiles; ++t)
    if (h->tile_off[t + 1] == h->tile_off[t]) h->tile_map.push_back(t);
  const int n_free = (int)h->tile_map.size();
  for (int t = 0; t < ntiles; ++t)
    if (h->tile_off[t + 1] != h->tile_off[t]) h->tile_map.push_back(t);
  h->n_free = n_free;
  h->n_forced = ntiles - n_free;
  int rc;
  if ((rc = upload(h, h->off_toff, h->tile_off.data(), h->tile_off.size() * sizeof(int)))) return rc;
  if ((rc = upload(h, h->off_tlist, h->tile_list.data(), h->tile_list.size() * sizeof(int)))) return rc;
  if ((rc = upload(h, h->off_tmap, h->tile_map.data(), h->tile_map.size() * sizeof(int)))) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  const double v = max_marker_speed(h);
  h->steps_to_rebin = v > 0.0 ? (int64_t)std::floor(kMoveMargin / v) : ((int64_t)1 << 60);
  if (h->steps_to_rebin < 1)
    return fail(BTDF_EINVAL, "a moving body's markers travel %g nodes per step; less than %d are allowed", v,
                kMoveMargin);
  return ok();
}

int btdf_step(btdf_t *h, int64_t n) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; step the batch");
    if (n < 0) return fail(BTDF_EINVAL, "negative step count");
    if (n == 0) return ok();
    int rc = ensure_device(h);
    if (rc) return rc;
    const LbmParams p = make_params(h);
    const IbParams ib = make_ib(h);
    if (blocking_active(h) && n >= h->depth) {
      if ((rc = run_blocked(h, p, ib, n))) return rc;
    } else if (!h->any_moving()) {
      if ((rc = run_steps(h, p, ib, n))) return rc;
    } else {
      for (int64_t left = n; left > 0;) {
        if (h->steps_to_rebin <= 0 && (rc = rebin(h))) return rc;
        const int64_t k = std::min(left, h->steps_to_rebin);
        if ((rc = run_steps(h, p, ib, k))) return rc;
        mirror_advance(h, k);
        h->steps_to_rebin -= k;
        left -= k;
      }
    }
    h->stepped = true;
    return ok();
  });
}

// two steps from buffer cur into 1 - cur (temporal blocking): the tiles near
// the bodies or the domain edges step twice by way of the third buffer X,
// with the marker kernel between; every other tile takes both steps at once
// (lbm2_kernel). The nodes just outside the near tiles (the ring) must hold
// their first step in X before the near tiles' second step: the two-step pass
// writes them, so it runs first. ev: 7 events (before/after the first marker
// kernel, after the near tiles' first step, after the second marker kernel,
// after their second step, before/after the two-step pass) or null.
static hipError_t launch_two_step(const btdf_t *h, const void *A, void *B, void *X, const unsigned char *near,
                                  const LbmParams &p, const int *fm, hipStream_t s) {
  // every level is a row of 1, 2 or 4 tiles (see remainder_pair)
  hipError_t e = hipSuccess;
  for (int g = 0; g < kLevels && e == hipSuccess; ++g) {
    const int ne = h->n_edge[g], ni = h->n_grp[g] - ne, *lv = fm + h->grp_start(g);
    if (ne) e = launch_lbm_edge2(h->prec, h->variant, kEdge | h->gkind[g], A, B, p, lv, ne, X, near, s);
    if (ni && e == hipSuccess) e = launch_lbm2(h->prec, h->variant, h->gkind[g] & 15, A, B, p, lv + ne, ni, X, near, s);
  }
  return e;
}

static int enqueue_pair(btdf_t *h, const LbmParams &p, const IbParams &ib, hipStream_t s, hipEvent_t *ev) {
  const void *A = h->ws + h->off_pop[h->cur];
  void *B = h->ws + h->off_pop[1 - h->cur];
  void *X = h->ws + h->off_pop3;
  const int *fm = h->at<int>(h->off_fmap);
  const unsigned char *near = h->at<unsigned char>(h->off_near);
  if (ev && ev[0]) HIPCHK(hipEventRecord(ev[0], s));
  HIPCHK(launch_ib(h->prec, A, p, ib, s));
  if (ev && ev[1]) HIPCHK(hipEventRecord(ev[1], s));
  if (ev && ev[5]) HIPCHK(hipEventRecord(ev[5], s));
  HIPCHK(launch_two_step(h, A, B, X, near, p, fm, s));
  if (ev && ev[6]) HIPCHK(hipEventRecord(ev[6], s));
  const int nb0 = h->n_groups();  // the near tiles start here in the map
  HIPCHK(launch_lbm(h->prec, h->variant, A, X, p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, A, X, p, s));
  if (ev && ev[2]) HIPCHK(hipEventRecord(ev[2], s));
  HIPCHK(launch_ib(h->prec, X, p, ib, s));
  if (ev && ev[3]) HIPCHK(hipEventRecord(ev[3], s));
  HIPCHK(launch_lbm(h->prec, h->variant, X, B, p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, X, B, p, s));
  if (ev && ev[4]) HIPCHK(hipEventRecord(ev[4], s));
  h->cur ^= 1;
  h->steps += 2;
  return ok();
}

// Fork a second stream from s for the blocked pass's smaller launches (the
// caller records join_ev on it after them and makes s wait for that).
static int fork_side(btdf_t *h, hipStream_t s) {
  if (!h->side) HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  if (!h->fork_ev) HIPCHK(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
  if (!h->join_ev) HIPCHK(hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(h->fork_ev, s));
  HIPCHK(hipStreamWaitEvent(h->side, h->fork_ev, 0));
  return ok();
}

// three steps from buffer cur into 1 - cur (three-step blocking): as a pair,
// with the near tiles' states n+1 and n+2 in X1 and X2 and the marker kernel
// before each of their steps. The three-step pass writes both rings, so it
// runs before the near tiles' second step; it runs after their first step,
// whose reads of A bring in the lines the pass's single tiles and pairs
// (which border near tiles) read for their halos, and these go first.
// ev: 9 events or null: marker kernel E0-E1, near step E1-E2, pass E5-E6,
// marker kernel E6-E3, near step E3-E4, marker kernel E4-E7, near step E7-E8.
static int enqueue_triple(btdf_t *h, const LbmParams &p, const IbParams &ib, hipStream_t s, hipEvent_t *ev) {
  const void *A = h->ws + h->off_pop[h->cur];
  void *B = h->ws + h->off_pop[1 - h->cur];
  void *X1 = h->ws + h->off_pop3;
  void *X2 = h->ws + h->off_pop4;
  const int *fm = h->at<int>(h->off_fmap);
  const unsigned char *near = h->at<unsigned char>(h->off_near);
  const int nb0 = h->n_groups();  // the near tiles start here in the map
  if (ev && ev[0]) HIPCHK(hipEventRecord(ev[0], s));
  HIPCHK(launch_ib(h->prec, A, p, ib, s));
  if (ev && ev[1]) HIPCHK(hipEventRecord(ev[1], s));
  HIPCHK(launch_lbm(h->prec, h->variant, A, X1, p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, A, X1, p, s));
  if (ev && ev[2]) HIPCHK(hipEventRecord(ev[2], s));
  // the pass: the smallest groups (which border near tiles) first, the
  // largest last; every launch but the largest interior groups' on a second
  // stream beside it (see enqueue_deep)
  if (ev && ev[5]) HIPCHK(hipEventRecord(ev[5], s));
  bool small = h->n_edge[0] > 0;
  for (int g = 1; g < kLevels; ++g) small = small || h->n_grp[g] > 0;
  const int n0 = h->n_grp[0] - h->n_edge[0];
  hipStream_t ss = s;
  if (small && n0 > 0) {
    const int rc = fork_side(h, s);
    if (rc) return rc;
    ss = h->side;
  }
  for (int g = kLevels - 1; g >= 0; --g) {
    const int ne = h->n_edge[g], ni = h->n_grp[g] - ne, *lv = fm + h->grp_start(g);
    if (ne) HIPCHK(launch_lbm_edge3(h->prec, h->variant, kEdge | h->gkind[g], A, B, p, lv, ne, X1, X2, near, ss));
    if (ni && g > 0) HIPCHK(launch_lbm3(h->prec, h->variant, h->gkind[g], A, B, p, lv + ne, ni, X1, X2, near, ss));
  }
  if (ss != s) HIPCHK(hipEventRecord(h->join_ev, ss));
  if (n0 > 0)
    HIPCHK(launch_lbm3(h->prec, h->variant, h->gkind[0], A, B, p, fm + h->n_edge[0], n0, X1, X2, near, s));
  if (ss != s) HIPCHK(hipStreamWaitEvent(s, h->join_ev, 0));
  if (ev && ev[6]) HIPCHK(hipEventRecord(ev[6], s));
  HIPCHK(launch_ib(h->prec, X1, p, ib, s));
  if (ev && ev[3]) HIPCHK(hipEventRecord(ev[3], s));
  HIPCHK(launch_lbm(h->prec, h->variant, X1, X2, p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, X1, X2, p, s));
  if (ev && ev[4]) HIPCHK(hipEventRecord(ev[4], s));
  HIPCHK(launch_ib(h->prec, X2, p, ib, s));
  if (ev && ev[7]) HIPCHK(hipEventRecord(ev[7], s));
  HIPCHK(launch_lbm(h->prec, h->variant, X2, B, p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, X2, B, p, s));
  if (ev && ev[8]) HIPCHK(hipEventRecord(ev[8], s));
  h->cur ^= 1;
  h->steps += 3;
  return ok();
}

// d = 4 or 5 steps from buffer cur into 1 - cur: as a triple, with the near
// tiles' states n+1 .. n+d-1 in X1 .. X(d-1) and the marker kernel before
// each of their steps. ev: 2d + 2 events or null: marker kernel E0-E1, near
// step E1-E2, pass E2-E3, then for each later step s = 1 .. d-1 the marker
// kernel E(2s+1)-E(2s+2) and the near step E(2s+2)-E(2s+3).
static int enqueue_deep(btdf_t *h, const LbmParams &p, const IbParams &ib, hipStream_t s, hipEvent_t *ev) {
  const int d = h->depth;
  const void *A = h->ws + h->off_pop[h->cur];
  void *B = h->ws + h->off_pop[1 - h->cur];
  // (X1 .. X4 are consecutive population buffers, which the pass addresses from X1)
  void *X[5] = {nullptr, h->ws + h->off_pop3, h->ws + h->off_pop4, h->ws + h->off_pop5, h->ws + h->off_pop6};
  const int *fm = h->at<int>(h->off_fmap);
  const unsigned *rwin = h->at<unsigned>(h->off_rwin);
  const int nb0 = h->n_groups();  // the near tiles start here in the map
  auto mark = [&](int k) -> hipError_t { return ev && ev[k] ? hipEventRecord(ev[k], s) : hipSuccess; };
  HIPCHK(mark(0));
  HIPCHK(launch_ib(h->prec, A, p, ib, s));
  HIPCHK(mark(1));
  HIPCHK(launch_lbm(h->prec, h->variant, A, X[1], p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
  if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, A, X[1], p, s));
  HIPCHK(mark(2));
  // the pass: the smaller groups' launches on a second stream, beside the
  // largest groups' launch (they are one to three waves of workgroups long,
  // and alone their tails would leave the GPU partly idle)
  bool small = false;
  for (int g = 1; g < kLevels; ++g) small = small || h->n_grp[g] > 0;
  if (small && h->n_grp[0]) {
    int rc;
    if ((rc = fork_side(h, s))) return rc;
    for (int g = kLevels - 1; g >= 1; --g)
      if (h->n_grp[g])
        HIPCHK(launch_lbm_deep(h->prec, h->variant, d, h->gkind[g], A, B, p, fm + h->grp_start(g), h->n_grp[g],
                               h->n_ring[g], X[1], rwin + h->grp_start(g), h->side));
    HIPCHK(hipEventRecord(h->join_ev, h->side));
    HIPCHK(launch_lbm_deep(h->prec, h->variant, d, h->gkind[0], A, B, p, fm, h->n_grp[0], h->n_ring[0], X[1], rwin,
                           s));
    HIPCHK(hipStreamWaitEvent(s, h->join_ev, 0));
  } else {
    for (int g = kLevels - 1; g >= 0; --g)
      if (h->n_grp[g])
        HIPCHK(launch_lbm_deep(h->prec, h->variant, d, h->gkind[g], A, B, p, fm + h->grp_start(g), h->n_grp[g],
                               h->n_ring[g], X[1], rwin + h->grp_start(g), s));
  }
  HIPCHK(mark(3));
  for (int k = 1; k < d; ++k) {
    void *dst = k + 1 < d ? X[k + 1] : B;
    HIPCHK(launch_ib(h->prec, X[k], p, ib, s));
    HIPCHK(mark(2 * k + 2));
    HIPCHK(launch_lbm(h->prec, h->variant, X[k], dst, p, TileRange{fm, nb0, h->n_near, 1}, ib, s));
    if (p.outlet == 2) HIPCHK(launch_conv_outlet(h->prec, X[k], dst, p, s));
    HIPCHK(mark(2 * k + 3));
  }
  h->cur ^= 1;
  h->steps += d;
  return ok();
}

static int enqueue_pass(btdf_t *h, const LbmParams &p, const IbParams &ib, hipStream_t s, hipEvent_t *ev) {
  if (h->depth >= 4) return enqueue_deep(h, p, ib, s, ev);
  return h->depth == 3 ? enqueue_triple(h, p, ib, s, ev) : enqueue_pair(h, p, ib, s, ev);
}

// a graph of graph_chunk / depth whole passes, starting from buffer 0
static int build_pass_graph(btdf_t *h, const LbmParams &p, const IbParams &ib, int passes) {
  drop_graph(h);
  if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  const int cur = h->cur;
  const int64_t steps = h->steps;
  h->cur = 0;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  for (int k = 0; k < passes && rc == 0; ++k) rc = enqueue_pass(h, p, ib, h->cap_stream, nullptr);
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  h->cur = cur;  // capturing ran nothing
  h->steps = steps;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(BTDF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph = nullptr;
    return fail(BTDF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  h->graph_depth = h->depth;
  return ok();
}

// n steps with temporal blocking: whole passes (replayed from graphs of
// graph_chunk / depth passes when a graph chunk is set), then single steps
static int run_blocked(btdf_t *h, const LbmParams &p, const IbParams &ib, int64_t n) {
  const int d = h->depth;
  const int per = h->graph_chunk / d;  // passes per graph
  int64_t left = n;
  int rc;
  if (per > 0 && left >= (int64_t)per * d + (h->cur ? 1 : 0)) {
    if (h->cur) {  // graphs start from buffer 0
      if ((rc = enqueue_step(h, p, ib, h->cur, h->stream, nullptr))) return rc;
      h->cur ^= 1;
      h->steps++;
      left--;
    }
    if ((!h->graph || h->graph_depth != d) && (rc = build_pass_graph(h, p, ib, per))) return rc;
    while (left >= (int64_t)per * d) {
      HIPCHK(hipGraphLaunch(h->graph, h->stream));
      left -= (int64_t)per * d;
      h->steps += (int64_t)per * d;
      h->cur = per & 1;  // each pass swaps the buffers once
      if (h->cur) break;
    }
  }
  for (; left >= d; left -= d)
    if ((rc = enqueue_pass(h, p, ib, h->stream, nullptr))) return rc;
  if (left >= 3 && remainder_triple(h)) {
    if ((rc = enqueue_triple(h, p, ib, h->stream, nullptr))) return rc;
    left -= 3;
  }
  if (left == 2 && remainder_pair(h)) {
    if ((rc = enqueue_pair(h, p, ib, h->stream, nullptr))) return rc;
    left = 0;
  }
  for (; left > 0; --left) {
    if ((rc = enqueue_step(h, p, ib, h->cur, h->stream, nullptr))) return rc;
    h->cur ^= 1;
    h->steps++;
  }
  return ok();
}

static bool blocking_active(const btdf_t *h) {
  return h->depth >= 2 && h->layout_ok && h->n_groups() > 0 && !h->any_moving();
}

// Whether two steps left over after three-step passes can take one two-step
// pass over the same tiles: a tile clear of the margins of three steps is
// clear of those of two, so the near set and the row groups of the
// three-step pass serve the two-step pass as they are (its groups along
// rows; not the groups two tiles tall).
static bool remainder_pair(const btdf_t *h) {
  if (h->depth < 3 || !variant_has_lbm2(h->variant, h->prec)) return false;
  for (int g = 0; g < kLevels; ++g) {
    if (!h->n_grp[g]) continue;
    const int code = h->gkind[g], w = code & 15;
    if (h->n_edge[g] && !variant_has_edge(h->variant, h->prec, 2, kEdge | code)) return false;
    if (h->n_grp[g] == h->n_edge[g]) continue;
    if (((code >> 4) & 15) != 1) return false;  // taller than one tile
    if (w > 1 && !variant_has_wide_lbm2(h->variant, h->prec, w)) return false;
  }
  return true;
}

// Whether three steps left over after deeper passes can take one three-step
// pass over the same tiles (the near set of a deeper pass covers that of
// three steps, and its groups are rows of tiles the three-step pass has).
static bool remainder_triple(const btdf_t *h) {
  if (h->depth < 4) return false;
  for (int g = 0; g < kLevels; ++g)
    if (h->n_grp[g] && (h->n_edge[g] || !variant_has_lbm3(h->variant, h->prec, h->gkind[g]))) return false;
  return true;
}

// n steps with HIP events around the launches: every launch of a step or a
// pass, or with pass_only just the blocked pass's launches (out[2] only;
// single steps and a two-step remainder carry no events), which keeps the
// events' own cost out of the steps being timed. out[0], out[1]: ms per step
// of the marker kernels and of the single-step lattice launches (means over
// the n steps); out[2]: the blocked pass's mean launch duration per step it
// covers; out[3]: the blocked pass's time per step of all n.
static int timed_impl(btdf_t *h, int64_t n, double *out, bool pass_only = false) {
  if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; step the batch");
  if (n <= 0) return fail(BTDF_EINVAL, "step count must be > 0");
  int rc = ensure_device(h);
  if (rc) return rc;
  const LbmParams p = make_params(h);
  const IbParams ib = make_ib(h);
  const int chunk = 256, NE = 12;  // events per entry
  HIPCHK(h->tev.reserve((size_t)NE * chunk));
  std::vector<hipEvent_t> ev(h->tev.ev.begin(), h->tev.ev.begin() + (size_t)NE * chunk);
  const int d = h->depth;
  // the pass's two events in an entry of d steps (deeper passes number
  // their events in launch order)
  const int pa = d >= 4 ? 2 : 5, pb = d >= 4 ? 3 : 6;
  if (pass_only)  // only the pass's two events of each entry are recorded
    for (size_t i = 0; i < ev.size(); ++i)
      if ((int)(i % NE) != pa && (int)(i % NE) != pb) ev[i] = nullptr;
  double tib = 0.0, tlbm = 0.0, tpair = 0.0;
  int64_t done = 0, pass_steps = 0;
  rc = ok();
  while (done < n && rc == 0) {
    // entries of this round: passes of d steps while d are left; three
    // left after deeper passes take one three-step pass, two left one
    // two-step pass (untimed with pass_only, so the pass's mean is that of
    // the d-step launches)
    const bool blk = blocking_active(h);
    const bool pairs = blk && n - done >= d;
    const bool rem3 = blk && !pairs && n - done >= 3 && remainder_triple(h);
    const bool rem2 = blk && !pairs && !rem3 && d >= 3 && n - done == 2 && remainder_pair(h);
    const int dk = pairs ? d : (rem3 ? 3 : (rem2 ? 2 : 1));  // steps per entry
    const int m = dk > 1 ? (int)std::min<int64_t>(chunk, (n - done) / dk) : (int)std::min<int64_t>(chunk, n - done);
    const bool moving = h->any_moving();
    for (int k = 0; k < m && rc == 0; ++k) {
      if (rem3) {
        rc = enqueue_triple(h, p, ib, h->stream, pass_only ? nullptr : &ev[NE * k]);
        continue;
      }
      if (rem2) {
        rc = enqueue_pair(h, p, ib, h->stream, pass_only ? nullptr : &ev[NE * k]);
        continue;
      }
      if (pairs) {
        rc = enqueue_pass(h, p, ib, h->stream, &ev[NE * k]);
        continue;
      }
      if (moving && h->steps_to_rebin <= 0 && (rc = rebin(h))) break;
      const StepEvents te{ev[NE * k], ev[NE * k + 1], ev[NE * k + 2], ev[NE * k + 3], ev[NE * k + 4], ev[NE * k + 5]};
      rc = enqueue_step(h, p, ib, h->cur, h->stream, pass_only ? nullptr : &te);
      h->cur ^= 1;
      h->steps++;
      if (moving) {
        mirror_advance(h, 1);
        h->steps_to_rebin--;
      }
    }
    if (rc) break;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      rc = fail(BTDF_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
      break;
    }
    for (int k = 0; k < m; ++k) {
      float a = 0.f, b = 0.f, c = 0.f, e4 = 0.f, f = 0.f, g = 0.f, gg = 0.f;
      hipEvent_t *E = &ev[NE * k];
      if (pass_only) {
        if (pairs) {
          (void)hipEventElapsedTime(&f, E[pa], E[pb]);
          tpair += f;
          pass_steps += dk;
        }
        continue;
      }
      if (dk >= 4) {  // a deeper pass: marker kernel and near step of each step, and the pass
        (void)hipEventElapsedTime(&a, E[0], E[1]);
        (void)hipEventElapsedTime(&b, E[1], E[2]);
        (void)hipEventElapsedTime(&f, E[2], E[3]);
        tib += a;
        tlbm += b;
        tpair += f;
        for (int s2 = 1; s2 < dk; ++s2) {
          (void)hipEventElapsedTime(&a, E[2 * s2 + 1], E[2 * s2 + 2]);
          (void)hipEventElapsedTime(&b, E[2 * s2 + 2], E[2 * s2 + 3]);
          tib += a;
          tlbm += b;
        }
        pass_steps += dk;
        continue;
      }
      if (dk > 1) {
        (void)hipEventElapsedTime(&a, E[0], E[1]);
        // the near tiles' first step: after the first marker kernel in a
        // triple, after the pass in a pair
        (void)hipEventElapsedTime(&b, dk == 3 ? E[1] : E[6], E[2]);
        // the second marker kernel: after the pass in a triple
        (void)hipEventElapsedTime(&c, dk == 3 ? E[6] : E[2], E[3]);
        (void)hipEventElapsedTime(&e4, E[3], E[4]);
        (void)hipEventElapsedTime(&f, E[5], E[6]);
        if (dk == 3) {
          (void)hipEventElapsedTime(&g, E[4], E[7]);
          (void)hipEventElapsedTime(&gg, E[7], E[8]);
        }
        tib += a + c + g;
        tlbm += b + e4 + gg;
        tpair += f;
        pass_steps += dk;
        continue;
      }
      (void)hipEventElapsedTime(&a, E[0], E[1]);
      (void)hipEventElapsedTime(&b, E[1], E[3]);
      tib += a;
      tlbm += b;
    }
    done += (int64_t)dk * m;
  }
  if (rc) return rc;
  h->stepped = true;
  out[0] = h->nb() ? tib / (double)n : 0.0;
  out[1] = tlbm / (double)n;
  out[2] = pass_steps ? tpair / (double)pass_steps : 0.0;
  out[3] = tpair / (double)n;
  return ok();
}

int btdf_step_timed(btdf_t *h, int64_t n, double *ms_ib, double *ms_lbm) {
  return guard([&]() -> int {
    if (!h || !ms_ib || !ms_lbm) return fail(BTDF_EINVAL, "NULL argument");
    double out[4];
    int rc = timed_impl(h, n, out);
    if (rc) return rc;
    *ms_ib = out[0];
    *ms_lbm = out[1] + out[3];
    return ok();
  });
}

int btdf_step_timed_split(btdf_t *h, int64_t n, double *ms) {
  return guard([&]() -> int {
    if (!h || !ms) return fail(BTDF_EINVAL, "NULL argument");
    double out[4];
    int rc = timed_impl(h, n, out);
    if (rc) return rc;
    ms[0] = out[0];
    ms[1] = out[1];
    ms[2] = out[2];
    return ok();
  });
}

int btdf_step_timed_pass(btdf_t *h, int64_t n, double *ms_pass) {
  return guard([&]() -> int {
    if (!h || !ms_pass) return fail(BTDF_EINVAL, "NULL argument");
    double out[4];
    int rc = timed_impl(h, n, out, true);
    if (rc) return rc;
    *ms_pass = out[2];
    return ok();
  });
}

int btdf_autotune(btdf_t *h, int64_t steps_per_trial, int *best_variant) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; tune the batch");
    if (steps_per_trial < 1) return fail(BTDF_EINVAL, "steps_per_trial must be >= 1");
    double best = 1e300;
    int bv = h->variant, bi = h->interior;
    for (int v = 0; v < num_variants(); ++v) {
      for (int in = 0; in < 2; ++in) {
        if (h->variant != v) {
          h->variant = v;
          h->layout_ok = false;  // (a shape that needs a larger workspace moves the state into one)
        }
        h->interior = in;
        drop_graph(h);
        double a = 0.0, l = 0.0;
        int rc = btdf_step_timed(h, steps_per_trial, &a, &l);
        if (rc) return rc;
        if (a + l < best) {
          best = a + l;
          bv = v;
          bi = in;
        }
      }
    }
    if (h->variant != bv) {
      h->variant = bv;
      h->layout_ok = false;
    }
    h->interior = bi;
    drop_graph(h);
    if (best_variant) *best_variant = bv;
    return ok();
  });
}

int btdf_forces(btdf_t *h, double *out, int cap_bodies) {
  return guard([&]() -> int {
    if (!h || (!out && h->nb() > 0)) return fail(BTDF_EINVAL, "NULL argument");
    if (cap_bodies < h->nb()) return fail(BTDF_EINVAL, "cap_bodies %d < %d bodies", cap_bodies, h->nb());
    const int nb = h->nb();
    if (h->steps == 0 || !h->ws) {
      for (int k = 0; k < 3 * nb; ++k) out[k] = 0.0;
      return h->ws ? check_flag(h) : ok();
    }
    int rc = ensure_device(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    if (nb > 0) {
      const long long slot = (h->steps - 1) % h->hist_cap;
      if (h->steps <= h->forces_from) {
        // no step since the body set changed or a state was loaded
        for (int k = 0; k < 3 * nb; ++k) out[k] = 0.0;
      } else {
        HIPCHK(hipMemcpy(out, h->ws + h->off_hist + (size_t)slot * nb * 3 * sizeof(double),
                         (size_t)nb * 3 * sizeof(double), hipMemcpyDeviceToHost));
      }
    }
    return check_flag(h);
  });
}

int btdf_force_history(btdf_t *h, double *out, int64_t max_steps, int64_t *n_written) {
  return guard([&]() -> int {
    if (!h || !n_written || (!out && max_steps > 0)) return fail(BTDF_EINVAL, "NULL argument");
    *n_written = 0;
    const int nb = h->nb();
    if (!h->ws || nb == 0 || max_steps <= 0) {
      h->hist_read = h->steps;
      return h->ws ? check_flag(h) : ok();
    }
    int rc = ensure_device(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    const int64_t pending = h->steps - std::max(h->hist_read, h->forces_from);
    const int64_t avail = std::min<int64_t>(pending, h->hist_cap);
    const int64_t first = h->steps - avail;
    const int64_t cnt = std::min<int64_t>(avail, max_steps);
    const size_t row = (size_t)nb * 3 * sizeof(double);
    int64_t k = 0;
    while (k < cnt) {
      const int64_t slot = (first + k) % h->hist_cap;
      const int64_t run = std::min<int64_t>(cnt - k, h->hist_cap - slot);
      HIPCHK(hipMemcpy((char *)out + (size_t)k * row, h->ws + h->off_hist + (size_t)slot * row,
                       (size_t)run * row, hipMemcpyDeviceToHost));
      k += run;
    }
    h->hist_read = first + cnt;
    *n_written = cnt;
    return check_flag(h);
  });
}

int btdf_init_equilibrium(btdf_t *h, const double *rho, const double *ux, const double *uy) {
  return guard([&]() -> int {
    if (!h || !ux || !uy) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    const size_t n = (size_t)h->nx * h->ny, d = sizeof(double);
    // stage the fields in the spare population buffer (at least 36 bytes per node)
    double *st = h->at<double>(h->off_pop[1 - h->cur]);
    HIPCHK(hipMemcpyAsync(st, ux, n * d, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(st + n, uy, n * d, hipMemcpyHostToDevice, h->stream));
    if (rho) HIPCHK(hipMemcpyAsync(st + 2 * n, rho, n * d, hipMemcpyHostToDevice, h->stream));
    LbmParams p = make_params(h);
    HIPCHK(launch_init_eq(h->prec, h->ws + h->off_pop[h->cur], p, st + 2 * n, st, st + n, h->rho0, rho != nullptr,
                          h->stream));
    h->stepped = false;
    if ((rc = clear_flag(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return ok();
  });
}

int btdf_get_macroscopic(btdf_t *h, double *rho, double *ux, double *uy) {
  return guard([&]() -> int {
    if (!h || !rho || !ux || !uy) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    const size_t n = (size_t)h->nx * h->ny, d = sizeof(double);
    double *st = h->at<double>(h->off_pop[1 - h->cur]);
    LbmParams p = make_params(h);
    HIPCHK(launch_macro(h->prec, h->ws + h->off_pop[h->cur], p, st, st + n, st + 2 * n, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(rho, st, n * d, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ux, st + n, n * d, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(uy, st + 2 * n, n * d, hipMemcpyDeviceToHost));
    return ok();
  });
}

int btdf_get_populations(btdf_t *h, double *dst) {
  return guard([&]() -> int {
    if (!h || !dst) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    const size_t n = (size_t)h->nx * h->ny;
    double *st = h->at<double>(h->off_pop[1 - h->cur]);
    LbmParams p = make_params(h);
    for (int q = 0; q < 9; ++q) {
      HIPCHK(launch_plane_to_f64(h->prec, h->ws + h->off_pop[h->cur], p, q, st, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(hipMemcpy(dst + (size_t)q * n, st, n * sizeof(double), hipMemcpyDeviceToHost));
    }
    return ok();
  });
}

int btdf_set_populations(btdf_t *h, const double *src) {
  return guard([&]() -> int {
    if (!h || !src) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    const size_t n = (size_t)h->nx * h->ny;
    double *st = h->at<double>(h->off_pop[1 - h->cur]);
    LbmParams p = make_params(h);
    for (int q = 0; q < 9; ++q) {
      HIPCHK(hipMemcpyAsync(st, src + (size_t)q * n, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
      HIPCHK(launch_f64_to_plane(h->prec, h->ws + h->off_pop[h->cur], p, q, st, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->stepped = false;
    if ((rc = clear_flag(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return ok();
  });
}

// whether ptr is device memory on the handle's device, the memory a kernel
// on the handle's stream may read or write
static int check_device_ptr(const btdf_t *h, const void *ptr) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();  // (clear the sticky error of an unknown pointer)
    return fail(BTDF_EINVAL, "the array is not memory HIP knows");
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (a.type != hipMemoryTypeDevice || a.device != dev)
    return fail(BTDF_EINVAL, "the array is not device memory on the handle's device");
  (void)h;
  return ok();
}

int btdf_get_populations_to(btdf_t *h, void *dst, int dst_on_device) {
  if (!dst_on_device) return btdf_get_populations(h, static_cast<double *>(dst));
  return guard([&]() -> int {
    if (!h || !dst) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    if ((rc = check_device_ptr(h, dst))) return rc;
    const size_t n = (size_t)h->nx * h->ny;
    LbmParams p = make_params(h);
    double *out = static_cast<double *>(dst);
    for (int q = 0; q < 9; ++q)
      HIPCHK(launch_plane_to_f64(h->prec, h->ws + h->off_pop[h->cur], p, q, out + (size_t)q * n, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return ok();
  });
}

int btdf_set_populations_from(btdf_t *h, const void *src, int src_on_device) {
  if (!src_on_device) return btdf_set_populations(h, static_cast<const double *>(src));
  return guard([&]() -> int {
    if (!h || !src) return fail(BTDF_EINVAL, "NULL argument");
    int rc = ensure_device(h);
    if (rc) return rc;
    if ((rc = check_device_ptr(h, src))) return rc;
    const size_t n = (size_t)h->nx * h->ny;
    LbmParams p = make_params(h);
    const double *in = static_cast<const double *>(src);
    for (int q = 0; q < 9; ++q)
      HIPCHK(launch_f64_to_plane(h->prec, h->ws + h->off_pop[h->cur], p, q, in + (size_t)q * n, h->stream));
    h->stepped = false;
    if ((rc = clear_flag(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return ok();
  });
}

int btdf_get_marker_data(btdf_t *h, double *rho_l, double *ux_l, double *uy_l, double *Fx, double *Fy) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    int rc = ensure_device(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    const size_t M = (size_t)std::max(h->nm(), 1), nm = (size_t)h->nm(), d = sizeof(double);
    double *outs[5] = {Fx, Fy, rho_l, ux_l, uy_l};
    for (int k = 0; k < 5; ++k)
      if (outs[k] && nm) HIPCHK(hipMemcpy(outs[k], h->ws + h->off_mk + (5 + k) * M * d, nm * d, hipMemcpyDeviceToHost));
    return ok();
  });
}

int btdf_marker_velocity(btdf_t *h, double *ux, double *uy) {
  return guard([&]() -> int {
    if (!h || !ux || !uy) return fail(BTDF_EINVAL, "NULL argument");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch");
    // the marker arrays on the device must be those of the last step, in the current layout
    if (!h->stepped || !h->layout_ok || !h->device_ok || !h->ws)
      return fail(BTDF_ESTATE, "no step since the state, the bodies or the layout last changed");
    const int nm = h->nm();
    if (nm == 0) return ok();
    if (h->any_moving())
      return fail(BTDF_ESTATE, "moving bodies: the markers have moved on since the last step's forces");
    std::vector<int> off, list;
    cover_lists(h, off, list);
    const size_t b_off = off.size() * sizeof(int), b_list = list.size() * sizeof(int);
    const size_t o_list = align256(b_off), o_out = o_list + align256(b_list);
    const size_t bytes = o_out + 2 * (size_t)nm * sizeof(double);
    char *buf = nullptr;
    hipError_t e = hipMalloc((void **)&buf, bytes);
    if (e != hipSuccess) return fail(BTDF_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    const LbmParams p = make_params(h);
    const IbParams ib = make_ib(h);
    double *out = reinterpret_cast<double *>(buf + o_out);
    e = hipMemcpyAsync(buf, off.data(), b_off, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(buf + o_list, list.data(), b_list, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = launch_marker_velocity(h->prec, h->ws + h->off_pop[h->cur], p, ib, reinterpret_cast<const int *>(buf),
                                 reinterpret_cast<const int *>(buf + o_list), out, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    std::vector<double> host(2 * (size_t)nm);
    if (e == hipSuccess) e = hipMemcpy(host.data(), out, host.size() * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(BTDF_EDEVICE, "marker velocity: %s", hipGetErrorString(e));
    for (int l = 0; l < nm; ++l) {
      ux[l] = host[2 * (size_t)l];
      uy[l] = host[2 * (size_t)l + 1];
    }
    return ok();
  });
}

static const uint64_t kStateMagic = 0x4254444653544154ULL;  // "BTDFSTAT"

size_t btdf_state_bytes(const btdf_t *h) {
  return guard_size([&]() -> size_t {
    if (!h) return 0;
    return 64 + 9 * (size_t)h->nx * h->ny * (size_t)h->prec;
  });
}

int btdf_save(btdf_t *h, void *dst, size_t bytes) {
  return guard([&]() -> int {
    if (!h || !dst) return fail(BTDF_EINVAL, "NULL argument");
    if (bytes < btdf_state_bytes(h)) return fail(BTDF_EINVAL, "buffer of %zu bytes < %zu", bytes, btdf_state_bytes(h));
    int rc = ensure_device(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    uint64_t hdr[8] = {kStateMagic, (uint64_t)h->prec, (uint64_t)h->nx, (uint64_t)h->ny, (uint64_t)h->steps, 0, 0, 0};
    std::memcpy(&hdr[5], &h->u0[0], 8);  // the reference state of the stored deviations
    std::memcpy(&hdr[6], &h->u0[1], 8);
    std::memcpy(dst, hdr, 64);
    const size_t row = (size_t)h->nx * h->prec;
    for (int q = 0; q < 9; ++q)
      HIPCHK(hipMemcpy2D((char *)dst + 64 + (size_t)q * h->ny * row, row,
                         h->ws + h->off_pop[h->cur] + (size_t)q * h->plane * h->prec, (size_t)h->pitch * h->prec,
                         row, (size_t)h->ny, hipMemcpyDeviceToHost));
    return ok();
  });
}

int btdf_load(btdf_t *h, const void *src, size_t bytes) {
  return guard([&]() -> int {
    if (!h || !src) return fail(BTDF_EINVAL, "NULL argument");
    if (bytes < btdf_state_bytes(h)) return fail(BTDF_EINVAL, "buffer of %zu bytes < %zu", bytes, btdf_state_bytes(h));
    uint64_t hdr[8];
    std::memcpy(hdr, src, 64);
    uint64_t r0, r1;
    std::memcpy(&r0, &h->u0[0], 8);
    std::memcpy(&r1, &h->u0[1], 8);
    if (hdr[0] != kStateMagic || hdr[1] != (uint64_t)h->prec || hdr[2] != (uint64_t)h->nx || hdr[3] != (uint64_t)h->ny ||
        hdr[5] != r0 || hdr[6] != r1)
      return fail(BTDF_EINVAL, "state does not match this handle (size, precision or initial velocity)");
    int rc = ensure_device(h);
    if (rc) return rc;
    h->stepped = false;
    const size_t row = (size_t)h->nx * h->prec;
    for (int q = 0; q < 9; ++q)
      HIPCHK(hipMemcpy2DAsync(h->ws + h->off_pop[h->cur] + (size_t)q * h->plane * h->prec, (size_t)h->pitch * h->prec,
                              (const char *)src + 64 + (size_t)q * h->ny * row, row, row, (size_t)h->ny,
                              hipMemcpyHostToDevice, h->stream));
    h->steps = (int64_t)hdr[4];
    h->hist_read = h->steps;
    h->forces_from = h->steps;
    long long ctr = (long long)h->steps;
    HIPCHK(hipMemcpyAsync(h->ws + h->off_ctl, &ctr, 8, hipMemcpyHostToDevice, h->stream));
    if ((rc = clear_flag(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return ok();
  });
}

int btdf_counts(const btdf_t *h, int *n_bodies, int *n_markers, int64_t *n_steps) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (n_bodies) *n_bodies = h->nb();
    if (n_markers) *n_markers = h->nm();
    if (n_steps) *n_steps = h->steps;
    return ok();
  });
}

int btdf_set_option(btdf_t *h, int key, int64_t value) {
  return guard([&]() -> int {
    if (!h) return fail(BTDF_EINVAL, "NULL handle");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch; set options on the batch");
    switch (key) {
      case BTDF_OPT_LBM_VARIANT:
        if (value < 0 || value >= num_variants()) return fail(BTDF_EINVAL, "variant %lld out of range", (long long)value);
        if (value != h->variant) {
          h->variant = (int)value;
          h->layout_ok = false;  // tiles change
          h->device_ok = false;
          drop_graph(h);
        }
        return ok();
      case BTDF_OPT_GRAPH_CHUNK:
        if (value < 0 || value > 4096) return fail(BTDF_EINVAL, "graph chunk must be in 0 .. 4096");
        if (value != h->graph_chunk) {
          h->graph_chunk = (int)value;
          drop_graph(h);
        }
        return ok();
      case BTDF_OPT_XCD_REMAP:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "xcd remap must be 0 or 1");
        h->xcd_remap = (int)value;
        drop_graph(h);
        return ok();
      case BTDF_OPT_INTERIOR_PATH:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "interior path flag must be 0 or 1");
        h->interior = (int)value;
        drop_graph(h);
        return ok();
      case BTDF_OPT_ROW_PAD:
      case BTDF_OPT_PLANE_PAD:
        if (value < 0 || value > (1 << 20) || (key == BTDF_OPT_PLANE_PAD && value % 64))
          return fail(BTDF_EINVAL, "padding must be in 0 .. 2^20 (planes: a multiple of 64)");
        if (h->state_ok) return fail(BTDF_ESTATE, "layout options must be set before the first device use");
        if (key == BTDF_OPT_ROW_PAD)
          h->row_pad = (int)value;
        else
          h->plane_pad = (int)value;
        h->layout_ok = false;
        return ok();
      case BTDF_OPT_ROW_ALIGN:
        if (value != 0 && (value < 4 || value > 4096 || (value & (value - 1))))
          return fail(BTDF_EINVAL, "row alignment must be 0 or a power of two in 4 .. 4096 bytes");
        if (h->state_ok) return fail(BTDF_ESTATE, "layout options must be set before the first device use");
        h->row_align = (int)value;
        h->layout_ok = false;
        return ok();
      case BTDF_OPT_EDGE_TILES:
        if (value != 0 && value != 1) return fail(BTDF_EINVAL, "edge tiles must be 0 (step singly) or 1 (blocked)");
        if (value != h->edge_tiles) {
          h->edge_tiles = (int)value;
          h->layout_ok = false;  // the tile lists
          h->device_ok = false;
          drop_graph(h);
        }
        return ok();
      case BTDF_OPT_TEMPORAL_BLOCKING:
        if (value < 0 || value > 5)
          return fail(BTDF_EINVAL, "temporal blocking must be 0 (off), 1 (the default depth) or 2 to 5 steps per pass");
        if (value != h->tblock) {
          h->tblock = (int)value;
          h->layout_ok = false;  // the tile lists and the third buffer
          h->device_ok = false;
          drop_graph(h);
        }
        return ok();
      case BTDF_OPT_FORCING_METHOD:
        if (value != BTDF_FORCING_DIRECT && value != BTDF_FORCING_IMPLICIT && value != BTDF_FORCING_RKPM)
          return fail(BTDF_EINVAL, "unknown forcing method %lld", (long long)value);
        if (value != BTDF_FORCING_DIRECT && h->nf != 1)
          return fail(BTDF_ESTATE, "the implicit and RKPM methods take one forcing pass (NF = 1)");
        if (value != BTDF_FORCING_DIRECT && h->any_moving())
          return fail(BTDF_ESTATE, "moving bodies need the direct forcing method");
        if (value != h->method) {
          h->method = (int)value;
          h->layout_ok = false;  // matrices and marker factors change
          h->device_ok = false;
          h->stepped = false;
          drop_graph(h);
        }
        return ok();
      case BTDF_OPT_FORCING_PASSES:
        if (value < 1 || value > 64) return fail(BTDF_EINVAL, "forcing passes must be in 1 .. 64");
        if (value != 1 && h->method != BTDF_FORCING_DIRECT)
          return fail(BTDF_ESTATE, "forcing passes need the direct forcing method");
        if (value != 1 && h->any_moving()) return fail(BTDF_ESTATE, "moving bodies take one forcing pass");
        if (value != h->nf) {
          h->nf = (int)value;
          h->layout_ok = false;  // the pass buffers change size
          h->device_ok = false;
          drop_graph(h);
        }
        return ok();
      default: return fail(BTDF_EINVAL, "unknown or read-only option %d", key);
    }
  });
}

int btdf_get_option(const btdf_t *h, int key, int64_t *value) {
  return guard([&]() -> int {
    if (!h || !value) return fail(BTDF_EINVAL, "NULL argument");
    int tx, ty;
    switch (key) {
      case BTDF_OPT_LBM_VARIANT: *value = h->variant; return ok();
      case BTDF_OPT_NUM_VARIANTS: *value = num_variants(); return ok();
      case BTDF_OPT_GRAPH_CHUNK: *value = h->graph_chunk; return ok();
      case BTDF_OPT_XCD_REMAP: *value = h->xcd_remap; return ok();
      case BTDF_OPT_TILE_X: variant_tile(h->variant, &tx, &ty); *value = tx; return ok();
      case BTDF_OPT_TILE_Y: variant_tile(h->variant, &tx, &ty); *value = ty; return ok();
      case BTDF_OPT_ROW_PAD: *value = h->row_pad; return ok();
      case BTDF_OPT_INTERIOR_PATH: *value = h->interior; return ok();
      case BTDF_OPT_FORCED_TILES:
        if (!h->layout_ok) compute_layout(const_cast<btdf_t *>(h));
        *value = h->n_forced;
        return ok();
      case BTDF_OPT_PLANE_PAD: *value = h->plane_pad; return ok();
      case BTDF_OPT_ROW_ALIGN: *value = h->row_align; return ok();
      case BTDF_OPT_FORCING_PASSES: *value = h->nf; return ok();
      case BTDF_OPT_FORCING_METHOD: *value = h->method; return ok();
      case BTDF_OPT_TEMPORAL_BLOCKING: *value = h->tblock; return ok();
      case BTDF_OPT_EDGE_TILES: *value = h->edge_tiles; return ok();
      case BTDF_OPT_FUSED_NODES:
        if (!h->layout_ok) compute_layout(const_cast<btdf_t *>(h));
        *value = blocking_active(h) ? h->pass_nodes : 0;
        return ok();
      case BTDF_OPT_EDGE_FUSED_TILES: {
        if (!h->layout_ok) compute_layout(const_cast<btdf_t *>(h));
        int k = 0;
        for (int g = 0; g < kLevels; ++g) k += group_tiles(h->gkind[g]) * h->n_edge[g];
        *value = blocking_active(h) ? k : 0;
        return ok();
      }
      case BTDF_OPT_FUSED_TILES:
        if (!h->layout_ok) compute_layout(const_cast<btdf_t *>(h));
        *value = blocking_active(h) ? h->pass_tiles() : 0;  // in lattice tiles
        return ok();
      case BTDF_OPT_STEPS_PER_PASS:
        if (!h->layout_ok) compute_layout(const_cast<btdf_t *>(h));
        *value = blocking_active(h) ? h->depth : 1;
        return ok();
      default: return fail(BTDF_EINVAL, "unknown option %d", key);
    }
  });
}

int btdf_calibrate_thickening_markers(int delta_kind, int n, const double *xy, double ds, double *drs_mean,
                                      double *drs_per_marker) {
  return guard([&]() -> int {
    if (!xy || !drs_mean) return fail(BTDF_EINVAL, "NULL argument");
    if (n < 1) return fail(BTDF_EINVAL, "need at least one marker");
    if (!valid_kind(delta_kind)) return fail(BTDF_EINVAL, "unknown delta kind %d", delta_kind);
    if (!(ds > 0.0) || !std::isfinite(ds)) return fail(BTDF_EINVAL, "ds must be > 0");
    for (int l = 0; l < 2 * n; ++l)
      if (!std::isfinite(xy[l]) || std::fabs(xy[l]) > 1e8) return fail(BTDF_EINVAL, "bad marker coordinate");
    const int S = stencil_size(delta_kind);
    // per marker: stencil base and weights; A_lm = ds sum_k W_lk W_mk (eq 22, dh = 1)
    std::vector<int> bx(n), by(n);
    std::vector<double> wx(4 * (size_t)n), wy(4 * (size_t)n);
    for (int l = 0; l < n; ++l) {
      bx[l] = stencil_base(delta_kind, xy[2 * l]);
      by[l] = stencil_base(delta_kind, xy[2 * l + 1]);
      for (int a = 0; a < S; ++a) {
        wx[4 * l + a] = phi_host(delta_kind, (double)(bx[l] + a) - xy[2 * l]);
        wy[4 * l + a] = phi_host(delta_kind, (double)(by[l] + a) - xy[2 * l + 1]);
      }
    }
    std::vector<double> A;
    try {
      A.assign((size_t)n * n, 0.0);
    } catch (...) {
      return fail(BTDF_ENOMEM, "out of host memory");
    }
    for (int l = 0; l < n; ++l) {
      for (int m = 0; m < n; ++m) {
        const int ox = bx[m] - bx[l], oy = by[m] - by[l];
        if (ox <= -S || ox >= S || oy <= -S || oy >= S) continue;
        double s = 0.0;
        for (int c = 0; c < S; ++c) {
          const int cm = c - oy;
          if (cm < 0 || cm >= S) continue;
          for (int a = 0; a < S; ++a) {
            const int am = a - ox;
            if (am < 0 || am >= S) continue;
            s += wx[4 * l + a] * wy[4 * l + c] * wx[4 * m + am] * wy[4 * m + cm];
          }
        }
        A[(size_t)l * n + m] = ds * s;
      }
    }
    // solve A x = 1 (eqs 24-25) by LU with partial pivoting
    std::vector<double> x(n, 1.0);
    double amax = 0.0;
    for (double v : A) amax = std::max(amax, std::fabs(v));
    for (int k = 0; k < n; ++k) {
      int piv = k;
      for (int r = k + 1; r < n; ++r)
        if (std::fabs(A[(size_t)r * n + k]) > std::fabs(A[(size_t)piv * n + k])) piv = r;
      if (!(std::fabs(A[(size_t)piv * n + k]) > 1e-13 * amax))
        return fail(BTDF_ESTATE, "matrix A is singular to working precision (markers too dense?)");
      if (piv != k) {
        for (int c = 0; c < n; ++c) std::swap(A[(size_t)k * n + c], A[(size_t)piv * n + c]);
        std::swap(x[k], x[piv]);
      }
      const double d = A[(size_t)k * n + k];
      for (int r = k + 1; r < n; ++r) {
        const double f = A[(size_t)r * n + k] / d;
        if (f == 0.0) continue;
        for (int c = k; c < n; ++c) A[(size_t)r * n + c] -= f * A[(size_t)k * n + c];
        x[r] -= f * x[k];
      }
    }
    for (int k = n - 1; k >= 0; --k) {
      double s = x[k];
      for (int c = k + 1; c < n; ++c) s -= A[(size_t)k * n + c] * x[c];
      x[k] = s / A[(size_t)k * n + k];
    }
    double mean = 0.0;
    for (int l = 0; l < n; ++l) mean += x[l];
    *drs_mean = mean / n;
    if (drs_per_marker)
      for (int l = 0; l < n; ++l) drs_per_marker[l] = x[l];
    return ok();
  });
}

int btdf_calibrate_thickening(int delta_kind, double D, int n_markers, double *drs_mean, double *drs_per_marker) {
  return guard([&]() -> int {
    if (!drs_mean) return fail(BTDF_EINVAL, "NULL argument");
    if (!(D > 0.0) || !std::isfinite(D) || D > 1e7) return fail(BTDF_EINVAL, "D must be > 0 (got %g)", D);
    if (n_markers < 3) return fail(BTDF_EINVAL, "need at least three markers");
    // the ring of btdf_add_body's usual input: X_l = (D/2)(cos t_l, sin t_l),
    // t_l = 2 pi l / n, about the node (0, 0); ds = pi D / n (arc spacing)
    std::vector<double> xy(2 * (size_t)n_markers);
    for (int l = 0; l < n_markers; ++l) {
      const double t = 2.0 * M_PI * l / n_markers;
      xy[2 * l] = 0.5 * D * std::cos(t);
      xy[2 * l + 1] = 0.5 * D * std::sin(t);
    }
    return btdf_calibrate_thickening_markers(delta_kind, n_markers, xy.data(), M_PI * D / n_markers, drs_mean,
                                             drs_per_marker);
  });
}

}  // extern "C"
