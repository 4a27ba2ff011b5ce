// btdf_launch.h -- host-side entry points of the kernels (internal to the library).
#pragma once

#include "btdf_device.h"

namespace btdf {

int num_variants();
void variant_tile(int v, int *tx, int *ty);

hipError_t launch_lbm(int prec, int variant, const void *A, void *B, const LbmParams &p, const TileRange &r,
                      const IbParams &ib, hipStream_t s);
hipError_t launch_ib(int prec, const void *A, const LbmParams &p, const IbParams &ib, hipStream_t s);
hipError_t launch_rigid_move(const MoveParams &mp, hipStream_t s);
// two steps A -> C over the listed groups of width lattice tiles; with near
// non-null, edge nodes next to a near tile also store their first step in X
hipError_t launch_lbm2(int prec, int variant, int width, const void *A, void *C, const LbmParams &p, const int *map,
                       int count, void *X, const unsigned char *near, hipStream_t s);
bool variant_has_wide_lbm2(int variant, int prec, int width);
// group shapes of the three-step pass, W | H << 4 for W x H lattice tiles
// (map entries name a group's lower-left tile)
constexpr int kGroup1x1 = 0x11, kGroup2x1 = 0x12, kGroup4x1 = 0x14;
constexpr int kGroup1x4 = 0x41;  // (edge groups only: the ends of a channel)
constexpr int kGroup2x2 = 0x22, kGroup1x2 = 0x21;  // (two tiles tall: passes of five steps)
constexpr int kNoGroup = 0;  // an unused level
// groups of tiles within reach of a domain edge, with the boundary readings
// in every step of the pass (btdf_edge.hip): the flag kEdge on a shape
constexpr int kEdge = 0x100;
constexpr int kEdge4x1 = kEdge | kGroup4x1, kEdge2x1 = kEdge | kGroup2x1, kEdge1x1 = kEdge | kGroup1x1;
constexpr int group_tiles(int code) { return (code & 15) * ((code >> 4) & 15); }
constexpr bool is_edge(int code) { return (code & kEdge) != 0; }
// a pass map entry names an edge group when this bit is set (tile ids are below it)
constexpr int kEdgeFlag = 1 << 30;
// A pass launches its groups level by level: up to kLevels shapes, the
// largest first in the tile map. A level's edge groups (map entries with
// kEdgeFlag, btdf_edge.h) come first in its list.
constexpr int kLevels = 4;
// three steps A -> C over the listed groups of the given shape; with near
// non-null, edge nodes next to a near tile also store their first and second
// steps in X1 and X2
hipError_t launch_lbm3(int prec, int variant, int code, const void *A, void *C, const LbmParams &p, const int *map,
                       int count, void *X1, void *X2, const unsigned char *near, hipStream_t s);
bool variant_has_lbm3(int variant, int prec, int code);
// batches: the groups of every case, gcase[k] / gtile[k] = case and first tile
hipError_t launch_lbm3_batch(int prec, int variant, int code, const CaseDesc *cases, const int *gcase,
                             const int *gtile, int count, int rt, int mask, int xcd, hipStream_t s);
bool variant_has_lbm2(int variant, int prec);
// Whether a pass of depth 2 or 3 takes edge groups of the given shape
// (kEdge and a row of 1, 2 or 4 tiles, or a column of 4)
bool variant_has_edge(int variant, int prec, int depth, int code);
// three steps A -> C over the listed edge groups (entries may carry kEdgeFlag);
// with near non-null, edge nodes next to a near tile also store their first
// and second steps in X1 and X2. Batches: gcase/gtile as for launch_lbm3_batch.
hipError_t launch_lbm_edge3(int prec, int variant, int code, const void *A, void *C, const LbmParams &p,
                            const int *map, int count, void *X1, void *X2, const unsigned char *near, hipStream_t s);
hipError_t launch_lbm_edge3_batch(int prec, int variant, int code, const CaseDesc *cases, const int *gcase,
                                  const int *gtile, int count, int rt, int mask, int xcd, hipStream_t s);
// two steps A -> C over the listed edge groups (entries may carry kEdgeFlag);
// with near non-null, edge nodes next to a near tile also store their first
// step in X
hipError_t launch_lbm_edge2(int prec, int variant, int code, const void *A, void *C, const LbmParams &p,
                            const int *map, int count, void *X, const unsigned char *near, hipStream_t s);
// four or five steps A -> C over the listed groups (rows of 1, 2 or 4
// lattice tiles, or two tiles tall, at least depth nodes from every domain
// edge); the first ring_groups of them border a near tile (rwin[k]: the
// near flags of the tiles around group k, bit 8 r + c for row r from the
// row below and column c from the column left of it), and their edge nodes also store
// their states n+1 .. n+depth-1 in the ring buffers, consecutive population
// buffers from ring (btdf_deep.hip)
bool variant_has_deep(int variant, int prec, int depth, int code);
hipError_t launch_lbm_deep(int prec, int variant, int depth, int code, const void *A, void *C, const LbmParams &p,
                           const int *map, int count, int ring_groups, void *ring, const unsigned *rwin,
                           hipStream_t s);
hipError_t launch_conv_outlet(int prec, const void *A, void *B, const LbmParams &p, hipStream_t s);
hipError_t launch_conv_outlet_batch(int prec, const CaseDesc *cases, int ncases, int mask_unstable, int rt,
                                    hipStream_t s);
hipError_t launch_marker_velocity(int prec, const void *A, const LbmParams &p, const IbParams &ib,
                                  const int *cover_off, const int *cover_list, double *out, hipStream_t s);
hipError_t launch_marker_velocity_tiles(int prec, const void *A, const LbmParams &p, const IbParams &ib, int tile_x,
                                        int tile_y, double *ux, double *uy, hipStream_t s);
hipError_t launch_lbm_batch(int prec, int variant, const CaseDesc *cases, const BatchMap &m, int rt,
                            hipStream_t s);
hipError_t launch_ib_batch(int prec, const CaseDesc *cases, const BatchMap &m, int rt, hipStream_t s);
hipError_t launch_adj_lattice(int prec, const void *A, const void *Gnext, void *Gout, const LbmParams &p,
                              const AdjParams &a, hipStream_t s);
hipError_t launch_adj_marker(int prec, const void *A, const void *Gnext, const LbmParams &p, const IbParams &ib,
                             const AdjParams &a, hipStream_t s);
hipError_t launch_adj_unpull(int prec, const void *G, const LbmParams &p, double *out, hipStream_t s);
hipError_t launch_init_uniform(int prec, void *A, const LbmParams &p, double r, double u, double v,
                               hipStream_t s);
hipError_t launch_init_eq(int prec, void *A, const LbmParams &p, const double *rho, const double *ux,
                          const double *uy, double rho0, int per_node_rho, hipStream_t s);
hipError_t launch_plane_to_f64(int prec, const void *A, const LbmParams &p, int q, double *out,
                               hipStream_t s);
hipError_t launch_f64_to_plane(int prec, void *A, const LbmParams &p, int q, const double *in,
                               hipStream_t s);
hipError_t launch_macro(int prec, const void *A, const LbmParams &p, double *rho, double *ux, double *uy,
                        hipStream_t s);

}  // namespace btdf
