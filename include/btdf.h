/*
 * btdf.h -- C ABI of the MI355X (gfx950) library for the boundary-thickening
 * direct-forcing immersed-boundary lattice Boltzmann method (BTDF-IB-LBM) of
 * Jiang & Liu, arXiv 1806.09403.
 *
 * One handle holds one 2-D D2Q9 simulation on one GPU: a grid of N_E
 * Eulerian nodes and any number of rigid bodies, each represented by N_L
 * Lagrangian markers with prescribed velocities U_b (Section 2.2). One time
 * step is Algorithm 1 (Section 2.4) with NF = 1:
 *   streaming, moments (eqs 9-10), interpolation of the unforced velocity to
 *   the markers (eqs 12, 14), the direct force F_b = 2 rho (U_b - D_I u*)
 *   (eq 20), spreading with the thickened solid shell drs (eqs 13, 15), the
 *   hydrodynamic force and torque on each body (eq 27), and the BGK collision
 *   with the Guo force term (eqs 5-7, 11).
 *
 * Units: lattice units, dh = dt = c = 1; node (i, j) sits at (x, y) = (i, j).
 *
 * Conventions shared by every call:
 *  - Every call returns an int status: BTDF_OK (0) or a negative BTDF_E*
 *    code. Nothing throws, aborts or exits across the ABI. The message of the
 *    last failure on the calling thread is returned by btdf_last_error().
 *  - A handle is used by one thread at a time.
 *  - "Host array" means memory the caller owns; the library copies what it
 *    needs during the call and keeps no pointer to it.
 *  - Host field arrays are double precision, row-major [ny][nx] (x fastest);
 *    population arrays are [9][ny][nx] with the D2Q9 order of eq 8:
 *    e = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
 *  - Device memory is either one caller-owned workspace (btdf_bind_workspace,
 *    e.g. a PyTorch tensor) or, if none is bound, allocated by the library.
 *  - Work is enqueued on the handle's HIP stream; calls documented as
 *    "synchronising" wait for that stream before returning.
 */
#ifndef BTDF_H
#define BTDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define BTDF_OK 0
#define BTDF_EINVAL (-1)    /* bad argument; nothing was changed */
#define BTDF_ENOMEM (-2)    /* host or device allocation failed, or workspace too small */
#define BTDF_EDEVICE (-3)   /* a HIP call or kernel launch failed */
#define BTDF_ESTATE (-4)    /* call not valid in the current state */
#define BTDF_EUNSTABLE (-5) /* the run went unstable (see btdf_step) */

/* ---- boundary kinds (btdf_grid.bc_*) ----
 * x ends: both PERIODIC, or VELOCITY_INLET (west) + ZERO_GRADIENT_OUTLET or
 *   CONVECTIVE_OUTLET (east). The channel ends are ghost columns i = 0 and
 *   i = nx-1 that are neither collided nor forced. After each collision the
 *   inlet ghost is set to the equilibrium (eq 6) at the inflow velocity with
 *   the density of column 1. A zero-gradient outlet ghost copies column
 *   nx-2; a convective outlet ghost follows d/dt + U d/dx = 0 with U the
 *   inflow speed (inflow_ux >= 0), implicit upwind:
 *   ghost(t+1) = (ghost(t) + U column_{nx-2}(t+1)) / (1 + U)
 *   (the far-field outflow of the paper's cylinder runs, Section 5.2).
 * y ends: both PERIODIC, or both BOUNCEBACK_WALL (halfway bounce-back), or
 *   both FREE_SLIP_WALL (du_x/dy = 0, u_y = 0; the far field of Section 5.2):
 *   a specular reflection, the population that left the upstream column
 *   towards the wall returns with its y component reversed. Walls sit at
 *   y = -1/2 and y = ny - 1/2. btdf_adjoint supports PERIODIC,
 *   BOUNCEBACK_WALL and ZERO_GRADIENT_OUTLET only. */
#define BTDF_PERIODIC 0
#define BTDF_VELOCITY_INLET 1
#define BTDF_ZERO_GRADIENT_OUTLET 2
#define BTDF_BOUNCEBACK_WALL 3
#define BTDF_FREE_SLIP_WALL 4
#define BTDF_CONVECTIVE_OUTLET 5

/* ---- forcing methods (BTDF_OPT_FORCING_METHOD) ----
 * DIRECT (default): F_l = 2 rho_l (U_l - D_I u*) (eq 20), spread with
 *   drs ds F_l: the thickened-shell method (or conventional direct forcing
 *   with thickening 1, multi direct forcing with NF > 1).
 * IMPLICIT: the implicit direct forcing of eq 17, F_b = (D_I D_E)^-1 times
 *   the direct force, one dense matrix per body (eq 21) formed and inverted
 *   on the host; identical to the implicit velocity correction of eqs
 *   32-35 (Appendix A) and independent of the thickening.
 * RKPM: the direct force spread with ds epsilon_l F_l, epsilon = A^-1 1 (row
 *   sums of A^-1, eq 22 with drs = dh; eq 36 / B54); the thickening is
 *   unused.
 * The hydrodynamic force of a body is minus the total force spread into the
 * fluid. Markers of different bodies are not coupled by the matrices. */
#define BTDF_FORCING_DIRECT 0
#define BTDF_FORCING_IMPLICIT 1
#define BTDF_FORCING_RKPM 2

/* ---- regularised delta functions (Section 4.3) ----
 * LINEAR2: 2-point, eq 37;  ROMA3: 3-point, eq 38;  PESKIN4: 4-point, eq 39;
 * COS4: the cosine 4-point kernel (1 + cos(pi r / 2)) / 4 on |r| <= 2.
 * Stencils: LINEAR2 floor(X) .. floor(X)+1; ROMA3 floor(X+1/2)-1 .. +1;
 * PESKIN4 and COS4 floor(X)-1 .. floor(X)+2 (per direction). */
#define BTDF_LINEAR2 2
#define BTDF_ROMA3 3
#define BTDF_PESKIN4 4
#define BTDF_COS4 5

/* ---- option keys (btdf_set_option / btdf_get_option) ---- */
#define BTDF_OPT_LBM_VARIANT 1   /* launch shape of the lattice kernel, 0 .. BTDF_OPT_NUM_VARIANTS-1 (default 6: 32x8 tiles) */
#define BTDF_OPT_NUM_VARIANTS 2  /* read-only: number of lattice launch shapes */
#define BTDF_OPT_GRAPH_CHUNK 3   /* steps per captured HIP graph; 0 = plain launches (default 0) */
#define BTDF_OPT_XCD_REMAP 4     /* 1 = map consecutive tiles to one XCD (default 1) */
#define BTDF_OPT_TILE_X 5        /* read-only: tile width of the current variant */
#define BTDF_OPT_TILE_Y 6        /* read-only: tile height of the current variant */
#define BTDF_OPT_ROW_PAD 7       /* elements added to each grid row (>= 0); only before the first device use */
#define BTDF_OPT_PLANE_PAD 8     /* elements added to each population plane, multiple of 64; same restriction */
#define BTDF_OPT_INTERIOR_PATH 9 /* 1 (default): waves away from every edge load from wave-uniform bases; 0: always the general pull */
#define BTDF_OPT_FORCED_TILES 11 /* read-only: lattice tiles touched by some marker's stencil */
#define BTDF_OPT_MASK_UNSTABLE 12 /* batches only: 1 (default) = a case that went unstable stops, the others go on */
#define BTDF_OPT_ROW_ALIGN 13     /* bytes (0 or a power of two 4..4096, default 128): each row starts on this
                                    boundary, pitch = round_up(nx, align) + row pad; only before the first device use */
#define BTDF_OPT_FORCING_METHOD 15 /* BTDF_FORCING_*: how the marker force is formed and spread (Section 3);
                                      stand-alone handles only, NF = 1, bodies of at most 2048 markers; the
                                      matrices are formed on the host when the bodies or the method change */
#define BTDF_OPT_TEMPORAL_BLOCKING 16 /* d steps per pass for the tiles at least d-1 nodes clear of every marker
                                         stencil and d nodes clear of the domain edges (at d = 2 or 3 with
                                         BTDF_OPT_EDGE_TILES, the edge tiles too): each node read and written
                                         once for d updates. The others step singly with the marker kernel
                                         between, and the pass gives them the intermediate states of the
                                         nodes just outside. Results are bit-identical to single steps.
                                         1 (default): five steps per pass in FP32 (three in FP64) on lattices
                                         of at least 2^20 nodes where the launch shape has them (32x8 lattice
                                         tiles), else the deepest below (3, or 2 for tiles one or two rows tall); smaller
                                         lattices step singly (the extra launches of a pass outweigh the
                                         bytes saved). 2 to 5: that depth where the shape has it, else the
                                         next lower; 0: off. In a batch (btdf_batch_set_option) any nonzero
                                         value means three steps per pass for every case, default on. Takes
                                         d-1 more population buffers. With a graph chunk k > 0 a graph holds
                                         k / d whole passes. Steps run singly instead with moving bodies or
                                         with a launch shape of more than one node per thread. Steps left
                                         over after whole passes, on a stand-alone handle: three after
                                         deeper passes take one three-step pass, two after passes of three
                                         or more one two-step pass, over the same tiles; otherwise (and in
                                         batches) they step singly. */
#define BTDF_OPT_EDGE_TILES 20        /* 1: tiles within reach of a domain edge (periodic seams, walls, the inlet and a
                                         zero-gradient outlet; not a convective outlet) also take the blocked pass,
                                         with the boundary readings in every step, in launches of their own; 0: they
                                         step singly with the near tiles. Default 0 for a stand-alone handle (its few
                                         edge tiles do not repay the launches' fixed cost), 1 in a batch (whose
                                         launches gather the edge tiles of every case). Results are bit-identical
                                         either way. */
#define BTDF_OPT_EDGE_FUSED_TILES 21  /* read-only: of BTDF_OPT_FUSED_TILES, the tiles within reach of a domain edge */
#define BTDF_OPT_FUSED_NODES 22       /* read-only: grid nodes in the blocked pass (tiles reaching past the grid
                                         counted by their nodes inside it); batches: over every case */
#define BTDF_OPT_FUSED_TILES 17       /* read-only: lattice tiles that take the blocked pass (0 when it is not active) */
#define BTDF_OPT_STEPS_PER_PASS 18    /* read-only: steps per pass of those tiles (1 when blocking is not active) */
#define BTDF_OPT_FORCING_PASSES 14 /* NF in 1..64 (default 1): direct-forcing passes per step (Sec. 2.3, eqs 29-31);
                                      each pass after the first re-interpolates the velocity corrected by the force
                                      spread so far and adds 2 rho_l (U - u) to the marker force; stand-alone
                                      handles only, and btdf_adjoint requires NF = 1 */

typedef struct btdf_grid {
  int32_t nx, ny;               /* nodes, ghost columns included; each >= 8 */
  int32_t bc_west, bc_east;     /* BTDF_PERIODIC pair or VELOCITY_INLET + ZERO_GRADIENT / CONVECTIVE_OUTLET */
  int32_t bc_south, bc_north;   /* BTDF_PERIODIC, BOUNCEBACK_WALL or FREE_SLIP_WALL pair */
  double inflow_ux, inflow_uy;  /* velocity of the inlet ghost column */
  double body_force_x;          /* uniform body-force density G (force per node) */
  double body_force_y;
  double rho0, ux0, uy0;        /* initial state: equilibrium at (rho0, u0) everywhere */
  int32_t precision;            /* 4: FP32 populations, 8: FP64 populations */
  int32_t history_capacity;     /* steps kept in the per-body force ring; 0 -> 4096 */
  void *hip_stream;             /* hipStream_t to enqueue on; NULL = the null stream */
  uint64_t flags;               /* reserved, must be 0 */
} btdf_grid;

typedef struct btdf_sim btdf_t;

/* Message of the last failed call on this thread ("" if none). The pointer
 * stays valid until the next call on the same thread. */
const char *btdf_last_error(void);

/* Create a simulation. tau > 1/2 is the BGK relaxation time (nu = (tau -
 * 1/2)/3, the relation stated after eq 7); delta_kind is one of BTDF_LINEAR2
 * .. BTDF_COS4; thickening = drs/dh > 0 is the solid-shell thickness of eq 15
 * (1.0 is conventional direct forcing, eq 28; the paper suggests 1.4, 1.9
 * and 2.6 for 2-, 3- and 4-point deltas, Section 4.4). No device memory is
 * touched until the first call that needs it; the populations then start
 * at the equilibrium (eq 6) at (rho0, u0), ghost columns included.
 * Errors: EINVAL (NULL pointers, nx or ny < 8, tau <= 1/2, unknown kind,
 * thickening <= 0, bad boundary combination, precision not 4 or 8, flags != 0).
 * ENOMEM. */
int btdf_create(const btdf_grid *g, double tau, int delta_kind, double thickening, btdf_t **out);

/* Free everything the library allocated (not a bound workspace). Waits for
 * the handle's stream. NULL is accepted. */
int btdf_destroy(btdf_t *h);

/* Device bytes the current grid and body set need in a caller-owned
 * workspace (256-byte aligned start required). 0 on a NULL handle. */
size_t btdf_workspace_bytes(const btdf_t *h);

/* Use dev[0 .. bytes) as all device memory of the handle from now on. The
 * caller keeps it alive until btdf_destroy or the next bind. If a state
 * exists it is moved into the new workspace (synchronising). Passing NULL
 * returns to library-owned memory. Errors: EINVAL (misaligned), ENOMEM
 * (bytes < btdf_workspace_bytes), EDEVICE. Adding a body may later raise the
 * requirement; calls that need device memory then return ENOMEM until a
 * large enough workspace is bound. */
int btdf_bind_workspace(btdf_t *h, void *dev, size_t bytes);

/* Enqueue all further work on hip_stream (NULL = null stream). */
int btdf_set_stream(btdf_t *h, void *hip_stream);

/* Add a rigid body of n >= 3 markers. xy: host array [n][2] of marker
 * positions X_l (eq 12); uv: host array [n][2] of prescribed velocities
 * U_b,l, or NULL for a body at rest; (cx, cy): the reference point of the
 * torque; ds > 0: the marker spacing of eq 15, or <= 0 for the polygon
 * perimeter / n. Markers may lie outside [0, nx) in a periodic direction
 * (their stencils wrap). In a non-periodic direction every stencil node must
 * be a fluid node (x in 1 .. nx-2 for a channel, y in 0 .. ny-1 for walls).
 * The body id (0, 1, ...) is written to *body_id if not NULL. Adding a body
 * resets the force history. Errors: EINVAL, ENOMEM. */
int btdf_add_body(btdf_t *h, int n, const double *xy, const double *uv, double cx, double cy,
                  double ds, int *body_id);

/* Replace the prescribed marker velocities of one body; uv: host [n][2].
 * Takes effect from the next enqueued step (synchronising). EINVAL for a
 * body that moves rigidly (its velocities follow the motion). */
int btdf_set_marker_velocity(btdf_t *h, int body, const double *uv);

/* Rigid motion of one body from the next step on (eq 4 for a rigid body
 * whose surface carries the fluid with it): translation (vx, vy) and
 * angular velocity omega (counter-clockwise, radians per step) about its
 * centre. The prescribed marker velocity becomes U_l = V + omega x (X_l - c)
 * at once; after every step the centre and angle advance by one step and
 * the markers are placed at c + R(theta) r_l, r_l their offsets from the
 * centre when the body was added. (0, 0, 0) holds the body where it is. A
 * marker may travel less than 2 nodes per step (|V| + |omega| max|r_l|);
 * the tile lists of the spreading carry a 2-node margin and are rebuilt on
 * the host before any marker can have left it, so a run with moving bodies
 * synchronises every few tens of steps. A step that would carry a stencil
 * out of the fluid region (non-periodic directions) fails with EINVAL
 * before it is enqueued. Moving bodies need the direct forcing with NF = 1
 * and are not covered by btdf_adjoint; stand-alone handles only. The motion
 * state is not part of a checkpoint. */
int btdf_set_body_motion(btdf_t *h, int body, double vx, double vy, double omega);

/* (cx, cy, theta, vx, vy, omega) of one body after the steps enqueued so
 * far (a fixed body reports its centre, zeros elsewhere). */
int btdf_get_body_state(const btdf_t *h, int body, double *state);

/* Marker positions, host [n_markers][2]. Synchronising. */
int btdf_get_marker_positions(btdf_t *h, double *xy);

/* Enqueue n >= 0 time steps (asynchronous). If during them a marker's
 * force became non-finite, a marker's interpolated |u*| exceeded 0.3, or a
 * node density became non-positive or non-finite, the next synchronising
 * call returns BTDF_EUNSTABLE (the flag stays set until the populations are
 * replaced by btdf_init_equilibrium, btdf_set_populations or btdf_load). */
int btdf_step(btdf_t *h, int64_t n);

/* Same as btdf_step, but times the kernels with HIP events on the handle's
 * stream and writes, in milliseconds per step, the duration of the marker
 * kernel (*ms_ib, 0 if no bodies) and of the lattice launches (*ms_lbm).
 * The events are created on the first timed call and kept until
 * btdf_destroy. Synchronising. */
int btdf_step_timed(btdf_t *h, int64_t n, double *ms_ib, double *ms_lbm);

/* As btdf_step_timed with the lattice time split: ms[0] marker kernels and
 * ms[1] single-step lattice kernels, means per step; ms[2] the blocked pass
 * of temporal blocking: its mean launch duration divided by the steps per
 * pass (over the passes taken, a two-step remainder pass included). */
int btdf_step_timed_split(btdf_t *h, int64_t n, double *ms);

/* Same as btdf_step, timing only the blocked pass of temporal blocking: HIP
 * events around the pass's launches alone (two per pass, on the stream the
 * pass runs on), so the recording costs the steps little. *ms_pass: the
 * mean launch duration of the full-depth passes divided by the steps per
 * pass, in milliseconds per step (0 when no such pass ran: blocking off, or
 * n below the steps per pass; a two-step remainder pass is not timed).
 * Synchronising. Errors as btdf_step. */
int btdf_step_timed_pass(btdf_t *h, int64_t n, double *ms_pass);

/* Hydrodynamic force and torque on every body at the last step:
 * out[3*b + 0..2] = (Fx, Fy, Tz), Fx,y = -drs ds sum_l F_l (eq 27, sign:
 * force of the fluid on the body), Tz = -drs ds sum_l (X_l - c) x F_l.
 * Zeros before the first step. Synchronising. Errors: EINVAL (cap_bodies <
 * number of bodies), EUNSTABLE (values still written). */
int btdf_forces(btdf_t *h, double *out, int cap_bodies);

/* Per-step (Fx, Fy, Tz) of every body for the steps not yet returned, oldest
 * first, at most max_steps of them: out[(k*nbodies + b)*3 + c]. Steps older
 * than the ring capacity are dropped. *n_written receives the count.
 * Synchronising. */
int btdf_force_history(btdf_t *h, double *out, int64_t max_steps, int64_t *n_written);

/* Replace the populations by the equilibrium (eq 6) of the host fields rho,
 * ux, uy ([ny][nx]; rho may be NULL for rho0 everywhere). Synchronising. */
int btdf_init_equilibrium(btdf_t *h, const double *rho, const double *ux, const double *uy);

/* Density and velocity of the current state, host [ny][nx] each. At fluid
 * nodes: rho = sum_q g_q and u* = (sum_q e_q g_q + G/2) / rho of the
 * streamed populations g_q(x) = f_q(x - e_q) (what the next step
 * interpolates); at channel ghost columns: plain moments of the ghost node.
 * Synchronising. */
int btdf_get_macroscopic(btdf_t *h, double *rho, double *ux, double *uy);

/* Post-collision populations f_q (full values, not deviations) as host FP64
 * [9][ny][nx]; set replaces them (rounded to the handle's precision) and
 * clears the instability flag. Synchronising. */
int btdf_get_populations(btdf_t *h, double *dst);
int btdf_set_populations(btdf_t *h, const double *src);
/* The same with the FP64 [9][ny][nx] array in host memory (on_device = 0)
 * or in device memory of the handle's device (on_device = 1). A device array
 * is written or read by kernels on the handle's stream, with no copy through
 * the host; the caller owns it and keeps it allocated for the call.
 * BTDF_EINVAL if it is not device memory on the handle's device (checked
 * with hipPointerGetAttributes). Synchronising. */
int btdf_get_populations_to(btdf_t *h, void *dst, int dst_on_device);
int btdf_set_populations_from(btdf_t *h, const void *src, int src_on_device);

/* Per-marker values of the last step (host arrays of length = total
 * markers, any may be NULL): interpolated rho_l and u*_l (eqs 12, 14) and
 * the direct force F_l (eq 20). Synchronising. */
int btdf_get_marker_data(btdf_t *h, double *rho_l, double *ux_l, double *uy_l, double *Fx,
                         double *Fy);

/* Velocity at every marker after the last step (host arrays of length =
 * total markers): the corrected velocity the collision used (eq 11, with
 * the body force and the immersed-boundary force of that step)
 * interpolated at the marker (eq 12). At rest markers its root mean square
 * is the boundary error of eq 45; in general U_b - u_b is the slip. Needs
 * a step since the state or the bodies last changed (ESTATE otherwise);
 * stand-alone handles without moving bodies only. Allocates a temporary device buffer for the
 * covering-marker lists. Synchronising. */
int btdf_marker_velocity(btdf_t *h, double *ux, double *uy);

/* For callers that cannot allocate memory (loops that forbid hipMalloc,
 * harnesses that allow no allocation): btdf_marker_velocity with no device
 * or host allocation. Same arguments, results and errors; it rebuilds each
 * stencil node's spread force from the tile marker lists already on the
 * device (the same markers in the same order) instead of building covering
 * lists, and stages the results in a fixed array of 2 x
 * BTDF_NOALLOC_MAX_MARKERS doubles (4 MiB) that each GPU the library runs
 * on holds until the process ends. Errors also: EINVAL when the handle has
 * more than BTDF_NOALLOC_MAX_MARKERS markers. Every call on one GPU shares
 * that array, so calls that overlap on one GPU (from several threads or
 * streams) race. Synchronising. */
#define BTDF_NOALLOC_MAX_MARKERS 262144
int btdf_marker_velocity_noalloc(btdf_t *h, double *ux, double *uy);

/* Checkpoint: the populations as the handle stores them (its precision, as
 * deviations from the equilibrium at the initial velocity of btdf_grid)
 * plus the step counter. btdf_state_bytes gives the size; save writes it
 * into the host buffer dst, load restores it (bit-identical resume) into a
 * handle of the same size, precision and initial velocity (else EINVAL).
 * Synchronising. */
size_t btdf_state_bytes(const btdf_t *h);
int btdf_save(btdf_t *h, void *dst, size_t bytes);
int btdf_load(btdf_t *h, const void *src, size_t bytes);

/* Number of bodies, total markers and steps taken so far. */
int btdf_counts(const btdf_t *h, int *n_bodies, int *n_markers, int64_t *n_steps);

/* Tuning knobs (BTDF_OPT_*). set returns EINVAL for unknown keys or values,
 * ESTATE for a layout option once the populations exist on the device. */
int btdf_set_option(btdf_t *h, int key, int64_t value);
int btdf_get_option(const btdf_t *h, int key, int64_t *value);

/* Autotuner: run steps_per_trial steps in every launch shape of the lattice
 * kernel (BTDF_OPT_LBM_VARIANT x BTDF_OPT_INTERIOR_PATH), timed with HIP
 * events, and keep the fastest. The trials advance the simulation by
 * 2 x NUM_VARIANTS x steps_per_trial steps (all launch shapes give
 * bit-identical results, so the trajectory is the one plain stepping gives). *best_variant (may be NULL) receives
 * the chosen variant. Synchronising. */
int btdf_autotune(btdf_t *h, int64_t steps_per_trial, int *best_variant);

/* ---- batches: many independent cases stepped together ----
 * A batch holds n_cases independent simulations (grids[c], taus[c],
 * delta_kinds[c], thickenings[c], as for btdf_create; one precision for all;
 * the stream of grids[0]). A batch step runs the marker kernel over the
 * markers of every case and the lattice kernel over the tiles of every case,
 * one launch each, so small cases fill the GPU together. Each case is an
 * ordinary handle (btdf_batch_case) for every state call (forces, history,
 * populations, macroscopic fields, marker data, save/load, counts); stepping,
 * binding, options and adding bodies go through the batch. With
 * BTDF_OPT_MASK_UNSTABLE (default on) a case whose instability flag is set
 * stops stepping and the others continue; btdf_batch_status reports which.
 * A stopped case's kernels store nothing from the moment they read its flag
 * set, so its populations are left as its last launches wrote them (tiles
 * may hold different steps); its state calls return BTDF_EUNSTABLE. The
 * other cases are bit-identical to running alone. */
typedef struct btdf_batch btdf_batch_t;

int btdf_batch_create(int n_cases, const btdf_grid *grids, const double *taus, const int *delta_kinds,
                      const double *thickenings, btdf_batch_t **out);
int btdf_batch_destroy(btdf_batch_t *b);
/* The handle of case i (owned by the batch; valid until btdf_batch_destroy). */
int btdf_batch_case(btdf_batch_t *b, int i, btdf_t **h);
int btdf_batch_add_body(btdf_batch_t *b, int case_id, int n, const double *xy, const double *uv, double cx,
                        double cy, double ds, int *body_id);
/* Device bytes for all cases. Adding bodies changes it; a caller-owned
 * workspace must then be replaced by a fresh one (ESTATE otherwise). */
size_t btdf_batch_workspace_bytes(const btdf_batch_t *b);
int btdf_batch_bind_workspace(btdf_batch_t *b, void *dev, size_t bytes);
int btdf_batch_set_stream(btdf_batch_t *b, void *hip_stream);
/* n steps of every case (asynchronous); graphs per BTDF_OPT_GRAPH_CHUNK. */
int btdf_batch_step(btdf_batch_t *b, int64_t n);
/* As btdf_step_timed: mean ms per step of the marker and lattice launches. */
int btdf_batch_step_timed(btdf_batch_t *b, int64_t n, double *ms_ib, double *ms_lbm);
/* unstable[c] = 1 if case c's instability flag is set (array of n_cases, may
 * be NULL); *n_steps = batch steps taken. Synchronising. */
int btdf_batch_status(btdf_batch_t *b, int *unstable, int64_t *n_steps);
/* Options: BTDF_OPT_LBM_VARIANT, _GRAPH_CHUNK, _XCD_REMAP, _INTERIOR_PATH, _MASK_UNSTABLE, _ROW_ALIGN,
   _TEMPORAL_BLOCKING, _EDGE_TILES. */
int btdf_batch_set_option(btdf_batch_t *b, int key, int64_t value);
int btdf_batch_get_option(const btdf_batch_t *b, int key, int64_t *value);
/* As btdf_autotune, for the batched launches. */
int btdf_batch_autotune(btdf_batch_t *b, int64_t steps_per_trial, int *best_variant);

/* ---- reverse mode: gradients of a weighted force history ----
 * J = sum over the n steps t and bodies b of hist_bar[t][b] . (Fx, Fy, Tz)
 * of that step (eq 27): any weighting of the force history, e.g. the time
 * mean of the drag coefficient, hist_bar[t][b] = (2 / (rho0 U^2 D n), 0, 0).
 * btdf_adjoint takes the n steps exactly as btdf_step(n) would (same kernels,
 * same final state, same history ring), then sweeps back through Algorithm 1
 * (Section 2.4) step by step with the transposes of its parts: boundary
 * columns, collision (eqs 5-7, 11), body force (eq 27), spreading (eqs 13,
 * 15), direct force (eq 20), interpolation (eqs 12, 14), moments (eqs 9-10)
 * and streaming. States of the forward run are kept all (checkpoint_every
 * >= n: a tape, no recomputation) or every K-th (checkpoint_every = K; 0
 * picks ceil(sqrt(n))), the states between checkpoints being recomputed one
 * segment at a time; both give bit-identical gradients. The arithmetic runs
 * in the handle's precision; gradients are returned in FP64.
 *   hist_bar  [n][n_bodies][3] host, FP64 (may be NULL without bodies)
 *   grads     host arrays to fill; any member may be NULL:
 *     populations [9][ny][nx]  dJ/d(populations before the first step)
 *     inflow      [2]          dJ/d(inlet velocity of the ghost column); the
 *                              initial state is an input of its own
 *     body_force  [2]          dJ/dG (uniform body-force density)
 *     marker_xy   [n_markers][2]  dJ/d(marker positions), through phi' of the
 *                              delta function (LINEAR2: one-sided at its kink)
 *     marker_uv   [n_markers][2]  dJ/d(prescribed marker velocities)
 *     centres     [n_bodies][2]   dJ/d(body centres) through the torque only
 *                              (moving a body also moves its markers)
 *   work      device memory of btdf_adjoint_workspace_bytes bytes, 256-byte
 *             aligned, or NULL (the library allocates and frees it)
 *   ms        [3] or NULL: milliseconds (HIP events) of the forward run, of
 *             the recomputation (summed; with checkpoints it runs on a second
 *             stream under the reverse steps of the segment above) and of the
 *             whole reverse sweep, recomputation included
 * Synchronising. Errors: EINVAL, ENOMEM, EUNSTABLE (the run went unstable:
 * no gradient), EDEVICE. */
typedef struct btdf_gradients {
  double *populations;
  double *inflow;
  double *body_force;
  double *marker_xy;
  double *marker_uv;
  double *centres;
} btdf_gradients;
size_t btdf_adjoint_workspace_bytes(btdf_t *h, int64_t n_steps, int64_t checkpoint_every);
int btdf_adjoint(btdf_t *h, int64_t n_steps, int64_t checkpoint_every, const double *hist_bar,
                 btdf_gradients *grads, void *work, size_t work_bytes, double *ms);

/* Boundary-thickness calibration on the host (no device), Section 2.3, for
 * a circular body of diameter D with n_markers equally spaced markers
 * X_l = (D/2)(cos t_l, sin t_l), t_l = 2 pi l / n_markers, about a node, and
 * ds = pi D / n_markers: the calibration below on that ring. *drs_mean
 * receives drs/dh of eq 26, drs_per_marker (length n_markers, may be NULL)
 * the local values of eq 25. Errors: EINVAL (D <= 0, n_markers < 3, bad
 * kind, NULL drs_mean), ESTATE (A singular to working precision: markers
 * much denser than the grid). */
int btdf_calibrate_thickening(int delta_kind, double D, int n_markers, double *drs_mean,
                              double *drs_per_marker);

/* The same calibration for any marker set: A_ij = (1/dh^2) sum_k phi_ik
 * phi_kj dh ds (eq 22) over the stencil nodes of the n markers xy ([n][2],
 * host), drs_vec = dh A^{-1} 1 (eq 25) and drs = mean(drs_vec) (eq 26),
 * with dh = 1. *drs_mean receives the mean, drs_per_marker (length n, may be
 * NULL) the local values. Errors: EINVAL (n < 1, bad kind, ds <= 0), ESTATE
 * (A singular to working precision). */
int btdf_calibrate_thickening_markers(int delta_kind, int n, const double *xy, double ds,
                                      double *drs_mean, double *drs_per_marker);

#ifdef __cplusplus
}
#endif

#endif /* BTDF_H */
