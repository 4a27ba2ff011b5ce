/*
 * btdf_oracle.c -- plain FP64 CPU oracle for one time step of the
 * boundary-thickening direct-forcing immersed-boundary lattice Boltzmann
 * method (BTDF-IB-LBM; Jiang & Liu, arXiv 1806.09403).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. It shares no code with
 * the HIP library: its own D2Q9 tables, its own delta functions, its own
 * loops. Everything is double precision. Every loop is the plain form of
 * the equation it cites; there is no blocking, no fusion and no reordering
 * beyond Algorithm 1 (Section 2.4) with NF = 1:
 *
 *   stream -> moments (eqs 9-10 with the body force, eq 11) ->
 *   interpolation (eqs 12, 14) -> direct force (eq 20) ->
 *   spreading with the thickened shell (eqs 13, 15) ->
 *   hydrodynamic force on each body (eq 27) ->
 *   equilibrium (eq 6), Guo force term (eq 7), BGK collision (eq 5) ->
 *   boundary columns.
 *
 * The state between steps is the post-collision population A_q(x); the
 * streaming of Algorithm 1 (last item) is therefore done at the start of
 * the next pass, g_q(x) = A_q(x - e_q).
 *
 * Readings taken where the paper is silent (listed with reasons in the
 * design notes of the repository):
 *  - rho in eq 20 is the marker-interpolated density D_I rho;
 *  - the hydrodynamic force on a body is minus the force the markers apply
 *    to the fluid, F_p = -drs*ds*sum_l F_l (eq 27 with the sign that makes
 *    the drag positive), and the torque about the body centre is
 *    T = -drs*ds*sum_l (X_l - c) x F_l;
 *  - u* includes half of the uniform body force G, so the immersed
 *    boundary corrects the total velocity (eq 11 applied to G);
 *  - the equilibrium and the Guo term use the corrected velocity of eq 11;
 *  - boundary columns: a velocity inlet is a ghost column i = 0 set to the
 *    equilibrium at the inlet velocity with the density of column 1 after
 *    collision; a zero-gradient outlet is a ghost column i = nx-1 copied
 *    from column nx-2; walls (south/north only) are halfway bounce-back;
 *    periodic directions wrap the node index;
 *  - the far-field conditions of the cylinder runs (Section 5.2): a
 *    free-slip wall (du_x/dy = 0, u_y = 0) is a specular reflection
 *    halfway between the edge row and the wall, and a convective outlet
 *    advects the ghost column with the inflow speed, implicit upwind;
 *  - stencil nodes are all nodes whose distance to the marker lies inside
 *    the support of the delta function (weights at the edge are zero).
 *
 * Besides the direct force of eq 20 (with NF passes, eqs 29-31), the
 * comparison methods of Section 3 are available per step: the implicit
 * direct forcing of eq 17 (equal to the implicit velocity correction of
 * eqs 32-35, Appendix A), one dense solve per body with D_I D_E built from
 * eq 21, markers of different bodies not coupled; and RKPM (eq 36 / B54),
 * the direct force spread with epsilon_l = row sums of A^-1 (eq 22). The
 * hydrodynamic force is minus the total force spread into the fluid.
 *
 * Layout: populations are [q][j][i] with i (x) fastest; nodes sit at
 * integer coordinates (x, y) = (i, j); lattice units dh = dt = 1.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PERIODIC 0
#define ORC_VELOCITY_INLET 1
#define ORC_ZERO_GRADIENT_OUTLET 2
#define ORC_BOUNCEBACK_WALL 3
#define ORC_FREE_SLIP_WALL 4
#define ORC_CONVECTIVE_OUTLET 5

#define ORC_LINEAR2 2
#define ORC_ROMA3 3
#define ORC_PESKIN4 4
#define ORC_COS4 5

/* D2Q9 velocities and weights, eq 8 and the weights stated after eq 7. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Mirror image of q in a wall parallel to x: the q' with e_q' = (e_qx, -e_qy). */
static int mirror_y(int q) {
  for (int p = 0; p < 9; ++p)
    if (EX[p] == EX[q] && EY[p] == -EY[q]) return p;
  return -1;
}

/* Opposite direction of q: the q' with e_q' = -e_q. */
static int opposite(int q) {
  for (int p = 0; p < 9; ++p)
    if (EX[p] == -EX[q] && EY[p] == -EY[q]) return p;
  return -1;
}

/* Regularised delta functions, Section 4.3. */
double oracle_delta(int kind, double r) {
  double a = fabs(r);
  switch (kind) {
    case ORC_LINEAR2: /* eq 37 */
      return a <= 1.0 ? 1.0 - a : 0.0;
    case ORC_ROMA3: /* eq 38 */
      if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
      if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
      return 0.0;
    case ORC_PESKIN4: /* eq 39 */
      if (a < 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
      if (a < 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
      return 0.0;
    case ORC_COS4: /* cosine 4-point kernel, (1 + cos(pi r / 2)) / 4 on |r| <= 2 */
      return a <= 2.0 ? 0.25 * (1.0 + cos(M_PI * a / 2.0)) : 0.0;
    default:
      return NAN;
  }
}

/* Half-width of the support of each delta function (drf/dh / 2). */
double oracle_delta_halfwidth(int kind) {
  switch (kind) {
    case ORC_LINEAR2: return 1.0;
    case ORC_ROMA3: return 1.5;
    case ORC_PESKIN4: return 2.0;
    case ORC_COS4: return 2.0;
    default: return -1.0;
  }
}

typedef struct {
  int nx, ny;
  int bc[4]; /* west, east, south, north */
  double tau;
  int kind;
  double drs; /* thickening * dh, dh = 1 */
  double G[2];
  double uin[2];
  /* grid */
  double *A;  /* post-collision populations [9][ny][nx] */
  double *g;  /* streamed populations [9][ny][nx] (fluid nodes only) */
  double *rho, *mx, *my;  /* moments of g */
  double *ux, *uy;        /* corrected velocity of the last collision */
  double *fx, *fy;        /* spread IB force density of the last step */
  /* markers */
  int nm, nm_cap;
  double *X, *Y, *Ub, *Vb;
  double *rho_l, *ux_l, *uy_l; /* interpolated rho and u* */
  double *Fx, *Fy;             /* direct force, eq 20 */
  int *body_of;
  /* bodies */
  int nb, nb_cap;
  int *off; /* markers of body b are off[b] .. off[b+1]-1 */
  double *cx, *cy, *ds;
  double *force; /* [nb][3]: Fx, Fy, Tz on each body, last step */
  long steps;
  int unstable; /* 0 = fine; 1 + body for a marker trigger; -1 for a node */
  int nf;       /* forcing passes per step (Algorithm 1 step 3; 1 = BTDF as proposed) */
  double *usx, *usy; /* u*^k at every node during the passes */
  double *dFx, *dFy; /* force increment of the current pass, per marker */
  int method;        /* ORC_DIRECT, ORC_IMPLICIT (IDF = IVC) or ORC_RKPM */
  double *sl;        /* per marker: the factor the spreading applies to F_l */
  /* rigid motion: per body a moving flag, angle, velocity and angular
   * velocity; per marker the offset from the centre at angle 0 */
  int *moving;
  double *theta, *bvx, *bvy, *bom;
  double *rx, *ry;
} oracle_t;

#define ORC_DIRECT 0
#define ORC_IMPLICIT 1
#define ORC_RKPM 2

static size_t nnode(const oracle_t *o) { return (size_t)o->nx * (size_t)o->ny; }
static size_t idx(const oracle_t *o, int q, int j, int i) {
  return ((size_t)q * o->ny + j) * o->nx + i;
}
static int x_periodic(const oracle_t *o) { return o->bc[0] == ORC_PERIODIC; }
static int y_periodic(const oracle_t *o) { return o->bc[2] == ORC_PERIODIC; }
/* Fluid columns: every column if x is periodic, else 1 .. nx-2 (ghosts at the ends). */
static int i_first(const oracle_t *o) { return x_periodic(o) ? 0 : 1; }
static int i_last(const oracle_t *o) { return x_periodic(o) ? o->nx - 1 : o->nx - 2; }
static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Equilibrium distribution, eq 6 with c = 1. */
static double feq(int q, double rho, double ux, double uy) {
  double eu = EX[q] * ux + EY[q] * uy;
  double uu = ux * ux + uy * uy;
  return WQ[q] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

oracle_t *oracle_create(int nx, int ny, const int *bc, double tau, int kind,
                        double thickening, double Gx, double Gy, double uin_x,
                        double uin_y, double rho0, double ux0, double uy0) {
  oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
  if (!o) return NULL;
  o->nx = nx;
  o->ny = ny;
  memcpy(o->bc, bc, 4 * sizeof(int));
  o->tau = tau;
  o->kind = kind;
  o->drs = thickening;
  o->G[0] = Gx;
  o->G[1] = Gy;
  o->uin[0] = uin_x;
  o->uin[1] = uin_y;
  size_t n = nnode(o);
  o->A = (double *)malloc(9 * n * sizeof(double));
  o->g = (double *)calloc(9 * n, sizeof(double));
  o->rho = (double *)calloc(n, sizeof(double));
  o->mx = (double *)calloc(n, sizeof(double));
  o->my = (double *)calloc(n, sizeof(double));
  o->ux = (double *)calloc(n, sizeof(double));
  o->uy = (double *)calloc(n, sizeof(double));
  o->fx = (double *)calloc(n, sizeof(double));
  o->fy = (double *)calloc(n, sizeof(double));
  o->off = (int *)calloc(1, sizeof(int));
  o->nf = 1;
  o->usx = (double *)calloc(n, sizeof(double));
  o->usy = (double *)calloc(n, sizeof(double));
  if (!o->A || !o->g || !o->rho || !o->mx || !o->my || !o->ux || !o->uy ||
      !o->fx || !o->fy || !o->off || !o->usx || !o->usy) {
    free(o);
    return NULL;
  }
  /* Initial state: equilibrium at (rho0, u0) everywhere, ghost columns included. */
  for (int q = 0; q < 9; ++q)
    for (size_t k = 0; k < n; ++k) o->A[(size_t)q * n + k] = feq(q, rho0, ux0, uy0);
  return o;
}

void oracle_destroy(oracle_t *o) {
  if (!o) return;
  free(o->A); free(o->g); free(o->rho); free(o->mx); free(o->my);
  free(o->ux); free(o->uy); free(o->fx); free(o->fy);
  free(o->X); free(o->Y); free(o->Ub); free(o->Vb);
  free(o->rho_l); free(o->ux_l); free(o->uy_l); free(o->Fx); free(o->Fy);
  free(o->body_of); free(o->off); free(o->cx); free(o->cy); free(o->ds);
  free(o->force);
  free(o->usx); free(o->usy); free(o->dFx); free(o->dFy); free(o->sl);
  free(o->rx); free(o->ry); free(o->moving); free(o->theta); free(o->bvx); free(o->bvy); free(o->bom);
  free(o);
}

/* Forcing passes per step (Algorithm 1 step 3 with NF passes: the multi
 * direct forcing of eqs 29-31 on the thickened spreading). */
void oracle_set_forcing_passes(oracle_t *o, int nf) { o->nf = nf < 1 ? 1 : nf; }

/* How the marker force is formed and spread: ORC_DIRECT (eq 20, the
 * default), ORC_IMPLICIT (eq 17: the implicit direct forcing, which
 * Appendix A shows is the implicit velocity correction of eqs 32-35) or
 * ORC_RKPM (eq 20 spread with the corrected operator of eq 36 / B54). */
void oracle_set_forcing_method(oracle_t *o, int method) { o->method = method; }

static int grow_markers(oracle_t *o, int need) {
  if (need <= o->nm_cap) return 0;
  int cap = need * 2;
  double **arrs[] = {&o->X, &o->Y, &o->Ub, &o->Vb, &o->rho_l, &o->ux_l, &o->uy_l, &o->Fx, &o->Fy,
                     &o->dFx, &o->dFy, &o->sl, &o->rx, &o->ry};
  for (int a = 0; a < 14; ++a) {
    double *p = (double *)realloc(*arrs[a], (size_t)cap * sizeof(double));
    if (!p) return -1;
    *arrs[a] = p;
  }
  int *b = (int *)realloc(o->body_of, (size_t)cap * sizeof(int));
  if (!b) return -1;
  o->body_of = b;
  o->nm_cap = cap;
  return 0;
}

/* Append one body of n markers. xy, uv are [n][2]; uv may be NULL (at rest).
 * Returns the body id, or -1. No validation: the tests only feed valid bodies. */
int oracle_add_body(oracle_t *o, int n, const double *xy, const double *uv,
                    double cx, double cy, double ds) {
  if (grow_markers(o, o->nm + n)) return -1;
  int b = o->nb;
  int *off = (int *)realloc(o->off, (size_t)(b + 2) * sizeof(int));
  double *pcx = (double *)realloc(o->cx, (size_t)(b + 1) * sizeof(double));
  double *pcy = (double *)realloc(o->cy, (size_t)(b + 1) * sizeof(double));
  double *pds = (double *)realloc(o->ds, (size_t)(b + 1) * sizeof(double));
  double *pf = (double *)realloc(o->force, (size_t)(b + 1) * 3 * sizeof(double));
  if (!off || !pcx || !pcy || !pds || !pf) return -1;
  o->off = off; o->cx = pcx; o->cy = pcy; o->ds = pds; o->force = pf;
  int *mv = (int *)realloc(o->moving, (size_t)(b + 1) * sizeof(int));
  if (!mv) return -1;
  o->moving = mv;
  double **barrs[] = {&o->theta, &o->bvx, &o->bvy, &o->bom};
  for (int a = 0; a < 4; ++a) {
    double *q = (double *)realloc(*barrs[a], (size_t)(b + 1) * sizeof(double));
    if (!q) return -1;
    *barrs[a] = q;
  }
  o->moving[b] = 0;
  o->theta[b] = o->bvx[b] = o->bvy[b] = o->bom[b] = 0.0;
  for (int l = 0; l < n; ++l) {
    int m = o->nm + l;
    o->X[m] = xy[2 * l];
    o->Y[m] = xy[2 * l + 1];
    o->Ub[m] = uv ? uv[2 * l] : 0.0;
    o->Vb[m] = uv ? uv[2 * l + 1] : 0.0;
    o->rho_l[m] = o->ux_l[m] = o->uy_l[m] = o->Fx[m] = o->Fy[m] = 0.0;
    o->body_of[m] = b;
    o->rx[m] = xy[2 * l] - cx;
    o->ry[m] = xy[2 * l + 1] - cy;
  }
  o->off[b] = o->nm;
  o->nm += n;
  o->off[b + 1] = o->nm;
  o->cx[b] = cx;
  o->cy[b] = cy;
  o->ds[b] = ds;
  o->force[3 * b] = o->force[3 * b + 1] = o->force[3 * b + 2] = 0.0;
  o->nb += 1;
  return b;
}

void oracle_set_marker_velocity(oracle_t *o, int b, const double *uv) {
  for (int m = o->off[b]; m < o->off[b + 1]; ++m) {
    int l = m - o->off[b];
    o->Ub[m] = uv[2 * l];
    o->Vb[m] = uv[2 * l + 1];
  }
}

/* Rigid motion of body b (eq 4 for a rigid body whose surface moves with
 * the fluid it carries): from now on the body translates with (vx, vy) and
 * turns with omega (counter-clockwise, per step) about its centre. The
 * markers' prescribed velocity becomes the rigid field at once,
 * U_l = V + omega x (X_l - c); after every step the centre and angle
 * advance by one step and the markers are placed at c + R(theta) r_l, with
 * r_l their offsets from the centre when the body was added. */
static void rigid_markers(oracle_t *o, int b) {
  double c = cos(o->theta[b]), s = sin(o->theta[b]);
  for (int m = o->off[b]; m < o->off[b + 1]; ++m) {
    o->X[m] = o->cx[b] + c * o->rx[m] - s * o->ry[m];
    o->Y[m] = o->cy[b] + s * o->rx[m] + c * o->ry[m];
    o->Ub[m] = o->bvx[b] - o->bom[b] * (o->Y[m] - o->cy[b]);
    o->Vb[m] = o->bvy[b] + o->bom[b] * (o->X[m] - o->cx[b]);
  }
}

void oracle_set_body_motion(oracle_t *o, int b, double vx, double vy, double omega) {
  o->moving[b] = 1;
  o->bvx[b] = vx;
  o->bvy[b] = vy;
  o->bom[b] = omega;
  for (int m = o->off[b]; m < o->off[b + 1]; ++m) {
    o->Ub[m] = vx - omega * (o->Y[m] - o->cy[b]);
    o->Vb[m] = vy + omega * (o->X[m] - o->cx[b]);
  }
}

/* (cx, cy, theta, vx, vy, omega) of body b. */
void oracle_body_state(const oracle_t *o, int b, double *out) {
  out[0] = o->cx[b]; out[1] = o->cy[b]; out[2] = o->theta[b];
  out[3] = o->bvx[b]; out[4] = o->bvy[b]; out[5] = o->bom[b];
}

void oracle_get_marker_positions(const oracle_t *o, double *xy) {
  for (int m = 0; m < o->nm; ++m) {
    xy[2 * m] = o->X[m];
    xy[2 * m + 1] = o->Y[m];
  }
}

static void move_bodies(oracle_t *o) {
  for (int b = 0; b < o->nb; ++b) {
    if (!o->moving[b]) continue;
    o->cx[b] += o->bvx[b];
    o->cy[b] += o->bvy[b];
    o->theta[b] += o->bom[b];
    rigid_markers(o, b);
  }
}

/* Streaming (Algorithm 1, last item, applied at the start of the next pass):
 * g_q(x) = A_q(x - e_q) at every fluid node, with the boundary readings above. */
static void stream(oracle_t *o) {
  int nx = o->nx, ny = o->ny;
  int i0 = i_first(o), i1 = i_last(o);
  for (int q = 0; q < 9; ++q) {
    int qb = opposite(q);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
      for (int i = i0; i <= i1; ++i) {
        int sj = j - EY[q];
        int si = i - EX[q];
        double val;
        if (sj < 0 || sj >= ny) {
          if (y_periodic(o)) {
            sj = wrap(sj, ny);
            if (x_periodic(o)) si = wrap(si, nx);
            val = o->A[idx(o, q, sj, si)];
          } else if (o->bc[sj < 0 ? 2 : 3] == ORC_FREE_SLIP_WALL) {
            /* specular reflection halfway between the edge row and the wall:
             * the population that left the neighbouring column towards the
             * wall returns with its normal component reversed */
            if (x_periodic(o)) si = wrap(si, nx);
            val = o->A[idx(o, mirror_y(q), j, si)];
          } else {
            /* halfway bounce-back: the population that left towards the wall returns */
            val = o->A[idx(o, qb, j, i)];
          }
        } else {
          if (x_periodic(o)) si = wrap(si, nx);
          val = o->A[idx(o, q, sj, si)];
        }
        o->g[idx(o, q, j, i)] = val;
      }
    }
  }
}

/* Zeroth and first moments of g (eqs 9-10). */
static void moments(oracle_t *o) {
  int i0 = i_first(o), i1 = i_last(o);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < o->ny; ++j) {
    for (int i = i0; i <= i1; ++i) {
      double r = 0.0, mx = 0.0, my = 0.0;
      for (int q = 0; q < 9; ++q) {
        double v = o->g[idx(o, q, j, i)];
        r += v;
        mx += EX[q] * v;
        my += EY[q] * v;
      }
      size_t k = (size_t)j * o->nx + i;
      o->rho[k] = r;
      o->mx[k] = mx;
      o->my[k] = my;
    }
  }
}

/* Node memory index of the (possibly out-of-range) integer coordinate (i, j):
 * periodic directions wrap; the tests keep non-periodic stencils inside the grid. */
static size_t node_of(const oracle_t *o, int i, int j) {
  if (x_periodic(o)) i = wrap(i, o->nx);
  if (y_periodic(o)) j = wrap(j, o->ny);
  return (size_t)j * o->nx + i;
}

/* Sum over the grid nodes k of W_lk W_mk, the weights of markers l and m at
 * node k (the node sum of eqs 21-22, with dh = 1). Node offsets from marker
 * m take the nearest periodic image. */
static double pair_weight(const oracle_t *o, int l, int m) {
  double h = oracle_delta_halfwidth(o->kind), s = 0.0;
  for (int j = (int)ceil(o->Y[l] - h); j <= (int)floor(o->Y[l] + h); ++j) {
    for (int i = (int)ceil(o->X[l] - h); i <= (int)floor(o->X[l] + h); ++i) {
      double dx = i - o->X[m], dy = j - o->Y[m];
      if (x_periodic(o)) dx -= o->nx * floor(dx / o->nx + 0.5);
      if (y_periodic(o)) dy -= o->ny * floor(dy / o->ny + 0.5);
      s += oracle_delta(o->kind, i - o->X[l]) * oracle_delta(o->kind, j - o->Y[l]) *
           oracle_delta(o->kind, dx) * oracle_delta(o->kind, dy);
    }
  }
  return s;
}

/* The matrix A of eq 22 (drs = dh) of body b, n x n row-major. */
static double *body_matrix_A(const oracle_t *o, int b, int *n_out) {
  int l0 = o->off[b], n = o->off[b + 1] - l0;
  double *A = (double *)malloc((size_t)n * n * sizeof(double));
  if (A)
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) A[(size_t)r * n + c] = o->ds[b] * pair_weight(o, l0 + r, l0 + c);
  *n_out = n;
  return A;
}

/* Solve M X = B in place for k right-hand sides (B is n x k, row-major) by
 * Gaussian elimination with partial pivoting; M is destroyed. Returns -1 on a
 * zero pivot. */
static int gauss_solve(double *M, double *B, int n, int k) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[(size_t)r * n + c]) > fabs(M[(size_t)p * n + c])) p = r;
    if (M[(size_t)p * n + c] == 0.0) return -1;
    if (p != c) {
      for (int t = 0; t < n; ++t) {
        double v = M[(size_t)c * n + t]; M[(size_t)c * n + t] = M[(size_t)p * n + t]; M[(size_t)p * n + t] = v;
      }
      for (int t = 0; t < k; ++t) {
        double v = B[(size_t)c * k + t]; B[(size_t)c * k + t] = B[(size_t)p * k + t]; B[(size_t)p * k + t] = v;
      }
    }
    for (int r = c + 1; r < n; ++r) {
      double f = M[(size_t)r * n + c] / M[(size_t)c * n + c];
      for (int t = c; t < n; ++t) M[(size_t)r * n + t] -= f * M[(size_t)c * n + t];
      for (int t = 0; t < k; ++t) B[(size_t)r * k + t] -= f * B[(size_t)c * k + t];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int t = 0; t < k; ++t) {
      double v = B[(size_t)c * k + t];
      for (int r = c + 1; r < n; ++r) v -= M[(size_t)c * n + r] * B[(size_t)r * k + t];
      B[(size_t)c * k + t] = v / M[(size_t)c * n + c];
    }
  }
  return 0;
}

/* Interpolation (eqs 12, 14) and eq 20 at every marker, then the implicit
 * force of eq 17 or the RKPM factors of eq B54, spreading, per-marker
 * spreading factors left in sl. */
static void implicit_or_rkpm(oracle_t *o) {
  double h = oracle_delta_halfwidth(o->kind);
  for (int m = 0; m < o->nm; ++m) {
    double X = o->X[m], Y = o->Y[m], rl = 0.0, ul = 0.0, vl = 0.0;
    for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
      for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
        double W = oracle_delta(o->kind, i - X) * oracle_delta(o->kind, j - Y);
        size_t k = node_of(o, i, j);
        rl += W * o->rho[k];
        ul += W * o->usx[k];
        vl += W * o->usy[k];
      }
    }
    o->rho_l[m] = rl;
    o->ux_l[m] = ul;
    o->uy_l[m] = vl;
    if (!(sqrt(ul * ul + vl * vl) <= 0.3) && o->unstable == 0) o->unstable = 1 + o->body_of[m];
    o->Fx[m] = 2.0 * rl * (o->Ub[m] - ul); /* eq 20; eq 17's right-hand side */
    o->Fy[m] = 2.0 * rl * (o->Vb[m] - vl);
  }
  for (int b = 0; b < o->nb; ++b) {
    int n, l0 = o->off[b];
    double *A = body_matrix_A(o, b, &n);
    if (!A) { o->unstable = 1 + b; continue; }
    if (o->method == ORC_IMPLICIT) {
      /* eq 17: (D_I D_E) F_b = 2 rho (U_b - D_I u*), with D_I D_E = drs A (eq 21) */
      double *rhs = (double *)malloc((size_t)n * 2 * sizeof(double));
      if (!rhs) { free(A); o->unstable = 1 + b; continue; }
      for (int r = 0; r < n; ++r) {
        rhs[2 * r] = o->Fx[l0 + r];
        rhs[2 * r + 1] = o->Fy[l0 + r];
      }
      for (size_t t = 0; t < (size_t)n * n; ++t) A[t] *= o->drs;
      if (gauss_solve(A, rhs, n, 2)) o->unstable = 1 + b;
      for (int r = 0; r < n; ++r) {
        o->Fx[l0 + r] = rhs[2 * r];
        o->Fy[l0 + r] = rhs[2 * r + 1];
        o->sl[l0 + r] = o->drs * o->ds[b];
      }
      free(rhs);
    } else {
      /* eq B54: epsilon_l = sum of row l of A^-1; the spreading D_EI epsilon */
      double *inv = (double *)calloc((size_t)n * n, sizeof(double));
      if (!inv) { free(A); o->unstable = 1 + b; continue; }
      for (int r = 0; r < n; ++r) inv[(size_t)r * n + r] = 1.0;
      if (gauss_solve(A, inv, n, n)) o->unstable = 1 + b;
      for (int r = 0; r < n; ++r) {
        double e = 0.0;
        for (int c = 0; c < n; ++c) e += inv[(size_t)r * n + c];
        o->sl[l0 + r] = o->ds[b] * e;
      }
      free(inv);
    }
    free(A);
  }
  for (int m = 0; m < o->nm; ++m) {
    int bad = !isfinite(o->Fx[m]) || !isfinite(o->Fy[m]);
    if (bad && o->unstable == 0) o->unstable = 1 + o->body_of[m];
    double X = o->X[m], Y = o->Y[m];
    for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
      for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
        double W = oracle_delta(o->kind, i - X) * oracle_delta(o->kind, j - Y);
        size_t k = node_of(o, i, j);
        o->fx[k] += W * o->sl[m] * o->Fx[m];
        o->fy[k] += W * o->sl[m] * o->Fy[m];
      }
    }
  }
}

/* Interpolation (eqs 12, 14), direct force (eq 20), spreading (eqs 13, 15)
 * and hydrodynamic force and torque (eq 27) for every marker, in NF forcing
 * passes (Algorithm 1 step 3; eqs 29-31 when NF > 1):
 *   u*^0 = u* (with G/2), F_b = 0, f = 0;
 *   for each pass: dF_l = 2 rho_l (U_b,l - D_I u*^{k-1}) (eq 20 / eq 29),
 *   F_b += dF, df = D_E dF (eqs 13, 15), f += df,
 *   u*^k = u*^{k-1} + df / (2 rho) at every node (eq 11 / eq 30).
 * rho_l = D_I rho is the same in every pass. Within a pass all markers see
 * the same u*^{k-1} (the interpolation of every marker happens before any
 * spreading). The marker data keep the first pass's rho_l and u*_l. */
static void immersed_boundary(oracle_t *o) {
  size_t n = nnode(o);
  double h = oracle_delta_halfwidth(o->kind);
  for (size_t k = 0; k < n; ++k) {
    o->fx[k] = o->fy[k] = 0.0;
    o->usx[k] = (o->mx[k] + 0.5 * o->G[0]) / o->rho[k]; /* u* with G/2 */
    o->usy[k] = (o->my[k] + 0.5 * o->G[1]) / o->rho[k];
  }
  for (int m = 0; m < o->nm; ++m) o->Fx[m] = o->Fy[m] = 0.0;

  for (int pass = 0; pass < (o->method == ORC_DIRECT ? o->nf : 0); ++pass) {
    /* interpolation + direct force increment */
    for (int m = 0; m < o->nm; ++m) {
      double X = o->X[m], Y = o->Y[m];
      double rl = 0.0, ul = 0.0, vl = 0.0;
      for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
        for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
          double W = oracle_delta(o->kind, i - X) * oracle_delta(o->kind, j - Y);
          size_t k = node_of(o, i, j);
          rl += W * o->rho[k];
          ul += W * o->usx[k];
          vl += W * o->usy[k];
        }
      }
      if (pass == 0) {
        o->rho_l[m] = rl;
        o->ux_l[m] = ul;
        o->uy_l[m] = vl;
        int bad = !(sqrt(ul * ul + vl * vl) <= 0.3);
        if (bad && o->unstable == 0) o->unstable = 1 + o->body_of[m];
      }
      rl = o->rho_l[m];
      o->dFx[m] = 2.0 * rl * (o->Ub[m] - ul); /* eq 20 / eq 29, dt = 1 */
      o->dFy[m] = 2.0 * rl * (o->Vb[m] - vl);
      o->Fx[m] += o->dFx[m];
      o->Fy[m] += o->dFy[m];
      int bad = !isfinite(o->Fx[m]) || !isfinite(o->Fy[m]);
      if (bad && o->unstable == 0) o->unstable = 1 + o->body_of[m];
    }
    /* spreading of the increment with the thickened solid shell:
     * df(x_k) += W dF_l drs ds / dh^2; then u*^k = u*^{k-1} + df / (2 rho) */
    for (int m = 0; m < o->nm; ++m) {
      double X = o->X[m], Y = o->Y[m];
      double s = o->drs * o->ds[o->body_of[m]];
      for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
        for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
          double W = oracle_delta(o->kind, i - X) * oracle_delta(o->kind, j - Y);
          size_t k = node_of(o, i, j);
          double dfx = W * o->dFx[m] * s, dfy = W * o->dFy[m] * s;
          o->fx[k] += dfx;
          o->fy[k] += dfy;
          o->usx[k] += 0.5 * dfx / o->rho[k];
          o->usy[k] += 0.5 * dfy / o->rho[k];
        }
      }
    }
  }

  if (o->method != ORC_DIRECT) implicit_or_rkpm(o);

  /* force and torque on each body: minus what its markers apply to the fluid */
  for (int b = 0; b < o->nb; ++b) {
    double sx = 0.0, sy = 0.0, tz = 0.0;
    for (int m = o->off[b]; m < o->off[b + 1]; ++m) {
      /* RKPM spreads s_l F_l with a factor of its own per marker */
      double w = o->method == ORC_RKPM ? o->sl[m] : 1.0;
      sx += w * o->Fx[m];
      sy += w * o->Fy[m];
      tz += w * ((o->X[m] - o->cx[b]) * o->Fy[m] - (o->Y[m] - o->cy[b]) * o->Fx[m]);
    }
    double s = o->method == ORC_RKPM ? 1.0 : o->drs * o->ds[b];
    o->force[3 * b] = -s * sx;
    o->force[3 * b + 1] = -s * sy;
    o->force[3 * b + 2] = -s * tz;
  }
}

/* Corrected velocity (eq 11), equilibrium (eq 6), Guo force (eq 7) and the
 * BGK collision (eq 5) at every fluid node, written into A. */
static void collide(oracle_t *o) {
  int i0 = i_first(o), i1 = i_last(o);
  double tau = o->tau;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int j = 0; j < o->ny; ++j) {
    for (int i = i0; i <= i1; ++i) {
      size_t k = (size_t)j * o->nx + i;
      double r = o->rho[k];
      double ftx = o->G[0] + o->fx[k];
      double fty = o->G[1] + o->fy[k];
      double ux = (o->mx[k] + 0.5 * ftx) / r;
      double uy = (o->my[k] + 0.5 * fty) / r;
      o->ux[k] = ux;
      o->uy[k] = uy;
      if (!(r > 0.0) || !isfinite(r)) bad = 1;
      for (int q = 0; q < 9; ++q) {
        double eu = EX[q] * ux + EY[q] * uy;
        double Fq = (1.0 - 1.0 / (2.0 * tau)) * WQ[q] *
                    ((3.0 * (EX[q] - ux) + 9.0 * eu * EX[q]) * ftx +
                     (3.0 * (EY[q] - uy) + 9.0 * eu * EY[q]) * fty);
        double gq = o->g[idx(o, q, j, i)];
        o->A[idx(o, q, j, i)] = gq - (gq - feq(q, r, ux, uy)) / tau + Fq;
      }
    }
  }
  if (bad && o->unstable == 0) o->unstable = -1;
}

/* Ghost columns of the channel: velocity inlet and zero-gradient outlet. */
static void boundary_columns(oracle_t *o) {
  int nx = o->nx;
  if (o->bc[0] == ORC_VELOCITY_INLET) {
    for (int j = 0; j < o->ny; ++j) {
      double r = 0.0;
      for (int q = 0; q < 9; ++q) r += o->A[idx(o, q, j, 1)];
      for (int q = 0; q < 9; ++q) o->A[idx(o, q, j, 0)] = feq(q, r, o->uin[0], o->uin[1]);
    }
  }
  if (o->bc[1] == ORC_ZERO_GRADIENT_OUTLET) {
    for (int j = 0; j < o->ny; ++j)
      for (int q = 0; q < 9; ++q) o->A[idx(o, q, j, nx - 1)] = o->A[idx(o, q, j, nx - 2)];
  }
  if (o->bc[1] == ORC_CONVECTIVE_OUTLET) {
    /* d(phi)/dt + U d(phi)/dx = 0 at the outlet, implicit upwind in time
     * and space with U the inflow speed: phi_N(t+1) = (phi_N(t) + U phi_{N-1}(t+1)) / (1 + U) */
    double U = o->uin[0];
    for (int j = 0; j < o->ny; ++j)
      for (int q = 0; q < 9; ++q)
        o->A[idx(o, q, j, nx - 1)] = (o->A[idx(o, q, j, nx - 1)] + U * o->A[idx(o, q, j, nx - 2)]) / (1.0 + U);
  }
}

void oracle_step(oracle_t *o, long n) {
  for (long s = 0; s < n; ++s) {
    stream(o);
    moments(o);
    immersed_boundary(o);
    collide(o);
    boundary_columns(o);
    move_bodies(o);
    o->steps += 1;
  }
}

/* Replace the state by the equilibrium of the given fields ([ny][nx] each;
 * rho may be NULL for rho = 1). Clears the instability flag. */
void oracle_init_equilibrium(oracle_t *o, const double *rho, const double *ux, const double *uy) {
  size_t n = nnode(o);
  for (int q = 0; q < 9; ++q)
    for (size_t k = 0; k < n; ++k)
      o->A[(size_t)q * n + k] = feq(q, rho ? rho[k] : 1.0, ux[k], uy[k]);
  o->unstable = 0;
}

void oracle_get_populations(const oracle_t *o, double *dst) {
  memcpy(dst, o->A, 9 * nnode(o) * sizeof(double));
}

void oracle_set_populations(oracle_t *o, const double *src) {
  memcpy(o->A, src, 9 * nnode(o) * sizeof(double));
  o->unstable = 0;
}

/* Macroscopic state of the current populations: at fluid nodes, rho and
 * u* = (sum e g + G/2) / rho of the streamed populations; at ghost columns,
 * plain moments of A at the ghost node. */
void oracle_get_macroscopic(oracle_t *o, double *rho, double *ux, double *uy) {
  stream(o);
  moments(o);
  int nx = o->nx;
  for (int j = 0; j < o->ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      if (i < i_first(o) || i > i_last(o)) {
        double r = 0.0, mx = 0.0, my = 0.0;
        for (int q = 0; q < 9; ++q) {
          double v = o->A[idx(o, q, j, i)];
          r += v;
          mx += EX[q] * v;
          my += EY[q] * v;
        }
        rho[k] = r;
        ux[k] = mx / r;
        uy[k] = my / r;
      } else {
        rho[k] = o->rho[k];
        ux[k] = (o->mx[k] + 0.5 * o->G[0]) / o->rho[k];
        uy[k] = (o->my[k] + 0.5 * o->G[1]) / o->rho[k];
      }
    }
  }
}

/* Per-marker quantities of the last step: interpolated rho and u*, and F_l. */
void oracle_marker_data(const oracle_t *o, double *rho_l, double *ux_l, double *uy_l,
                        double *Fx, double *Fy) {
  for (int m = 0; m < o->nm; ++m) {
    rho_l[m] = o->rho_l[m];
    ux_l[m] = o->ux_l[m];
    uy_l[m] = o->uy_l[m];
    Fx[m] = o->Fx[m];
    Fy[m] = o->Fy[m];
  }
}

/* Velocity at the markers after forcing: D_I applied to the corrected
 * velocity u of eq 11 from the last collision. Feeds the boundary error of
 * eq 45. */
void oracle_marker_corrected_velocity(const oracle_t *o, double *ux_c, double *uy_c) {
  double h = oracle_delta_halfwidth(o->kind);
  for (int m = 0; m < o->nm; ++m) {
    double X = o->X[m], Y = o->Y[m], su = 0.0, sv = 0.0;
    for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
      for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
        double W = oracle_delta(o->kind, i - X) * oracle_delta(o->kind, j - Y);
        size_t k = node_of(o, i, j);
        su += W * o->ux[k];
        sv += W * o->uy[k];
      }
    }
    ux_c[m] = su;
    uy_c[m] = sv;
  }
}

void oracle_get_force_field(const oracle_t *o, double *fx, double *fy) {
  memcpy(fx, o->fx, nnode(o) * sizeof(double));
  memcpy(fy, o->fy, nnode(o) * sizeof(double));
}

void oracle_body_forces(const oracle_t *o, double *out) {
  memcpy(out, o->force, (size_t)o->nb * 3 * sizeof(double));
}

int oracle_unstable(const oracle_t *o) { return o->unstable; }
long oracle_steps(const oracle_t *o) { return o->steps; }
int oracle_num_markers(const oracle_t *o) { return o->nm; }
int oracle_num_bodies(const oracle_t *o) { return o->nb; }

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the parallel loops use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set the threads of the parallel loops (n >= 1). Results do not depend on
 * it: the marker loops are serial and every node is written by one thread. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ======================================================================
 * Reverse mode. The step above is a differentiable map
 *   A_{t+1} = Step(A_t; U_b, X, c, u_in, G)
 * that also emits the body forces h_t (Fx, Fy, Tz per body, eq 27). For a
 * scalar J = sum_t sum_b hbar_t . h_t (hbar given), oracle_adjoint returns
 * dJ/dA_0, dJ/du_in, dJ/dG, dJ/dX_l, dJ/dU_b,l and dJ/dc_b (the centre
 * enters the torque only). It runs the n forward steps keeping every state
 * (a full tape: the oracle is for small grids), then walks back through the
 * steps, each time recomputing the step's intermediates from its stored
 * state and applying the transposes of its parts in reverse order:
 *   boundary columns -> collision (eqs 5-7, 11) -> body force (eq 27) ->
 *   spreading (eqs 13, 15) -> direct force (eq 20) -> interpolation
 *   (eqs 12, 14) -> u* of the moments -> moments (eqs 9-10) -> streaming.
 * Positions enter through the weights W_lk = phi(x_k - X_l) phi(y_k - Y_l),
 * whose derivative uses phi' (oracle_delta_deriv).
 * ====================================================================== */

/* d phi / d r of the delta functions of Section 4.3 (one-sided 0 outside
 * the support; LINEAR2 takes -sign(r), its kink at r = 0 having no
 * derivative). */
double oracle_delta_deriv(int kind, double r) {
  double a = fabs(r), s = r < 0.0 ? -1.0 : 1.0;
  switch (kind) {
    case ORC_LINEAR2:
      return a < 1.0 ? -s : 0.0;
    case ORC_ROMA3:
      if (a <= 0.5) return s * (-a / sqrt(1.0 - 3.0 * a * a));
      if (a < 1.5) {
        double b = 1.0 - a;
        return s * (-3.0 - 3.0 * b / sqrt(1.0 - 3.0 * b * b)) / 6.0;
      }
      return 0.0;
    case ORC_PESKIN4:
      if (a < 1.0) return s * (-2.0 + (2.0 - 4.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
      if (a < 2.0) return s * (-2.0 - (6.0 - 4.0 * a) / sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
      return 0.0;
    case ORC_COS4:
      return a <= 2.0 ? -s * (M_PI / 8.0) * sin(M_PI * a / 2.0) : 0.0;
    default:
      return NAN;
  }
}

/* Where the streaming of node (i, j), direction q, reads A: the element
 * index of the source (see stream()). */
static size_t stream_source(const oracle_t *o, int q, int j, int i) {
  int sj = j - EY[q], si = i - EX[q];
  if (sj < 0 || sj >= o->ny) {
    if (y_periodic(o)) {
      sj = wrap(sj, o->ny);
      if (x_periodic(o)) si = wrap(si, o->nx);
      return idx(o, q, sj, si);
    }
    return idx(o, opposite(q), j, i);
  }
  if (x_periodic(o)) si = wrap(si, o->nx);
  return idx(o, q, sj, si);
}

/* d feq_q / d rho at fixed u, and d feq_q / d u at fixed rho (eq 6). */
static double feq_drho(int q, double ux, double uy) { return feq(q, 1.0, ux, uy); }
static void feq_du(int q, double rho, double ux, double uy, double *dx, double *dy) {
  double eu = EX[q] * ux + EY[q] * uy;
  *dx = WQ[q] * rho * (3.0 * EX[q] + 9.0 * eu * EX[q] - 3.0 * ux);
  *dy = WQ[q] * rho * (3.0 * EY[q] + 9.0 * eu * EY[q] - 3.0 * uy);
}

/* n steps forward from the current state (the state advances by n, as with
 * oracle_step), then the reverse sweep. hist_bar is [n][nb][3]; every
 * output may be NULL; outputs are overwritten, not accumulated:
 * pop_bar [9][ny][nx], inflow_bar [2], force_bar [2], xy_bar [nm][2],
 * uv_bar [nm][2], centre_bar [nb][2]. Returns 0, or -1 when memory fails
 * or the forward run went unstable. */
int oracle_adjoint(oracle_t *o, long n, const double *hist_bar, double *pop_bar,
                   double *inflow_bar, double *force_bar, double *xy_bar, double *uv_bar,
                   double *centre_bar) {
  const size_t N = nnode(o), S = 9 * N;
  const int nx = o->nx, ny = o->ny, nb = o->nb, nm = o->nm;
  const int i0 = i_first(o), i1 = i_last(o);
  const double tau = o->tau, h = oracle_delta_halfwidth(o->kind);
  double *tape = (double *)malloc((size_t)(n + 1) * S * sizeof(double));
  double *hist = (double *)malloc((size_t)(n > 0 ? n : 1) * (nb > 0 ? nb : 1) * 3 * sizeof(double));
  double *Abar = (double *)calloc(S, sizeof(double));
  double *Bbar = (double *)malloc(S * sizeof(double));
  double *gbar = (double *)malloc(S * sizeof(double));
  double *fbx = (double *)malloc(N * sizeof(double)), *fby = (double *)malloc(N * sizeof(double));
  double *Fbx = (double *)malloc((size_t)(nm > 0 ? nm : 1) * sizeof(double));
  double *Fby = (double *)malloc((size_t)(nm > 0 ? nm : 1) * sizeof(double));
  double gin[2] = {0.0, 0.0}, gG[2] = {0.0, 0.0};
  double *gxy = (double *)calloc((size_t)(nm > 0 ? nm : 1) * 2, sizeof(double));
  double *guv = (double *)calloc((size_t)(nm > 0 ? nm : 1) * 2, sizeof(double));
  double *gc = (double *)calloc((size_t)(nb > 0 ? nb : 1) * 2, sizeof(double));
  int rc = 0;
  int any_moving = 0;
  for (int b = 0; b < o->nb; ++b) any_moving |= o->moving[b];
  if (o->nf != 1 || o->method != ORC_DIRECT || o->bc[1] == ORC_CONVECTIVE_OUTLET ||
      o->bc[2] == ORC_FREE_SLIP_WALL || any_moving) {
    /* the reverse mode covers one forcing pass and the bounce-back / zero-gradient boundaries */
    rc = -1;
    goto done;
  }
  if (!tape || !hist || !Abar || !Bbar || !gbar || !fbx || !fby || !Fbx || !Fby || !gxy || !guv || !gc) {
    rc = -1;
    goto done;
  }

  /* forward, keeping every state and the body forces of every step */
  memcpy(tape, o->A, S * sizeof(double));
  for (long t = 0; t < n; ++t) {
    oracle_step(o, 1);
    memcpy(tape + (size_t)(t + 1) * S, o->A, S * sizeof(double));
    memcpy(hist + (size_t)t * nb * 3, o->force, (size_t)nb * 3 * sizeof(double));
  }
  if (o->unstable) {
    rc = -1;
    goto done;
  }

  /* Abar holds dJ/dA_{t+1}; J does not read the final state */
  for (long t = n - 1; t >= 0; --t) {
    const double *Anext = tape + (size_t)(t + 1) * S;
    /* recompute the intermediates of step t from its state */
    memcpy(o->A, tape + (size_t)t * S, S * sizeof(double));
    stream(o);
    moments(o);
    immersed_boundary(o);

    /* boundary columns (applied last in the forward step, so first here) */
    memcpy(Bbar, Abar, S * sizeof(double));
    if (o->bc[1] == ORC_ZERO_GRADIENT_OUTLET) {
      for (int j = 0; j < ny; ++j)
        for (int q = 0; q < 9; ++q) {
          Bbar[idx(o, q, j, nx - 2)] += Bbar[idx(o, q, j, nx - 1)];
          Bbar[idx(o, q, j, nx - 1)] = 0.0;
        }
    }
    if (o->bc[0] == ORC_VELOCITY_INLET) {
      for (int j = 0; j < ny; ++j) {
        double r = 0.0; /* density of column 1 after collision */
        for (int q = 0; q < 9; ++q) r += Anext[idx(o, q, j, 1)];
        double rbar = 0.0;
        for (int q = 0; q < 9; ++q) {
          double bb = Bbar[idx(o, q, j, 0)];
          double dx, dy;
          feq_du(q, r, o->uin[0], o->uin[1], &dx, &dy);
          rbar += bb * feq_drho(q, o->uin[0], o->uin[1]);
          gin[0] += bb * dx;
          gin[1] += bb * dy;
          Bbar[idx(o, q, j, 0)] = 0.0;
        }
        for (int q = 0; q < 9; ++q) Bbar[idx(o, q, j, 1)] += rbar;
      }
    }

    /* collision at every fluid node: B_q = g_q - (g_q - feq_q(rho, u)) / tau + F_q,
     * u = (m + f/2) / rho, f = G + f_IB */
    memset(gbar, 0, S * sizeof(double));
    for (size_t k = 0; k < N; ++k) fbx[k] = fby[k] = 0.0;
    for (int j = 0; j < ny; ++j) {
      for (int i = i0; i <= i1; ++i) {
        size_t k = (size_t)j * nx + i;
        double r = o->rho[k];
        double ftx = o->G[0] + o->fx[k], fty = o->G[1] + o->fy[k];
        double ux = (o->mx[k] + 0.5 * ftx) / r, uy = (o->my[k] + 0.5 * fty) / r;
        double c = 1.0 - 1.0 / (2.0 * tau);
        double rbar = 0.0, ubx = 0.0, uby = 0.0, ftbx = 0.0, ftby = 0.0;
        for (int q = 0; q < 9; ++q) {
          double bb = Bbar[idx(o, q, j, i)];
          double eu = EX[q] * ux + EY[q] * uy;
          double ef = EX[q] * ftx + EY[q] * fty;
          double dx, dy;
          feq_du(q, r, ux, uy, &dx, &dy);
          gbar[idx(o, q, j, i)] += (1.0 - 1.0 / tau) * bb;
          rbar += bb * feq_drho(q, ux, uy) / tau;
          /* d F_q / d u and d F_q / d f of eq 7 */
          ubx += bb * (dx / tau + c * WQ[q] * (-3.0 * ftx + 9.0 * ef * EX[q]));
          uby += bb * (dy / tau + c * WQ[q] * (-3.0 * fty + 9.0 * ef * EY[q]));
          ftbx += bb * c * WQ[q] * (3.0 * (EX[q] - ux) + 9.0 * eu * EX[q]);
          ftby += bb * c * WQ[q] * (3.0 * (EY[q] - uy) + 9.0 * eu * EY[q]);
        }
        /* u = (m + f/2) / rho */
        double mbx = ubx / r, mby = uby / r;
        ftbx += 0.5 * ubx / r;
        ftby += 0.5 * uby / r;
        rbar -= (ubx * ux + uby * uy) / r;
        for (int q = 0; q < 9; ++q) gbar[idx(o, q, j, i)] += rbar + EX[q] * mbx + EY[q] * mby;
        fbx[k] = ftbx;
        fby[k] = ftby;
        gG[0] += ftbx;
        gG[1] += ftby;
      }
    }

    /* body force and torque (eq 27), then spreading (eqs 13, 15): dJ/dF_l */
    for (int m = 0; m < nm; ++m) {
      int b = o->body_of[m];
      double s = o->drs * o->ds[b];
      const double *hb = hist_bar + ((size_t)t * nb + b) * 3;
      double X = o->X[m], Y = o->Y[m];
      /* F_b = -s sum F_l ; T_b = -s sum (X_l - c) x F_l */
      double Fbarx = -s * hb[0] + s * hb[2] * (Y - o->cy[b]);
      double Fbary = -s * hb[1] - s * hb[2] * (X - o->cx[b]);
      gxy[2 * m] += -s * hb[2] * o->Fy[m];
      gxy[2 * m + 1] += s * hb[2] * o->Fx[m];
      for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
        for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
          double px = oracle_delta(o->kind, i - X), py = oracle_delta(o->kind, j - Y);
          double dpx = -oracle_delta_deriv(o->kind, i - X) * py; /* dW/dX */
          double dpy = -px * oracle_delta_deriv(o->kind, j - Y); /* dW/dY */
          size_t k = node_of(o, i, j);
          Fbarx += px * py * s * fbx[k];
          Fbary += px * py * s * fby[k];
          double fdot = s * (o->Fx[m] * fbx[k] + o->Fy[m] * fby[k]);
          gxy[2 * m] += dpx * fdot;
          gxy[2 * m + 1] += dpy * fdot;
        }
      }
      Fbx[m] = Fbarx;
      Fby[m] = Fbary;
    }
    for (int b = 0; b < nb; ++b) { /* the centre enters the torque only */
      const double *hb = hist_bar + ((size_t)t * nb + b) * 3;
      const double *Fb = hist + ((size_t)t * nb + b) * 3;
      gc[2 * b] += -hb[2] * Fb[1];
      gc[2 * b + 1] += hb[2] * Fb[0];
    }

    /* direct force (eq 20) and interpolation (eqs 12, 14) */
    for (int m = 0; m < nm; ++m) {
      double X = o->X[m], Y = o->Y[m];
      double rl = o->rho_l[m], ul = o->ux_l[m], vl = o->uy_l[m];
      /* F = 2 rho_l (U_b - u*_l) */
      double rlbar = 2.0 * (Fbx[m] * (o->Ub[m] - ul) + Fby[m] * (o->Vb[m] - vl));
      double ulbar = -2.0 * rl * Fbx[m], vlbar = -2.0 * rl * Fby[m];
      guv[2 * m] += 2.0 * rl * Fbx[m];
      guv[2 * m + 1] += 2.0 * rl * Fby[m];
      for (int j = (int)ceil(Y - h); j <= (int)floor(Y + h); ++j) {
        for (int i = (int)ceil(X - h); i <= (int)floor(X + h); ++i) {
          double px = oracle_delta(o->kind, i - X), py = oracle_delta(o->kind, j - Y);
          double W = px * py;
          double dpx = -oracle_delta_deriv(o->kind, i - X) * py;
          double dpy = -px * oracle_delta_deriv(o->kind, j - Y);
          size_t k = node_of(o, i, j);
          double r = o->rho[k];
          double us = (o->mx[k] + 0.5 * o->G[0]) / r, vs = (o->my[k] + 0.5 * o->G[1]) / r;
          double v = rlbar * r + ulbar * us + vlbar * vs;
          gxy[2 * m] += dpx * v;
          gxy[2 * m + 1] += dpy * v;
          /* node adjoints of rho and u* = (m + G/2) / rho */
          double usbar = W * ulbar, vsbar = W * vlbar;
          double rbar = W * rlbar - (usbar * us + vsbar * vs) / r;
          double mbx = usbar / r, mby = vsbar / r;
          gG[0] += 0.5 * usbar / r;
          gG[1] += 0.5 * vsbar / r;
          int jj = (int)(k / (size_t)nx), ii = (int)(k % (size_t)nx);
          for (int q = 0; q < 9; ++q) gbar[idx(o, q, jj, ii)] += rbar + EX[q] * mbx + EY[q] * mby;
        }
      }
    }

    /* streaming: g_q(x) = A(source) for every fluid node, so the adjoint of
     * the state collects each g's adjoint at its source */
    memset(Abar, 0, S * sizeof(double));
    for (int q = 0; q < 9; ++q)
      for (int j = 0; j < ny; ++j)
        for (int i = i0; i <= i1; ++i) Abar[stream_source(o, q, j, i)] += gbar[idx(o, q, j, i)];
  }

  /* back to the final state, with the intermediates of the last step as
   * oracle_step leaves them (the step is recomputed from its stored state) */
  if (n > 0) {
    memcpy(o->A, tape + (size_t)(n - 1) * S, S * sizeof(double));
    stream(o);
    moments(o);
    immersed_boundary(o);
    collide(o);
    boundary_columns(o);
  }
  if (pop_bar) memcpy(pop_bar, Abar, S * sizeof(double));
  if (inflow_bar) { inflow_bar[0] = gin[0]; inflow_bar[1] = gin[1]; }
  if (force_bar) { force_bar[0] = gG[0]; force_bar[1] = gG[1]; }
  if (xy_bar) memcpy(xy_bar, gxy, (size_t)nm * 2 * sizeof(double));
  if (uv_bar) memcpy(uv_bar, guv, (size_t)nm * 2 * sizeof(double));
  if (centre_bar) memcpy(centre_bar, gc, (size_t)nb * 2 * sizeof(double));
done:
  free(tape); free(hist); free(Abar); free(Bbar); free(gbar); free(fbx); free(fby);
  free(Fbx); free(Fby); free(gxy); free(guv); free(gc);
  return rc;
}
