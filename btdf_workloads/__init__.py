"""Seeded synthetic workloads for the BTDF-IB-LBM step.

This module is the only code shared by the HIP library's tests and the
FP64 oracle. It holds configuration and geometry only -- grid sizes,
boundary kinds, relaxation times, marker rings, random cylinder centres
and initial velocity fields -- and none of the method's arithmetic
(no equilibria, deltas, forcing or collision).

Geometry conventions (lattice units, dh = dt = 1): node (i, j) sits at
(x, y) = (i, j); a cylinder of diameter D centred at c carries N_L markers
at X_l = c + (D/2)(cos t_l, sin t_l), t_l = 2 pi l / N_L, with the arc
spacing ds = pi D / N_L (Section 4.2 discusses the choice of ds/dh).
"""
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# boundary kinds (west, east, south, north)
PERIODIC, VELOCITY_INLET, ZERO_GRADIENT_OUTLET, BOUNCEBACK_WALL = 0, 1, 2, 3
FREE_SLIP_WALL, CONVECTIVE_OUTLET = 4, 5
# regularised delta kinds: 2-point (eq 37), 3-point (eq 38), 4-point (eq 39), cosine 4-point
LINEAR2, ROMA3, PESKIN4, COS4 = 2, 3, 4, 5
KIND_NAMES = {LINEAR2: "linear2", ROMA3: "roma3", PESKIN4: "peskin4", COS4: "cos4"}
# boundary thickness drs/dh suggested for 2-, 3- and 4-point deltas (Section 4.4);
# the cosine kernel has the 4-point support and takes the 4-point value.
PAPER_THICKENING = {LINEAR2: 1.4, ROMA3: 1.9, PESKIN4: 2.6, COS4: 2.6}

CHANNEL = (VELOCITY_INLET, ZERO_GRADIENT_OUTLET, PERIODIC, PERIODIC)
FULLY_PERIODIC = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
# the far-field boundaries of the paper's cylinder runs (Section 5.2)
FAR_FIELD = (VELOCITY_INLET, CONVECTIVE_OUTLET, FREE_SLIP_WALL, FREE_SLIP_WALL)


@dataclass
class Body:
    xy: np.ndarray                  # [n, 2] marker positions
    uv: Optional[np.ndarray]        # [n, 2] prescribed marker velocities (None = at rest)
    cx: float
    cy: float
    ds: float
    D: float = 0.0


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    bc: Tuple[int, int, int, int]
    tau: float
    kind: int
    thickening: float
    G: Tuple[float, float] = (0.0, 0.0)
    inflow: Tuple[float, float] = (0.0, 0.0)
    init: Tuple[float, float, float] = (1.0, 0.0, 0.0)   # rho0, ux0, uy0
    init_uy: Optional[np.ndarray] = None                # optional [ny, nx] initial u_y field
    bodies: List[Body] = field(default_factory=list)
    steps: int = 0
    precision: int = 8
    U: float = 0.0
    D: float = 0.0

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    @property
    def n_markers(self) -> int:
        return sum(b.xy.shape[0] for b in self.bodies)

    def init_fields(self):
        """Initial (ux, uy) as [ny, nx] arrays (rho is init[0] everywhere)."""
        ux = np.full((self.ny, self.nx), float(self.init[1]))
        uy = np.full((self.ny, self.nx), float(self.init[2]))
        if self.init_uy is not None:
            uy = uy + self.init_uy
        return ux, uy


def cylinder_markers(cx, cy, D, n):
    t = 2.0 * np.pi * np.arange(n) / n
    return np.stack([cx + 0.5 * D * np.cos(t), cy + 0.5 * D * np.sin(t)], axis=1)


def cylinder_body(cx, cy, D, n=None, uv=None) -> Body:
    if n is None:
        n = int(round(np.pi * D))
    return Body(xy=cylinder_markers(cx, cy, D, n), uv=uv, cx=float(cx), cy=float(cy),
                ds=float(np.pi * D / n), D=float(D))


def tau_from_nu(nu):
    """Relaxation time of a lattice viscosity (the relation stated after eq 7)."""
    return 0.5 + 3.0 * nu


def c1(kind=COS4, thickening=None, steps=2000) -> Case:
    """FP64 correctness case: 200x120 channel, D = 16 cylinder at (60, 60), Re = 40."""
    U, D = 0.02, 16.0
    return Case(name="c1-channel-200x120-Re40", nx=200, ny=120, bc=CHANNEL,
                tau=tau_from_nu(0.008), kind=kind,
                thickening=PAPER_THICKENING[kind] if thickening is None else thickening,
                inflow=(U, 0.0), init=(1.0, U, 0.0),
                bodies=[cylinder_body(60.0, 60.0, D, 50)], steps=steps, precision=8, U=U, D=D)


def shedding_perturbation(nx, ny, U, D, xc, yc):
    """Deterministic u_y bump one diameter behind the cylinder that triggers shedding."""
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return 0.01 * U * np.exp(-((x - xc - D) ** 2 + (y - yc) ** 2) / (D / 2.0) ** 2)


def c2(kind=COS4, perturb=True, steps=100000, precision=4) -> Case:
    """Unsteady shedding: 2000x800 channel, D = 80 at (400, 400), Re = 200."""
    U, D = 0.05, 80.0
    return Case(name="c2-channel-2000x800-Re200", nx=2000, ny=800, bc=CHANNEL,
                tau=tau_from_nu(0.02), kind=kind, thickening=PAPER_THICKENING[kind],
                inflow=(U, 0.0), init=(1.0, U, 0.0),
                init_uy=shedding_perturbation(2000, 800, U, D, 400.0, 400.0) if perturb else None,
                bodies=[cylinder_body(400.0, 400.0, D, 251)], steps=steps,
                precision=precision, U=U, D=D)


def v40(re=40.0, kind=ROMA3, U=0.05, precision=4, perturb=None, D=40, ds=1.0, thickening=None) -> Case:
    """The paper's cylinder validation (Section 5.2, Table 3): a 40D x 40D
    domain meshed with 40 D + 1 nodes a side (1601 x 1601 at D/dh = 40), the
    cylinder at (18D, 20D), uniform inflow, free-slip top and bottom,
    convective outflow; by default the 3-point delta with its thickening 1.9
    (Section 4.4) and markers ds = dh apart (126 at D = 40). thickening=1.0
    is the conventional direct forcing (drs = dh). nu = U D / Re. An
    unsteady run (Re above the onset of shedding) gets a u_y bump behind the
    cylinder to break the symmetry; perturb=False/True overrides."""
    D = int(D)
    n = 40 * D + 1
    xc, yc = 18.0 * D, 20.0 * D
    if perturb is None:
        perturb = re > 46.0
    bump = 10.0 * shedding_perturbation(n, n, U, D, xc, yc) if perturb else None
    n_mk = int(round(np.pi * D / ds))
    drs = PAPER_THICKENING[kind] if thickening is None else float(thickening)
    return Case(name="v40-%dx%d-Re%g" % (n, n, re), nx=n, ny=n, bc=FAR_FIELD,
                tau=tau_from_nu(U * D / re), kind=kind, thickening=drs,
                inflow=(U, 0.0), init=(1.0, U, 0.0), init_uy=bump,
                bodies=[cylinder_body(xc, yc, float(D), n_mk)], steps=0, precision=precision, U=U,
                D=float(D))


def random_centres(n, L, dmin, seed=0, max_draws=1_000_000):
    """Sequential rejection sampling of n centres in a periodic L x L box whose
    periodic distances are all >= dmin (draw order: rng.random(2) * L)."""
    rng = np.random.default_rng(seed)
    pts = np.empty((n, 2))
    k = 0
    draws = 0
    while k < n:
        if draws >= max_draws:
            raise RuntimeError("could not place %d centres" % n)
        p = rng.random(2) * L
        draws += 1
        if k:
            d = np.abs(pts[:k] - p)
            d = np.minimum(d, L - d)
            if np.min(d[:, 0] ** 2 + d[:, 1] ** 2) < dmin * dmin:
                continue
        pts[k] = p
        k += 1
    return pts


def c3(kind=COS4, n=8192, n_bodies=2000, D=24.0, gap=4.0, seed=0, steps=10000, precision=4) -> Case:
    """Particle-laden throughput case: fully periodic n x n lattice, uniform body
    force, n_bodies fixed cylinders of 75 markers each (150 000 markers at 2000)."""
    centres = random_centres(n_bodies, float(n), D + gap, seed=seed)
    bodies = [cylinder_body(c[0], c[1], D, int(round(np.pi * D))) for c in centres]
    U = 0.042
    return Case(name="c3-periodic-%dx%d-%dcyl" % (n, n, n_bodies), nx=n, ny=n, bc=FULLY_PERIODIC,
                tau=0.8, kind=kind, thickening=PAPER_THICKENING[kind], G=(2.5e-6, 0.0),
                init=(1.0, U, 0.0), bodies=bodies, steps=steps, precision=precision, U=U, D=D)


def c4(seed=0, steps=5000):
    """256 independent channel cases of uneven size and Re (batched mode)."""
    rng = np.random.default_rng(seed)
    uw = rng.random(256)
    Ds = rng.uniform(8.0, 48.0, 256)
    Res = rng.uniform(0.1, 200.0, 256)
    U = 0.02
    cases = []
    for k in range(256):
        W = int(2 * round(128 * 8 ** uw[k] / 2))
        H = W // 2
        D = float(Ds[k])
        nu = U * D / Res[k]
        cases.append(Case(name="c4-%03d" % k, nx=W, ny=H, bc=CHANNEL, tau=tau_from_nu(nu),
                          kind=COS4, thickening=PAPER_THICKENING[COS4], inflow=(U, 0.0),
                          init=(1.0, U, 0.0), bodies=[cylinder_body(W / 4.0, H / 2.0, D)],
                          steps=steps, precision=4, U=U, D=D))
    return cases


def c5(steps=5000, precision=4) -> Case:
    """Adjoint case: 800x400 channel, D = 40 at (200, 200), Re = 100."""
    U, D = 0.04, 40.0
    return Case(name="c5-channel-800x400-Re100", nx=800, ny=400, bc=CHANNEL,
                tau=tau_from_nu(0.016), kind=COS4, thickening=PAPER_THICKENING[COS4],
                inflow=(U, 0.0), init=(1.0, U, 0.0), bodies=[cylinder_body(200.0, 200.0, D, 126)],
                steps=steps, precision=precision, U=U, D=D)


def random_case(seed, nx=37, ny=29, kind=COS4, bc=FULLY_PERIODIC, n_bodies=2, precision=8,
                G=(1e-5, -4e-6), moving=True, tau=0.7, D_range=(4.0, 9.0)) -> Case:
    """Small seeded case with several bodies, prescribed marker velocities, a
    body force and a smooth non-uniform initial flow (parity tests)."""
    rng = np.random.default_rng(seed)
    bodies = []
    margin = 5.0
    for b in range(n_bodies):
        D = float(rng.uniform(*D_range))
        lo_x = margin + D / 2 if bc[0] != PERIODIC else 0.0
        hi_x = nx - 1 - margin - D / 2 if bc[0] != PERIODIC else float(nx)
        lo_y = margin + D / 2 if bc[2] != PERIODIC else 0.0
        hi_y = ny - 1 - margin - D / 2 if bc[2] != PERIODIC else float(ny)
        cx, cy = float(rng.uniform(lo_x, hi_x)), float(rng.uniform(lo_y, hi_y))
        n = int(rng.integers(7, 23))
        uv = rng.uniform(-0.02, 0.02, size=(n, 2)) if moving else None
        body = cylinder_body(cx, cy, D, n, uv)
        bodies.append(body)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    uy0 = 0.01 * np.sin(2 * np.pi * x / nx + 0.3) * np.cos(2 * np.pi * y / ny)
    inflow = (0.03, 0.0) if bc[0] == VELOCITY_INLET else (0.0, 0.0)
    return Case(name="random-%d" % seed, nx=nx, ny=ny, bc=bc, tau=tau, kind=kind,
                thickening=PAPER_THICKENING[kind], G=G, inflow=inflow, init=(1.0, 0.02, 0.0),
                init_uy=uy0, bodies=bodies, steps=10, precision=precision, U=0.02, D=0.0)
