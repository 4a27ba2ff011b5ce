"""GPU parity of the far-field boundaries of the cylinder runs (Section 5.2):
free-slip walls (specular reflection) and the convective outlet, alone and
combined with the other boundary kinds, against the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

pytestmark = pytest.mark.gpu

SLIP_Y = (W.PERIODIC, W.PERIODIC, W.FREE_SLIP_WALL, W.FREE_SLIP_WALL)
CONV_PERIODIC_Y = (W.VELOCITY_INLET, W.CONVECTIVE_OUTLET, W.PERIODIC, W.PERIODIC)
CONV_WALLS = (W.VELOCITY_INLET, W.CONVECTIVE_OUTLET, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL)
ZG_SLIP = (W.VELOCITY_INLET, W.ZERO_GRADIENT_OUTLET, W.FREE_SLIP_WALL, W.FREE_SLIP_WALL)


def log(msg):
    print(msg, flush=True)


def oracle_of(c):
    s = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    if c.init_uy is not None:
        ux, uy = c.init_fields()
        s.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    return s


def gpu_of(c, precision=8):
    from paper_1806_09403_amd import Sim
    return Sim.from_case(c, precision=precision)


CASES = [
    # (seed, nx, ny, kind, bc, reference velocity)
    (20, 151, 61, W.ROMA3, W.FAR_FIELD, (0.02, 0.0)),
    (21, 97, 45, W.COS4, W.FAR_FIELD, (0.02, 0.015)),
    (22, 120, 50, W.PESKIN4, SLIP_Y, (0.02, -0.01)),
    (23, 90, 40, W.LINEAR2, CONV_PERIODIC_Y, (0.02, 0.0)),
    (24, 110, 44, W.COS4, CONV_WALLS, (0.02, 0.0)),
    (25, 100, 48, W.ROMA3, ZG_SLIP, (0.03, 0.01)),
]


@pytest.mark.parametrize("seed,nx,ny,kind,bc,uref", CASES)
def test_fp64_steps_match_oracle(seed, nx, ny, kind, bc, uref):
    log("far-field parity seed=%d %dx%d kind=%d bc=%s uref=%s" % (seed, nx, ny, kind, bc, uref))
    c = W.random_case(seed, nx=nx, ny=ny, kind=kind, bc=bc, n_bodies=2, D_range=(5.0, 9.0))
    c = dataclasses.replace(c, init=(1.0, *uref))
    o, g = oracle_of(c), gpu_of(c)
    for step in range(8):
        o.step(1)
        g.step(1)
        assert o.unstable == 0, step
        assert np.max(np.abs(g.populations() - o.populations())) < 1e-14, step
        Fo, Fg = o.forces(), g.forces()
        assert np.max(np.abs(Fg - Fo)) < 1e-12 * np.max(np.abs(Fo)), step
    g.close()


def test_fp32_one_step_from_same_state():
    c = W.random_case(26, nx=180, ny=70, kind=W.ROMA3, bc=W.FAR_FIELD, n_bodies=2)
    c = dataclasses.replace(c, init=(1.0, 0.02, 0.01))
    g = gpu_of(c, precision=4)
    g.step(9)
    o = oracle_of(c)
    o.set_populations(g.populations())
    o.step(1)
    g.step(1)
    d = np.max(np.abs(g.populations() - o.populations()))
    log("  far-field fp32 one-step max |df| = %.3e" % d)
    assert d < 2e-7
    assert np.max(np.abs(g.forces() - o.forces())) < 1e-12 * np.max(np.abs(o.forces()))
    g.close()


def test_uniform_inflow_stays_uniform_in_both_precisions():
    from paper_1806_09403_amd import Sim
    for prec, tol in ((8, 1e-15), (4, 1e-7)):
        s = Sim(64, 32, 0.8, W.ROMA3, 1.9, W.FAR_FIELD, (0.05, 0.0), (0.0, 0.0), (1.0, 0.05, 0.0), prec)
        f0 = s.populations()
        s.step(500)
        assert np.max(np.abs(s.populations() - f0)) < tol, prec
        s.close()


def test_interior_path_keeps_the_convective_outlet():
    from paper_1806_09403_amd import _lib
    log("interior path at the convective outlet, every launch shape")
    c = W.random_case(27, nx=513, ny=20, kind=W.ROMA3, bc=W.FAR_FIELD, n_bodies=1, D_range=(3.0, 4.0))
    o = oracle_of(c)
    o.step(3)
    ref = o.populations()
    g0 = gpu_of(c)
    for v in range(g0.get_option(_lib.OPT_NUM_VARIANTS)):
        g = gpu_of(c)
        g.set_option(_lib.OPT_LBM_VARIANT, v)
        g.set_option(_lib.OPT_INTERIOR_PATH, 1)
        g.step(3)
        assert np.max(np.abs(g.populations() - ref)) < 1e-14, v
        g.close()
    g0.close()


def test_batch_of_far_field_cases_equals_single_runs():
    from paper_1806_09403_amd import BatchSim
    cases = [W.random_case(30 + k, nx=80 + 8 * k, ny=40, kind=W.COS4, bc=bc, n_bodies=1)
             for k, bc in enumerate((W.FAR_FIELD, SLIP_Y, CONV_WALLS))]
    bs = BatchSim(cases, precision=4)
    bs.step(12)
    for k, c in enumerate(cases):
        g = gpu_of(c, precision=4)
        g.step(12)
        assert np.array_equal(bs.cases[k].populations(), g.populations()), k
        g.close()
    bs.close()


def test_refusals():
    from paper_1806_09403_amd import BtdfError, Sim
    with pytest.raises(BtdfError):   # mixed wall kinds
        Sim(32, 16, 0.8, W.ROMA3, 1.9, (W.PERIODIC, W.PERIODIC, W.FREE_SLIP_WALL, W.BOUNCEBACK_WALL))
    with pytest.raises(BtdfError):   # a convective outlet against the flow
        Sim(32, 16, 0.8, W.ROMA3, 1.9, W.FAR_FIELD, (-0.01, 0.0))
    with pytest.raises(BtdfError):   # an outlet without an inlet
        Sim(32, 16, 0.8, W.ROMA3, 1.9, (W.PERIODIC, W.CONVECTIVE_OUTLET, W.PERIODIC, W.PERIODIC))
    c = W.random_case(31, nx=40, ny=24, kind=W.ROMA3, bc=W.FAR_FIELD, n_bodies=1)
    g = gpu_of(c)
    with pytest.raises(BtdfError):
        g.adjoint(2, np.zeros((2, 1, 3)))
    g.close()
