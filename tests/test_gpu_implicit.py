"""GPU parity of the comparison forcing methods of Section 3: the implicit
direct forcing (eq 17, identical to the implicit velocity correction of
eqs 32-35) and RKPM (eq 36 / B54), against the oracle."""
import dataclasses

import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def oracle_of(c, method):
    s = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    if c.init_uy is not None:
        ux, uy = c.init_fields()
        s.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    s.set_forcing_method(method)
    return s


def gpu_of(c, method, precision=8):
    from paper_1806_09403_amd import Sim, _lib
    s = Sim.from_case(c, precision=precision)
    s.set_option(_lib.OPT_FORCING_METHOD, method)
    assert s.get_option(_lib.OPT_FORCING_METHOD) == method
    return s


CASES = [
    # (seed, nx, ny, kind, bc)
    (50, 140, 80, W.ROMA3, W.FULLY_PERIODIC),
    (51, 150, 70, W.COS4, W.CHANNEL),
    (52, 110, 64, W.PESKIN4, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL)),
    (53, 130, 60, W.LINEAR2, W.FAR_FIELD),
]


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("seed,nx,ny,kind,bc", CASES)
def test_fp64_steps_match_oracle(seed, nx, ny, kind, bc, method):
    log("implicit/rkpm parity method=%d seed=%d kind=%d" % (method, seed, kind))
    c = W.random_case(seed, nx=nx, ny=ny, kind=kind, bc=bc, n_bodies=3, D_range=(6.0, 10.0))
    o, g = oracle_of(c, method), gpu_of(c, method)
    for step in range(5):
        o.step(1)
        g.step(1)
        assert o.unstable == 0, step
        assert np.max(np.abs(g.populations() - o.populations())) < 1e-13, step
        mo, mg = o.marker_data(), g.marker_data()
        scale = np.max(np.abs(mo["Fx"])) + np.max(np.abs(mo["Fy"]))
        for k in ("Fx", "Fy"):
            assert np.max(np.abs(mg[k] - mo[k])) < 1e-10 * scale, (step, k)
        Fo, Fg = o.forces(), g.forces()
        assert np.max(np.abs(Fg - Fo)) < 1e-10 * np.max(np.abs(Fo)), step
    g.close()


@pytest.mark.parametrize("method", [1, 2])
def test_fp32_one_step_from_same_state(method):
    c = W.random_case(54, nx=160, ny=90, kind=W.ROMA3, bc=W.CHANNEL, n_bodies=3, D_range=(6.0, 10.0))
    g = gpu_of(c, method, precision=4)
    g.step(6)
    o = oracle_of(c, method)
    o.set_populations(g.populations())
    o.step(1)
    g.step(1)
    d = np.max(np.abs(g.populations() - o.populations()))
    log("  method %d fp32 one-step max |df| = %.3e" % (method, d))
    assert d < 2e-7
    mo, mg = o.marker_data(), g.marker_data()
    for k in ("Fx", "Fy"):
        assert np.max(np.abs(mg[k] - mo[k])) < 1e-10 * np.max(np.abs(mo[k]))
    g.close()


def test_implicit_enforces_the_marker_velocity_exactly():
    """eq 16 with a uniform density: after one implicit step from a uniform
    flow the velocity at every marker is the prescribed one."""
    from paper_1806_09403_amd import Sim, _lib
    s = Sim(64, 64, 0.8, W.ROMA3, 1.9, W.FULLY_PERIODIC, init=(1.0, 0.04, 0.01), precision=8)
    b = W.cylinder_body(30.3, 31.7, 12.0, 38)
    uv = np.random.default_rng(5).uniform(-0.01, 0.01, size=(38, 2))
    s.add_body(b.xy, uv, b.cx, b.cy, b.ds)
    s.set_option(_lib.OPT_FORCING_METHOD, 1)
    s.step(1)
    u, v = s.marker_velocity()
    assert max(np.max(np.abs(u - uv[:, 0])), np.max(np.abs(v - uv[:, 1]))) < 1e-13
    s.close()


def test_launch_shapes_and_graphs_are_bit_identical():
    from paper_1806_09403_amd import _lib
    c = W.random_case(55, nx=150, ny=64, n_bodies=2, D_range=(6.0, 9.0))
    for method in (1, 2):
        ref = None
        for v, chunk in ((6, 0), (6, 5), (0, 0), (11, 7)):
            g = gpu_of(c, method, precision=4)
            g.set_option(_lib.OPT_LBM_VARIANT, v)
            g.set_option(_lib.OPT_GRAPH_CHUNK, chunk)
            g.step(4)
            g.step(11)
            out = (g.populations(), g.force_history(15))
            if ref is None:
                ref = out
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), (method, v, chunk)
            g.close()


def test_method_change_mid_run_and_refusals():
    from paper_1806_09403_amd import BtdfError, Sim, _lib
    c = W.random_case(56, nx=100, ny=60, kind=W.ROMA3, bc=W.CHANNEL, n_bodies=2, D_range=(6.0, 9.0))
    o, g = oracle_of(c, 0), gpu_of(c, 0)
    for method in (0, 1, 2, 0, 2):
        o.set_forcing_method(method)
        g.set_option(_lib.OPT_FORCING_METHOD, method)
        o.step(2)
        g.step(2)
        assert np.max(np.abs(g.populations() - o.populations())) < 1e-13, method
    with pytest.raises(BtdfError):
        g.set_option(_lib.OPT_FORCING_PASSES, 3)      # RKPM takes one pass
    with pytest.raises(BtdfError):
        g.set_option(_lib.OPT_FORCING_METHOD, 7)
    with pytest.raises(BtdfError):
        g.adjoint(2, np.zeros((2, 2, 3)))
    g.set_option(_lib.OPT_FORCING_METHOD, 0)
    g.set_option(_lib.OPT_FORCING_PASSES, 3)
    with pytest.raises(BtdfError):
        g.set_option(_lib.OPT_FORCING_METHOD, 1)      # passes need the direct method
    g.close()
    # a body beyond the matrix limit is refused when the run starts
    s = Sim(400, 400, 0.8, W.ROMA3, 1.9, init=(1.0, 0.02, 0.0))
    b = W.cylinder_body(200.0, 200.0, 300.0, 2100)
    s.add_body(b.xy, None, b.cx, b.cy, b.ds)
    s.set_option(_lib.OPT_FORCING_METHOD, 2)
    with pytest.raises(BtdfError):
        s.step(1)
    s.close()
