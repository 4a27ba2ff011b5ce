"""GPU parity of the forcing passes (multi direct forcing, eqs 29-31).

With NF > 1 passes per step the HIP path (a first marker kernel that caches
each stencil node's rho and u*, then one small kernel per further pass that
rebuilds the spread force from the covering-marker lists) must agree with
the oracle's passes, which spread every force increment onto a grid-sized
field. FP64 populations: the same few-ulp bar as one pass. FP32 populations:
one step from the same state, marker forces in FP64 to 1e-12 relative.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def oracle_of(c, nf):
    s = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    if c.init_uy is not None:
        ux, uy = c.init_fields()
        s.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    s.set_forcing_passes(nf)
    return s


def gpu_of(c, nf, precision=8):
    from paper_1806_09403_amd import Sim, _lib
    s = Sim.from_case(c, precision=precision)
    s.set_option(_lib.OPT_FORCING_PASSES, nf)
    assert s.get_option(_lib.OPT_FORCING_PASSES) == nf
    return s


def compare(o, g, step, pop_tol=1e-14):
    fo, fg = o.populations(), g.populations()
    assert np.max(np.abs(fg - fo)) < pop_tol, step
    mo, mg = o.marker_data(), g.marker_data()
    scale = max(1e-300, np.max(np.abs(mo["Fx"])) + np.max(np.abs(mo["Fy"])))
    for k in ("Fx", "Fy"):
        assert np.max(np.abs(mg[k] - mo[k])) < 1e-12 * scale, (step, k)
    for k in ("rho", "ux", "uy"):
        assert np.max(np.abs(mg[k] - mo[k])) < 1e-14, (step, k)
    Fo, Fg = o.forces(), g.forces()
    assert np.max(np.abs(Fg - Fo)) < 1e-12 * max(1e-300, np.max(np.abs(Fo))), step


CASES = [
    # (seed, nx, ny, kind, bc, nf)
    (0, 197, 83, W.COS4, W.FULLY_PERIODIC, 3),
    (1, 131, 70, W.ROMA3, W.CHANNEL, 5),
    (2, 70, 61, W.PESKIN4, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), 2),
    (3, 90, 37, W.LINEAR2, (W.VELOCITY_INLET, W.ZERO_GRADIENT_OUTLET, W.BOUNCEBACK_WALL,
                            W.BOUNCEBACK_WALL), 4),
]


@pytest.mark.parametrize("seed,nx,ny,kind,bc,nf", CASES)
def test_fp64_passes_match_oracle(seed, nx, ny, kind, bc, nf):
    log("mdf fp64 parity seed=%d %dx%d kind=%d nf=%d" % (seed, nx, ny, kind, nf))
    c = W.random_case(seed, nx=nx, ny=ny, kind=kind, bc=bc, n_bodies=3, D_range=(4.0, 9.0))
    o, g = oracle_of(c, nf), gpu_of(c, nf)
    for step in range(6):
        o.step(1)
        g.step(1)
        assert o.unstable == 0, step
        compare(o, g, step)
    g.close()


def test_body_across_the_periodic_seam():
    """A body centred on the corner of a fully periodic grid: the covering
    lists must wrap in both directions."""
    log("mdf periodic seam")
    c = W.random_case(4, nx=64, ny=48, kind=W.COS4, bc=W.FULLY_PERIODIC, n_bodies=0)
    b = W.cylinder_body(0.3, 47.6, 9.0)
    o = oracle_of(c, 3)
    o.add_body(b.xy, None, b.cx, b.cy, b.ds)
    from paper_1806_09403_amd import _lib
    g = gpu_of(c, 1)
    g.add_body(b.xy, None, b.cx, b.cy, b.ds)
    g.set_option(_lib.OPT_FORCING_PASSES, 3)
    for step in range(4):
        o.step(1)
        g.step(1)
        compare(o, g, step)
    g.close()


def test_change_of_passes_mid_run():
    """Switch NF between steps (the pass buffers are re-laid out); the state
    and the force ring carry over."""
    from paper_1806_09403_amd import _lib
    log("mdf change of NF mid-run")
    c = W.random_case(5, nx=100, ny=60, kind=W.ROMA3, bc=W.CHANNEL, n_bodies=2, D_range=(5.0, 8.0))
    o, g = oracle_of(c, 1), gpu_of(c, 1)
    ho = []
    for nf, n in ((1, 3), (4, 3), (2, 2), (1, 2)):
        o.set_forcing_passes(nf)
        g.set_option(_lib.OPT_FORCING_PASSES, nf)
        for _ in range(n):
            o.step(1)
            g.step(1)
            ho.append(o.forces())
        compare(o, g, nf)
    ho, hg = np.stack(ho), g.force_history(10)
    assert ho.shape == hg.shape == (10, 2, 3)
    assert np.max(np.abs(hg - ho)) < 1e-12 * np.max(np.abs(ho))
    g.close()


@pytest.mark.parametrize("kind,bc", [(W.COS4, W.FULLY_PERIODIC), (W.ROMA3, W.CHANNEL)])
def test_fp32_one_step_from_same_state(kind, bc):
    log("mdf fp32 one step kind=%d" % kind)
    c = W.random_case(6, nx=203, ny=77, kind=kind, bc=bc, n_bodies=3)
    g = gpu_of(c, 4, precision=4)
    g.step(7)
    f = g.populations()
    o = oracle_of(c, 4)
    o.set_populations(f)
    o.step(1)
    g.step(1)
    d = np.max(np.abs(g.populations() - o.populations()))
    log("  fp32 nf=4 one-step max |df| = %.3e" % d)
    assert d < 2e-7
    mo, mg = o.marker_data(), g.marker_data()
    for k in ("Fx", "Fy"):
        assert np.max(np.abs(mg[k] - mo[k])) < 1e-12 * np.max(np.abs(mo[k]))
    assert np.max(np.abs(g.forces() - o.forces())) < 1e-12 * np.max(np.abs(o.forces()))
    g.close()


def test_graph_replay_and_launch_shapes_are_bit_identical():
    from paper_1806_09403_amd import _lib
    log("mdf graph and launch shapes")
    c = W.random_case(7, nx=150, ny=64, n_bodies=2)
    ref = None
    for v, chunk in ((6, 0), (6, 5), (0, 0), (11, 7)):
        g = gpu_of(c, 3, precision=4)
        g.set_option(_lib.OPT_LBM_VARIANT, v)
        g.set_option(_lib.OPT_GRAPH_CHUNK, chunk)
        for n in (4, 11):
            g.step(n)
        out = (g.populations(), g.force_history(15))
        if ref is None:
            ref = out
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), (v, chunk)
        g.close()


def test_slip_falls_with_passes_on_gpu():
    """The marker slip after one step (eq 45's boundary error) falls as NF
    grows; measured as |U_b - D_I u| with u the corrected velocity the
    oracle computes from the GPU's populations."""
    errs = []
    c = W.random_case(8, nx=64, ny=64, kind=W.ROMA3, bc=W.FULLY_PERIODIC, n_bodies=0)
    b = W.cylinder_body(30.3, 31.6, 12.0)
    for nf in (1, 2, 4, 8):
        from paper_1806_09403_amd import _lib
        g = gpu_of(c, 1)
        g.add_body(b.xy, None, b.cx, b.cy, b.ds)
        g.set_option(_lib.OPT_FORCING_PASSES, nf)
        g.step(1)
        o = oracle_of(c, nf)
        o.add_body(b.xy, None, b.cx, b.cy, b.ds)
        o.step(1)
        assert np.max(np.abs(g.populations() - o.populations())) < 1e-14
        u, v = o.marker_corrected_velocity()
        errs.append(float(np.sqrt(np.mean(u * u + v * v))))
        g.close()
    log("  slip by NF: %s" % errs)
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:])), errs


def test_option_limits_and_refusals():
    from paper_1806_09403_amd import BatchSim, BtdfError, _lib
    c = W.random_case(9, nx=64, ny=40, n_bodies=1)
    g = gpu_of(c, 1)
    for bad in (0, 65, -1):
        with pytest.raises(BtdfError):
            g.set_option(_lib.OPT_FORCING_PASSES, bad)
    assert g.get_option(_lib.OPT_FORCING_PASSES) == 1
    g.set_option(_lib.OPT_FORCING_PASSES, 2)
    with pytest.raises(BtdfError):
        g.adjoint(3, np.zeros((3, 1, 3)))
    g.close()
    bs = BatchSim([c, c], precision=8)
    with pytest.raises(BtdfError):
        bs.set_option(_lib.OPT_FORCING_PASSES, 2)
    bs.close()
