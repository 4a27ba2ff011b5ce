"""The boundary-velocity diagnostic (eq 45's u_b) on the GPU against the
oracle: the corrected velocity of the last step (eq 11) interpolated at
every marker (eq 12)."""
import dataclasses

import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

pytestmark = pytest.mark.gpu


def oracle_of(c, nf=1):
    s = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    if c.init_uy is not None:
        ux, uy = c.init_fields()
        s.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    s.set_forcing_passes(nf)
    return s


def gpu_of(c, precision=8, nf=1):
    from paper_1806_09403_amd import Sim, _lib
    s = Sim.from_case(c, precision=precision)
    s.set_option(_lib.OPT_FORCING_PASSES, nf)
    return s


@pytest.mark.parametrize("seed,bc,kind,nf", [
    (40, W.FULLY_PERIODIC, W.COS4, 1),
    (41, W.CHANNEL, W.ROMA3, 1),
    (42, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), W.PESKIN4, 1),
    (43, W.FAR_FIELD, W.ROMA3, 3),
    (44, W.FULLY_PERIODIC, W.LINEAR2, 5),
])
def test_fp64_marker_velocity_matches_oracle(seed, bc, kind, nf):
    print("marker velocity seed=%d nf=%d" % (seed, nf), flush=True)
    c = W.random_case(seed, nx=120, ny=70, kind=kind, bc=bc, n_bodies=3, D_range=(5.0, 9.0))
    c = dataclasses.replace(c, init=(1.0, 0.02, 0.01))
    o, g = oracle_of(c, nf), gpu_of(c, nf=nf)
    for n in (1, 4):
        o.step(n)
        g.step(n)
        uo, vo = o.marker_corrected_velocity()
        ug, vg = g.marker_velocity()
        assert np.max(np.abs(ug - uo)) < 1e-14 and np.max(np.abs(vg - vo)) < 1e-14, n
    g.close()


def test_fp32_marker_velocity_from_same_state():
    c = W.random_case(45, nx=150, ny=80, kind=W.COS4, bc=W.CHANNEL, n_bodies=3)
    g = gpu_of(c, precision=4)
    g.step(5)
    o = oracle_of(c)
    o.set_populations(g.populations())
    o.step(1)
    g.step(1)
    uo, vo = o.marker_corrected_velocity()
    ug, vg = g.marker_velocity()
    d = max(np.max(np.abs(ug - uo)), np.max(np.abs(vg - vo)))
    print("  fp32 marker velocity max diff %.3e" % d, flush=True)
    assert d < 1e-6
    g.close()


def test_needs_a_step_after_each_change():
    from paper_1806_09403_amd import BtdfError
    c = W.random_case(46, nx=60, ny=40, n_bodies=1)
    g = gpu_of(c)
    with pytest.raises(BtdfError):
        g.marker_velocity()
    g.step(2)
    g.marker_velocity()
    g.set_populations(g.populations())
    with pytest.raises(BtdfError):
        g.marker_velocity()
    g.step(1)
    g.marker_velocity()
    b = W.cylinder_body(40.0, 20.0, 5.0)
    g.add_body(b.xy, None, b.cx, b.cy, b.ds)
    with pytest.raises(BtdfError):
        g.marker_velocity()
    g.step(1)
    u, v = g.marker_velocity()
    assert u.shape == (c.bodies[0].xy.shape[0] + b.xy.shape[0],)
    g.close()
