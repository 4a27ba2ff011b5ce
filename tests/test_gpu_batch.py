"""Batched mode: many independent cases stepped by one launch per kernel.

Every case of a batch must evolve exactly as the same case run on its own
(bit for bit: the batched kernels run the same per-tile and per-marker code
on the same data), a case that trips the instability guard stops while the
others go on, and graph replay and the autotuner leave the results
untouched. FP64 batches are also checked against the oracle directly.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

pytestmark = pytest.mark.gpu


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


def mixed_cases():
    """Uneven sizes, every boundary kind and delta, 0 to 3 bodies."""
    return [
        W.random_case(20, nx=197, ny=83, kind=W.COS4, bc=W.FULLY_PERIODIC, n_bodies=3),
        W.random_case(21, nx=64, ny=40, kind=W.ROMA3, bc=W.CHANNEL, n_bodies=1),
        W.random_case(22, nx=131, ny=70, kind=W.PESKIN4,
                      bc=(W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), n_bodies=2),
        W.random_case(23, nx=33, ny=17, kind=W.LINEAR2, bc=W.FULLY_PERIODIC, n_bodies=0),
        W.random_case(24, nx=90, ny=37, kind=W.LINEAR2,
                      bc=(W.VELOCITY_INLET, W.ZERO_GRADIENT_OUTLET, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL),
                      n_bodies=1),
    ]


def single(c, precision, variant=None, interior=None):
    from paper_1806_09403_amd import Sim
    from paper_1806_09403_amd._lib import OPT_INTERIOR_PATH, OPT_LBM_VARIANT
    s = Sim.from_case(c, precision=precision)
    if variant is not None:
        s.set_option(OPT_LBM_VARIANT, variant)
    if interior is not None:
        s.set_option(OPT_INTERIOR_PATH, interior)
    return s


def assert_same(batch_case, ref, nb, steps, what):
    fb, fr = batch_case.populations(), ref.populations()
    assert np.array_equal(fb, fr), what
    if nb:
        hb, hr = batch_case.force_history(steps), ref.force_history(steps)
        assert hb.shape == hr.shape and np.array_equal(hb, hr), what


@pytest.mark.parametrize("precision", [8, 4])
def test_batch_equals_single_runs(precision):
    from paper_1806_09403_amd import BatchSim
    cases = mixed_cases()
    log("batch of %d mixed cases, precision %d" % (len(cases), precision))
    b = BatchSim(cases, precision=precision)
    refs = [single(c, precision) for c in cases]
    for n in (1, 4, 7):
        b.step(n)
        for r in refs:
            r.step(n)
        for k, c in enumerate(cases):
            assert_same(b.cases[k], refs[k], len(c.bodies), n, (precision, n, k))
    unstable, steps = b.status()
    assert not unstable.any() and steps == 12
    for k in range(len(cases)):
        assert b.cases[k].counts()[2] == 12


def test_batch_fp64_matches_oracle():
    from paper_1806_09403_amd import BatchSim
    cases = mixed_cases()[:3]
    log("fp64 batch vs oracle")
    b = BatchSim(cases, precision=8)
    os_ = [oracle_of(c) for c in cases]
    for step in range(5):
        b.step(1)
        for o in os_:
            o.step(1)
        for k, o in enumerate(os_):
            assert np.max(np.abs(b.cases[k].populations() - o.populations())) < 1e-14, (step, k)
            if cases[k].bodies:
                Fo = o.forces()
                assert np.max(np.abs(b.cases[k].forces() - Fo)) < 1e-12 * np.max(np.abs(Fo)), (step, k)


@pytest.mark.parametrize("variant,interior", [(0, 0), (2, 1), (6, 1), (16, 0)])
def test_batch_launch_shapes(variant, interior):
    from paper_1806_09403_amd import BatchSim
    from paper_1806_09403_amd._lib import OPT_INTERIOR_PATH, OPT_LBM_VARIANT, OPT_XCD_REMAP
    cases = mixed_cases()
    log("batch launch shape variant=%d interior=%d" % (variant, interior))
    b = BatchSim(cases, precision=4)
    b.set_option(OPT_LBM_VARIANT, variant)
    b.set_option(OPT_INTERIOR_PATH, interior)
    b.set_option(OPT_XCD_REMAP, variant & 1)
    refs = [single(c, 4) for c in cases]
    b.step(9)
    for r in refs:
        r.step(9)
    for k, c in enumerate(cases):
        assert_same(b.cases[k], refs[k], len(c.bodies), 9, k)


def test_batch_graph_replay():
    from paper_1806_09403_amd import BatchSim
    from paper_1806_09403_amd._lib import OPT_GRAPH_CHUNK
    cases = mixed_cases()
    log("batch graph replay")
    a, g = BatchSim(cases, precision=4), BatchSim(cases, precision=4)
    g.set_option(OPT_GRAPH_CHUNK, 6)
    for n in (1, 13, 6, 20):           # odd starts, partial chunks
        a.step(n)
        g.step(n)
        for k in range(len(cases)):
            assert np.array_equal(a.cases[k].populations(), g.cases[k].populations()), (n, k)
    for k, c in enumerate(cases):
        if c.bodies:
            assert np.array_equal(a.cases[k].force_history(40), g.cases[k].force_history(40)), k


def test_batch_masks_unstable_case():
    from paper_1806_09403_amd import BatchSim
    from paper_1806_09403_amd._lib import BtdfUnstable, OPT_MASK_UNSTABLE
    good = mixed_cases()[:2]
    # a channel whose inflow is beyond the marker-velocity guard (|u*| > 0.3)
    bad = W.Case(name="too-fast", nx=80, ny=40, bc=W.CHANNEL, tau=0.6, kind=W.COS4,
                 thickening=W.PAPER_THICKENING[W.COS4], inflow=(0.35, 0.0), init=(1.0, 0.35, 0.0),
                 bodies=[W.cylinder_body(20.0, 20.0, 8.0)], steps=10, precision=4, U=0.35, D=8.0)
    cases = [good[0], bad, good[1]]
    log("batch masking of an unstable case")
    b = BatchSim(cases, precision=4)
    assert b.get_option(OPT_MASK_UNSTABLE) == 1
    refs = [single(c, 4) for c in good]
    b.step(10)
    for r in refs:
        r.step(10)
    unstable, steps = b.status()
    assert list(unstable) == [False, True, False] and steps == 10
    assert_same(b.cases[0], refs[0], len(good[0].bodies), 10, 0)
    assert_same(b.cases[2], refs[1], len(good[1].bodies), 10, 2)
    with pytest.raises(BtdfUnstable):
        b.cases[1].forces()
    b.cases[0].forces()
    # the same case on its own trips the same guard
    s = single(bad, 4)
    s.step(1)
    with pytest.raises(BtdfUnstable):
        s.forces()


def test_batch_autotune_keeps_results():
    from paper_1806_09403_amd import BatchSim
    from paper_1806_09403_amd._lib import OPT_LBM_VARIANT, OPT_NUM_VARIANTS
    cases = mixed_cases()
    log("batch autotune")
    b = BatchSim(cases, precision=4)
    nv = b.get_option(OPT_NUM_VARIANTS)
    best = b.autotune(steps_per_trial=1)
    assert 0 <= best < nv and b.get_option(OPT_LBM_VARIANT) == best
    done = b.status()[1]
    assert done == 2 * nv
    b.step(5)
    refs = [single(c, 4) for c in cases]
    for r in refs:
        r.step(done + 5)
    for k in range(len(cases)):
        assert np.array_equal(b.cases[k].populations(), refs[k].populations()), k


def test_single_autotune_keeps_results():
    from paper_1806_09403_amd._lib import OPT_NUM_VARIANTS
    c = mixed_cases()[0]
    s, r = single(c, 4), single(c, 4)
    nv = s.get_option(OPT_NUM_VARIANTS)
    s.autotune(steps_per_trial=1)
    s.step(3)
    r.step(2 * nv + 3)
    assert np.array_equal(s.populations(), r.populations())


def test_batch_add_body_after_steps_moves_state():
    from paper_1806_09403_amd import BatchSim
    cases = mixed_cases()[:3]
    log("batch: body added after stepping")
    b = BatchSim(cases, precision=8)
    refs = [single(c, 8) for c in cases]
    b.step(3)
    for r in refs:
        r.step(3)
    extra = W.cylinder_body(30.0, 20.0, 6.0)
    b.add_body(0, extra.xy, extra.uv, extra.cx, extra.cy, extra.ds)
    refs[0].add_body(extra.xy, extra.uv, extra.cx, extra.cy, extra.ds)
    b.step(4)
    for r in refs:
        r.step(4)
    for k in range(3):
        assert np.array_equal(b.cases[k].populations(), refs[k].populations()), k


def test_c4_cases_batched_equal_single():
    """The first cases of the 256-case uneven channel workload (FP32)."""
    from paper_1806_09403_amd import BatchSim
    cases = W.c4()[:24]
    log("c4 first 24 cases, 30 steps")
    b = BatchSim(cases, precision=4)
    b.step(30)
    unstable, _ = b.status()
    for k, c in enumerate(cases):
        r = single(c, 4)
        r.step(30)
        if unstable[k]:
            continue
        assert np.array_equal(b.cases[k].populations(), r.populations()), k
        assert np.array_equal(b.cases[k].force_history(30), r.force_history(30)), k
        r.close()


@pytest.mark.parametrize("edge", [1, 0])
@pytest.mark.parametrize("precision", [4, 8])
def test_batch_blocking_equals_single_steps(precision, edge):
    """Three steps per pass in a batch (every case's near tiles stepped singly
    in one launch per step, every case's other tiles in the batched pass;
    edge = 1, the default, also the tiles within reach of each case's
    edges) give the bits of the unblocked batch, after every call: step
    counts that leave 0, 1 or 2 steps over, and cases with and without far
    tiles."""
    from paper_1806_09403_amd import BatchSim
    from paper_1806_09403_amd._lib import OPT_EDGE_TILES, OPT_STEPS_PER_PASS, OPT_TEMPORAL_BLOCKING
    cases = mixed_cases() + [W.random_case(25, nx=300, ny=160, kind=W.COS4, bc=W.CHANNEL, n_bodies=2),
                             W.random_case(26, nx=260, ny=150, kind=W.ROMA3, bc=W.FAR_FIELD, n_bodies=1)]
    log("batch blocking prec=%d edge=%d" % (precision, edge))
    a = BatchSim(cases, precision=precision, options={OPT_TEMPORAL_BLOCKING: 0})
    b = BatchSim(cases, precision=precision, options={OPT_EDGE_TILES: edge})
    assert b.get_option(OPT_EDGE_TILES) == edge
    assert a.get_option(OPT_STEPS_PER_PASS) == 1 and b.get_option(OPT_STEPS_PER_PASS) == 3
    for n in (1, 2, 7, 20, 3):
        a.step(n)
        b.step(n)
        for k in range(len(cases)):
            assert np.array_equal(a.cases[k].populations(), b.cases[k].populations()), (n, k)
    for k, c in enumerate(cases):
        if c.bodies:
            assert np.array_equal(a.cases[k].force_history(40), b.cases[k].force_history(40)), k
    a.close()
    b.close()
