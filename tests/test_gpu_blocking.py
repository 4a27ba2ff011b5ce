"""Temporal blocking (two to five steps per pass for tiles away from the
markers; at two or three steps, tiles at the domain edges with the boundary
readings in every step) gives bit-identical results to single steps, for
every boundary set, ragged edge, forcing method, precision and launch shape
that has the blocked pass."""
import dataclasses

import numpy as np
import pytest

import btdf_workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def run(c, blocking, steps, precision=4, options=None, timed=False):
    from paper_1806_09403_amd import Sim, _lib
    s = Sim.from_case(c, precision=precision)
    for k, v in (options or {}).items():
        s.set_option(k, v)
    s.set_option(_lib.OPT_TEMPORAL_BLOCKING, blocking)
    fused = s.get_option(_lib.OPT_FUSED_TILES)
    if fused:
        # the depth asked for, or the deepest below it that the launch shape has
        assert 2 <= s.get_option(_lib.OPT_STEPS_PER_PASS) <= (5 if blocking == 1 else blocking)
    for n in steps:
        if timed == "pass":
            s.step_timed_pass(n)
        elif timed:
            s.step_timed_split(n)
        else:
            s.step(n)
    out = (s.populations(), s.force_history(200), fused)
    s.close()
    return out


def bodies_case(seed, nx, ny, bc, kind=W.COS4, n=6):
    c = W.random_case(seed, nx=nx, ny=ny, kind=kind, bc=bc, n_bodies=n, D_range=(6.0, 12.0))
    return c


CASES = [
    ("periodic", 41, 512, 256, W.FULLY_PERIODIC),
    ("channel", 42, 400, 200, W.CHANNEL),
    ("walls", 43, 300, 160, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL)),
    ("far-field", 44, 420, 180, W.FAR_FIELD),
    # the outlet's ghost column alone in the last tile column, ragged rows
    ("channel-ragged", 45, 417, 203, W.CHANNEL),
    ("walls-ragged", 46, 300, 165, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL)),
]


@pytest.mark.parametrize("depth,edge", [(2, 0), (2, 1), (3, 0), (3, 1), (4, 0), (5, 0)])
@pytest.mark.parametrize("precision", [4, 8])
@pytest.mark.parametrize("name,seed,nx,ny,bc", CASES)
def test_blocked_steps_are_bit_identical(name, seed, nx, ny, bc, precision, depth, edge):
    """edge = 1: the tiles within reach of the domain edges take the pass too
    (every case here has some: periodic seams, walls, inlet and outlet)."""
    from paper_1806_09403_amd import Sim, _lib
    log("blocking %s prec=%d depth=%d edge=%d" % (name, precision, depth, edge))
    c = bodies_case(seed, nx, ny, bc)
    steps = (1, 2, 7, 8, 20)   # leftovers of every size after whole passes
    ref = run(c, 0, steps, precision)
    got = run(c, depth, steps, precision, options={_lib.OPT_EDGE_TILES: edge})
    assert got[2] > 0 and ref[2] == 0
    s = Sim.from_case(c, precision=precision)
    s.set_option(_lib.OPT_TEMPORAL_BLOCKING, depth)
    s.set_option(_lib.OPT_EDGE_TILES, edge)
    assert s.get_option(_lib.OPT_STEPS_PER_PASS) == depth
    assert (s.get_option(_lib.OPT_EDGE_FUSED_TILES) > 0) == bool(edge)
    s.close()
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("depth", [2, 3, 4, 5])
@pytest.mark.parametrize("opts", ["passes", "implicit", "rkpm", "timed", "timed-pass"])
def test_blocking_with_other_features(opts, depth):
    from paper_1806_09403_amd import _lib
    c = bodies_case(45, 384, 192, W.CHANNEL, kind=W.ROMA3)
    o = {"passes": {_lib.OPT_FORCING_PASSES: 3}, "implicit": {_lib.OPT_FORCING_METHOD: 1},
         "rkpm": {_lib.OPT_FORCING_METHOD: 2}, "timed": {}, "timed-pass": {}}[opts]
    timed = "pass" if opts == "timed-pass" else opts.endswith("timed")
    ref = run(c, 0, (3, 10, 13), 4, o, timed=timed)
    got = run(c, depth, (3, 10, 13), 4, o, timed=timed)
    assert got[2] > 0
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("depth,min_active", [(2, 10), (3, 6), (5, 6)])
def test_every_launch_shape_with_the_blocked_pass(depth, min_active):
    """Every launch shape, the edge tiles in the pass wherever the shape
    has it for them."""
    from paper_1806_09403_amd import Sim, _lib
    c = bodies_case(46, 520, 260, W.FULLY_PERIODIC)
    ref = run(c, 0, (9,))
    s = Sim.from_case(c, precision=4)
    nv = s.get_option(_lib.OPT_NUM_VARIANTS)
    s.close()
    active = 0
    for v in range(nv):
        got = run(c, depth, (9,), options={_lib.OPT_LBM_VARIANT: v, _lib.OPT_EDGE_TILES: 1})
        active += got[2] > 0
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), v
    log("  %d launch shapes with a pass of depth %d or less" % (active, depth))
    assert active >= min_active


def test_default_depth_follows_the_lattice_size():
    """By default lattices of 2^20 nodes or more take five steps per pass in
    FP32 and three in FP64, and smaller ones step singly; a depth asked for
    explicitly applies to any size."""
    from paper_1806_09403_amd import Sim, _lib
    big = bodies_case(47, 1024, 1024, W.FULLY_PERIODIC)
    small = bodies_case(47, 512, 256, W.FULLY_PERIODIC)
    for prec in (4, 8):
        s = Sim.from_case(big, precision=prec)
        assert s.get_option(_lib.OPT_TEMPORAL_BLOCKING) == 1
        assert s.get_option(_lib.OPT_STEPS_PER_PASS) == (5 if prec == 4 else 3)
        s.set_option(_lib.OPT_TEMPORAL_BLOCKING, 4)
        assert s.get_option(_lib.OPT_STEPS_PER_PASS) == 4
        s.set_option(_lib.OPT_TEMPORAL_BLOCKING, 3)
        assert s.get_option(_lib.OPT_STEPS_PER_PASS) == 3
        s.set_option(_lib.OPT_TEMPORAL_BLOCKING, 2)
        assert s.get_option(_lib.OPT_STEPS_PER_PASS) == 2
        s.close()
        s = Sim.from_case(small, precision=prec)
        assert s.get_option(_lib.OPT_STEPS_PER_PASS) == 1
        s.set_option(_lib.OPT_TEMPORAL_BLOCKING, 3)
        assert s.get_option(_lib.OPT_STEPS_PER_PASS) == 3
        s.close()


def test_moving_bodies_step_singly_under_blocking():
    from paper_1806_09403_amd import Sim, _lib
    outs = []
    for blocking in (0, 3):   # (3: asked for explicitly, whatever the lattice size)
        s = Sim(256, 128, 0.8, W.ROMA3, 1.9, W.FULLY_PERIODIC, init=(1.0, 0.02, 0.0), precision=4)
        b = W.cylinder_body(100.3, 60.2, 12.0, 38)
        s.add_body(b.xy, None, b.cx, b.cy, b.ds)
        s.set_option(_lib.OPT_TEMPORAL_BLOCKING, blocking)
        s.set_body_motion(0, 0.03, 0.0, 0.001)
        assert s.get_option(_lib.OPT_FUSED_TILES) == 0
        s.step(50)
        outs.append(s.populations())
        s.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("depth,chunk,edge", [(3, 7, 0), (3, 9, 1), (3, 12, 0), (2, 6, 1), (2, 8, 0), (4, 9, 0),
                                              (4, 13, 0), (5, 10, 0), (5, 15, 0)])
def test_blocked_passes_in_graphs(depth, chunk, edge):
    """Graphs of chunk // depth whole passes (an even or an odd number of
    passes, so graphs are entered from either buffer, with single steps
    before and after) give the bits of eager single steps, checked after
    every call: each call replays the graph one or more times, with the
    program's own synchronising reads between the calls."""
    from paper_1806_09403_amd import Sim, _lib
    log("blocked graphs depth=%d chunk=%d edge=%d" % (depth, chunk, edge))
    c = bodies_case(49, 384, 192, W.CHANNEL)
    ref = Sim.from_case(c, precision=4)
    ref.set_option(_lib.OPT_TEMPORAL_BLOCKING, 0)
    got = Sim.from_case(c, precision=4)
    got.set_option(_lib.OPT_GRAPH_CHUNK, chunk)
    got.set_option(_lib.OPT_TEMPORAL_BLOCKING, depth)
    got.set_option(_lib.OPT_EDGE_TILES, edge)
    assert got.get_option(_lib.OPT_STEPS_PER_PASS) == depth
    for n in (1, 25, 2, 30, 19):
        ref.step(n)
        got.step(n)
        assert np.array_equal(got.populations(), ref.populations()), n
        assert np.array_equal(got.force_history(200), ref.force_history(200)), n
    ref.close()
    got.close()


@pytest.mark.parametrize("depth", [0, 2, 3, 4, 5])
def test_pass_timing_reports_the_pass(depth):
    """btdf_step_timed_pass: a positive time per step when passes ran, 0
    without blocking; the steps are the same as plain ones."""
    from paper_1806_09403_amd import Sim, _lib
    c = bodies_case(48, 512, 256, W.FULLY_PERIODIC)
    ref = run(c, 0, (10,))
    s = Sim.from_case(c, precision=4)
    s.set_option(_lib.OPT_TEMPORAL_BLOCKING, depth)
    ms = s.step_timed_pass(10)
    log("  depth %d: pass %.4f ms per step" % (depth, ms))
    assert (ms > 0) == (depth > 0)
    assert np.array_equal(s.populations(), ref[0])
    s.close()
