"""btdf_marker_velocity_noalloc, the entry point that allocates nothing,
against btdf_marker_velocity on the same handles: the corrected velocity of
the last step (eq 11) interpolated at every marker (eq 12). Two calls in a
row share the fixed staging array, the second with fewer markers; a third
goes back to the first handle."""
import dataclasses

import numpy as np
import pytest

import btdf_workloads as W


def both(g):
    from paper_1806_09403_amd import api
    h = g._workspace()
    u0, v0 = api.btdf_marker_velocity(h)
    nm = u0.shape[0]
    # caller-owned outputs, filled with a marker value first
    u1, v1 = np.full(nm, np.nan), np.full(nm, np.nan)
    api.btdf_marker_velocity_noalloc(h, u1, v1)
    return u0, v0, u1, v1


def check(u0, v0, u1, v1, tol, what):
    scale = max(np.max(np.abs(u0)), np.max(np.abs(v0)), 1e-30)
    d = max(np.max(np.abs(u1 - u0)), np.max(np.abs(v1 - v0))) / scale
    same = np.array_equal(u0, u1) and np.array_equal(v0, v1)
    print("  %s: %d markers, max rel diff %.3e, bit-identical %s" % (what, u0.shape[0], d, same), flush=True)
    assert np.all(np.isfinite(u1)) and np.all(np.isfinite(v1))
    assert d <= tol


@pytest.mark.gpu
def test_noalloc_marker_velocity_matches_the_allocating_call():
    from paper_1806_09403_amd import Sim
    # the 8192^2 particle-laden lattice with its 2000 cylinders (150 000
    # markers), FP32, stepped in the benchmark's launch configuration
    print("no-alloc call 1: 8192^2, 2000 cylinders, FP32", flush=True)
    big = Sim.from_case(W.c3(), precision=4)
    big.step(7)  # two three-step passes and one single step
    check(*both(big), 1e-6, "8192^2 FP32")
    # a smaller FP64 channel with three bodies
    print("no-alloc call 2: 150x90 channel, FP64", flush=True)
    c = W.random_case(47, nx=150, ny=90, kind=W.ROMA3, bc=W.CHANNEL, n_bodies=3, D_range=(5.0, 9.0))
    c = dataclasses.replace(c, init=(1.0, 0.02, 0.01))
    small = Sim.from_case(c, precision=8)
    small.step(4)
    check(*both(small), 1e-12, "channel FP64")
    # the larger handle again, after the smaller call left its results behind
    print("no-alloc call 3: 8192^2 again", flush=True)
    big.step(2)
    check(*both(big), 1e-6, "8192^2 FP32, again")
    small.close()
    big.close()


def test_noalloc_rejects_more_markers_than_its_array():
    """The limit is checked on the host before any device work."""
    from paper_1806_09403_amd import BtdfError, _lib, api
    h = api.btdf_create(4096, 4096, 0.8, W.COS4, 2.6)
    try:
        n = _lib.NOALLOC_MAX_MARKERS + 1
        t = 2.0 * np.pi * np.arange(n) / n
        xy = np.stack([2048.0 + 1500.0 * np.cos(t), 2048.0 + 1500.0 * np.sin(t)], axis=1)
        api.btdf_add_body(h, xy, None, 2048.0, 2048.0, 0.0)
        u, v = np.empty(n), np.empty(n)
        with pytest.raises(BtdfError) as e:
            api.btdf_marker_velocity_noalloc(h, u, v)
        assert e.value.code == _lib.EINVAL and "at most" in str(e.value)
    finally:
        api.btdf_destroy(h)
