"""Pins of the regularised delta functions (Section 4.3, eqs 37-39, and the
cosine 4-point kernel) in both host implementations (C loop oracle and the
numpy dense brute force): closed-form values and the moment identities
every one of these kernels is built to satisfy."""
import numpy as np
import pytest

from oracle import dense
from oracle import oracle as orc

KINDS = [orc.LINEAR2, orc.ROMA3, orc.PESKIN4, orc.COS4]
HALF = {orc.LINEAR2: 1.0, orc.ROMA3: 1.5, orc.PESKIN4: 2.0, orc.COS4: 2.0}


def impls(kind):
    return [lambda r: orc.delta(kind, r), lambda r: dense.phi(kind, r)]


def node_sums(phi, X, power=1, moment=0, parity=None):
    lo, hi = int(np.floor(X - 3)), int(np.ceil(X + 3))
    js = np.arange(lo, hi + 1)
    if parity is not None:
        js = js[js % 2 == parity]
    r = js - X
    return np.sum(r ** moment * phi(r) ** power)


@pytest.mark.parametrize("kind", KINDS)
def test_partition_of_unity(oracle_lib, kind):
    # sum_j phi(j - X) = 1 for every X (the partition-of-unity condition behind eqs 18-19)
    rng = np.random.default_rng(1)
    for phi in impls(kind):
        for X in np.concatenate([rng.uniform(-3, 3, 200), [0.0, 0.5, 1.0, -0.5, 0.25]]):
            assert abs(node_sums(phi, X) - 1.0) < 1e-14


@pytest.mark.parametrize("kind", [orc.LINEAR2, orc.ROMA3, orc.PESKIN4])
def test_first_moment_zero(oracle_lib, kind):
    rng = np.random.default_rng(2)
    for phi in impls(kind):
        for X in rng.uniform(-3, 3, 200):
            assert abs(node_sums(phi, X, moment=1)) < 1e-14


def test_cosine_first_moment_not_zero(oracle_lib):
    # the cosine kernel does not reproduce linear functions: the moment is
    # (1/4) sum_j r_j cos(pi r_j / 2) != 0 away from integer and half-integer X
    for phi in impls(orc.COS4):
        assert abs(node_sums(phi, 0.3, moment=1)) > 1e-3


@pytest.mark.parametrize("kind,val", [(orc.ROMA3, 0.5), (orc.PESKIN4, 3 / 8), (orc.COS4, 3 / 8)])
def test_sum_of_squares(oracle_lib, kind, val):
    rng = np.random.default_rng(3)
    for phi in impls(kind):
        for X in rng.uniform(-3, 3, 200):
            assert abs(node_sums(phi, X, power=2) - val) < 1e-14


@pytest.mark.parametrize("kind", [orc.PESKIN4, orc.COS4])
def test_even_odd_sums(oracle_lib, kind):
    rng = np.random.default_rng(4)
    for phi in impls(kind):
        for X in rng.uniform(-3, 3, 100):
            assert abs(node_sums(phi, X, parity=0) - 0.5) < 1e-14
            assert abs(node_sums(phi, X, parity=1) - 0.5) < 1e-14


@pytest.mark.parametrize("kind,values", [
    (orc.LINEAR2, {0.0: 1.0, 0.5: 0.5, 1.0: 0.0}),
    (orc.ROMA3, {0.0: 2 / 3, 1.0: 1 / 6, 0.5: 0.5, 1.5: 0.0}),
    (orc.PESKIN4, {0.0: 0.5, 1.0: 0.25, 2.0: 0.0}),
    (orc.COS4, {0.0: 0.5, 1.0: 0.25, 2.0: 0.0}),
])
def test_closed_form_values(oracle_lib, kind, values):
    for phi in impls(kind):
        for r, v in values.items():
            assert abs(float(phi(np.array(r))) - v) < 1e-15
            assert abs(float(phi(np.array(-r))) - v) < 1e-15


@pytest.mark.parametrize("kind", KINDS)
def test_support_and_continuity(oracle_lib, kind):
    h = HALF[kind]
    for phi in impls(kind):
        r = np.linspace(-h - 1, h + 1, 2001)
        v = phi(r)
        assert np.all(v[np.abs(r) > h] == 0.0)
        assert np.all(v >= 0.0)
        # continuous: no jump bigger than the slope bound times the step
        assert np.max(np.abs(np.diff(v))) < 2.0 * (r[1] - r[0])
