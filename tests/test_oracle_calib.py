"""Pins of the boundary-thickness calibration (Section 2.3, eqs 22-26).

* Flat periodic wall on a node line with ds = dh: the x-part of A is a
  circulant whose rows sum to one (partition of unity), so A 1 = (sum_j
  phi(j - y0)^2) 1 exactly and drs = 1 / sum phi^2 solves eq 24: 2 for the
  3-point kernel, 8/3 for the 4-point kernels, 1 or 2 for the 2-point one
  on / halfway between node lines.
* Cylinder: the mean thickness sits near the values the paper suggests
  (Section 4.4) and follows the trends it describes for Fig. 4 (larger for
  wider kernels, smaller for larger ds, a plateau for 3- and 4-point kernels).
"""
import json
import os

import numpy as np
import pytest

import btdf_workloads as W
from oracle import calib, dense

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
SUM_SQ = {W.ROMA3: 0.5, W.PESKIN4: 3 / 8, W.COS4: 3 / 8}


def wall(L, y0):
    return np.stack([np.arange(L, dtype=float), np.full(L, y0)], 1)


@pytest.mark.parametrize("kind", [W.LINEAR2, W.ROMA3, W.PESKIN4, W.COS4])
@pytest.mark.parametrize("y0", [0.0, 0.3, 0.5])
def test_flat_wall_row_sums(kind, y0):
    L = 32
    A = calib.matrix_A(kind, wall(L, y0), 1.0, period_x=L)
    js = np.arange(-4, 5)
    s2 = np.sum(dense.phi(kind, js - y0) ** 2)
    assert np.allclose(A @ np.ones(L), s2, rtol=0, atol=1e-14)
    if kind in SUM_SQ:
        assert abs(s2 - SUM_SQ[kind]) < 1e-15
        # eq 24 holds with the uniform thickness 1 / sum phi^2
        drs = np.full(L, 1.0 / SUM_SQ[kind])
        assert np.allclose(A @ drs, 1.0, rtol=0, atol=1e-13)


def test_flat_wall_solve_roma3():
    # the 3-point circulant is non-singular at ds = dh (symbol 2/3 + cos(k)/3 >= 1/3)
    for y0 in (0.0, 0.21, 0.5):
        v = calib.thickness_vector(W.ROMA3, wall(32, y0), 1.0, period_x=32)
        assert np.allclose(v, 2.0, rtol=0, atol=1e-12)


def test_flat_wall_solve_linear2():
    v0 = calib.thickness_vector(W.LINEAR2, wall(32, 0.0), 1.0, period_x=32)
    v5 = calib.thickness_vector(W.LINEAR2, wall(32, 0.5), 1.0, period_x=32)
    assert np.allclose(v0, 1.0, atol=1e-12) and np.allclose(v5, 2.0, atol=1e-12)


@pytest.mark.parametrize("kind,name", [(W.LINEAR2, "linear2"), (W.ROMA3, "roma3"),
                                       (W.PESKIN4, "peskin4"), (W.COS4, "peskin4")])
@pytest.mark.parametrize("D", [20.0, 40.0])
def test_cylinder_mean_near_paper(kind, name, D):
    n = int(round(np.pi * D))
    xy = W.cylinder_markers(0.0, 0.0, D, n)
    m = calib.thickness_mean(kind, xy, np.pi * D / n)
    assert abs(m - GOLD["suggested_thickness"]["drs_over_dh"][name]) < 0.15


def mean_at(kind, D, ratio):
    n = int(round(np.pi * D / ratio))
    return calib.thickness_mean(kind, W.cylinder_markers(0.0, 0.0, D, n), np.pi * D / n)


def test_fig4_trends():
    for D in (20.0, 40.0):
        at1 = [mean_at(k, D, 1.0) for k in (W.LINEAR2, W.ROMA3, W.PESKIN4)]
        assert at1[0] < at1[1] < at1[2]                      # grows with drf
        for k in (W.LINEAR2, W.ROMA3, W.PESKIN4, W.COS4):
            assert mean_at(k, D, 0.5) > mean_at(k, D, 2.0)    # falls with ds
        for k in (W.ROMA3, W.PESKIN4, W.COS4):                # plateau
            vals = [mean_at(k, D, r) for r in (0.75, 1.0, 1.5)]
            assert max(vals) - min(vals) < 0.03
