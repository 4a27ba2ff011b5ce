"""The library's thickness calibration (eqs 22, 25, 26) swept as in Fig. 4,
against the oracle's dense-matrix calibration on the same markers."""
import math

import numpy as np
import pytest

import btdf_workloads as W
from oracle import calib


@pytest.mark.parametrize("kind", [W.LINEAR2, W.ROMA3, W.PESKIN4, W.COS4])
def test_sweep_matches_the_oracle_and_the_fig4_trends(kind):
    from paper_1806_09403_amd import sweeps
    rows = sweeps.calibration(kinds=(kind,), D_values=(20,), ds_values=(0.5, 1.0, 1.5), log=lambda m: None)
    for r in rows:
        n = int(round(math.pi * r["D"] / r["ds"]))
        b = W.cylinder_body(0.3 + 2.0 * r["D"], 0.6 + 2.0 * r["D"], float(r["D"]), n)
        ref = calib.thickness_mean(kind, b.xy, b.ds)
        assert abs(r["drs_mean"] - ref) < 1e-9 * ref
    drs = [r["drs_mean"] for r in rows]
    # Fig. 4: the calibrated thickness falls as markers spread and levels off near ds = dh
    assert drs[0] > drs[1] >= drs[2] - 0.05
    assert abs(drs[1] - W.PAPER_THICKENING[kind]) < 0.25
