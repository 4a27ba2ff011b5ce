"""The oracle's forcing passes (Algorithm 1 step 3 with NF > 1, eqs 29-31).

One pass is the method as proposed and must equal the default step. Many
passes are a fixed-point iteration whose limit the paper names: the
implicit direct force (eq 17), at which the corrected velocity interpolated
to the markers equals the prescribed one. That limit is computed here
independently, with dense D_I / D_E matrices (eqs 14, 15) and a linear
solve, from the streamed populations formed by whole-array shifts.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.dense import E, interpolation_matrix
from oracle.oracle import OracleSim


def make(kind, thickening, nf, nx=32, ny=32, u0=(0.03, 0.01), D=8.0):
    o = OracleSim(nx, ny, W.FULLY_PERIODIC, 0.7, kind, thickening, (0.0, 0.0), (0.0, 0.0), (1.0, *u0))
    b = W.cylinder_body(15.3, 16.6, D)
    o.add_body(b.xy, None, b.cx, b.cy, b.ds)
    # a non-uniform density, so that the 1/rho of the corrected velocity matters
    y, x = np.mgrid[0:ny, 0:nx]
    rho = 1.0 + 0.05 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)
    o.init_equilibrium(np.full((ny, nx), u0[0]), np.full((ny, nx), u0[1]), rho)
    o.set_forcing_passes(nf)
    return o, b


def test_one_pass_is_the_default():
    c = W.random_case(3, nx=40, ny=30, kind=W.COS4, bc=W.CHANNEL, n_bodies=1)
    runs = []
    for nf in (None, 1):
        o = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
        for b in c.bodies:
            o.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
        if nf is not None:
            o.set_forcing_passes(nf)
        o.step(5)
        runs.append((o.populations(), o.forces()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("kind,thickening", [(W.ROMA3, 1.0), (W.ROMA3, 1.9), (W.LINEAR2, 1.4)])
def test_many_passes_reach_the_implicit_force(kind, thickening):
    o, b = make(kind, thickening, nf=4000)
    A = o.populations()
    o.step(1)
    md = o.marker_data()
    # the implicit force from the same state, with dense operators
    g = np.stack([np.roll(A[q], shift=(E[1, q], E[0, q]), axis=(0, 1)) for q in range(9)])
    rho = g.sum(axis=0).ravel()
    usx = (np.tensordot(E[0], g, axes=(0, 0)).ravel()) / rho
    usy = (np.tensordot(E[1], g, axes=(0, 0)).ravel()) / rho
    DI = interpolation_matrix(kind, 32, 32, b.xy[:, 0], b.xy[:, 1])
    DE = DI.T * (thickening * b.ds)
    M = DI @ (DE / rho[:, None]) / 2.0
    Fx = np.linalg.solve(M, 0.0 - DI @ usx)
    Fy = np.linalg.solve(M, 0.0 - DI @ usy)
    scale = np.max(np.abs(np.concatenate([Fx, Fy])))
    assert np.max(np.abs(md["Fx"] - Fx)) < 1e-8 * scale
    assert np.max(np.abs(md["Fy"] - Fy)) < 1e-8 * scale
    # the corrected velocity at the markers is the prescribed one (at rest)
    u, v = o.marker_corrected_velocity()
    assert max(np.max(np.abs(u)), np.max(np.abs(v))) < 1e-10


@pytest.mark.parametrize("kind,thickening", [(W.ROMA3, 1.0), (W.COS4, 2.6)])
def test_slip_falls_with_passes(kind, thickening):
    """The boundary error (eq 45) of one step decreases with the number of
    passes (the direction of Fig. 16(b))."""
    errs = []
    for nf in (1, 2, 4, 8, 16, 64):
        o, _ = make(kind, thickening, nf)
        o.step(1)
        u, v = o.marker_corrected_velocity()
        errs.append(np.sqrt(np.mean(u * u + v * v)))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
