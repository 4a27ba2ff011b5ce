"""The oracle's implicit forcing (IDF, eq 17 = IVC, eqs 32-35 by Appendix A)
and RKPM (eq 36 / B54) against what the paper and the mathematics fix:

* eq 16: with a uniform density the implicit force makes the corrected
  velocity at every marker equal the prescribed one, exactly;
* Appendix A: the implicit method does not depend on the shell thickness;
* the implicit force and the RKPM spreading equal dense numpy linear
  algebra on D_I (eq 14) built independently over the whole periodic grid;
* RKPM with markers too far apart to share a node: A is diagonal with
  A_ll = ds (sum phi^2)^2, so RKPM is the direct forcing whose spreading
  factor drs ds is 1 / (sum phi^2)^2 = 4 (3-point) or 64/9 (4-point).
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.dense import interpolation_matrix
from oracle.oracle import OracleSim

IMPLICIT, RKPM = OracleSim.IMPLICIT, OracleSim.RKPM


def uniform_flow(kind=W.ROMA3, drs=1.9, n=48, U=(0.04, 0.01), bodies=((20.3, 23.7, 10.0, 31),)):
    o = OracleSim(n, n, W.FULLY_PERIODIC, 0.8, kind, drs, init=(1.0, *U))
    out = []
    for cx, cy, D, nm in bodies:
        b = W.cylinder_body(cx, cy, D, nm)
        b.xy = np.mod(b.xy, n)   # positions given inside the periodic grid
        rng = np.random.default_rng(int(cx * 10))
        uv = rng.uniform(-0.01, 0.01, size=(nm, 2))
        o.add_body(b.xy, uv, b.cx, b.cy, b.ds)
        out.append((b, uv))
    return o, out


@pytest.mark.parametrize("kind", [W.ROMA3, W.PESKIN4, W.COS4])
def test_implicit_force_enforces_the_marker_velocity(kind):
    for method, exact in ((IMPLICIT, True), (0, False)):
        o, bodies = uniform_flow(kind, bodies=((14.3, 15.7, 9.0, 28), (36.1, 33.2, 7.0, 22)))
        o.set_forcing_method(method)
        o.step(1)
        u, v = o.marker_corrected_velocity()
        uv = np.concatenate([b[1] for b in bodies])
        err = max(np.max(np.abs(u - uv[:, 0])), np.max(np.abs(v - uv[:, 1])))
        assert (err < 1e-13) == exact, (method, err)


def test_implicit_does_not_depend_on_the_thickness():
    runs = []
    for drs in (1.0, 1.9, 2.6):
        o, _ = uniform_flow(drs=drs)
        o.set_forcing_method(IMPLICIT)
        o.step(3)
        runs.append((drs, o.populations(), o.forces(), o.marker_data()["Fx"]))
    for drs, f, F, Fx in runs[1:]:
        assert np.max(np.abs(f - runs[0][1])) < 1e-15
        assert np.max(np.abs(F - runs[0][2])) < 1e-12 * np.max(np.abs(runs[0][2]))
        assert np.max(np.abs(drs * Fx - runs[0][3])) < 1e-12 * np.max(np.abs(runs[0][3]))


def random_state(o, n, seed):
    rng = np.random.default_rng(seed)
    o.init_equilibrium(0.03 + 0.01 * rng.uniform(-1, 1, (n, n)), 0.01 * rng.uniform(-1, 1, (n, n)),
                       1.0 + 0.01 * rng.uniform(-1, 1, (n, n)))


@pytest.mark.parametrize("kind,drs,cx,cy", [(W.ROMA3, 1.9, 19.3, 20.2), (W.PESKIN4, 1.0, 19.3, 20.2),
                                             (W.COS4, 2.6, 1.3, 38.8)])
def test_implicit_force_equals_a_dense_solve(kind, drs, cx, cy):
    """(1.3, 38.8): a body across both periodic seams of the 40 x 40 grid,
    its markers given on both sides of each seam."""
    n = 40
    o, bodies = uniform_flow(kind, drs, n=n, bodies=((cx, cy, 10.0, 31),))
    random_state(o, n, 3)
    o.set_forcing_method(IMPLICIT)
    o.step(1)
    md = o.marker_data()
    b, uv = bodies[0]
    rhs = np.stack([2 * md["rho"] * (uv[:, 0] - md["ux"]), 2 * md["rho"] * (uv[:, 1] - md["uy"])], axis=1)
    D = interpolation_matrix(kind, n, n, b.xy[:, 0], b.xy[:, 1])
    M = drs * b.ds * (D @ D.T)          # eq 21: D_I D_E
    F = np.linalg.solve(M, rhs)         # eq 17
    scale = np.max(np.abs(F))
    assert np.max(np.abs(md["Fx"] - F[:, 0])) < 1e-10 * scale
    assert np.max(np.abs(md["Fy"] - F[:, 1])) < 1e-10 * scale
    # the spread force is D_E F (eq 13)
    fx, fy = o.force_field()
    assert np.max(np.abs(fx.ravel() - drs * b.ds * D.T @ F[:, 0])) < 1e-12 * scale
    assert np.max(np.abs(fy.ravel() - drs * b.ds * D.T @ F[:, 1])) < 1e-12 * scale


@pytest.mark.parametrize("kind", [W.ROMA3, W.COS4])
def test_rkpm_spreading_equals_dense_row_sums(kind):
    n = 40
    o, bodies = uniform_flow(kind, 1.9, n=n, bodies=((19.3, 20.2, 10.0, 31),))
    random_state(o, n, 4)
    o.set_forcing_method(RKPM)
    o.step(1)
    md = o.marker_data()
    b, uv = bodies[0]
    # the marker force is eq 20 (B52)
    assert np.max(np.abs(md["Fx"] - 2 * md["rho"] * (uv[:, 0] - md["ux"]))) < 1e-15
    D = interpolation_matrix(kind, n, n, b.xy[:, 0], b.xy[:, 1])
    A = b.ds * (D @ D.T)                                  # eq 22
    eps = np.linalg.inv(A).sum(axis=1)                    # B54
    fx, fy = o.force_field()
    ex = D.T @ (b.ds * eps * md["Fx"])
    ey = D.T @ (b.ds * eps * md["Fy"])
    scale = np.max(np.abs(ex)) + np.max(np.abs(ey))
    assert np.max(np.abs(fx.ravel() - ex)) < 1e-10 * scale
    assert np.max(np.abs(fy.ravel() - ey)) < 1e-10 * scale
    # and the body force is minus the total spread force
    F = o.forces()[0]
    assert abs(F[0] + fx.sum()) < 1e-10 * abs(F[0]) and abs(F[1] + fy.sum()) < 1e-10 * max(abs(F[1]), 1e-12)


@pytest.mark.parametrize("kind,shell", [(W.ROMA3, 4.0), (W.PESKIN4, 64.0 / 9.0)])
def test_rkpm_with_isolated_markers_is_a_fixed_shell(kind, shell):
    """Markers 7.65 apart share no node; sum_i phi(x - i)^2 is 1/2 (3-point)
    and 3/8 (4-point) at every offset, so A_ll = ds (sum phi^2)^2."""
    n = 48
    t = np.linspace(0.0, 2 * np.pi, 9, endpoint=False)
    xy = np.stack([24.3 + 10.0 * np.cos(t), 23.9 + 10.0 * np.sin(t)], axis=1)   # 7.65 apart
    ds = 0.8
    runs = []
    for method, drs in ((RKPM, 1.9), (0, shell / ds)):   # direct forcing spreads drs ds F
        o = OracleSim(n, n, W.FULLY_PERIODIC, 0.8, kind, drs, init=(1.0, 0.03, 0.0))
        o.add_body(xy, None, 24.3, 23.9, ds)
        random_state(o, n, 5)
        o.set_forcing_method(method)
        o.step(4)
        runs.append((o.populations(), o.forces()))
    assert np.max(np.abs(runs[0][0] - runs[1][0])) < 1e-15
    assert np.max(np.abs(runs[0][1] - runs[1][1])) < 1e-12 * np.max(np.abs(runs[1][1]))
