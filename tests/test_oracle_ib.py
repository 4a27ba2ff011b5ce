"""Pins of the oracle's immersed-boundary part (Sections 2.2-2.3, 3.1, 5.2).

* interpolation reproduces constant fields (all kernels) and linear fields
  (kernels with a zero first moment) exactly (eqs 12, 14);
* spreading is the adjoint of interpolation: sum_k f_k dh^2 equals
  sum_l F_l ds drs (both sides of eq 27), and D_E = drs ds D_I^T (eq 15);
* uniform flow with markers moving at the flow velocity gives F = 0 (eq 20);
* steady force balance on a periodic box driven by a body force: the drag
  on the body equals the total driving force (fixes the sign and the
  drs ds factor of eq 27);
* a rotating cylinder in fluid at rest feels a retarding torque;
* the loop oracle equals the dense-matrix brute force step by step;
* mirror symmetry of the cylinder channel;
* the thickened shell cuts the no-slip error (eq 45) against conventional
  direct forcing (drs = dh, eq 28) -- the paper's central claim.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle import dense
from oracle.oracle import OracleSim

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def from_case(c):
    s = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    ux, uy = c.init_fields()
    s.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    return s


def pre_streamed_equilibrium(nx, ny, ufun):
    """Populations A with A_q(x) = feq_q(1, u(x + e_q)), so that the streamed
    populations at x are exactly the equilibrium of u(x); feq from dense."""
    y, x = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    A = np.empty((9, ny, nx))
    for q in range(9):
        ux, uy = ufun(x + EX[q], y + EY[q])
        A[q] = dense.equilibrium(np.ones((ny, nx)), ux, uy)[q]
    return A


@pytest.mark.parametrize("kind", [W.LINEAR2, W.ROMA3, W.PESKIN4, W.COS4])
def test_interpolation_reproduces_constant_and_linear(oracle_lib, kind):
    nx = ny = 40
    rng = np.random.default_rng(5)
    xy = np.column_stack([rng.uniform(15, 25, 12), rng.uniform(15, 25, 12)])
    a, bx, by = 0.01, 3e-4, -2e-4

    def lin(x, y):
        return a + bx * x + by * y, -a + by * x + bx * y

    def const(x, y):
        return np.full_like(x, 0.013), np.full_like(x, -0.007)

    for fun, exact_linear in ((const, True), (lin, kind != W.COS4)):
        s = OracleSim(nx, ny, W.FULLY_PERIODIC, 0.8, kind, 1.0)
        s.add_body(xy, None, 20.0, 20.0, 1.0)
        s.set_populations(pre_streamed_equilibrium(nx, ny, fun))
        s.step(1)
        md = s.marker_data()
        ux, uy = fun(xy[:, 0], xy[:, 1])
        assert np.allclose(md["rho"], 1.0, rtol=0, atol=1e-14)
        err = max(np.max(np.abs(md["ux"] - ux)), np.max(np.abs(md["uy"] - uy)))
        if exact_linear:
            assert err < 1e-15
        else:
            assert err > 1e-8  # the cosine kernel has a non-zero first moment


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spread_adjoint_and_eq27(oracle_lib, seed):
    c = W.random_case(seed, nx=31, ny=26, n_bodies=3)
    s = from_case(c)
    s.step(3)
    md = s.marker_data()
    fx, fy = s.force_field()
    ds_l = np.concatenate([np.full(b.xy.shape[0], b.ds) for b in c.bodies])
    # eq 27: sum_l F_l ds drs == sum_k f_k dh^2
    assert abs(np.sum(md["Fx"] * ds_l) * c.thickening - fx.sum()) < 1e-15 * max(1, np.abs(fx).sum())
    assert abs(np.sum(md["Fy"] * ds_l) * c.thickening - fy.sum()) < 1e-15 * max(1, np.abs(fy).sum())
    # body forces are minus the per-body sums
    F = s.forces()
    m0 = 0
    for b, body in enumerate(c.bodies):
        sl = slice(m0, m0 + body.xy.shape[0])
        m0 += body.xy.shape[0]
        assert abs(F[b, 0] + body.ds * c.thickening * md["Fx"][sl].sum()) < 1e-17 + 1e-14 * abs(F[b, 0])
    # D_E = drs ds D_I^T: the spread field equals the dense transpose applied to F
    X = np.concatenate([b.xy[:, 0] for b in c.bodies])
    Y = np.concatenate([b.xy[:, 1] for b in c.bodies])
    DI = dense.interpolation_matrix(c.kind, c.nx, c.ny, X, Y)
    f_dense = (DI.T * (c.thickening * ds_l)[None, :]) @ md["Fx"]
    assert np.max(np.abs(f_dense - fx.ravel())) < 1e-16 + 1e-14 * np.max(np.abs(fx))


def test_uniform_flow_markers_comoving(oracle_lib):
    u0 = (0.03, -0.01)
    for kind in (W.ROMA3, W.COS4):
        s = OracleSim(48, 40, W.FULLY_PERIODIC, 0.7, kind, 2.0, init=(1.0,) + u0)
        body = W.cylinder_body(20.3, 18.7, 12.0)
        s.add_body(body.xy, np.tile(u0, (body.xy.shape[0], 1)), body.cx, body.cy, body.ds)
        f0 = s.populations()
        s.step(20)
        md = s.marker_data()
        assert np.max(np.abs(md["Fx"])) < 1e-15 and np.max(np.abs(md["Fy"])) < 1e-15
        assert np.max(np.abs(s.populations() - f0)) < 1e-15


def test_steady_force_balance(oracle_lib):
    # periodic box driven by G: at steady state the total momentum is constant,
    # so the drag on the cylinder (eq 27 with the body sign) equals N G
    nx = ny = 32
    G = 2e-6
    s = OracleSim(nx, ny, W.FULLY_PERIODIC, 1.0, W.ROMA3, 1.9, G=(G, 0.0))
    body = W.cylinder_body(15.5, 16.2, 8.0)
    s.add_body(body.xy, None, body.cx, body.cy, body.ds)
    s.step(30000)
    F = s.forces()[0]
    assert abs(F[0] / (nx * ny * G) - 1) < 1e-6
    assert abs(F[1]) < 1e-6 * nx * ny * G


def test_momentum_budget_each_step(oracle_lib):
    c = W.random_case(7, nx=30, ny=24, n_bodies=2)
    s = from_case(c)
    one = np.ones(9)
    for _ in range(4):
        p0 = np.einsum("q,qij->", EX, s.populations())
        s.step(1)
        p1 = np.einsum("q,qij->", EX, s.populations())
        drag = s.forces()[:, 0].sum()
        assert abs((p1 - p0) - (c.nx * c.ny * c.G[0] - drag)) < 1e-14 * (abs(p0) + abs(drag)) * 10


def test_rotating_cylinder_torque_sign(oracle_lib):
    s = OracleSim(48, 48, W.FULLY_PERIODIC, 0.8, W.PESKIN4, 2.6)
    body = W.cylinder_body(24.0, 24.0, 16.0)
    omega = 0.002
    r = body.xy - np.array([body.cx, body.cy])
    uv = omega * np.column_stack([-r[:, 1], r[:, 0]])
    s.add_body(body.xy, uv, body.cx, body.cy, body.ds)
    s.step(200)
    F = s.forces()[0]
    assert F[2] < 0
    assert abs(F[0]) < 1e-12 * abs(F[2]) * 100 and abs(F[1]) < 1e-12 * abs(F[2]) * 100


@pytest.mark.parametrize("kind", [W.LINEAR2, W.ROMA3, W.PESKIN4, W.COS4])
def test_loop_oracle_equals_dense_brute_force(oracle_lib, kind):
    nx, ny = 12, 10
    rng = np.random.default_rng(kind)
    tau, drs, G = 0.71, W.PAPER_THICKENING[kind], (2e-5, 1e-5)
    d = dense.DenseSim(nx, ny, tau, kind, drs, G)
    s = OracleSim(nx, ny, W.FULLY_PERIODIC, tau, kind, drs, G)
    bodies = [((3.3, 4.1), 3.0, 5), ((9.4, 8.7), 2.5, 4)]   # the second one wraps
    for (cx, cy), D, n in bodies:
        xy = W.cylinder_markers(cx, cy, D, n)
        uv = rng.uniform(-0.01, 0.01, (n, 2))
        d.add_body(xy, uv, cx, cy, np.pi * D / n)
        s.add_body(xy, uv, cx, cy, np.pi * D / n)
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    A0 = dense.equilibrium(1 + 0.01 * np.cos(2 * np.pi * x / nx), 0.02 * np.sin(2 * np.pi * y / ny),
                           0.01 * np.cos(2 * np.pi * (x + y) / nx))
    d.A = A0.copy()
    s.set_populations(A0)
    for _ in range(10):
        d.step()
        s.step(1)
        assert np.max(np.abs(s.populations() - d.A)) < 1e-14
        assert np.max(np.abs(s.forces() - d.forces)) < 1e-16 + 1e-13 * np.max(np.abs(d.forces))


def c1_run(kind, thickening, steps):
    c = W.c1(kind=kind, thickening=thickening, steps=steps)
    s = from_case(c)
    s.step(steps)
    return c, s


def test_channel_mirror_symmetry(oracle_lib):
    c, s = c1_run(W.COS4, None, 2000)
    F = s.forces()[0]
    assert F[0] > 0                                   # drag opposes the flow
    assert abs(F[1]) <= 1e-10 * abs(F[0])
    _, u, v = s.macroscopic()
    j = np.arange(c.ny)
    mirror = (2 * 60 - j) % c.ny
    assert np.max(np.abs(v + v[mirror])) < 1e-12 * np.max(np.abs(u))
    assert np.max(np.abs(u - u[mirror])) < 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("kind,ratio", [(W.ROMA3, 0.5), (W.PESKIN4, 0.5), (W.COS4, 0.75)])
def test_thickening_cuts_boundary_error(oracle_lib, kind, ratio):
    errs = {}
    for th in (W.PAPER_THICKENING[kind], 1.0):
        c, s = c1_run(kind, th, 2000)
        uc, vc = s.marker_corrected_velocity()
        errs[th] = np.sqrt(np.mean(uc ** 2 + vc ** 2))     # eq 45 (U_b = 0)
    assert errs[W.PAPER_THICKENING[kind]] < ratio * errs[1.0]
