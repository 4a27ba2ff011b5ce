"""GPU reverse mode (btdf_adjoint) through the C ABI.

FP64: every gradient equals the FP64 oracle's adjoint on small cases of
every boundary kind and delta (the oracle's adjoint is itself pinned to
central differences of its forward step). Checkpointed and taped sweeps are
bit-identical, and the forward run inside btdf_adjoint leaves exactly the
state and history plain stepping leaves. On the 800x400 Re = 100 channel
(126 markers, 5000 steps) the FP64 adjoint's gradients of the mean drag
coefficient (inflow speed, cylinder centre, marker velocities) agree with
FP64 central differences of the GPU forward run to 1e-4; the FP32 adjoint
meets that bound for marker velocities norm-wise but not for the inflow
speed and the centre (an expected failure that states the measured errors).
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def oracle_of(c):
    o = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        o.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    if c.init_uy is not None:
        ux, uy = c.init_fields()
        o.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    return o


def gpu_of(c, precision):
    from paper_1806_09403_amd import Sim
    return Sim.from_case(c, precision=precision)


CASES = [
    # (seed, nx, ny, kind, bc, n_bodies, n_steps)
    (1, 24, 20, W.COS4, W.FULLY_PERIODIC, 2, 6),
    (2, 18, 16, W.ROMA3, W.CHANNEL, 1, 10),
    (3, 26, 20, W.PESKIN4, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), 2, 5),
    (4, 18, 17, W.COS4, (W.VELOCITY_INLET, W.ZERO_GRADIENT_OUTLET, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), 1, 10),
    (5, 25, 19, W.LINEAR2, W.FULLY_PERIODIC, 2, 4),
    (8, 150, 70, W.COS4, W.FULLY_PERIODIC, 3, 7),  # several adjoint tiles, ragged edges, bodies across the periodic edges
]
KEYS = [("populations", "populations"), ("inflow", "inflow"), ("body_force", "body_force"),
        ("marker_xy", "xy"), ("marker_uv", "uv"), ("centres", "centres")]


def small_case(seed, nx, ny, kind, bc, nbody):
    c = W.random_case(seed, nx=nx, ny=ny, kind=kind, bc=bc, n_bodies=nbody, D_range=(4.0, 6.0))
    if bc[0] == W.VELOCITY_INLET:
        c.inflow = (0.03, 0.004)
    return c


@pytest.mark.parametrize("seed,nx,ny,kind,bc,nbody,n", CASES)
def test_fp64_adjoint_matches_oracle(seed, nx, ny, kind, bc, nbody, n):
    log("fp64 adjoint vs oracle seed=%d %dx%d kind=%d" % (seed, nx, ny, kind))
    c = small_case(seed, nx, ny, kind, bc, nbody)
    hbar = np.random.default_rng(200 + seed).standard_normal((n, nbody, 3))
    go = oracle_of(c).adjoint(n, hbar)
    s = gpu_of(c, 8)
    gg, ms = s.adjoint(n, hbar, checkpoint_every=0)
    for gk, ok in KEYS:
        ref, got = go[ok], gg[gk]
        scale = max(np.max(np.abs(ref)), 1e-300) if ref.size else 1.0
        assert got.shape == ref.shape, gk
        assert np.max(np.abs(got - ref), initial=0.0) <= 1e-11 * scale + 1e-300, (gk, np.max(np.abs(got - ref)), scale)


@pytest.mark.parametrize("precision", [8, 4])
def test_checkpointing_is_bit_identical_and_leaves_the_forward_state(precision):
    c = small_case(8, 150, 70, W.COS4, W.FULLY_PERIODIC, 3)
    n = 23
    hbar = np.random.default_rng(9).standard_normal((n, 3, 3))
    ref = gpu_of(c, precision)
    ref.step(n)
    f_ref, h_ref = ref.populations(), ref.force_history(n)
    results = []
    for K in (0, 1, 4, 7, n, 10 * n):
        s = gpu_of(c, precision)
        g, _ = s.adjoint(n, hbar, checkpoint_every=K)
        assert np.array_equal(s.populations(), f_ref), K
        assert np.array_equal(s.force_history(n), h_ref), K
        results.append(g)
    for g in results[1:]:
        for k in g:
            assert np.array_equal(g[k], results[0][k]), k


def test_fp32_adjoint_close_to_fp64():
    c = small_case(8, 150, 70, W.COS4, W.FULLY_PERIODIC, 3)
    n = 15
    hbar = np.random.default_rng(10).standard_normal((n, 3, 3))
    g64, _ = gpu_of(c, 8).adjoint(n, hbar)
    g32, _ = gpu_of(c, 4).adjoint(n, hbar)
    for k in ("marker_uv", "marker_xy", "body_force", "centres"):
        scale = np.max(np.abs(g64[k]))
        assert np.max(np.abs(g32[k] - g64[k])) <= 2e-4 * scale, k


def c5_J(U, dx=0.0, dy=0.0, uv=None, precision=8, steps=5000):
    """Mean drag coefficient of the 800x400 channel over `steps` steps, with
    inflow and initial flow U, the cylinder moved by (dx, dy)."""
    from paper_1806_09403_amd import Sim
    c = W.c5(steps=steps, precision=precision)
    b = c.bodies[0]
    s = Sim(c.nx, c.ny, c.tau, c.kind, c.thickening, c.bc, (U, 0.0), c.G, (1.0, U, 0.0), precision,
            history_capacity=steps)
    s.add_body(b.xy + np.array([dx, dy]), b.uv if uv is None else uv, b.cx + dx, b.cy + dy, b.ds)
    s.step(steps)
    h = s.force_history(steps)
    s.close()
    return float(np.mean(2.0 * h[:, 0, 0] / (U * U * c.D)))


def feq_dU(U, nx, ny):
    """d/dU of the initial populations feq_q(1, (U, 0)) at every node."""
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    d = w * (3.0 * ex + 9.0 * ex * ex * U - 3.0 * U)
    return np.broadcast_to(d[:, None, None], (9, ny, nx))


def c5_adjoint(precision, n, K=0):
    from paper_1806_09403_amd import Sim
    c = W.c5(precision=precision)
    U, D = c.U, c.D
    b = c.bodies[0]
    s = Sim(c.nx, c.ny, c.tau, c.kind, c.thickening, c.bc, (U, 0.0), c.G, (1.0, U, 0.0), precision,
            history_capacity=n)
    s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    hbar = np.zeros((n, 1, 3))
    hbar[:, 0, 0] = 2.0 / (U * U * D) / n
    g, ms = s.adjoint(n, hbar, checkpoint_every=K)
    hist = s.force_history(n)
    J = float(np.mean(2.0 * hist[:, 0, 0] / (U * U * D)))
    # dJ/dU: through the inlet and the initial state feq(1, U) (the flow's
    # response), plus the explicit -2 J / U of the coefficient's 1/U^2
    dU_flow = g["inflow"][0] + float(np.sum(g["populations"] * feq_dU(U, c.nx, c.ny)))
    dU = dU_flow - 2.0 * J / U
    dx = float(np.sum(g["marker_xy"][:, 0]) + g["centres"][0, 0])
    dy = float(np.sum(g["marker_xy"][:, 1]) + g["centres"][0, 1])
    log("  precision %d: J = %.8f dJ/dU %.8e (flow part %.8e) dJ/dx %.8e dJ/dy %.3e; "
        "ms fwd %.1f recompute (overlapped) %.1f sweep %.1f" % (precision, J, dU, dU_flow, dx, dy, *ms))
    s.close()
    return dict(J=J, dU=dU, dU_flow=dU_flow, dx=dx, dy=dy, xy=g["marker_xy"], cx=g["centres"][0, 0],
                uv=g["marker_uv"])


UV_SAMPLES = ((0, 0), (16, 1), (31, 0), (31, 1), (70, 0), (70, 1))  # not (0, 1): zero by symmetry


@pytest.fixture(scope="module")
def c5_gradients():
    """FP64 and FP32 adjoints of the mean drag over 5000 steps and FP64
    central differences of the GPU forward run (h = 1e-4) for dJ/dU, dJ/dx_c,
    dJ/dy_c and six marker velocities."""
    c = W.c5()
    U, n, h = c.U, 5000, 1e-4
    log("c5 adjoint: 800x400, 126 markers, %d steps, sqrt(N) checkpoints" % n)
    a64 = c5_adjoint(8, n)
    a32 = c5_adjoint(4, n)
    fd = dict(dU=(c5_J(U + h) - c5_J(U - h)) / (2 * h),
              dx=(c5_J(U, dx=h) - c5_J(U, dx=-h)) / (2 * h),
              dy=(c5_J(U, dy=h) - c5_J(U, dy=-h)) / (2 * h))
    nm = c.bodies[0].xy.shape[0]
    fd["uv"] = {}
    for l, comp in UV_SAMPLES:
        uv = np.zeros((nm, 2))
        uv[l, comp] = h
        fd["uv"][l, comp] = (c5_J(U, uv=uv) - c5_J(U, uv=-uv)) / (2 * h)
    log("  FD: dJ/dU %.8e dJ/dx %.8e dJ/dy %.3e" % (fd["dU"], fd["dx"], fd["dy"]))
    for p, a in (("FP64", a64), ("FP32", a32)):
        log("  %s relative errors: dJ/dU %.2e dJ/dx_c %.2e; dJ/dU_b %s" % (
            p, abs(a["dU"] / fd["dU"] - 1), abs(a["dx"] / fd["dx"] - 1),
            " ".join("%.1e" % abs(a["uv"][k] / fd["uv"][k] - 1) for k in UV_SAMPLES)))
    return a64, a32, fd


@pytest.mark.slow
def test_c5_fp64_gradients_match_central_differences(c5_gradients):
    """FP64 adjoint: dJ/dU, dJ/dx_c and six dJ/dU_b within 1e-4 relative of
    FP64 central differences; dJ/dy_c (zero by the channel's symmetry up to
    the half-node offset of the centre) within 1e-4 of |dJ/dx_c|."""
    a64, _, fd = c5_gradients
    tol = 1e-4
    assert abs(a64["dU"] - fd["dU"]) <= tol * abs(fd["dU"])
    assert abs(a64["dx"] - fd["dx"]) <= tol * abs(fd["dx"])
    assert abs(a64["dy"] - fd["dy"]) <= tol * abs(fd["dx"])
    for k in UV_SAMPLES:
        assert abs(a64["uv"][k] - fd["uv"][k]) <= tol * abs(fd["uv"][k]), k


@pytest.mark.slow
def test_c5_fp32_flow_response_matches_fp64(c5_gradients):
    """FP32 adjoint against FP64: the flow-response part of dJ/dU (inlet and
    initial state), every marker's dJ/dX_l and dJ/dU_b, within 1e-4 of the
    FP64 values' scale; the sampled dJ/dU_b within 1e-4 of central
    differences relative to the largest sampled entry (norm-wise)."""
    a64, a32, fd = c5_gradients
    tol = 1e-4
    assert abs(a32["dU_flow"] - a64["dU_flow"]) <= tol * abs(a64["dU_flow"])
    assert np.max(np.abs(a32["xy"] - a64["xy"])) <= tol * np.max(np.abs(a64["xy"]))
    assert np.max(np.abs(a32["uv"] - a64["uv"])) <= tol * np.max(np.abs(a64["uv"]))
    scale = max(abs(v) for v in fd["uv"].values())
    for k in UV_SAMPLES:
        assert abs(a32["uv"][k] - fd["uv"][k]) <= tol * scale, k


@pytest.mark.slow
@pytest.mark.xfail(strict=False, reason="FP32 misses 1e-4: measured dJ/dU 3.3e-4 and dJ/dx_c 1.3e-3 relative, "
                   "dJ/dU_b 1.4e-4 entry-wise on one of six sampled markers. "
                   "The FP32 forward's mean drag is 9.4e-5 off FP64 (a per-step bias present from the "
                   "first hundred steps), which enters dJ/dU through -2J/U; dJ/dx_c is a sum of "
                   "per-marker terms that cancel to 1e-3 of their size")
def test_c5_fp32_gradients_within_1e4_of_central_differences(c5_gradients):
    """The FP32 target: dJ/dU, dJ/dx_c and each sampled dJ/dU_b within 1e-4
    relative of FP64 central differences."""
    _, a32, fd = c5_gradients
    assert abs(a32["dU"] - fd["dU"]) <= 1e-4 * abs(fd["dU"])
    assert abs(a32["dx"] - fd["dx"]) <= 1e-4 * abs(fd["dx"])
    for k in UV_SAMPLES:
        assert abs(a32["uv"][k] - fd["uv"][k]) <= 1e-4 * abs(fd["uv"][k]), k


def torch_equilibrium(rho, ux, uy, nx, ny):
    """feq_q(rho, (ux, uy)) of eq 6, uniform, as a differentiable [9, ny, nx] tensor."""
    import torch
    ex = torch.tensor([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=torch.float64)
    ey = torch.tensor([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=torch.float64)
    w = torch.tensor([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=torch.float64)
    eu = ex * ux + ey * uy
    f = w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))
    return f[:, None, None].expand(9, ny, nx).contiguous()


def test_autograd_rollout_matches_finite_differences():
    """J = mean drag coefficient through torch: the initial state and the
    inflow built from U, the markers placed around a centre; gradients by
    loss.backward() against central differences of the same FP64 run."""
    import torch
    from paper_1806_09403_amd.autograd import RolloutSpec, rollout
    nx, ny, D, n, U0 = 120, 60, 10.0, 300, 0.04
    body = W.cylinder_body(30.0, 30.0, D)
    nl = body.xy.shape[0]
    offsets = torch.from_numpy(body.xy - np.array([body.cx, body.cy]))
    spec = RolloutSpec(nx, ny, W.tau_from_nu(U0 * D / 40.0), n, (nl,), (body.ds,), W.COS4,
                       W.PAPER_THICKENING[W.COS4], W.CHANNEL, 8, 0, (U0, 0.0))

    def J_of(U, c, uv):
        zero = torch.zeros((), dtype=torch.float64)
        hist = rollout(spec, torch_equilibrium(1.0, U, zero, nx, ny), torch.stack([U, zero]),
                       torch.zeros(2, dtype=torch.float64), c[None, :] + offsets, uv, c[None, :])
        return torch.mean(2.0 * hist[:, 0, 0] / (U * U * D))

    U = torch.tensor(U0, dtype=torch.float64, requires_grad=True)
    c = torch.tensor([body.cx, body.cy], dtype=torch.float64, requires_grad=True)
    uv = torch.zeros((nl, 2), dtype=torch.float64, requires_grad=True)
    J = J_of(U, c, uv)
    J.backward()
    h = 1e-5
    with torch.no_grad():
        fdU = (J_of(U + h, c, uv) - J_of(U - h, c, uv)).item() / (2 * h)
        e0 = torch.tensor([h, 0.0], dtype=torch.float64)
        fdx = (J_of(U, c + e0, uv) - J_of(U, c - e0, uv)).item() / (2 * h)
        duv = torch.zeros_like(uv)
        duv[5, 1] = h
        fduv = (J_of(U, c, uv + duv) - J_of(U, c, uv - duv)).item() / (2 * h)
    log("autograd: dJ/dU %.8e FD %.8e; dJ/dcx %.8e FD %.8e; dJ/dV_5 %.8e FD %.8e"
        % (U.grad.item(), fdU, c.grad[0].item(), fdx, uv.grad[5, 1].item(), fduv))
    assert abs(U.grad.item() - fdU) <= 1e-6 * abs(fdU)
    assert abs(c.grad[0].item() - fdx) <= 1e-5 * abs(fdx)
    assert abs(uv.grad[5, 1].item() - fduv) <= 1e-6 * abs(fduv)
