"""The oracle's reverse mode against the derivative's definition.

J = sum_t sum_b hbar_t,b . (Fx, Fy, Tz)_t,b over n steps of the oracle's
own forward step (itself pinned by the other oracle tests). Every gradient
the adjoint returns -- initial populations, inflow velocity, uniform body
force, marker positions, marker velocities, body centres -- is checked
against central differences of J along random directions, on small cases
covering every boundary kind and delta function. A mirror-symmetric
channel pins the symmetry the exact gradient must have, and phi' is pinned
against differences of phi.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.oracle import OracleSim, delta, delta_deriv


def build(c, xy=None, uv=None, centres=None, inflow=None, G=None, pop=None):
    o = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G if G is None else G,
                  c.inflow if inflow is None else inflow, c.init)
    at = 0
    for b, body in enumerate(c.bodies):
        n = body.xy.shape[0]
        bxy = body.xy if xy is None else xy[at:at + n]
        buv = body.uv if uv is None else uv[at:at + n]
        cx, cy = (body.cx, body.cy) if centres is None else centres[b]
        o.add_body(bxy, buv, cx, cy, body.ds)
        at += n
    if pop is not None:
        o.set_populations(pop)
    elif c.init_uy is not None:
        ux, uy = c.init_fields()
        o.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    return o


def history(o, n):
    out = []
    for _ in range(n):
        o.step(1)
        out.append(o.forces())
    return np.array(out)


def base_params(c):
    o = build(c)
    pop = o.populations()
    xy = np.concatenate([b.xy for b in c.bodies]) if c.bodies else np.zeros((0, 2))
    uv = np.concatenate([b.uv if b.uv is not None else np.zeros_like(b.xy) for b in c.bodies]) \
        if c.bodies else np.zeros((0, 2))
    centres = np.array([[b.cx, b.cy] for b in c.bodies]).reshape(-1, 2)
    return dict(pop=pop, inflow=np.array(c.inflow, float), G=np.array(c.G, float), xy=xy, uv=uv,
                centres=centres)


def J_of(c, n, hbar, p):
    o = build(c, xy=p["xy"], uv=p["uv"], centres=p["centres"], inflow=tuple(p["inflow"]),
              G=tuple(p["G"]), pop=p["pop"])
    return float(np.sum(hbar * history(o, n)))


CASES = [
    # (seed, nx, ny, kind, bc, n_bodies, n_steps)
    (1, 24, 20, W.COS4, W.FULLY_PERIODIC, 2, 6),
    (2, 18, 16, W.ROMA3, W.CHANNEL, 1, 10),  # narrow: the ends reach the body within the run
    (3, 26, 20, W.PESKIN4, (W.PERIODIC, W.PERIODIC, W.BOUNCEBACK_WALL, W.BOUNCEBACK_WALL), 2, 5),
    (4, 18, 17, W.COS4, (W.VELOCITY_INLET, W.ZERO_GRADIENT_OUTLET, W.BOUNCEBACK_WALL,
                         W.BOUNCEBACK_WALL), 1, 10),
    (5, 25, 19, W.LINEAR2, W.FULLY_PERIODIC, 2, 4),
]

KEYS = [("pop", "populations", 1e-6), ("inflow", "inflow", 1e-5), ("G", "body_force", 1e-6),
        ("xy", "xy", 1e-5), ("uv", "uv", 1e-5), ("centres", "centres", 1e-5)]


@pytest.mark.parametrize("seed,nx,ny,kind,bc,nbody,n", CASES)
def test_adjoint_matches_central_differences(seed, nx, ny, kind, bc, nbody, n):
    c = W.random_case(seed, nx=nx, ny=ny, kind=kind, bc=bc, n_bodies=nbody, D_range=(4.0, 6.0))
    if bc[0] == W.VELOCITY_INLET:
        c.inflow = (0.03, 0.004)
    rng = np.random.default_rng(100 + seed)
    hbar = rng.standard_normal((n, len(c.bodies), 3))
    p0 = base_params(c)
    o = build(c)
    g = o.adjoint(n, hbar)
    # the adjoint run leaves the same state and forces as plain stepping
    r = build(c)
    hist = history(r, n)
    assert np.array_equal(o.populations(), r.populations())
    assert np.array_equal(o.forces(), hist[-1])
    for key, gkey, h in KEYS:
        if p0[key].size == 0:
            continue
        v = rng.standard_normal(p0[key].shape)
        if key == "pop":
            v *= 1e-3
        if key == "inflow" and bc[0] != W.VELOCITY_INLET:
            continue  # no inlet: J does not depend on it (checked below)
        pp = dict(p0)
        pm = dict(p0)
        pp[key] = p0[key] + h * v
        pm[key] = p0[key] - h * v
        fd = (J_of(c, n, hbar, pp) - J_of(c, n, hbar, pm)) / (2 * h)
        ad = float(np.sum(g[gkey] * v))
        scale = max(abs(fd), 1e-12)
        assert abs(ad - fd) <= 2e-6 * scale + 1e-13, (key, ad, fd)
    if bc[0] != W.VELOCITY_INLET:
        assert np.all(g["inflow"] == 0.0)


def test_adjoint_is_linear_in_hist_bar():
    c = W.random_case(7, nx=22, ny=18, kind=W.COS4, bc=W.FULLY_PERIODIC, n_bodies=1, D_range=(4.0, 5.0))
    rng = np.random.default_rng(7)
    a, b = rng.standard_normal((2, 4, 1, 3))
    ga = build(c).adjoint(4, a)
    gb = build(c).adjoint(4, b)
    gab = build(c).adjoint(4, 2.0 * a - 3.0 * b)
    for k in ga:
        ref = 2.0 * ga[k] - 3.0 * gb[k]
        assert np.allclose(gab[k], ref, rtol=1e-10, atol=1e-14 * max(1.0, np.max(np.abs(ref)))), k


def test_mirror_symmetric_channel_gradients():
    """Cylinder on the centre line of a periodic-y channel: the flow is
    symmetric about y = y_c, so for J = mean drag the exact gradient w.r.t.
    the centre's y is zero, marker-velocity gradients of mirror markers are
    equal in x and opposite in y."""
    U, D, nx, ny = 0.04, 8.0, 48, 32
    yc = ny / 2.0
    body = W.cylinder_body(16.0, yc, D, 24)
    c = W.Case(name="mirror", nx=nx, ny=ny, bc=W.CHANNEL, tau=0.6, kind=W.COS4,
               thickening=W.PAPER_THICKENING[W.COS4], inflow=(U, 0.0), init=(1.0, U, 0.0),
               bodies=[body], precision=8, U=U, D=D)
    n = 8
    hbar = np.zeros((n, 1, 3))
    hbar[:, 0, 0] = 2.0 / (U * U * D) / n
    g = build(c).adjoint(n, hbar)
    # d J / d y_c with the body moved rigidly: sum of the marker y gradients + the centre's own
    dyc = np.sum(g["xy"][:, 1]) + g["centres"][0, 1]
    dxc = np.sum(g["xy"][:, 0]) + g["centres"][0, 0]
    assert abs(dyc) <= 1e-9 * abs(dxc)
    # marker l at angle 2 pi l / N mirrors to marker (N - l) % N
    N = body.xy.shape[0]
    mirror = (N - np.arange(N)) % N
    scale = np.max(np.abs(g["uv"]))
    assert np.max(np.abs(g["uv"][:, 0] - g["uv"][mirror, 0])) <= 1e-10 * scale
    assert np.max(np.abs(g["uv"][:, 1] + g["uv"][mirror, 1])) <= 1e-10 * scale
    assert abs(g["inflow"][1]) <= 1e-9 * abs(g["inflow"][0])


@pytest.mark.parametrize("kind", [W.ROMA3, W.PESKIN4, W.COS4, W.LINEAR2])
def test_delta_derivative_matches_differences(kind):
    r = np.linspace(-2.4, 2.4, 97) + 0.0123
    if kind == W.LINEAR2:
        r = r[np.abs(np.abs(r) - 1.0) > 1e-3]
        r = r[np.abs(r) > 1e-3]
    h = 1e-6
    fd = (delta(kind, r + h) - delta(kind, r - h)) / (2 * h)
    assert np.max(np.abs(delta_deriv(kind, r) - fd)) < 1e-7
    # sum_i phi'(i - X) = 0 for every X (derivative of the partition of unity)
    for X in (0.1, 0.37, 0.5, 0.93):
        i = np.arange(-4, 6)
        assert abs(np.sum(delta_deriv(kind, i - X))) < 1e-12
