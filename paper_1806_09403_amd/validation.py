"""Flow past a stationary cylinder (Section 5.2, Table 3) run on the GPU:
drag and lift coefficients (eq 44 and its cross-stream counterpart), the
Strouhal number and the recirculation length behind the cylinder.

The coefficients are normalised with the far-field density, the mean
density of the first fluid column: with a velocity inlet and a convective
or zero-gradient outlet the boundaries leave the mean density free (scaling
every population by c maps a solution to a solution), so the density level
a long run settles at is not exactly 1.
"""
import math

import numpy as np

from . import _lib
from .sim import Sim


def coefficients(hist, U, D, rho=1.0, body=0):
    """C_D and C_L series from a force history [steps, bodies, 3]."""
    q = 0.5 * rho * U * U * D
    return hist[:, body, 0] / q, hist[:, body, 1] / q


def mean_and_deviation(x):
    """The paper's a +- b for an oscillating coefficient: the mean and the
    largest deviation from it (half the peak-to-peak swing)."""
    x = np.asarray(x, dtype=np.float64)
    return float(x.mean()), float(0.5 * (x.max() - x.min()))


def strouhal(cl, U, D):
    """St = f D / U from the upward zero crossings of C_L - mean(C_L)
    (linear interpolation between steps, dt = 1)."""
    c = np.asarray(cl, dtype=np.float64)
    c = c - c.mean()
    up = np.nonzero((c[:-1] < 0.0) & (c[1:] >= 0.0))[0]
    if len(up) < 3:
        return float("nan")
    t = up + (-c[up]) / (c[up + 1] - c[up])
    period = (t[-1] - t[0]) / (len(t) - 1)
    return float(D / (period * U))


def wake_length(ux_line, x_rear, D):
    """Recirculation length in diameters: from the rear of the cylinder to
    the first point downstream where u_x on the centre line turns from
    negative to non-negative (linear interpolation between nodes)."""
    u = np.asarray(ux_line, dtype=np.float64)
    i = int(math.ceil(x_rear))
    while i + 1 < len(u) and not (u[i] < 0.0):
        i += 1  # skip the shell, where u can still be >= 0
    while i + 1 < len(u) and u[i + 1] < 0.0:
        i += 1
    if i + 1 >= len(u):
        return float("nan")
    x0 = i + (-u[i]) / (u[i + 1] - u[i])
    return float((x0 - x_rear) / D)


def boundary_error(ub, vb, U):
    """Eq 45 for markers at rest: the root mean square of the velocity
    interpolated at the markers, in units of the inflow speed."""
    return float(np.sqrt(np.mean(np.asarray(ub) ** 2 + np.asarray(vb) ** 2)) / U)


def _sim(case, precision, graph_chunk, forcing_passes, method=0):
    s = Sim.from_case(case, precision=precision)
    s.set_option(_lib.OPT_GRAPH_CHUNK, graph_chunk)
    if forcing_passes != 1:
        s.set_option(_lib.OPT_FORCING_PASSES, forcing_passes)
    if method:
        s.set_option(_lib.OPT_FORCING_METHOD, method)
    return s


def run_steady(case, max_steps=200_000, min_steps=40_000, check_every=4000, tol=1e-3, precision=None,
               graph_chunk=50, forcing_passes=1, method=0, log=None):
    """Step until C_D has changed by less than tol (relative) over each of
    two successive check intervals (at least min_steps); then C_D, C_L and
    the wake length of the single body. Acoustic waves trapped between the
    inlet and the walls keep C_D moving by about 1e-3 relative for a long
    time, so tol is not set tighter by default."""
    U, D, body = case.U, case.D, case.bodies[0]
    s = _sim(case, precision, graph_chunk, forcing_passes, method)
    try:
        hist, steps, converged = [], 0, False
        while steps < max_steps and not converged:
            s.step(check_every)
            steps += check_every
            hist.append(s.forces()[0, 0] / (0.5 * U * U * D))
            if log:
                log("  step %d  C_D(rho=1) %.6f" % (steps, hist[-1]))
            converged = (steps >= min_steps and len(hist) >= 3 and
                         all(abs(hist[-k] - hist[-k - 1]) < tol * abs(hist[-1]) for k in (1, 2)))
        ub, vb = s.marker_velocity()
        rho, ux, _ = s.macroscopic()
        rho_inf = float(rho[:, 1].mean())
        F = s.forces()[0]
        q = 0.5 * rho_inf * U * U * D
        jc = int(round(body.cy))
        return {"steps": steps, "converged": bool(converged), "Cd": float(F[0] / q), "Cl": float(F[1] / q),
                "rho_inf": rho_inf, "Lw": wake_length(ux[jc, :], body.cx + 0.5 * D, D),
                "boundary_error": boundary_error(ub, vb, U)}
    finally:
        s.close()


def run_unsteady(case, warmup=100_000, window=40_000, precision=None, graph_chunk=50, forcing_passes=1,
                 method=0, log=None):
    """Run warmup steps, then record window steps: C_D and C_L as mean +-
    largest deviation, and the Strouhal number from C_L."""
    U, D = case.U, case.D
    s = _sim(case, precision, graph_chunk, forcing_passes, method)
    piece = 4000   # below the force ring's default capacity of 4096
    try:
        done = 0
        while done < warmup:
            n = min(piece, warmup - done)
            s.step(n)
            s.force_history(n)   # drain
            done += n
            if log:
                log("  warmup step %d  C_L %.4f" % (done, s.forces()[0, 1] / (0.5 * U * U * D)))
        parts = []
        got = 0
        while got < window:
            n = min(piece, window - got)
            s.step(n)
            parts.append(s.force_history(n))
            got += n
        hist = np.concatenate(parts, axis=0)
        rho, _, _ = s.macroscopic()
        rho_inf = float(rho[:, 1].mean())
        cd, cl = coefficients(hist, U, D, rho_inf)
        cd_m, cd_d = mean_and_deviation(cd)
        cl_m, cl_d = mean_and_deviation(cl)
        return {"steps": warmup + window, "Cd": cd_m, "Cd_dev": cd_d, "Cl_mean": cl_m, "Cl_dev": cl_d,
                "St": strouhal(cl, U, D), "rho_inf": rho_inf}
    finally:
        s.close()
