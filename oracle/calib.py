"""Boundary-thickness calibration of Section 2.3 (eqs 22, 25, 26), FP64.

TEST INFRASTRUCTURE. Builds the interpolation matrix D_I of a marker set
over the nodes of its stencils, forms A = (1/dh^2) D_I D_I^T dh ds (eq 22),
solves A drs = dh 1 (eqs 24-25) and averages (eq 26). numpy's dense solve
is the only library step.
"""
import numpy as np

from .dense import phi

HALF = {2: 1.0, 3: 1.5, 4: 2.0, 5: 2.0}


def interpolation_matrix(kind, xy, dh=1.0, period_x=None):
    """D_I (N_L x N_E) over every node within the support of some marker.

    With ``period_x`` the x direction is periodic with that many nodes
    (node x-coordinates 0 .. period_x-1, minimum-image distances)."""
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    h = HALF[kind] * dh
    y0 = int(np.floor((xy[:, 1].min() - h) / dh))
    y1 = int(np.ceil((xy[:, 1].max() + h) / dh))
    if period_x is None:
        x0 = int(np.floor((xy[:, 0].min() - h) / dh))
        x1 = int(np.ceil((xy[:, 0].max() + h) / dh))
        xs = np.arange(x0, x1 + 1) * dh
    else:
        xs = np.arange(period_x) * dh
    ys = np.arange(y0, y1 + 1) * dh
    YY, XX = np.meshgrid(ys, xs, indexing="ij")
    xk, yk = XX.ravel(), YY.ravel()
    dx = xk[None, :] - xy[:, 0:1]
    if period_x is not None:
        L = period_x * dh
        dx = (dx + L / 2) % L - L / 2
    dy = yk[None, :] - xy[:, 1:2]
    return phi(kind, dx / dh) * phi(kind, dy / dh)


def matrix_A(kind, xy, ds, dh=1.0, period_x=None):
    """eq 22: A_ij = (1/dh^2) sum_k phi_ik phi_kj dh ds."""
    D = interpolation_matrix(kind, xy, dh, period_x)
    return (D @ D.T) * (dh * ds) / dh ** 2


def thickness_vector(kind, xy, ds, dh=1.0, period_x=None):
    """eq 25: drs = A^{-1} 1 dh."""
    A = matrix_A(kind, xy, ds, dh, period_x)
    return np.linalg.solve(A, np.ones(A.shape[0])) * dh


def thickness_mean(kind, xy, ds, dh=1.0, period_x=None):
    """eq 26: the uniform thickness is the mean of the local ones."""
    return float(np.mean(thickness_vector(kind, xy, ds, dh, period_x)))
