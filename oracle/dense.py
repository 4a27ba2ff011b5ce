"""Dense-matrix brute force of the BTDF-IB-LBM step on tiny periodic grids.

TEST INFRASTRUCTURE. This is a second, independent host implementation,
written as the paper writes the method: the interpolation operator D_I is
built as a dense N_L x N_E matrix (eq 14), the spreading operator as the
dense N_E x N_L matrix D_E of eq 15, the force as eq 20 and the body force
as both sides of eq 27. Streaming is a whole-array shift per direction and
the collision is eqs 5-7 on whole arrays. It is only usable for grids of a
few hundred nodes, and exists to pin the loop oracle in ``btdf_oracle.c``.
Fully periodic grids only (minimum-image distances).
"""
import numpy as np

# eq 8: columns are e_0 .. e_8
E = np.array([[0, 1, 0, -1, 0, 1, -1, -1, 1],
              [0, 0, 1, 0, -1, 1, 1, -1, -1]], dtype=np.int64)
# weights stated after eq 7
WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

LINEAR2, ROMA3, PESKIN4, COS4 = 2, 3, 4, 5


def phi(kind, r):
    """Delta functions of eqs 37-39 and the cosine 4-point kernel, on arrays."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    if kind == LINEAR2:
        return np.where(a <= 1.0, 1.0 - a, 0.0)
    if kind == ROMA3:
        inner = (1.0 + np.sqrt(np.clip(1.0 - 3.0 * a * a, 0.0, None))) / 3.0
        outer = (5.0 - 3.0 * a - np.sqrt(np.clip(1.0 - 3.0 * (1.0 - a) ** 2, 0.0, None))) / 6.0
        return np.where(a <= 0.5, inner, np.where(a <= 1.5, outer, 0.0))
    if kind == PESKIN4:
        inner = (3.0 - 2.0 * a + np.sqrt(np.clip(1.0 + 4.0 * a - 4.0 * a * a, 0.0, None))) / 8.0
        outer = (5.0 - 2.0 * a - np.sqrt(np.clip(-7.0 + 12.0 * a - 4.0 * a * a, 0.0, None))) / 8.0
        return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))
    if kind == COS4:
        return np.where(a <= 2.0, 0.25 * (1.0 + np.cos(np.pi * a / 2.0)), 0.0)
    raise ValueError(kind)


def equilibrium(rho, ux, uy):
    """eq 6, c = 1, on arrays; returns [9, ...]."""
    eu = E[0][:, None, None] * ux[None] + E[1][:, None, None] * uy[None]
    uu = ux * ux + uy * uy
    return WQ[:, None, None] * rho[None] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu[None])


def min_image(d, n):
    return (d + n / 2.0) % n - n / 2.0


def interpolation_matrix(kind, nx, ny, X, Y):
    """D_I of eq 14 with dh = 1 over every node of a periodic nx x ny grid."""
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    xk = ii.ravel().astype(np.float64)
    yk = jj.ravel().astype(np.float64)
    dx = min_image(xk[None, :] - X[:, None], nx)
    dy = min_image(yk[None, :] - Y[:, None], ny)
    return phi(kind, dx) * phi(kind, dy)


class DenseSim:
    """Fully periodic BTDF-IB-LBM with dense operators (Algorithm 1, NF = 1)."""

    def __init__(self, nx, ny, tau, kind, thickening, G=(0.0, 0.0)):
        self.nx, self.ny, self.tau, self.kind = nx, ny, tau, kind
        self.drs = thickening
        self.G = np.array(G, dtype=np.float64)
        self.A = equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
        self.X = np.zeros(0)
        self.Y = np.zeros(0)
        self.Ub = np.zeros(0)
        self.Vb = np.zeros(0)
        self.ds_l = np.zeros(0)
        self.bodies = []  # (first marker, count, cx, cy, ds)
        self.forces = np.zeros((0, 3))

    def add_body(self, xy, uv, cx, cy, ds):
        xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
        uv = np.zeros_like(xy) if uv is None else np.asarray(uv, dtype=np.float64).reshape(-1, 2)
        self.bodies.append((self.X.size, xy.shape[0], cx, cy, ds))
        self.X = np.concatenate([self.X, xy[:, 0]])
        self.Y = np.concatenate([self.Y, xy[:, 1]])
        self.Ub = np.concatenate([self.Ub, uv[:, 0]])
        self.Vb = np.concatenate([self.Vb, uv[:, 1]])
        self.ds_l = np.concatenate([self.ds_l, np.full(xy.shape[0], ds)])

    def step(self):
        nx, ny, tau = self.nx, self.ny, self.tau
        # streaming: g_q(x) = A_q(x - e_q)
        g = np.stack([np.roll(self.A[q], shift=(E[1, q], E[0, q]), axis=(0, 1)) for q in range(9)])
        # eqs 9-10 and u* with half of the body force (eq 11 applied to G)
        rho = g.sum(axis=0)
        mx = np.tensordot(E[0], g, axes=(0, 0))
        my = np.tensordot(E[1], g, axes=(0, 0))
        usx = (mx + 0.5 * self.G[0]) / rho
        usy = (my + 0.5 * self.G[1]) / rho
        fx = np.zeros(nx * ny)
        fy = np.zeros(nx * ny)
        self.forces = np.zeros((len(self.bodies), 3))
        if self.X.size:
            DI = interpolation_matrix(self.kind, nx, ny, self.X, self.Y)       # eq 14
            DE = DI.T * (self.drs * self.ds_l)[None, :]                          # eq 15, dh = 1
            rho_l = DI @ rho.ravel()
            Fx = 2.0 * rho_l * (self.Ub - DI @ usx.ravel())                      # eq 20
            Fy = 2.0 * rho_l * (self.Vb - DI @ usy.ravel())
            fx = DE @ Fx                                                         # eq 13
            fy = DE @ Fy
            self.Fx, self.Fy, self.rho_l = Fx, Fy, rho_l
            for b, (m0, n, cx, cy, ds) in enumerate(self.bodies):
                sl = slice(m0, m0 + n)
                # eq 27 (left side), force on the body = minus force on the fluid
                s = ds * self.drs
                self.forces[b, 0] = -s * Fx[sl].sum()
                self.forces[b, 1] = -s * Fy[sl].sum()
                self.forces[b, 2] = -s * np.sum((self.X[sl] - cx) * Fy[sl] - (self.Y[sl] - cy) * Fx[sl])
        self.fx = fx.reshape(ny, nx)
        self.fy = fy.reshape(ny, nx)
        # eq 11, eq 6, eq 7, eq 5
        ftx = self.G[0] + self.fx
        fty = self.G[1] + self.fy
        ux = (mx + 0.5 * ftx) / rho
        uy = (my + 0.5 * fty) / rho
        feq = equilibrium(rho, ux, uy)
        ex = E[0][:, None, None]
        ey = E[1][:, None, None]
        eu = ex * ux[None] + ey * uy[None]
        Fq = (1 - 1 / (2 * tau)) * WQ[:, None, None] * (
            (3 * (ex - ux[None]) + 9 * eu * ex) * ftx[None] +
            (3 * (ey - uy[None]) + 9 * eu * ey) * fty[None])
        self.A = g - (g - feq) / tau + Fq
