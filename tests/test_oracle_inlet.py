"""The oracle's velocity inlet (Section 5.2's Dirichlet inflow).

The paper prescribes the inflow velocity at the inlet and gives no discrete
rule for the density there. The reading taken is the zero-gradient
extrapolation of the density from the first fluid column: after each
collision the ghost column i = 0 is set to the equilibrium (eq 6) at the
inflow velocity with the density rho(1, y) = sum_q f_q(1, y) of the
post-collision state. Two pins fix that reading in the oracle:

* directly: the ghost column after a step equals eq 6 evaluated by the
  numpy brute force (``oracle/dense.equilibrium``) at column 1's density,
  on a state whose columns 1 and 2 have clearly different densities;
* through mass conservation: streaming and the collision conserve mass, so
  the change of the fluid mass over the next step is the net flux through
  the two channel ends. All of it but the inlet ghost's contribution is
  read from the state itself; what the ghost must have supplied is then
  the closed form sum_{e_x = 1} f_eq = rho (1 + 3U + 3U^2) / 6 (eq 6 at
  u = (U, 0), summed over q = 1, 5, 8) times column 1's density.
"""
import numpy as np
import pytest

import btdf_workloads as W
from oracle.dense import equilibrium
from oracle.oracle import OracleSim

EAST = [1, 5, 8]  # e_x = +1 (D2Q9 order of eq 8)
WEST = [3, 6, 7]  # e_x = -1


def channel_state(nx, ny, U, seed, outlet=W.ZERO_GRADIENT_OUTLET):
    """A channel whose density varies strongly along x and y (columns 1 and
    2 differ by about 5%)."""
    rng = np.random.default_rng(seed)
    bc = (W.VELOCITY_INLET, outlet, W.PERIODIC, W.PERIODIC)
    s = OracleSim(nx, ny, bc, 0.7, W.COS4, 2.6, inflow=(U, 0.0))
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    rho = 1.0 + 0.05 * np.sin(2 * np.pi * x / 5.0 + 0.3) + 0.02 * np.cos(2 * np.pi * y / ny) \
        + 0.005 * rng.uniform(-1, 1, size=(ny, nx))
    ux = U + 0.01 * rng.uniform(-1, 1, size=(ny, nx))
    uy = 0.01 * rng.uniform(-1, 1, size=(ny, nx))
    s.init_equilibrium(ux, uy, rho)
    return s


@pytest.mark.parametrize("U", [0.0, 0.02, 0.08])
def test_inlet_ghost_is_the_equilibrium_at_column_one_density(U):
    nx, ny = 23, 11
    s = channel_state(nx, ny, U, seed=1)
    for _ in range(2):
        s.step(1)
        f = s.populations()
        rho1 = f[:, :, 1].sum(axis=0)
        rho2 = f[:, :, 2].sum(axis=0)
        assert np.max(np.abs(rho1 - rho2)) > 1e-3  # the two readings differ here
        want = equilibrium(rho1[:, None], np.full((ny, 1), U), np.zeros((ny, 1)))[:, :, 0]
        assert np.max(np.abs(f[:, :, 0] - want)) <= 1e-15 * np.max(np.abs(want))
        other = equilibrium(rho2[:, None], np.full((ny, 1), U), np.zeros((ny, 1)))[:, :, 0]
        assert np.max(np.abs(f[:, :, 0] - other)) > 1e-5


@pytest.mark.parametrize("outlet", [W.ZERO_GRADIENT_OUTLET, W.CONVECTIVE_OUTLET])
@pytest.mark.parametrize("U", [0.01, 0.05])
def test_inlet_mass_inflow_follows_column_one_density(U, outlet):
    nx, ny = 19, 9
    s = channel_state(nx, ny, U, seed=2, outlet=outlet)
    s.step(1)  # the ghost columns now hold what the reading sets
    fa = s.populations()
    s.step(1)
    fb = s.populations()
    mass_a = fa[:, :, 1:nx - 1].sum()
    mass_b = fb[:, :, 1:nx - 1].sum()
    # fluxes of the step a -> b read from state a (periodic y: summing over
    # all rows makes the diagonal shifts irrelevant)
    out_west = fa[WEST, :, 1].sum()
    out_east = fa[EAST, :, nx - 2].sum()
    in_east = fa[WEST, :, nx - 1].sum()
    in_west = mass_b - mass_a + out_west + out_east - in_east
    rho1 = fa[:, :, 1].sum(axis=0)
    want = rho1.sum() * (1.0 + 3.0 * U + 3.0 * U * U) / 6.0
    assert abs(in_west - want) <= 1e-13 * abs(want)
    rho2 = fa[:, :, 2].sum(axis=0)
    assert abs(in_west - rho2.sum() * (1.0 + 3.0 * U + 3.0 * U * U) / 6.0) > 1e-6
