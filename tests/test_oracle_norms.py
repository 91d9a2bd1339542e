"""Pins of the oracle's diagnostics (Sim.norms) against closed forms.

The wall heat flux of Eq. pool-heat-flux uses a one-sided second-order
difference at y = 0, which is exact on quadratic profiles; the discrete
norms are checked on fields whose mean, rms and max are known."""
import numpy as np
import pytest

from oracle import thermo as th
from oracle.step import ADIABATIC, DIRICHLET, FREE, Params, Sim

A = 2.0 / 49.0
EOS = th.EOS(A)
T86 = 0.86 * EOS.Tc
RV, RL, _ = th.maxwell(EOS, T86)


@pytest.mark.parametrize("b,c", [(2e-4, 0.0), (-3e-4, 1e-5), (1e-4, -2e-6)])
def test_wall_flux_exact_on_quadratic_profiles(b, c):
    """Uniform liquid between walls, constant conductivity lambda,
    T = T0 + b y + c y^2: the flux lambda dT/dy at y = 0 is lambda b at
    every node.  The held (Dirichlet) nodes average exactly that; the wall
    sum counts it on the nodes that are not adiabatic and divides by nx."""
    nx, ny = 10, 9
    kinds = np.array([ADIABATIC, DIRICHLET, DIRICHLET, FREE, ADIABATIC,
                      DIRICHLET, ADIABATIC, ADIABATIC, DIRICHLET, FREE])
    T0 = T86
    lam_l = lam_v = 1.95
    p = Params(nx=nx, ny=ny, a=A, rho_l=RL, rho_v=RV, walls=True, rho_w_bottom=RL, rho_w_top=RL,
               thermal=True, cv=5.0, lambda_l=lam_l, lambda_v=lam_v, t_bottom_kind=kinds,
               t_bottom_val=np.full(nx, T0))
    s = Sim(p)
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    s.init_fields(np.full((ny, nx), RL), T=T0 + b * y + c * y * y)
    n = s.norms()
    held = int(np.count_nonzero(kinds == DIRICHLET))
    not_adiabatic = int(np.count_nonzero(kinds != ADIABATIC))
    assert n["n_heater"] == held
    assert abs(n["q_heater"] - lam_l * b) <= 1e-12 * abs(lam_l * b)
    assert abs(n["q_bottom"] - lam_l * b * not_adiabatic / nx) <= 1e-12 * abs(lam_l * b)


def test_wall_flux_is_zero_without_walls_and_heater_mean_is_per_node():
    """Periodic lattices have no wall: both fluxes are 0 and no node is
    averaged.  With walls and a linear profile whose slope differs between
    two held groups the heater flux is the node mean of the two slopes."""
    nx, ny = 6, 5
    p = Params(nx=nx, ny=ny, a=A, rho_l=RL, rho_v=RV, thermal=True, cv=5.0)
    s = Sim(p)
    s.init_fields(np.full((ny, nx), RV), T=np.full((ny, nx), T86))
    n = s.norms()
    assert n["q_bottom"] == 0.0 and n["q_heater"] == 0.0 and n["n_heater"] == 0
    kinds = np.array([DIRICHLET, DIRICHLET, ADIABATIC, DIRICHLET, ADIABATIC, ADIABATIC])
    p = Params(nx=nx, ny=ny, a=A, rho_l=RL, rho_v=RV, walls=True, rho_w_bottom=RV, rho_w_top=RV,
               thermal=True, cv=5.0, lambda_l=0.7, lambda_v=0.7, t_bottom_kind=kinds,
               t_bottom_val=np.full(nx, T86))
    s = Sim(p)
    slope = np.array([1e-4, 3e-4, 9e-3, -2e-4, 9e-3, 9e-3])  # adiabatic slopes must not count
    y = np.arange(ny, dtype=float)[:, None]
    s.init_fields(np.full((ny, nx), RV), T=T86 + slope[None, :] * y)
    n = s.norms()
    assert n["n_heater"] == 3
    assert abs(n["q_heater"] - 0.7 * (1e-4 + 3e-4 - 2e-4) / 3) <= 1e-12 * 0.7 * 1e-4
    assert abs(n["q_bottom"] - 0.7 * (1e-4 + 3e-4 - 2e-4) / nx) <= 1e-12 * 0.7 * 1e-4


def test_discrete_norms_of_a_two_valued_field():
    """Periodic lattice, rho = r1 on half the nodes and r2 on the other half
    (rows), T likewise: mean |.| = (r1 + r2)/2, rms = sqrt((r1^2 + r2^2)/2),
    max = max(r1, r2); mass = N (r1 + r2)/2; nothing is non-finite.  (rho
    is the sum of the populations, so it carries one rounding.)"""
    nx, ny = 4, 6
    r1, r2 = 0.5, 5.5
    t1, t2 = 0.9 * EOS.Tc, 0.87 * EOS.Tc
    rho = np.where(np.arange(ny)[:, None] < ny // 2, r1, r2) * np.ones((1, nx))
    T = np.where(np.arange(ny)[:, None] < ny // 2, t1, t2) * np.ones((1, nx))
    s = Sim(Params(nx=nx, ny=ny, a=A, rho_l=RL, rho_v=RV))
    s.init_fields(rho, T=T)
    n = s.norms()
    N = nx * ny
    assert abs(n["mass"] - N * (r1 + r2) / 2) <= 1e-13 * n["mass"]
    assert abs(n["rho_mean"] - (r1 + r2) / 2) <= 1e-15 * 3
    assert abs(n["l1_rho"] - (r1 + r2) / 2) <= 1e-15 * 3
    assert abs(n["l2_rho"] - np.sqrt((r1 ** 2 + r2 ** 2) / 2)) <= 1e-15 * 4
    assert abs(n["linf_rho"] - r2) <= 2e-15 * r2
    assert abs(n["l1_T"] - (t1 + t2) / 2) <= 1e-15
    assert abs(n["l2_T"] - np.sqrt((t1 ** 2 + t2 ** 2) / 2)) <= 1e-15
    assert n["linf_T"] == t1
    assert n["nonfinite"] == 0


def test_umax_of_a_uniform_flow():
    """Uniform density and velocity: no force, u = (j + F/2)/rho = u0."""
    nx, ny = 5, 4
    ux, uy = 0.03, -0.04
    s = Sim(Params(nx=nx, ny=ny, a=A, rho_l=RL, rho_v=RV))
    s.init_fields(np.full((ny, nx), 2.0), np.full((ny, nx), ux), np.full((ny, nx), uy),
                  np.full((ny, nx), T86))
    assert abs(s.norms()["umax"] - 0.05) <= 1e-15
