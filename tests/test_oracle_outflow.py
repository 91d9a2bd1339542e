"""Pins of the oracle's zero-gradient outflow (the open end of the 1-D
boiling problem, Sec. 4.2): uniform flows cross it untouched, the top row's
incoming populations are those of the row below, and the Stefan problem
(Eq. stefan-analytical) is followed on a short column."""
import numpy as np
import pytest

from oracle import lattice as lat
from oracle import thermo as th
from oracle.step import ADIABATIC, DIRICHLET, Params, Sim

A = 2.0 / 49.0
EOS = th.EOS(A)
T86 = 0.86 * EOS.Tc
RV, RL, PS = th.maxwell(EOS, T86)


@pytest.mark.parametrize("uy", [0.0, 0.01, -0.01])
def test_uniform_flow_crosses_the_outflow(uy):
    """Uniform density and velocity: the bottom wall disturbs the rows near
    it (a few rows per step), the outflow nothing, so after 3 steps the
    upper rows are unchanged to rounding."""
    nx, ny, rho0 = 5, 32, 2.0
    p = Params(nx=nx, ny=ny, a=A, sigma=0.1, kappa=0.2, rho_l=RL, rho_v=RV, walls=True,
               outflow_top=True, rho_w_bottom=1.0, thermal=True, cv=5.0,
               t_bottom_kind=DIRICHLET, t_bottom_val=0.9 * EOS.Tc, t_top_kind=ADIABATIC)
    s = Sim(p)
    s.init_fields(np.full((ny, nx), rho0), ux=np.full((ny, nx), 0.004),
                  uy=np.full((ny, nx), uy), T=np.full((ny, nx), 0.95 * EOS.Tc))
    f0 = s.populations().copy()
    r0, ux0, uy0, T0 = s.fields()
    s.step(3)
    r, ux, uy_, T = s.fields()
    top = slice(16, ny)
    np.testing.assert_allclose(s.populations()[:, top], f0[:, top], rtol=0, atol=1e-15 * rho0)
    np.testing.assert_allclose(r[top], r0[top], rtol=1e-15)
    np.testing.assert_allclose(uy_[top], uy0[top], atol=1e-16)
    np.testing.assert_array_equal(T[top], T0[top])
    # the disturbance of the wall did reach the lower rows
    assert np.abs(r[:3] - rho0).max() > 1e-6


def test_top_row_takes_the_incoming_populations_of_the_row_below():
    rng = np.random.default_rng(4)
    nx, ny = 6, 9
    p = Params(nx=nx, ny=ny, a=A, sigma=0.1, kappa=0.1, rho_l=RL, rho_v=RV, walls=True,
               outflow_top=True, rho_w_bottom=rng.uniform(0.5, 6, nx))
    s = Sim(p)
    s.init_fields(rng.uniform(0.5, 6.0, (ny, nx)), ux=rng.uniform(-0.01, 0.01, (ny, nx)),
                  uy=rng.uniform(-0.01, 0.01, (ny, nx)), T=np.full((ny, nx), T86))
    for _ in range(3):
        f = s.populations()
        for i in np.nonzero(lat.CY < 0)[0]:
            np.testing.assert_array_equal(f[i, ny - 1], f[i, ny - 2])
        # the top row is an ordinary node: its momentum is that of its populations
        m = s.macro()
        np.testing.assert_allclose(m["rho"][ny - 1], f[:, ny - 1].sum(0), rtol=1e-15)
        np.testing.assert_allclose(m["jy"][ny - 1], (f[:, ny - 1] * lat.CY[:, None]).sum(0),
                                   atol=1e-15)
        s.step(1)


def test_stefan_column_follows_the_similarity_solution():
    """Second parameter set of Sec. 4.2 on a column of 96 nodes (a = 6.12e-2,
    c_v = 10, lambda 15 / 1, T_w = 0.9 T_c, hydrophobic hot wall; Ja must be
    the printed 0.076): the vapour film grows from the wall and the front
    stays within 30 % below 2 beta sqrt(alpha_v t) (Eq. stefan-analytical)
    up to t = 4000.  The scheme is compressible (expansion cooling at the
    front through the last term of Eq. energy-equation), so the similarity
    solution of the incompressible limit is a reference, not a limit."""
    a = 6.12e-2
    eos = th.EOS(a)
    Ts, Tw = 0.86 * eos.Tc, 0.9 * eos.Tc
    rv, rl, _ = th.maxwell(eos, Ts)
    sigma = th.fit_sigma(eos, Ts)
    ny, nx, cv, lam_l, lam_v = 96, 1, 10.0, 15.0, 1.0
    p = Params(nx=nx, ny=ny, a=a, sigma=sigma, kappa=0.0, rho_l=rl, rho_v=rv, walls=True,
               outflow_top=True, rho_w_bottom=rv, thermal=True, cv=cv, lambda_l=lam_l,
               lambda_v=lam_v, s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1,
               t_bottom_kind=DIRICHLET, t_bottom_val=Tw, t_top_kind=ADIABATIC)
    s = Sim(p)
    s.init_fields(np.full((ny, nx), rl), T=np.full((ny, nx), Ts))
    ja = cv * (Tw - Ts) / th.latent_heat(eos, Ts)
    assert abs(ja - 0.076) < 1e-3
    beta = th.stefan_beta(ja)
    alpha_v = lam_v / (cv * rv)
    mid = 0.5 * (rl + rv)

    def front():
        r = s.fields()[0][:, 0]
        k = int(np.nonzero(r < mid)[0].max())
        return k + (r[k] - mid) / (r[k] - r[k + 1])

    times = (500, 1000, 2000, 4000)
    pos = []
    for n in times:
        s.step(n - s.n)
        pos.append(front())
    exact = [2 * beta * np.sqrt(alpha_v * t) for t in times]
    print("Ja", ja, "beta", beta, "front", np.round(pos, 2), "similarity", np.round(exact, 2))
    assert all(b > a for a, b in zip(pos, pos[1:]))
    for a_, e in zip(pos, exact):
        assert 0.7 < a_ / e < 1.0
    # the liquid pushed out through the open end carries the mass away
    assert s.fields()[0].sum() < rl * ny - 0.5 * (rl - rv) * pos[-1]
