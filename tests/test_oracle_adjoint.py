"""Pins of the oracle's heater gradient (complex-step differentiation of the
oracle's step): central differences in float64, exact zeros where the
heater value is overridden, linearity of the directional derivative."""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as adj
from oracle import thermo as th
from oracle.step import Params

DIRICHLET = 1


def tiny_case(nx=16, ny=14, nsteps=12, seed=3):
    """Droplet near a heated bottom row inside a Dirichlet ring."""
    eos = th.EOS(2.0 / 49.0)
    Tsat = 0.86 * eos.Tc
    rv, rl, _ = th.maxwell(eos, Tsat)
    Tout = 0.95 * eos.Tc
    rng = np.random.default_rng(seed)
    tb = Tout * (1.0 + 0.01 * rng.uniform(-1, 1, nx))
    p = Params(nx=nx, ny=ny, a=2.0 / 49.0, sigma=0.1, kappa=0.1, rho_l=rl, rho_v=rv, thermal=True,
               cv=6.0, lambda_l=2 / 3, lambda_v=2 / 3, t_side_dirichlet=True, t_side_val=Tout,
               t_bottom_kind=np.full(nx, DIRICHLET), t_bottom_val=tb,
               t_top_kind=np.full(nx, DIRICHLET), t_top_val=np.full(nx, Tout),
               **wl.DROPLET_RATES)
    rho, T = wl.droplet(nx, ny, 3.5, 1.2, rl, rv, Tsat, Tout, centre=(nx / 2, 5.0), seed=seed)
    return p, rho, T, nsteps, 0.5 * (rl + rv), (rl - rv) / 8.0


def test_complex_step_matches_central_differences():
    p, rho, T, n, rm, w = tiny_case()
    g = adj.heater_gradient(p, rho, T, n, rm, w, entries=[3, 7, 8, 12])
    h = 2e-6
    for x, gx in g.items():
        tp = p.t_bottom_val.copy()
        tm = p.t_bottom_val.copy()
        tp[x] += h
        tm[x] -= h
        fd = (adj.evaporated_mass(p, rho, T, n, rm, w, tp) -
              adj.evaporated_mass(p, rho, T, n, rm, w, tm)) / (2 * h)
        print(x, gx, fd)
        assert abs(gx) > 1e-3
        assert abs(gx - fd) <= 1e-6 * abs(gx), (x, gx, fd)


def test_overridden_heater_entries_have_zero_gradient():
    """Columns 0 and nx-1 are held at the side value: the corner entries of
    the bottom profile never enter the computation."""
    p, rho, T, n, rm, w = tiny_case()
    g = adj.heater_gradient(p, rho, T, n, rm, w, entries=[0, p.nx - 1])
    assert g[0] == 0.0 and g[p.nx - 1] == 0.0


def test_directional_derivative_is_linear():
    p, rho, T, n, rm, w = tiny_case(nsteps=6)
    g = adj.heater_gradient(p, rho, T, n, rm, w)
    v = np.random.default_rng(1).normal(size=p.nx)
    d = adj.heater_directional_derivative(p, rho, T, n, rm, w, v)
    gv = sum(v[x] * g[x] for x in g)
    assert abs(d - gv) <= 1e-12 * max(abs(d), np.abs(list(g.values())).max())
