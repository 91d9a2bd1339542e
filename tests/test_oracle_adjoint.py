"""Pins of the oracle's heater gradient (complex-step differentiation of the
oracle's step): central differences in float64, exact zeros where the
heater value is overridden, linearity of the directional derivative."""
import numpy as np
import pytest

import cases
from oracle import adjoint as adj


def tiny_case(nx=16, ny=14, nsteps=12, seed=3):
    """Droplet near a heated bottom row inside a Dirichlet ring."""
    c, rho, T, rm, w = cases.heater_case(nx, ny, seed=seed)
    return cases.oracle_params(c), rho, T, nsteps, rm, w


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
