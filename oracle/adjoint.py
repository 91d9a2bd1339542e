"""Gradient of the evaporated liquid mass with respect to the bottom-row
Dirichlet temperatures (the heater profile), by complex-step
differentiation of the oracle's time step.

Test infrastructure only (see oracle/__init__.py).

Objective.  The liquid mass of a density field is M_l = sum_x rho H(rho)
with the smooth indicator H(rho) = (1 + tanh((rho - rho_mid) / width)) / 2;
the evaporated mass after N steps is J = M_l(rho^0) - M_l(rho^N), rho^n the
density the step n reads (Eq. DensityAndVelocityRelationToF).  The heater
profile enters as the DIRICHLET values of the bottom row (rule R8 of
oracle/step.py), held at initialisation and after every RK stage of the
energy equation.

Method.  Every operation of the oracle's step is an analytic function of
its inputs (no branch depends on the perturbed values), so for a real
direction v and h << 1, J(Tb + i h v) = J(Tb) + i h dJ/dTb . v + O(h^2),
and dJ/dTb . v = Im J(Tb + i h v) / h to rounding, with no cancellation.
One complex run gives one directional derivative; unit vectors give the
gradient entries.  Parity pin: central differences in float64
(tests/test_oracle_adjoint.py).
"""
import dataclasses

import numpy as np

from .step import Sim


def smooth_liquid_mass(rho, rho_mid, width):
    return (rho * 0.5 * (1.0 + np.tanh((rho - rho_mid) / width))).sum()


def evaporated_mass(params, rho0, T0, nsteps, rho_mid, width, t_bottom_val=None):
    """J for the heater profile t_bottom_val (real or complex)."""
    p = params if t_bottom_val is None else dataclasses.replace(
        params, t_bottom_val=np.asarray(t_bottom_val))
    cplx = np.iscomplexobj(p.t_bottom_val)
    s = Sim(p, dtype=np.complex128 if cplx else np.float64)
    s.init_fields(rho0, None, None, T0)
    m0 = smooth_liquid_mass(s.fields()[0], rho_mid, width)
    s.step(nsteps)
    return m0 - smooth_liquid_mass(s.fields()[0], rho_mid, width)


def heater_directional_derivative(params, rho0, T0, nsteps, rho_mid, width, v, h=1e-30):
    """dJ/dTb . v by one complex-step run."""
    tb = np.asarray(params.t_bottom_val, dtype=np.float64) + 1j * h * np.asarray(v, np.float64)
    return float(np.imag(evaporated_mass(params, rho0, T0, nsteps, rho_mid, width, tb)) / h)


def heater_gradient(params, rho0, T0, nsteps, rho_mid, width, entries=None, h=1e-30):
    """dJ/dTb[x] for x in entries (default: all nx), one complex run each."""
    nx = params.nx
    entries = range(nx) if entries is None else entries
    out = {}
    for x in entries:
        v = np.zeros(nx)
        v[x] = 1.0
        out[x] = heater_directional_derivative(params, rho0, T0, nsteps, rho_mid, width, v, h)
    return out
