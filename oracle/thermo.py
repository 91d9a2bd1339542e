"""Thermodynamics of the method: Peng-Robinson EOS, pseudopotential,
Maxwell coexistence, latent heat, the sigma fit, the planar surface
tension, the kappa rule and the Stefan similarity constant.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed
  Eq. peng-robinson   p_EOS(rho, T); T_c, p_c from a, b (Sec. 2.1)
  Eq. psi             psi = sqrt(2 (p_EOS - rho/3) / G), G = -1
  Eq. energy-equation (dp/dT)_rho needed by the compression term
  Sec. 3.2            Maxwell rule for the coexistence densities
  Eq. integral_coexistence_curve   sigma fit by the secant method from
                      -16 G sigma_0 = 2
  Eq. surface_tension / Eq. gamma-meshes-relation   gamma and kappa
  Eq. stefan-analytical  similarity constant beta
  Sec. 4.2            latent heat "from the Peng-Robinson EOS"

Readings (where the paper is silent):
  * h_fg is the integral of T (dp/dT)_rho / rho^2 over the coexistence
    interval, the latent heat of an EOS with constant c_v (it equals the
    Clausius-Clapeyron value; the tests check that identity).
  * The planar profile used for gamma in continuum form solves the normal
    mechanical balance p_EOS + 2 sigma G^2 psi'^2 + (G/4) psi psi'' = p_sat,
    the balance whose first integral is Eq. integral_coexistence_curve; it
    does not depend on kappa, so gamma = (1 - kappa) gamma(kappa = 0).

Parity pins (tests/test_oracle_thermo.py): criticality of the EOS at T_c,
equal PR fugacities at the Maxwell densities (textbook closed form),
wall densities 0.38 / 6.50 and diffusivities 0.23 / 0.26 printed in
Secs. 4.2-4.3, Clausius-Clapeyron for h_fg and the Jakob numbers printed
in Secs. 4.1-4.2, sigma against Table 2, kappa against Sec. 3.2 (loose),
beta against its small-Ja series.
"""
import math
import warnings
from dataclasses import dataclass

import numpy as np
from scipy import integrate, special

G_DEFAULT = -1.0

# Peng-Robinson constants as printed in Eq. peng-robinson
PR_OMEGA_A = 0.45724
PR_OMEGA_B = 0.0778
PR_K0, PR_K1, PR_K2 = 0.37464, 1.54226, 0.2699


def critical_temperature(a, b, R=1.0):
    """T_c from a = 0.45724 R^2 T_c^2 / p_c and b = 0.0778 R T_c / p_c."""
    return PR_OMEGA_B * a / (PR_OMEGA_A * b * R)


def critical_pressure(a, b, R=1.0):
    return PR_OMEGA_B * R * critical_temperature(a, b, R) / b


@dataclass
class EOS:
    """Peng-Robinson EOS in lattice units (Eq. peng-robinson)."""

    a: float
    b: float = 2.0 / 21.0
    R: float = 1.0
    omega: float = 0.344
    G: float = G_DEFAULT

    @property
    def Tc(self):
        return critical_temperature(self.a, self.b, self.R)

    @property
    def kw(self):
        """the acentric slope 0.37464 + 1.54226 w - 0.2699 w^2"""
        w = self.omega
        return PR_K0 + PR_K1 * w - PR_K2 * w * w

    def alpha(self, T):
        return (1.0 + self.kw * (1.0 - np.sqrt(T / self.Tc))) ** 2

    def p(self, rho, T):
        b = self.b
        return rho * self.R * T / (1.0 - b * rho) - self.a * self.alpha(T) * rho**2 / (
            1.0 + 2.0 * b * rho - b * b * rho**2
        )

    def dp_drho(self, rho, T):
        b = self.b
        D = 1.0 + 2.0 * b * rho - b * b * rho**2
        return self.R * T / (1.0 - b * rho) ** 2 - self.a * self.alpha(T) * 2.0 * rho * (
            1.0 + b * rho
        ) / D**2

    def dp_dT(self, rho, T):
        """(dp/dT) at constant rho, used by Eq. energy-equation."""
        b = self.b
        D = 1.0 + 2.0 * b * rho - b * b * rho**2
        s = np.sqrt(T / self.Tc)
        return rho * self.R / (1.0 - b * rho) + self.a * rho**2 * self.kw * (
            1.0 + self.kw * (1.0 - s)
        ) / (np.sqrt(T * self.Tc) * D)

    def psi_radicand(self, rho, T):
        """2 (p_EOS - rho/3) / G; must be > 0 (Eq. psi)."""
        return 2.0 * (self.p(rho, T) - rho / 3.0) / self.G

    def psi(self, rho, T):
        return np.sqrt(self.psi_radicand(rho, T))

    def dpsi_drho(self, rho, T):
        # psi^2 = 2 (p - rho/3)/G  ->  2 psi psi' = 2 (p' - 1/3)/G
        return (self.dp_drho(rho, T) - 1.0 / 3.0) / (self.G * self.psi(rho, T))


# ----------------------------------------------------------------------------
# Maxwell construction (Sec. 3.2 uses the Maxwell rule as the target of the
# sigma fit).  Brute force: spinodals by scanning the sign of dp/drho on a
# grid, branch roots by bisection, then bisection on p_sat until the
# equal-area condition  int_{v_l}^{v_v} (p - p_sat) dv = 0  holds.
# ----------------------------------------------------------------------------
def _bisect(fun, lo, hi, tol=1e-15, maxit=400):
    flo = fun(lo)
    for _ in range(maxit):
        mid = 0.5 * (lo + hi)
        fm = fun(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if hi - lo <= tol * max(1.0, abs(mid)):
            break
    return 0.5 * (lo + hi)


def spinodals(eos, T, n=200001):
    """Densities of the local max (vapour spinodal) and local min (liquid
    spinodal) of p(rho) at T < T_c."""
    rmax = (1.0 - 1e-9) / eos.b
    r = np.linspace(1e-6, rmax * 0.999, n)
    dp = eos.dp_drho(r, T)
    sgn = np.sign(dp)
    idx = np.nonzero(sgn[1:] != sgn[:-1])[0]
    if len(idx) < 2:
        raise ValueError("no two-phase region at this temperature")
    fn = lambda x: eos.dp_drho(x, T)
    s1 = _bisect(fn, r[idx[0]], r[idx[0] + 1])
    s2 = _bisect(fn, r[idx[1]], r[idx[1] + 1])
    return s1, s2


def maxwell(eos, T):
    """Coexistence (rho_v, rho_l, p_sat) of the EOS at temperature T."""
    s1, s2 = spinodals(eos, T)
    pmax = eos.p(s1, T)
    pmin = eos.p(s2, T)
    rmax = (1.0 - 1e-12) / eos.b

    def roots(p0):
        rv = _bisect(lambda x: eos.p(x, T) - p0, 1e-14, s1)
        rl = _bisect(lambda x: eos.p(x, T) - p0, s2, rmax)
        return rv, rl

    def area(p0):
        rv, rl = roots(p0)
        # int_{v_l}^{v_v} (p - p0) dv with v = 1/rho  ->  int_{rv}^{rl} (p-p0)/rho^2 drho
        val, _ = integrate.quad(lambda x: (eos.p(x, T) - p0) / x**2, rv, rl,
                                epsabs=1e-15, epsrel=1e-13, limit=200)
        return val

    lo = max(pmin, 1e-14)
    hi = pmax
    # area(p0) decreases with p0: positive at lo, negative at hi
    p_sat = _bisect(area, lo + 1e-15 * abs(hi), hi - 1e-15 * abs(hi), tol=1e-15)
    rv, rl = roots(p_sat)
    return rv, rl, p_sat


def latent_heat(eos, T, coex=None):
    """h_fg = int_{rho_v}^{rho_l} T (dp/dT)_rho / rho^2 drho (constant c_v)."""
    rv, rl, _ = coex if coex is not None else maxwell(eos, T)
    val, _ = integrate.quad(lambda x: T * eos.dp_dT(x, T) / x**2, rv, rl,
                            epsabs=1e-14, epsrel=1e-12, limit=200)
    return val


# ----------------------------------------------------------------------------
# sigma fit, Eq. integral_coexistence_curve
# ----------------------------------------------------------------------------
def coexistence_integral(eos, T, sigma, coex=None):
    """int_{rho_v}^{rho_l} (p_sat - p_EOS) psi_dot / psi^(1 - 16 G sigma) drho
    evaluated at the Maxwell densities."""
    rv, rl, ps = coex if coex is not None else maxwell(eos, T)
    expo = 1.0 - 16.0 * eos.G * sigma

    def integrand(x):
        return (ps - eos.p(x, T)) * eos.dpsi_drho(x, T) / eos.psi(x, T) ** expo

    val, _ = integrate.quad(integrand, rv, rl, epsabs=1e-15, epsrel=1e-13, limit=400)
    return val


def fit_sigma(eos, T, coex=None, tol=1e-13, maxit=60):
    """Secant root of Eq. integral_coexistence_curve in sigma, started from
    -16 G sigma_0 = 2 as the paper prescribes."""
    coex = coex if coex is not None else maxwell(eos, T)
    s0 = 2.0 / (-16.0 * eos.G)
    s1 = s0 * 0.95
    f0 = coexistence_integral(eos, T, s0, coex)
    f1 = coexistence_integral(eos, T, s1, coex)
    for _ in range(maxit):
        if f1 == f0:
            break
        s2 = s1 - f1 * (s1 - s0) / (f1 - f0)
        s0, f0 = s1, f1
        s1 = s2
        f1 = coexistence_integral(eos, T, s1, coex)
        if abs(s1 - s0) < tol:
            break
    return s1


# ----------------------------------------------------------------------------
# planar surface tension, Eq. surface_tension, continuum profile
# ----------------------------------------------------------------------------
def planar_gamma_continuum(eos, T, sigma, kappa=0.0, coex=None, n=400001):
    """gamma = (G/6)(1-kappa) int psi psi'' dx = -(G/6)(1-kappa) int psi'^2 dx
    for one planar interface whose profile solves the normal balance
    p_EOS + 2 sigma G^2 psi'^2 + (G/4) psi psi'' = p_sat.

    With Y(rho) = psi'^2, the balance integrates to
      Y = (8/G) psi^(-16 G sigma) int_{rho_v}^{rho} (p_sat - p) psi^(16 G sigma - 1) psi_dot
    and int psi'^2 dx = int |psi_dot| sqrt(Y) drho along the interface."""
    rv, rl, ps = coex if coex is not None else maxwell(eos, T)
    G = eos.G
    r = np.linspace(rv, rl, n)
    psi = eos.psi(r, T)
    pd = eos.dpsi_drho(r, T)
    e = 16.0 * G * sigma
    inner = (ps - eos.p(r, T)) * psi ** (e - 1.0) * pd
    cum = integrate.cumulative_trapezoid(inner, r, initial=0.0)
    Y = (8.0 / G) * psi ** (-e) * cum
    Y = np.maximum(Y, 0.0)
    I = integrate.trapezoid(np.abs(pd) * np.sqrt(Y), r)
    return -(G / 6.0) * (1.0 - kappa) * I


def kappa_for_target(gamma_target, gamma_kappa0):
    """Eq. surface_tension: gamma(kappa) = (1-kappa) gamma(0)  ->  kappa."""
    return 1.0 - gamma_target / gamma_kappa0


def refinement_parameters(a_base, L0, Ls, Tr=0.86, b=2.0 / 21.0, omega=0.344,
                          kappa0=0.0):
    """Sec. 3: per mesh L, a = a_base (L0/L)^2 (Eq. a-deltax), sigma from
    Eq. integral_coexistence_curve, kappa from Eq. gamma-meshes-relation
    with the continuum planar gamma.  Returns a list of dicts."""
    out = []
    eos0 = EOS(a_base, b, 1.0, omega)
    T0 = Tr * eos0.Tc
    c0 = maxwell(eos0, T0)
    s0 = fit_sigma(eos0, T0, c0)
    g0 = planar_gamma_continuum(eos0, T0, s0, kappa0, c0)
    for L in Ls:
        a = a_base * (L0 / L) ** 2
        eos = EOS(a, b, 1.0, omega)
        T = Tr * eos.Tc
        c = maxwell(eos, T)
        s = fit_sigma(eos, T, c)
        gk0 = planar_gamma_continuum(eos, T, s, 0.0, c)
        target = g0 * (L0 / L)
        kap = kappa_for_target(target, gk0) if L != L0 else kappa0
        out.append(dict(L=L, a=a, Tc=eos.Tc, T=T, rho_v=c[0], rho_l=c[1], p_sat=c[2],
                        sigma=s, kappa=kap, gamma=target))
    return out


# ----------------------------------------------------------------------------
# Stefan problem, Eq. stefan-analytical
# ----------------------------------------------------------------------------
def stefan_beta(ja):
    """beta with beta exp(beta^2) erf(beta) = Ja / sqrt(pi), by bisection."""
    target = ja / math.sqrt(math.pi)
    f = lambda b: b * math.exp(b * b) * special.erf(b) - target
    hi = 1.0
    while f(hi) < 0:
        hi *= 2.0
    return _bisect(f, 0.0, hi, tol=1e-15)


def coexistence_for_sigma(eos, T, sigma):
    """Planar coexistence densities predicted by the continuum theory for a
    given sigma: p(rho_v) = p(rho_l) = p0 and Eq. integral_coexistence_curve
    (with p0 in place of p_sat) vanishes.  Bisection on p0."""
    s1, s2 = spinodals(eos, T)
    pmax, pmin = eos.p(s1, T), eos.p(s2, T)
    rmax = (1.0 - 1e-12) / eos.b
    expo = 1.0 - 16.0 * eos.G * sigma

    def roots(p0):
        rv = _bisect(lambda x: eos.p(x, T) - p0, 1e-14, s1)
        rl = _bisect(lambda x: eos.p(x, T) - p0, s2, rmax)
        return rv, rl

    def resid(p0):
        rv, rl = roots(p0)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            val, _ = integrate.quad(
                lambda x: (p0 - eos.p(x, T)) * eos.dpsi_drho(x, T) / eos.psi(x, T) ** expo,
                rv, rl, epsabs=1e-15, epsrel=1e-13, limit=400)
        return val

    lo = max(pmin, 1e-14) + 1e-15 * abs(pmax)
    hi = pmax - 1e-15 * abs(pmax)
    p0 = _bisect(resid, lo, hi, tol=1e-15)
    rv, rl = roots(p0)
    return rv, rl, p0
