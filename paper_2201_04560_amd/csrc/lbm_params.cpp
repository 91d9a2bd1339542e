// Host parameter pipeline of the mesh-refinement procedure (Sec. 3):
// Peng-Robinson critical temperature, Maxwell coexistence, the sigma fit of
// Eq. integral_coexistence_curve and the planar surface tension of
// Eq. surface_tension; the latent heat and the Stefan constant of
// Eq. stefan-analytical (Sec. 4.2).  Plain float64 C++, no GPU.
#include <cmath>
#include <functional>

#include "../../include/lbm_pp.h"

namespace {

struct PR {
  double a, b, R, kw, Tc;
  PR(double a_, double b_, double R_, double omega) : a(a_), b(b_), R(R_) {
    kw = 0.37464 + 1.54226 * omega - 0.2699 * omega * omega;
    Tc = 0.0778 * a / (0.45724 * b * R);
  }
  double alpha(double T) const {
    const double s = 1.0 + kw * (1.0 - std::sqrt(T / Tc));
    return s * s;
  }
  double p(double rho, double T) const {
    const double br = b * rho;
    return rho * R * T / (1.0 - br) - a * alpha(T) * rho * rho / (1.0 + 2.0 * br - br * br);
  }
  double dp(double rho, double T) const {
    const double br = b * rho, D = 1.0 + 2.0 * br - br * br;
    return R * T / ((1.0 - br) * (1.0 - br)) - a * alpha(T) * 2.0 * rho * (1.0 + br) / (D * D);
  }
  // d alpha / dT
  double dalpha(double T) const {
    const double s = 1.0 + kw * (1.0 - std::sqrt(T / Tc));
    return -kw * s / std::sqrt(T * Tc);
  }
  // antiderivative of p dv in the specific volume v = 1/rho
  double int_p_dv(double v, double T) const {
    const double s2 = std::sqrt(2.0);
    return R * T * std::log(v - b) -
           a * alpha(T) / (2.0 * s2 * b) * std::log((v + b - s2 * b) / (v + b + s2 * b));
  }
};

double bisect(const std::function<double(double)>& f, double lo, double hi, int maxit = 300) {
  double flo = f(lo);
  for (int i = 0; i < maxit; ++i) {
    const double mid = 0.5 * (lo + hi);
    const double fm = f(mid);
    if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else { hi = mid; }
    if (hi - lo <= 1e-16 * std::fabs(mid)) break;
  }
  return 0.5 * (lo + hi);
}

// composite 8-point Gauss-Legendre on [lo, hi] with n panels
double gauss(const std::function<double(double)>& f, double lo, double hi, int n = 256) {
  static const double xg[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                               0.9602898564975363};
  static const double wg[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                               0.1012285362903763};
  const double h = (hi - lo) / n;
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    const double c = lo + (k + 0.5) * h, r = 0.5 * h;
    for (int j = 0; j < 4; ++j) s += wg[j] * (f(c - r * xg[j]) + f(c + r * xg[j]));
  }
  return s * 0.5 * h;
}

bool spinodals(const PR& e, double T, double& s1, double& s2) {
  const int n = 20000;
  const double rmax = 0.999 / e.b;
  double prev = e.dp(1e-6, T);
  int found = 0;
  for (int i = 1; i <= n; ++i) {
    const double r = 1e-6 + (rmax - 1e-6) * i / n;
    const double d = e.dp(r, T);
    if ((d > 0) != (prev > 0)) {
      const double lo = 1e-6 + (rmax - 1e-6) * (i - 1) / n;
      const double root = bisect([&](double x) { return e.dp(x, T); }, lo, r);
      if (found == 0) s1 = root; else s2 = root;
      if (++found == 2) return true;
    }
    prev = d;
  }
  return false;
}

bool maxwell(const PR& e, double T, double& rv, double& rl, double& ps) {
  double s1, s2;
  if (!spinodals(e, T, s1, s2)) return false;
  const double pmax = e.p(s1, T), pmin = std::fmax(e.p(s2, T), 1e-300);
  const double rtop = (1.0 - 1e-12) / e.b;
  auto roots = [&](double p0, double& v, double& l) {
    v = bisect([&](double x) { return e.p(x, T) - p0; }, 1e-14, s1);
    l = bisect([&](double x) { return e.p(x, T) - p0; }, s2, rtop);
  };
  // equal area in closed form: int_{v_l}^{v_v} (p - p0) dv
  auto area = [&](double p0) {
    double v, l;
    roots(p0, v, l);
    const double vv = 1.0 / v, vl = 1.0 / l;
    return e.int_p_dv(vv, T) - e.int_p_dv(vl, T) - p0 * (vv - vl);
  };
  ps = bisect(area, pmin * (1 + 1e-15), pmax * (1 - 1e-15));
  roots(ps, rv, rl);
  return true;
}

double coex_integral(const PR& e, double G, double T, double sigma, double rv, double rl, double ps) {
  const double expo = 1.0 - 16.0 * G * sigma;
  return gauss(
      [&](double r) {
        const double psi = std::sqrt(2.0 * (e.p(r, T) - r / 3.0) / G);
        const double dpsi = (e.dp(r, T) - 1.0 / 3.0) / (G * psi);
        return (ps - e.p(r, T)) * dpsi / std::pow(psi, expo);
      },
      rv, rl, 512);
}

}  // namespace

extern "C" {

double lbm_pr_critical_temperature(double a, double b, double R) {
  return 0.0778 * a / (0.45724 * b * R);
}

lbm_status lbm_pr_latent_heat(double a, double b, double R, double omega, double T, double rho_v,
                              double rho_l, double* h_fg) {
  if (!(a > 0) || !(b > 0) || !(R > 0) || !(T > 0) || !h_fg) return LBM_E_INVAL;
  if (!(rho_v > 0) || !(rho_l > rho_v) || !(b * rho_l < 1.0)) return LBM_E_INVAL;
  PR e(a, b, R, omega);
  if (!(T < e.Tc)) return LBM_E_INVAL;
  // h_fg = T int (dp/dT)_rho / rho^2 drho over [rho_v, rho_l], with
  // (dp/dT)_rho = rho R / (1 - b rho) - a alpha'(T) rho^2 / (1 + 2 b rho - b^2 rho^2):
  // the first part integrates to R ln(rho / (1 - b rho)), the second, with
  // 1 + 2 b rho - b^2 rho^2 = 2 - (b rho - 1)^2, to
  // ln((sqrt2 + b rho - 1) / (sqrt2 - b rho + 1)) / (2 sqrt2 b)
  const double s2 = std::sqrt(2.0);
  auto F = [&](double r) {
    const double w = b * r - 1.0;
    return R * std::log(r / (1.0 - b * r)) -
           a * e.dalpha(T) * std::log((s2 + w) / (s2 - w)) / (2.0 * s2 * b);
  };
  const double h = T * (F(rho_l) - F(rho_v));
  if (!std::isfinite(h)) return LBM_E_INVAL;
  *h_fg = h;
  return LBM_OK;
}

lbm_status lbm_stefan_beta(double ja, double* beta) {
  if (!(ja >= 0.0) || !std::isfinite(ja) || !beta) return LBM_E_INVAL;
  // g(beta) = sqrt(pi) beta exp(beta^2) erf(beta) rises from 0 and exceeds
  // any finite Ja before beta = 6 (g(6) > 1e16)
  const double sp = std::sqrt(M_PI);
  auto g = [&](double x) { return sp * x * std::exp(x * x) * std::erf(x) - ja; };
  double lo = 0.0, hi = 1.0;
  while (g(hi) < 0.0) {
    lo = hi;
    hi *= 2.0;
    if (hi > 64.0) return LBM_E_INVAL;
  }
  for (int i = 0; i < 200 && hi - lo > 1e-17 * hi; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (g(mid) < 0.0) lo = mid; else hi = mid;
  }
  *beta = 0.5 * (lo + hi);
  return LBM_OK;
}

lbm_status lbm_pr_maxwell(double a, double b, double R, double omega, double T, double* rho_v,
                          double* rho_l, double* p_sat) {
  if (!(a > 0) || !(b > 0) || !(R > 0) || !(T > 0) || !rho_v || !rho_l || !p_sat) return LBM_E_INVAL;
  PR e(a, b, R, omega);
  if (!(T < e.Tc)) return LBM_E_INVAL;
  double rv, rl, ps;
  if (!maxwell(e, T, rv, rl, ps)) return LBM_E_INVAL;
  *rho_v = rv;
  *rho_l = rl;
  *p_sat = ps;
  return LBM_OK;
}

lbm_status lbm_fit_sigma(double a, double b, double R, double omega, double G, double T, double* sigma) {
  if (!sigma || !(G < 0)) return LBM_E_INVAL;
  PR e(a, b, R, omega);
  double rv, rl, ps;
  if (!(T > 0 && T < e.Tc) || !maxwell(e, T, rv, rl, ps)) return LBM_E_INVAL;
  // secant from -16 G sigma_0 = 2
  double s0 = 2.0 / (-16.0 * G), s1 = 0.95 * s0;
  double f0 = coex_integral(e, G, T, s0, rv, rl, ps), f1 = coex_integral(e, G, T, s1, rv, rl, ps);
  for (int it = 0; it < 60 && f1 != f0; ++it) {
    const double s2 = s1 - f1 * (s1 - s0) / (f1 - f0);
    s0 = s1;
    f0 = f1;
    s1 = s2;
    f1 = coex_integral(e, G, T, s1, rv, rl, ps);
    if (std::fabs(s1 - s0) < 1e-13) break;
  }
  if (!std::isfinite(s1)) return LBM_E_INVAL;
  *sigma = s1;
  return LBM_OK;
}

lbm_status lbm_planar_gamma(double a, double b, double R, double omega, double G, double T, double sigma,
                            double* gamma0) {
  if (!gamma0 || !(G < 0)) return LBM_E_INVAL;
  PR e(a, b, R, omega);
  double rv, rl, ps;
  if (!(T > 0 && T < e.Tc) || !maxwell(e, T, rv, rl, ps)) return LBM_E_INVAL;
  // psi'^2 as a function of rho from the first integral of the normal
  // balance p + 2 sigma G^2 psi'^2 + (G/4) psi psi'' = p_sat; Simpson sums
  const int n = 200000;
  const double h = (rl - rv) / n, ex = 16.0 * G * sigma;
  double cum = 0.0, total = 0.0, prev_in = 0.0, prev_out = 0.0;
  for (int i = 0; i <= n; ++i) {
    const double r = rv + h * i;
    const double psi = std::sqrt(2.0 * (e.p(r, T) - r / 3.0) / G);
    const double dpsi = (e.dp(r, T) - 1.0 / 3.0) / (G * psi);
    const double in = (ps - e.p(r, T)) * std::pow(psi, ex - 1.0) * dpsi;
    if (i > 0) cum += 0.5 * h * (in + prev_in);
    double Y = (8.0 / G) * std::pow(psi, -ex) * cum;
    if (Y < 0) Y = 0;
    const double out = std::fabs(dpsi) * std::sqrt(Y);
    if (i > 0) total += 0.5 * h * (out + prev_out);
    prev_in = in;
    prev_out = out;
  }
  *gamma0 = -(G / 6.0) * total;
  return LBM_OK;
}

lbm_status lbm_refinement_level(double a_base, double dx, double Tr, double b, double R, double omega,
                                double G, double kappa0, double gy0, int64_t steps0, lbm_level* out) {
  if (!out || !(dx > 0) || !(Tr > 0 && Tr < 1) || !(a_base > 0)) return LBM_E_INVAL;
  lbm_level L{};
  L.dx = dx;
  // Eq. a-deltax: a = a_base (dx / dx0)^2, b fixed, T_c proportional to a
  L.a = a_base * dx * dx;
  L.Tc = lbm_pr_critical_temperature(L.a, b, R);
  L.T = Tr * L.Tc;
  lbm_status s = lbm_pr_maxwell(L.a, b, R, omega, L.T, &L.rho_v, &L.rho_l, &L.p_sat);
  if (s != LBM_OK) return s;
  // Eq. integral_coexistence_curve for sigma
  s = lbm_fit_sigma(L.a, b, R, omega, G, L.T, &L.sigma);
  if (s != LBM_OK) return s;
  // Eq. gamma-meshes-relation: gamma(dx) = gamma(dx0) dx / dx0, with
  // gamma = (1 - kappa) gamma(kappa = 0) from Eq. surface_tension
  double base_sigma, g_base, g0;
  const double Tb = Tr * lbm_pr_critical_temperature(a_base, b, R);
  s = lbm_fit_sigma(a_base, b, R, omega, G, Tb, &base_sigma);
  if (s != LBM_OK) return s;
  s = lbm_planar_gamma(a_base, b, R, omega, G, Tb, base_sigma, &g_base);
  if (s != LBM_OK) return s;
  s = lbm_planar_gamma(L.a, b, R, omega, G, L.T, L.sigma, &g0);
  if (s != LBM_OK) return s;
  L.gamma = (1.0 - kappa0) * g_base * dx;
  L.kappa = dx == 1.0 ? kappa0 : 1.0 - L.gamma / g0;
  // Table 1: g ~ dx^3; viscous regime: steps ~ dx^-2
  L.gy = gy0 * dx * dx * dx;
  L.steps = int64_t(std::llround(double(steps0) / (dx * dx)));
  *out = L;
  return LBM_OK;
}

}  // extern "C"
