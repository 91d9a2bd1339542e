// Device-side building blocks of the pseudopotential LBM step (gfx950).
//
// Everything here is float64 unless a template parameter says otherwise:
// the Peng-Robinson EOS and the pseudopotential (Eqs. peng-robinson, psi)
// are always evaluated in float64, also by the float32-storage kernels,
// because psi differences near the spinodal lose all digits in float32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kLanes = 64;               // one wavefront per workgroup
constexpr int kHaloY = 3;                // RK2 energy update reaches 3 rows
// x halo (columns recomputed on each side of a 64-lane strip): 3 for the
// same reason, 4 with walls because the wall closure reads psi at x +- 1
inline int halo_x(int walls) { return walls ? 4 : 3; }
inline int tile_x(int walls) { return kLanes - 2 * halo_x(walls); }
constexpr int kNewtonWall = 8;           // Newton steps of the wall closure

enum { T_FREE = 0, T_DIRICHLET = 1, T_ADIABATIC = 2 };
enum : uint32_t { ERR_RHO = 1u, ERR_RADICAND = 2u, ERR_TEMP = 4u, ERR_NAN = 8u };

// float64 constants of the model, precomputed on the host
struct Phys {
  double a, b, R, G, kw, inv_Tc, Tc, inv_b, inv_sqrtTc, akw_isTc;  // akw_isTc = a kw / sqrt(T_c)
  double sigma, kappa;
  double s_e, s_z, s_j, s_q;
  double sig_e, sig_z;       // 12 sigma / (1/s_e - 1/2), 12 sigma / (1/s_z - 1/2)
  double eta_l, eta_v, rho_l, rho_v, inv_drho;
  double gy;
  double cv, lambda_l, lambda_v, dlam;  // dlam = (lambda_l - lambda_v)/(rho_l - rho_v)
  double t_side_val;
  double rho_ref;
  double two_G;     // 2 / G: the radicand of Eq. psi without a division
  int wall_mod;     // 1: modified-psi walls (the wall tables hold G_w)
  int outflow_top;  // 1: the top row is a zero-gradient outflow, not a wall
};

// constants of the collision and the energy update in the compute type C
template <class C>
struct PhysC {
  C s_e, s_z, s_q;
  C snu_const;             // used when eta_l == eta_v
  C eta_l, eta_v, rho_v, inv_drho;
  C lambda_v, dlam, inv_cv;
  C kw, inv_sqrtTc, akw_isTc;
  int snu_varies;
};

// per-column boundary tables (device pointers, nx entries each)
struct Tables {
  const double* rho_w_b;
  const double* rho_w_t;
  const double* tv_b;
  const double* tv_t;
  const int32_t* tk_b;
  const int32_t* tk_t;
};

// ---------------------------------------------------------------- EOS
// sqrt(alpha(T)) = 1 + kw (1 - sqrt(T / T_c))
__device__ __forceinline__ double sqrt_alpha(double T, const Phys& p) {
  return 1.0 + p.kw * (1.0 - sqrt(T * p.inv_Tc));
}

__device__ __forceinline__ double p_eos(double rho, double T, const Phys& p) {
  const double br = p.b * rho;
  const double sa = sqrt_alpha(T, p);
  return rho * p.R * T / (1.0 - br) - p.a * (sa * sa) * rho * rho / (1.0 + 2.0 * br - br * br);
}

__device__ __forceinline__ double dp_drho(double rho, double T, const Phys& p) {
  const double br = p.b * rho;
  const double sa = sqrt_alpha(T, p);
  const double om = 1.0 - br;
  const double D = 1.0 + 2.0 * br - br * br;
  return p.R * T / (om * om) - p.a * (sa * sa) * 2.0 * rho * (1.0 + br) / (D * D);
}

// (dp/dT)_rho of Eq. energy-equation
__device__ __forceinline__ double dp_dT(double rho, double T, const Phys& p) {
  const double br = p.b * rho;
  const double D = 1.0 + 2.0 * br - br * br;
  return rho * p.R / (1.0 - br) +
         p.a * rho * rho * p.kw * sqrt_alpha(T, p) / (sqrt(T * p.Tc) * D);
}

// psi radicand 2 (p - rho/3) / G
__device__ __forceinline__ double psi_radicand(double rho, double T, const Phys& p) {
  return 2.0 * (p_eos(rho, T, p) - rho / 3.0) / p.G;
}

// pseudopotential with the domain checks of the method; bits go to err
__device__ __forceinline__ double psi_checked(double rho, double T, const Phys& p, uint32_t& err) {
  const double rad = psi_radicand(rho, T, p);
  if (!(rho > 0.0) || !(rho < p.inv_b)) err |= ERR_RHO;
  if (!(T > 0.0)) err |= ERR_TEMP;
  if (!(rad > 0.0)) err |= ERR_RADICAND;
  return sqrt(rad);
}

__device__ __forceinline__ double dpsi_drho(double rho, double T, double psi, const Phys& p) {
  return (dp_drho(rho, T, p) - 1.0 / 3.0) / (p.G * psi);
}

// ------------------------------------------- fast float64 rcp / rsqrt / sqrt
// Hardware estimates refined by two Newton steps: ~1 ulp, not correctly
// rounded (the IEEE expansions cost 2-3x the instructions).
// NR: Newton steps (2 by default; 1 where the result feeds float32 storage)
template <int NR = 2>
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
  }
  return r;
}
template <int NR = 2>
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const double t = fma(-h * y, y, 0.5);
    y = fma(y, t, y);
  }
  return y;
}
__device__ __forceinline__ float rsq_c(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_c(double x) { return rsq64<2>(x); }
__device__ __forceinline__ float rcp_c(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_c(double x) { return rcp64<2>(x); }

// EOS terms of one node, shared by psi (stage A) and (dp/dT)_rho (energy
// stages): A1 = rho R / (1 - b rho), A2 = rho^2 / (1 + 2 b rho - b^2 rho^2),
// rsqT = 1 / sqrt(T); p = A1 T - a alpha(T) A2.
struct EosNode {
  double A1, A2, rsqT, rad;
};
template <int NR = 2>
__device__ __forceinline__ EosNode eos_node(double rho, double T, const Phys& p) {
  EosNode e;
  const double br = p.b * rho;
  const double om = 1.0 - br;
  const double D = 1.0 + 2.0 * br - br * br;
  const double inv = rcp64<NR>(om * D);
  e.A1 = rho * p.R * D * inv;
  e.A2 = rho * rho * om * inv;
  e.rsqT = rsq64<NR>(T);
  const double sa = 1.0 + p.kw * (1.0 - T * e.rsqT * p.inv_sqrtTc);
  const double pr = e.A1 * T - p.a * (sa * sa) * e.A2;
  e.rad = (pr - rho * (1.0 / 3.0)) * p.two_G;
  return e;
}
// psi = sqrt(rad) with the domain checks of the method
template <int NR = 2>
__device__ __forceinline__ double psi_fast(double rho, double T, const EosNode& e, const Phys& p,
                                           uint32_t& err) {
  if (!(rho > 0.0) || !(rho < p.inv_b)) err |= ERR_RHO;
  if (!(T > 0.0)) err |= ERR_TEMP;
  if (!(e.rad > 0.0)) err |= ERR_RADICAND;
  const double y = rsq64<NR>(e.rad);
  double s = e.rad * y;  // one Newton correction of the root itself
  return fma(0.5 * y, fma(-s, s, e.rad), s);
}

// ----------------------------------------------------------- wall closure
// Zou-He at a wet wall node with prescribed momentum -F/2, F = F^m + F^b:
// the wall density solves rho + sgn (psi(rho) B + gy (rho - rbk)) / 2 = K
// (sgn = +1 bottom, -1 top), where F^m_y = psi(rho) B and the buoyancy
// F^b_y = gy (rho - rbk) takes rbk, the mean density with every wall node
// counted at its known part K.  Fixed number of Newton steps from rho = K.
__device__ __forceinline__ double wall_coef_B(double nb_c, double nb_p, double nb_m, double psi_w,
                                              double sgn, const Phys& p) {
  const double nbsum = nb_c / 3.0 + (nb_p + nb_m) / 12.0;
  return -p.G * sgn * (nbsum - 0.5 * psi_w);
}

__device__ __forceinline__ double wall_density(double K, double B, double T, double sgn,
                                               const Phys& p, double rbk) {
  double r = K;
#pragma unroll 1
  for (int it = 0; it < kNewtonWall; ++it) {
    const double ps = sqrt(psi_radicand(r, T, p));
    const double g = r + sgn * 0.5 * (ps * B + p.gy * (r - rbk)) - K;
    const double dg = 1.0 + sgn * 0.5 * (dpsi_drho(r, T, ps, p) * B + p.gy);
    r = r - g / dg;
  }
  return r;
}

// Modified-psi walls (Eq. mod-psi-based-formula): F^m_y = sgn (-G psi nbsum
// + G_w psi^2 / 2) with nbsum the fluid neighbours' weighted psi, so zero
// fluid velocity asks rho + (-G psi nbsum + G_w psi^2 / 2) / 2 = K at both
// walls; Newton from rho = K
__device__ __forceinline__ double wall_density_mod(double K, double nbsum, double gw, double T,
                                                   double sgn, const Phys& p, double rbk) {
  double r = K;
#pragma unroll 1
  for (int it = 0; it < kNewtonWall; ++it) {
    const double ps = sqrt(psi_radicand(r, T, p));
    const double dps = dpsi_drho(r, T, ps, p);
    const double g = r + 0.5 * (-p.G * ps * nbsum + 0.5 * gw * ps * ps) + sgn * 0.5 * p.gy * (r - rbk) - K;
    const double dg = 1.0 + 0.5 * (-p.G * nbsum + gw * ps) * dps + sgn * 0.5 * p.gy;
    r = r - g / dg;
  }
  return r;
}

// ------------------------------------------------------------ utilities
__device__ __forceinline__ int pmod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// a modulo n for a in [-3, n + 3): one compare-and-add unless n < 3
__device__ __forceinline__ int wrap3(int a, int n) {
  if (n < 3) return pmod(a, n);
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanes);
  return v;
}

// Sum of n values in one fixed order, the same in every caller: lane l
// adds entries l, l + 64, ... into eight interleaved accumulators (eight
// loads in flight), then the accumulators and the lanes combine.  ld(i)
// loads entry i.
template <class LD>
__device__ __forceinline__ double fixed_order_sum(LD ld, int n, int lane) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = lane;
  for (; i + 7 * kLanes < n; i += 8 * kLanes) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += ld(i + k * kLanes);
  }
  for (; i < n; i += kLanes) a[0] += ld(i);  // fewer than 8 left per lane
  return wave_sum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kLanes));
  return v;
}

// temperature boundary kind of node (y, x): side columns, then top, then bottom
__device__ __forceinline__ int t_kind(int y, int x, int nx, int ny, int side_dir, const Tables& t,
                                      double& val, const Phys& p) {
  if (side_dir && (x == 0 || x == nx - 1)) {
    val = p.t_side_val;
    return T_DIRICHLET;
  }
  if (y == ny - 1) {
    val = t.tv_t[x];
    return t.tk_t[x];
  }
  if (y == 0) {
    val = t.tv_b[x];
    return t.tk_b[x];
  }
  val = 0.0;
  return T_FREE;
}

}  // namespace lbm
