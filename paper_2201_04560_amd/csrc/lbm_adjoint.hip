// Reverse mode of the time step: gradient of the evaporated liquid mass
// with respect to the bottom-row Dirichlet temperatures (the heater
// profile), for periodic lattices without gravity with the energy equation
// on (Sec. 2, Eqs. DensityAndVelocityRelationToF to energy-equation).
//
// Objective.  M_l = sum_x rho H(rho), H = (1 + tanh((rho - rho_mid)/width))/2,
// J = M_l(start) - M_l(end), rho the density a step reads.
//
// Schedule.  The forward pass runs the fused step kernel and stores the
// state (post-collision populations + T) every `ckpt` steps.  The backward
// pass walks the segments last to first: it re-runs the fused kernel over
// the segment from its checkpoint, each step writing straight into the
// segment's next state slot (identical bits: same kernel, same tiling), then
// reverses the steps one by one.  Each reversed step is a chain of plain float64 kernels, one node per
// thread, each a local map or a radius-1 gather (the transposed stencil of a
// forward scatter), so that no atomics are needed:
//   fm1  rho, j, psi from the stored state (pull-stream)
//   fm2  F^m, Q (kappa term), u
//   fm3  the RK2 stage temperature T*
//   per RK stage, second then first, one kernel each (k_ea_stage): the
//        adjoint of the temperature boundary rule (the Dirichlet bottom
//        values accumulate into the gradient) and the local partials of K on
//        the workgroup's tile plus a one-node ring into LDS, then the
//        transposed stencils gathered from there; the first stage's kernel
//        goes on with
//   ca   the adjoint of the MRT collision with the forcing S and the C term,
//        of u = (j + F/2)/rho and of the moments, gathering the adjoint of
//        the pull-stream from what the previous reversed step wrote
//   fa   adjoint of F^m and Q with respect to psi, then of psi(rho, T)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm_pp.h"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

constexpr int kThreads = 256;

__constant__ int d_cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int d_cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ double d_wi[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};
__constant__ double d_we[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Lallemand-Luo rows (rho, e, zeta, jx, qx, jy, qy, pxx, pxy) and their squared norms
__constant__ double d_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},     {-4, -1, -1, -1, -1, 2, 2, 2, 2}, {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},  {0, -2, 0, 2, 0, 1, -1, -1, 1},   {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},  {0, 1, -1, 1, -1, 0, 0, 0, 0},    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
__constant__ double d_Mn[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};

struct Geo {
  int nx, ny, pitch;
  long long plane;
  int fp32;
  double rho_ref;
};

// float64 scratch fields, dense index y * nx + x
enum Field {
  F_RHO, F_JX, F_JY, F_PSI, F_FX, F_FY, F_QXX, F_QYY, F_QXY, F_UX, F_UY, F_T, F_TS,
  F_THAT, F_AM2, F_AM1, F_TSH,
  F_RHOE, F_UXE, F_UYE,
  F_FXH, F_FYH, F_QXXH, F_QYYH, F_QXYH, F_PSIS,
  // two sets (reversed steps alternate): adjoints of rho through psi and of
  // the streamed populations, written by one reversed step, gathered by the next
  F_RHOPSI, F_RHOPSI1, F_FH0, F_FH1 = F_FH0 + 9,
  F_PH0 = F_FH1 + 9, kNumFields = F_PH0 + 9
};

struct Fields {
  double* f[kNumFields];
};

// the forward quantities each reversed step recomputes from its stored state
// (written by k_fm1, k_fm2, k_fm3, read by the adjoint kernels); they are kept
// per step of a segment, so that the recompute runs beside the reversal
constexpr int kFwd[] = {F_RHO, F_JX, F_JY, F_PSI, F_T, F_FX, F_FY, F_QXX, F_QYY, F_QXY, F_UX, F_UY, F_TS};
constexpr int kNumFwd = sizeof(kFwd) / sizeof(kFwd[0]);

struct BC {
  const int32_t* tk_b;
  const int32_t* tk_t;
  const double* tv_b;
  const double* tv_t;
  int side;
  double side_val;
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ int kind_at(const BC& bc, int x, int y, int nx, int ny) {
  if (bc.side && (x == 0 || x == nx - 1)) return T_DIRICHLET;
  if (y == 0) return bc.tk_b[x];
  if (y == ny - 1) return bc.tk_t[x];
  return T_FREE;
}

__device__ __forceinline__ double dir_val(const BC& bc, int x, int y, int nx) {
  if (bc.side && (x == 0 || x == nx - 1)) return bc.side_val;
  return y == 0 ? bc.tv_b[x] : bc.tv_t[x];
}

template <class S>
__device__ __forceinline__ double pop(const S* P, const Geo& g, int i, int x, int y) {
  const double v = double(P[i * g.plane + (long long)y * g.pitch + x]);
  if constexpr (sizeof(S) == 4) return v + d_we[i] * g.rho_ref;
  else return v;
}

// T (dp/dT)_rho and its partial derivatives (Eq. peng-robinson)
__device__ __forceinline__ void g_tdpdt(double rho, double T, const Phys& p, double& g, double& gT, double& gr) {
  const double br = p.b * rho, om = 1.0 - br, D = 1.0 + 2.0 * br - br * br;
  const double s = sqrt(T * p.inv_Tc);
  const double akw = p.a * p.kw;
  const double h = (1.0 + p.kw - p.kw * s) * s;  // (1 + kw (1 - s)) s
  const double r2D = rho * rho / D;
  g = rho * p.R * T / om + akw * r2D * h;
  const double dh_ds = 1.0 + p.kw - 2.0 * p.kw * s;
  gT = rho * p.R / om + akw * r2D * dh_ds * (s / (2.0 * T));
  const double dr2D = (2.0 * rho * D - rho * rho * (2.0 * p.b - 2.0 * p.b * p.b * rho)) / (D * D);
  gr = p.R * T / (om * om) + akw * h * dr2D;
}

__device__ __forceinline__ double psi_of(double rho, double T, const Phys& p) {
  return sqrt(2.0 * (p_eos(rho, T, p) - rho / 3.0) / p.G);
}

#define NODE_LOOP                                                  \
  const int id = blockIdx.x * blockDim.x + threadIdx.x;            \
  if (id >= g.nx * g.ny) return;                                   \
  const int x = id % g.nx, y = id / g.nx;                          \
  (void)x;                                                         \
  (void)y

#define NB(arr, i) arr[wrapi(y + d_cy[i], g.ny) * g.nx + wrapi(x + d_cx[i], g.nx)]

// ------------------------------------------------------------ forward parts
template <class S>
__global__ __launch_bounds__(kThreads) void k_fm1(const S* __restrict__ P, const S* __restrict__ T, Geo g,
                                                  Phys ph, Fields F) {
  NODE_LOOP;
  double r = 0, jx = 0, jy = 0;
  #pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double fi = pop(P, g, i, wrapi(x - d_cx[i], g.nx), wrapi(y - d_cy[i], g.ny));
    r += fi;
    jx += d_cx[i] * fi;
    jy += d_cy[i] * fi;
  }
  const double t = double(T[(long long)y * g.pitch + x]);
  F.f[F_RHO][id] = r;
  F.f[F_JX][id] = jx;
  F.f[F_JY][id] = jy;
  F.f[F_PSI][id] = psi_of(r, t, ph);
  F.f[F_T][id] = t;
}

__global__ __launch_bounds__(kThreads) void k_fm2(Geo g, Phys ph, Fields F) {
  NODE_LOOP;
  const double* psi = F.f[F_PSI];
  const double p0 = psi[id];
  double sx = 0, sy = 0, qxx = 0, qyy = 0, qxy = 0;
  #pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double pn = NB(psi, i);
    sx += d_wi[i] * pn * d_cx[i];
    sy += d_wi[i] * pn * d_cy[i];
    const double d = d_wi[i] * (pn - p0);
    qxx += d * d_cx[i] * d_cx[i];
    qyy += d * d_cy[i] * d_cy[i];
    qxy += d * d_cx[i] * d_cy[i];
  }
  const double fx = -ph.G * p0 * sx, fy = -ph.G * p0 * sy;
  const double k = ph.kappa * ph.G * 0.5 * p0;
  const double r = F.f[F_RHO][id];
  F.f[F_FX][id] = fx;
  F.f[F_FY][id] = fy;
  F.f[F_QXX][id] = k * qxx;
  F.f[F_QYY][id] = k * qyy;
  F.f[F_QXY][id] = k * qxy;
  F.f[F_UX][id] = (F.f[F_JX][id] + 0.5 * fx) / r;
  F.f[F_UY][id] = (F.f[F_JY][id] + 0.5 * fy) / r;
}

// K(phi) of Eq. energy-equation at (x, y) with rho, u held (isotropic
// radius-1 stencils: grad = sum W_i phi(x + c_i) c_i, lap = 6 sum w_i (phi_nb - phi))
template <class PhiF>
__device__ double energy_K(PhiF phi, const Fields& F, const Geo& g, const Phys& ph, int x, int y) {
  const double* rho = F.f[F_RHO];
  const double* ux = F.f[F_UX];
  const double* uy = F.f[F_UY];
  const int id = y * g.nx + x;
  const double p0 = phi(x, y);
  double gx = 0, gy = 0, lap = 0, grx = 0, gry = 0, du = 0;
  #pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int xn = wrapi(x + d_cx[i], g.nx), yn = wrapi(y + d_cy[i], g.ny);
    const int n = yn * g.nx + xn;
    const double pn = phi(xn, yn);
    gx += d_wi[i] * pn * d_cx[i];
    gy += d_wi[i] * pn * d_cy[i];
    lap += d_we[i] * (pn - p0);
    grx += d_wi[i] * rho[n] * d_cx[i];
    gry += d_wi[i] * rho[n] * d_cy[i];
    du += d_wi[i] * (ux[n] * d_cx[i] + uy[n] * d_cy[i]);
  }
  lap *= 6.0;
  const double r = rho[id];
  const double lam = ph.lambda_v + ph.dlam * (r - ph.rho_v);
  const double rcv = 1.0 / (r * ph.cv);
  return -(ux[id] * gx + uy[id] * gy) + (lam * lap + ph.dlam * (grx * gx + gry * gy)) * rcv -
         p0 * dp_dT(r, p0, ph) * du * rcv;
}

__global__ __launch_bounds__(kThreads) void k_fm3(Geo g, Phys ph, BC bc, Fields F) {
  NODE_LOOP;
  const double* Tn = F.f[F_T];
  auto phi = [&](int xx, int yy) { return Tn[yy * g.nx + xx]; };
  const int k = kind_at(bc, x, y, g.nx, g.ny);
  double v;
  if (k == T_DIRICHLET) {
    v = dir_val(bc, x, y, g.nx);
  } else {
    const int ys = k == T_ADIABATIC ? (y == 0 ? 1 : g.ny - 2) : y;
    v = phi(x, ys) + 0.5 * energy_K(phi, F, g, ph, x, ys);
  }
  F.f[F_TS][id] = v;
}

// ------------------------------------------------------- energy adjoint
// am = adjoint of the stage value before the boundary rule; Dirichlet
// bottom entries (not the side columns) accumulate into grad
__device__ __forceinline__ double ea_mask(const double* __restrict__ gin, double* __restrict__ am,
                                          double* __restrict__ grad, const Geo& g, const BC& bc, int id, int x,
                                          int y) {
  const int k = kind_at(bc, x, y, g.nx, g.ny);
  double a = 0.0;
  if (k == T_DIRICHLET) {
    if (y == 0 && !(bc.side && (x == 0 || x == g.nx - 1))) grad[x] += gin[id];
  } else if (k == T_FREE) {
    a = gin[id];
    if (y == 1 && kind_at(bc, x, 0, g.nx, g.ny) == T_ADIABATIC) a += gin[x];
    if (y == g.ny - 2 && kind_at(bc, x, g.ny - 1, g.nx, g.ny) == T_ADIABATIC) a += gin[(g.ny - 1) * g.nx + x];
  }
  am[id] = a;
  return a;
}

// value of the mask at (x, y) (ea_mask without its side effects)
__device__ __forceinline__ double ea_mask_val(const double* __restrict__ gin, const Geo& g, const BC& bc, int id,
                                              int x, int y) {
  const int k = kind_at(bc, x, y, g.nx, g.ny);
  double a = 0.0;
  if (k == T_FREE) {
    a = gin[id];
    if (y == 1 && kind_at(bc, x, 0, g.nx, g.ny) == T_ADIABATIC) a += gin[x];
    if (y == g.ny - 2 && kind_at(bc, x, g.ny - 1, g.nx, g.ny) == T_ADIABATIC) a += gin[(g.ny - 1) * g.nx + x];
  }
  return a;
}

// coefficients of the local partials of w * K(phi) at one node that its
// neighbours' transposed stencils gather
struct EaCoef {
  double cux, cuy, c1, c2x, c2y, c3, dx, dy;
};
// the local partials of w * K(phi) at (x, y): the gathered coefficients, and
// the node's own terms (philoc: d/dphi(x); rl, uxl, uyl: d/drho, d/du)
__device__ __forceinline__ void ea_coef_at(double w, const double* __restrict__ phi_arr, const Geo& g,
                                           const Phys& ph, const Fields& F, int id, int x, int y, EaCoef& c,
                                           double& philoc, double& rl, double& uxl, double& uyl) {
  const double* rho = F.f[F_RHO];
  const double* ux = F.f[F_UX];
  const double* uy = F.f[F_UY];
  const double p0 = phi_arr[id];
  double gx = 0, gy = 0, lap = 0, grx = 0, gry = 0, du = 0;
  #pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int n = wrapi(y + d_cy[i], g.ny) * g.nx + wrapi(x + d_cx[i], g.nx);
    const double pn = phi_arr[n];
    gx += d_wi[i] * pn * d_cx[i];
    gy += d_wi[i] * pn * d_cy[i];
    lap += d_we[i] * (pn - p0);
    grx += d_wi[i] * rho[n] * d_cx[i];
    gry += d_wi[i] * rho[n] * d_cy[i];
    du += d_wi[i] * (ux[n] * d_cx[i] + uy[n] * d_cy[i]);
  }
  lap *= 6.0;
  const double r = rho[id];
  const double lam = ph.lambda_v + ph.dlam * (r - ph.rho_v);
  const double rcv = 1.0 / (r * ph.cv);
  const double glx = ph.dlam * grx, gly = ph.dlam * gry;
  double gg, gT, gr;
  g_tdpdt(r, p0, ph, gg, gT, gr);
  c.cux = w * ux[id];
  c.cuy = w * uy[id];
  c.c1 = w * lam * rcv;
  c.c2x = w * glx * rcv;
  c.c2y = w * gly * rcv;
  c.c3 = w * gg * rcv;
  c.dx = w * gx * rcv;
  c.dy = w * gy * rcv;
  // d lap / d phi(x) = -6 (1 - w_0)
  philoc = -6.0 * (1.0 - 4.0 / 9.0) * w * lam * rcv - w * gT * du * rcv;
  const double num = lam * lap + glx * gx + gly * gy - gg * du;
  rl = w * (-num * rcv / r + (ph.dlam * lap - gr * du) * rcv);
  uxl = -w * gx;
  uyl = -w * gy;
}

// ----------------------------------------------------- collision adjoint
// The adjoint of the pull-stream f_i(x) = P_i(x - c_i) is gathered here: the
// adjoint of the collided population i at x is that of the streamed one at
// x + c_i plus that of rho there through psi, both written by the previous
// reversed step into the other set.  The first reversed step reads the seed
// (F_PH0) instead.  This step writes its own outputs into set `set`.
template <class S>
__device__ __forceinline__ void ca_at(const S* __restrict__ P, const Geo& g, const Phys& ph, const Fields& F,
                                      int thermal, int set, bool seeded, int id, int x, int y) {
  double f[9], fs[9];
  const double* rpsi = F.f[F_RHOPSI + (set ^ 1)];
  #pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[i] = pop(P, g, i, wrapi(x - d_cx[i], g.nx), wrapi(y - d_cy[i], g.ny));
    if (seeded) {
      fs[i] = F.f[F_PH0 + i][id];
    } else {
      const int n = wrapi(y + d_cy[i], g.ny) * g.nx + wrapi(x + d_cx[i], g.nx);
      fs[i] = F.f[F_FH0 + 9 * (set ^ 1) + i][n] + rpsi[n];
    }
  }
  const double r = F.f[F_RHO][id], ux = F.f[F_UX][id], uy = F.f[F_UY][id];
  const double fx = F.f[F_FX][id], fy = F.f[F_FY][id], psi = F.f[F_PSI][id];
  const double qxx = F.f[F_QXX][id], qyy = F.f[F_QYY][id], qxy = F.f[F_QXY][id];
  const double eta = ph.eta_v + (ph.eta_l - ph.eta_v) * (r - ph.rho_v) * ph.inv_drho;
  const double snu = 1.0 / (3.0 * eta + 0.5);
  const double dsnu = -3.0 * (ph.eta_l - ph.eta_v) * ph.inv_drho * snu * snu;
  double m[9], ms[9];
  #pragma unroll
  for (int k = 0; k < 9; ++k) {
    double s = 0, t = 0;
    #pragma unroll
    for (int i = 0; i < 9; ++i) {
      s += d_M[k][i] * f[i];
      t += d_M[k][i] * fs[i];
    }
    m[k] = s;
    ms[k] = t / d_Mn[k];  // adjoint of m* (M^-T = diag(1/n) M)
  }
  const double u2 = ux * ux + uy * uy;
  const double meq7 = r * (ux * ux - uy * uy), meq8 = r * ux * uy;
  const double uf = ux * fx + uy * fy, fm2 = fx * fx + fy * fy;
  const double A = ph.sig_e / (psi * psi), B = ph.sig_z / (psi * psi);
  const double S7 = 2.0 * (ux * fx - uy * fy), S8 = ux * fy + uy * fx;
  const double lam[9] = {1.0, ph.s_e, ph.s_z, ph.s_j, ph.s_q, ph.s_j, ph.s_q, snu, snu};
  // direct path m -> m*: (1 - Lambda); rho row: s_rho cancels (m_0 = meq_0)
  double mh[9];
  #pragma unroll
  for (int k = 0; k < 9; ++k) mh[k] = (1.0 - lam[k]) * ms[k];
  double rh = ms[0] * 1.0;  // meq_0 = rho with rate lam[0] = 1 (same total as any s_rho)
  double uxh = 0, uyh = 0;
  // Lambda(rho) through s_nu (rows pxx, pxy)
  const double snuh = ms[7] * (-(m[7] - meq7) - 0.5 * S7 - (qxx - qyy)) + ms[8] * (-(m[8] - meq8) - 0.5 * S8 - qxy);
  rh += snuh * dsnu;
  // equilibrium moments
  const double e1 = lam[1] * ms[1], e2 = lam[2] * ms[2], e3 = lam[3] * ms[3], e4 = lam[4] * ms[4];
  const double e5 = lam[5] * ms[5], e6 = lam[6] * ms[6], e7 = lam[7] * ms[7], e8 = lam[8] * ms[8];
  rh += e1 * (-2.0 + 3.0 * u2) + e2 * (1.0 - 3.0 * u2) + (e3 - e4) * ux + (e5 - e6) * uy + e7 * (ux * ux - uy * uy) +
        e8 * ux * uy;
  uxh += 6.0 * r * ux * (e1 - e2) + r * (e3 - e4) + 2.0 * r * ux * e7 + r * uy * e8;
  uyh += 6.0 * r * uy * (e1 - e2) + r * (e5 - e6) - 2.0 * r * uy * e7 + r * ux * e8;
  // forcing S, weights (1 - Lambda/2)
  const double s1 = (1.0 - 0.5 * lam[1]) * ms[1], s2 = (1.0 - 0.5 * lam[2]) * ms[2];
  const double s3 = (1.0 - 0.5 * lam[3]) * ms[3], s4 = (1.0 - 0.5 * lam[4]) * ms[4];
  const double s5 = (1.0 - 0.5 * lam[5]) * ms[5], s6 = (1.0 - 0.5 * lam[6]) * ms[6];
  const double s7 = (1.0 - 0.5 * lam[7]) * ms[7], s8 = (1.0 - 0.5 * lam[8]) * ms[8];
  const double ufh = 6.0 * (s1 - s2);
  const double fm2h = A * s1 - B * s2;
  const double psih = -2.0 / psi * (A * fm2 * s1 - B * fm2 * s2);
  double fxh = (s3 - s4) + 2.0 * ux * s7 + uy * s8 + ux * ufh + 2.0 * fx * fm2h;
  double fyh = (s5 - s6) - 2.0 * uy * s7 + ux * s8 + uy * ufh + 2.0 * fy * fm2h;
  uxh += 2.0 * fx * s7 + fy * s8 + fx * ufh;
  uyh += -2.0 * fy * s7 + fx * s8 + fy * ufh;
  // C term (kappa)
  const double qxxh = 1.5 * ph.s_e * ms[1] - 1.5 * ph.s_z * ms[2] - snu * ms[7];
  const double qyyh = 1.5 * ph.s_e * ms[1] - 1.5 * ph.s_z * ms[2] + snu * ms[7];
  const double qxyh = -snu * ms[8];
  // energy equation's use of rho and u
  if (thermal) {
    rh += F.f[F_RHOE][id];
    uxh += F.f[F_UXE][id];
    uyh += F.f[F_UYE][id];
  }
  // u = (j + F/2) / rho
  const double jxh = uxh / r, jyh = uyh / r;
  fxh += 0.5 * uxh / r;
  fyh += 0.5 * uyh / r;
  rh -= (uxh * ux + uyh * uy) / r;
  // f* = M^-1 m*, m = M f, rho = sum f, j = sum f c
  #pragma unroll
  for (int i = 0; i < 9; ++i) {
    double s = 0;
    #pragma unroll
    for (int k = 0; k < 9; ++k) s += d_M[k][i] * mh[k];
    F.f[F_FH0 + 9 * set + i][id] = s + rh + d_cx[i] * jxh + d_cy[i] * jyh;
  }
  F.f[F_FXH][id] = fxh;
  F.f[F_FYH][id] = fyh;
  F.f[F_QXXH][id] = qxxh;
  F.f[F_QYYH][id] = qyyh;
  F.f[F_QXYH][id] = qxyh;
  F.f[F_PSIS][id] = psih;
}
template <class S>
__global__ __launch_bounds__(kThreads) void k_ca(const S* __restrict__ P, Geo g, Phys ph, Fields F, int thermal,
                                                 int set, int seeded) {
  NODE_LOOP;
  ca_at(P, g, ph, F, thermal, set, seeded != 0, id, x, y);
}
// Reversal of one RK stage in one kernel (periodic lattices): each workgroup
// computes the local partials of its kEaTx x kEaTy tile and a one-node ring
// around it into LDS (the ring's mask values are read, not written), then
// every node of the tile gathers its neighbours' coefficients (the
// transposed stencils).  Owned nodes keep the side effects: am, the
// Dirichlet bottom entries of grad (one thread per column), the energy
// equation's adjoints of rho and u (FIRST: the stage that starts them), and
// out = base1 + (base2 or the node's own mask value) + the adjoint of phi.
// CA: the collision adjoint of the node follows (it reads only the node's
// own results of the stage).
// The workgroup has a thread for each of the extended tile's positions: the
// tile's own (or, in a tile cut by the lattice edge, their periodic images)
// and the 84 of the ring, so that no thread evaluates two positions one
// after the other (with one thread per tile node some evaluated three: the
// 256^2 x 500-step backward took 19.1 ms float32 / 19.7 ms float64 on
// MI355X, 18.0 / 18.5 ms with this layout; gradients bit-identical).
constexpr int kEaTx = 32, kEaTy = 8;
constexpr int kEaRing = 2 * (kEaTx + 2) + 2 * kEaTy;
constexpr int kEaThreads = (kEaTx * kEaTy + kEaRing + 63) / 64 * 64;
template <bool FIRST, bool CA, class S>
__global__ __launch_bounds__(kEaThreads) void k_ea_stage(const S* __restrict__ P, const double* __restrict__ gin,
                                                           double* __restrict__ am, double* __restrict__ grad,
                                                           BC bc, const double* __restrict__ phi_arr, double wfac,
                                                           double* __restrict__ out,
                                                           const double* __restrict__ base1, int own_base2, Geo g,
                                                           Phys ph, Fields F, int set, int seeded) {
  constexpr int EX = kEaTx + 2, EY = kEaTy + 2, NE = EX * EY;
  __shared__ double s_c[8][EY][EX];
  const int t = threadIdx.x;
  const int tx = t % kEaTx, ty = t / kEaTx;
  const int x0 = blockIdx.x * kEaTx, y0 = blockIdx.y * kEaTy;
  const int x = x0 + tx, y = y0 + ty;
  const bool owned = x < g.nx && y < g.ny;
  const int id = owned ? y * g.nx + x : 0;
  auto put = [&](int ex, int ey, const EaCoef& c) {
    s_c[0][ey][ex] = c.cux;
    s_c[1][ey][ex] = c.cuy;
    s_c[2][ey][ex] = c.c1;
    s_c[3][ey][ex] = c.c2x;
    s_c[4][ey][ex] = c.c2y;
    s_c[5][ey][ex] = c.c3;
    s_c[6][ey][ex] = c.dx;
    s_c[7][ey][ex] = c.dy;
  };
  static_assert(kEaTx * kEaTy + kEaRing == NE, "extended tile = tile + ring");
  double philoc = 0, rl = 0, uxl = 0, uyl = 0, a_own = 0;
  const bool tile_thread = t < kEaTx * kEaTy;
  if (tile_thread && owned) {
    // the mask with its side effects (ea_mask), then the node's partials
    a_own = ea_mask(gin, am, grad, g, bc, id, x, y);
    EaCoef c;
    ea_coef_at(wfac * a_own, phi_arr, g, ph, F, id, x, y, c, philoc, rl, uxl, uyl);
    put(tx + 1, ty + 1, c);
  } else if (t < NE) {
    // another position of the extended tile: a tile position past the
    // lattice edge (periodic image, x0 - 1 + ex wrapped) or one of the ring
    // (q: bottom row, top row, left column, right column)
    int ex, ey;
    if (tile_thread) {
      ex = tx + 1;
      ey = ty + 1;
    } else {
      const int q = t - kEaTx * kEaTy;
      if (q < EX) {
        ex = q;
        ey = 0;
      } else if (q < 2 * EX) {
        ex = q - EX;
        ey = EY - 1;
      } else if (q < 2 * EX + kEaTy) {
        ex = 0;
        ey = q - 2 * EX + 1;
      } else {
        ex = EX - 1;
        ey = q - 2 * EX - kEaTy + 1;
      }
    }
    const int xr = pmod(x0 - 1 + ex, g.nx), yr = pmod(y0 - 1 + ey, g.ny);
    const int idr = yr * g.nx + xr;
    EaCoef c;
    double d0, d1, d2, d3;
    ea_coef_at(wfac * ea_mask_val(gin, g, bc, idr, xr, yr), phi_arr, g, ph, F, idr, xr, yr, c, d0, d1, d2, d3);
    put(ex, ey, c);
  }
  __syncthreads();
  if (!tile_thread || !owned) return;
  // transposed stencils: the neighbour x - c_i sees this node as its i
  double ph_ = philoc, rh = 0, uxh = 0, uyh = 0;
  #pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int ex = tx + 1 - d_cx[i], ey = ty + 1 - d_cy[i];
    const double cx = d_cx[i], cy = d_cy[i], W = d_wi[i];
    ph_ += W * (-(s_c[0][ey][ex] * cx + s_c[1][ey][ex] * cy) + s_c[3][ey][ex] * cx + s_c[4][ey][ex] * cy) +
           6.0 * d_we[i] * s_c[2][ey][ex];
    rh += ph.dlam * W * (s_c[6][ey][ex] * cx + s_c[7][ey][ex] * cy);
    uxh -= W * cx * s_c[5][ey][ex];
    uyh -= W * cy * s_c[5][ey][ex];
  }
  if (FIRST) {
    F.f[F_RHOE][id] = rl + rh;
    F.f[F_UXE][id] = uxl + uxh;
    F.f[F_UYE][id] = uyl + uyh;
  } else {
    F.f[F_RHOE][id] += rl + rh;
    F.f[F_UXE][id] += uxl + uxh;
    F.f[F_UYE][id] += uyl + uyh;
  }
  out[id] = (base1 ? base1[id] : 0.0) + (own_base2 ? a_own : 0.0) + ph_;
  if constexpr (CA) ca_at(P, g, ph, F, 1, set, seeded != 0, id, x, y);
}

// adjoint of F^m, Q with respect to psi (gather), then of psi(rho, T); the
// part that reaches rho goes to set `set`
__global__ __launch_bounds__(kThreads) void k_fa(Geo g, Phys ph, Fields F, int set) {
  NODE_LOOP;
  const double* psi = F.f[F_PSI];
  const double p0 = psi[id];
  const double kG2 = ph.kappa * ph.G * 0.5;
  double h = F.f[F_PSIS][id] +
             (F.f[F_FXH][id] * F.f[F_FX][id] + F.f[F_FYH][id] * F.f[F_FY][id] + F.f[F_QXXH][id] * F.f[F_QXX][id] +
              F.f[F_QYYH][id] * F.f[F_QYY][id] + F.f[F_QXYH][id] * F.f[F_QXY][id]) /
                 p0 -
             kG2 * p0 * (F.f[F_QXXH][id] + F.f[F_QYYH][id]);
  #pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int n = wrapi(y - d_cy[i], g.ny) * g.nx + wrapi(x - d_cx[i], g.nx);
    const double cx = d_cx[i], cy = d_cy[i];
    h += d_wi[i] * psi[n] *
         (-ph.G * (F.f[F_FXH][n] * cx + F.f[F_FYH][n] * cy) +
          kG2 * (F.f[F_QXXH][n] * cx * cx + F.f[F_QYYH][n] * cy * cy + F.f[F_QXYH][n] * cx * cy));
  }
  const double r = F.f[F_RHO][id];
  const double t = F.f[F_T][id];
  const double inv = 1.0 / (ph.G * p0);
  F.f[F_RHOPSI + set][id] = h * (dp_drho(r, t, ph) - 1.0 / 3.0) * inv;
  F.f[F_THAT][id] += h * dp_dT(r, t, ph) * inv;
}

// ------------------------------------------------ objective and its seed
template <class S>
__device__ __forceinline__ double rho_read(const S* P, const Geo& g, int x, int y) {
  double r = 0;
  #pragma unroll
  for (int i = 0; i < 9; ++i) r += pop(P, g, i, wrapi(x - d_cx[i], g.nx), wrapi(y - d_cy[i], g.ny));
  return r;
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_mass(const S* __restrict__ P, Geo g, double rm, double wd,
                                                   double* __restrict__ part) {
  __shared__ double sh[kThreads];
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0;
  if (id < g.nx * g.ny) {
    const int x = id % g.nx, y = id / g.nx;
    const double r = rho_read(P, g, x, y);
    v = r * 0.5 * (1.0 + tanh((r - rm) / wd));
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kThreads) void k_sum(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  double v = 0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += part[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// dJ/dP_i(y) = -dJ (H + rho H')(y + c_i); the temperature adjoint starts at 0
template <class S>
__global__ __launch_bounds__(kThreads) void k_seed(const S* __restrict__ P, Geo g, double rm, double wd, double dJ,
                                                   Fields F) {
  NODE_LOOP;
  for (int i = 0; i < 9; ++i) {
    const int xn = wrapi(x + d_cx[i], g.nx), yn = wrapi(y + d_cy[i], g.ny);
    const double r = rho_read(P, g, xn, yn);
    const double t = tanh((r - rm) / wd);
    const double H = 0.5 * (1.0 + t), dH = 0.5 * (1.0 - t * t) / wd;
    F.f[F_PH0 + i][id] = -dJ * (H + r * dH);
  }
  F.f[F_THAT][id] = 0.0;
}

// start state: its Dirichlet bottom row holds the heater values
__global__ __launch_bounds__(kThreads) void k_grad_init(const double* __restrict__ that, double* __restrict__ grad,
                                                        Geo g, BC bc) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  if (kind_at(bc, x, 0, g.nx, g.ny) == T_DIRICHLET && !(bc.side && (x == 0 || x == g.nx - 1))) grad[x] += that[x];
}

__global__ __launch_bounds__(kThreads) void k_zero(double* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

size_t al(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

struct lbm_adjoint {
  lbm_ctx* c = nullptr;
  int nsteps = 0, ckpt = 0, nck = 0;
  double rm = 0, wd = 1;
  char* buf = nullptr;
  size_t bytes = 0;
  size_t fbytes = 0, tbytes = 0, slot = 0;
  size_t off_ck = 0, off_seg = 0, off_fin = 0, off_fields = 0, off_grad = 0, off_part = 0, off_out = 0, off_fwd = 0;
  int64_t start_step = 0;
  double m0 = 0;
  bool forward_done = false;
  uint64_t gen = 0;  // the context's generation at the end of the forward pass
  double fwd_ms = 0, bwd_ms = 0;
  Fields F{};
  Geo g{};
  BC bc{};
  // the backward replays segment k - 1 on a stream of its own while segment
  // k is reversed; segment k's states use slot set k & 1
  hipStream_t replay = nullptr;
  hipEvent_t ev_start = nullptr, ev_replayed[2] = {nullptr, nullptr}, ev_reversed[2] = {nullptr, nullptr};

  char* slot_ptr(size_t off, int k) const { return buf + off + size_t(k) * slot; }
  // the fields with the forward quantities of step s of segment k in place
  Fields fields_at(int k, int s) const {
    Fields r = F;
    const size_t fb = al(size_t(g.nx) * g.ny * 8);
    char* base = buf + off_fwd + (size_t((k & 1) * ckpt + s) * kNumFwd) * fb;
    for (int j = 0; j < kNumFwd; ++j) r.f[kFwd[j]] = reinterpret_cast<double*>(base + size_t(j) * fb);
    return r;
  }
  ~lbm_adjoint() {
    for (hipEvent_t e : {ev_start, ev_replayed[0], ev_replayed[1], ev_reversed[0], ev_reversed[1]})
      if (e) (void)hipEventDestroy(e);
    if (replay) (void)hipStreamDestroy(replay);
  }
};

static void adj_sizes(const lbm_params& p, int nsteps, int ckpt, size_t& fbytes, size_t& tbytes, size_t& slot,
                      size_t& total, size_t offs[8]) {
  Layout L;
  make_layout(p, L);
  fbytes = size_t(9 * L.plane) * L.elem;
  tbytes = size_t(L.pitch) * p.ny * L.elem;
  slot = al(fbytes) + al(tbytes);
  const int nck = (nsteps + ckpt - 1) / ckpt;
  const size_t nodes = size_t(p.nx) * p.ny;
  const int nblk = int((nodes + kThreads - 1) / kThreads);
  size_t o = 0;
  offs[0] = o; o += size_t(nck) * slot;                      // checkpoints
  offs[1] = o; o += 2 * size_t(ckpt) * slot;                 // segment states, two sets
  offs[2] = o; o += slot;                                    // final state
  offs[3] = o; o += size_t(kNumFields) * al(nodes * 8);      // float64 fields
  offs[4] = o; o += al(size_t(p.nx) * 8);                    // gradient
  offs[5] = o; o += al(size_t(nblk) * 8);                    // partial sums
  offs[6] = o; o += 256;                                     // scalar out
  offs[7] = o; o += 2 * size_t(ckpt) * kNumFwd * al(nodes * 8);  // recomputed forward fields, two sets
  total = o;
}

static lbm_status adj_check_params(const lbm_params* p, int nsteps, int ckpt) {
  if (!p || nsteps < 1 || ckpt < 1) return LBM_E_INVAL;
  if (p->walls || p->gy != 0.0 || !p->thermal) return LBM_E_UNSUPPORTED;
  if (p->nx < 3 || p->ny < 3) return LBM_E_INVAL;
  return LBM_OK;
}

template <class S>
static void copy_state(lbm_adjoint* a, char* dst, bool to_ctx) {
  lbm_ctx* c = a->c;
  char* f = static_cast<char*>(c->f(c->cur));
  char* T = static_cast<char*>(c->T(c->Tcur));
  if (to_ctx) {
    (void)hipMemcpyAsync(f, dst, a->fbytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(T, dst + al(a->fbytes), a->tbytes, hipMemcpyDeviceToDevice, c->stream);
  } else {
    (void)hipMemcpyAsync(dst, f, a->fbytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(dst + al(a->fbytes), T, a->tbytes, hipMemcpyDeviceToDevice, c->stream);
  }
}

template <class S>
static hipError_t liquid_mass(lbm_adjoint* a, const char* state, double* out_dev) {
  const int nodes = a->g.nx * a->g.ny, nblk = (nodes + kThreads - 1) / kThreads;
  double* part = reinterpret_cast<double*>(a->buf + a->off_part);
  hipLaunchKernelGGL(k_mass<S>, dim3(nblk), dim3(kThreads), 0, a->c->stream, reinterpret_cast<const S*>(state),
                     a->g, a->rm, a->wd, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, a->c->stream, part, nblk, out_dev);
  return hipGetLastError();
}

// the forward quantities of the step at the state stored in `state`, into
// the per-step fields F (on the replay stream, after the state's replay)
template <class S>
static hipError_t recompute_step(const lbm_adjoint* a, const char* state, bool thermal_on, const Fields& F,
                                 hipStream_t st) {
  const S* P = reinterpret_cast<const S*>(state);
  const S* T = reinterpret_cast<const S*>(state + al(a->fbytes));
  const Geo& g = a->g;
  const Phys& ph = a->c->ph;
  const int nodes = g.nx * g.ny;
  const dim3 grid((nodes + kThreads - 1) / kThreads), blk(kThreads);
  hipLaunchKernelGGL(k_fm1<S>, grid, blk, 0, st, P, T, g, ph, F);
  hipLaunchKernelGGL(k_fm2, grid, blk, 0, st, g, ph, F);
  if (thermal_on) hipLaunchKernelGGL(k_fm3, grid, blk, 0, st, g, ph, a->bc, F);
  return hipGetLastError();
}

// the reversed energy update of one step up to its first RK stage, F
// holding the step's forward quantities: stage 2 (T' = BC(T + K(T*)))
// reversed in one kernel; stage 1 is reversed together with the collision
// in reverse_step_rest
template <class S>
static hipError_t reverse_energy(lbm_adjoint* a, bool thermal_on, const Fields& F) {
  const Geo& g = a->g;
  const Phys& ph = a->c->ph;
  double* grad = reinterpret_cast<double*>(a->buf + a->off_grad);
  hipStream_t st = a->c->stream;
  const dim3 tiles((g.nx + kEaTx - 1) / kEaTx, (g.ny + kEaTy - 1) / kEaTy), tblk(kEaThreads);
  if (thermal_on)
    hipLaunchKernelGGL((k_ea_stage<true, false, S>), tiles, tblk, 0, st, nullptr, F.f[F_THAT], F.f[F_AM2], grad,
                       a->bc, F.f[F_TS], 1.0, F.f[F_TSH], nullptr, 0, g, ph, F, 0, 0);
  return hipGetLastError();
}

template <class S>
static hipError_t reverse_step_rest(lbm_adjoint* a, const char* state, bool thermal_on, int64_t j,
                                    const Fields& F) {
  const S* P = reinterpret_cast<const S*>(state);
  const Geo& g = a->g;
  const Phys& ph = a->c->ph;
  double* grad = reinterpret_cast<double*>(a->buf + a->off_grad);
  hipStream_t st = a->c->stream;
  const int nodes = g.nx * g.ny;
  const dim3 grid((nodes + kThreads - 1) / kThreads), blk(kThreads);
  const dim3 tiles((g.nx + kEaTx - 1) / kEaTx, (g.ny + kEaTy - 1) / kEaTy), tblk(kEaThreads);
  // j counts the reversed steps from 0: the first reads the seed, each later
  // one gathers what the previous one wrote into the other set
  const int set = int(j & 1), seeded = j == 0;
  if (thermal_on)
    // stage 1 (T* = BC(T + K(T)/2)) and the collision: the adjoint of T is
    // that of stage 2's mask, of stage 1's mask and of phi
    hipLaunchKernelGGL((k_ea_stage<false, true, S>), tiles, tblk, 0, st, P, F.f[F_TSH], F.f[F_AM1], grad, a->bc,
                       F.f[F_T], 0.5, F.f[F_THAT], F.f[F_AM2], 1, g, ph, F, set, seeded);
  else
    hipLaunchKernelGGL(k_ca<S>, grid, blk, 0, st, P, g, ph, F, 0, set, seeded);
  hipLaunchKernelGGL(k_fa, grid, blk, 0, st, g, ph, F, set);
  return hipGetLastError();
}

extern "C" {

lbm_status lbm_adjoint_bytes(const lbm_params* p, int32_t nsteps, int32_t ckpt_every, size_t* bytes) {
  if (!bytes) return LBM_E_INVAL;
  lbm_status s = adj_check_params(p, nsteps, ckpt_every);
  if (s != LBM_OK) return s;
  size_t fb, tb, sl, tot, offs[8];
  adj_sizes(*p, nsteps, ckpt_every, fb, tb, sl, tot, offs);
  *bytes = tot;
  return LBM_OK;
}

lbm_status lbm_adjoint_create(lbm_ctx* c, int32_t nsteps, int32_t ckpt_every, double rho_mid, double width,
                              void* dev_buf, size_t bytes, lbm_adjoint** out) {
  if (!c || !out) return LBM_E_INVAL;
  *out = nullptr;
  lbm_status s = adj_check_params(&c->p, nsteps, ckpt_every);
  if (s == LBM_E_UNSUPPORTED)
    return fail(c, s, "the adjoint covers periodic lattices without gravity with the energy equation on");
  if (s != LBM_OK) return fail(c, s, "invalid adjoint arguments");
  if (!(width > 0)) return fail(c, LBM_E_INVAL, "width must be > 0");
  if (!dev_buf || reinterpret_cast<uintptr_t>(dev_buf) % 256)
    return fail(c, LBM_E_INVAL, "adjoint buffer must be non-null and 256-byte aligned");
  size_t offs[8], tot;
  lbm_adjoint* a = new (std::nothrow) lbm_adjoint();
  if (!a) return LBM_E_NOMEM;
  adj_sizes(c->p, nsteps, ckpt_every, a->fbytes, a->tbytes, a->slot, tot, offs);
  if (bytes < tot) {
    delete a;
    return fail(c, LBM_E_NOMEM, "adjoint buffer smaller than lbm_adjoint_bytes()");
  }
  a->c = c;
  a->nsteps = nsteps;
  a->ckpt = ckpt_every;
  a->nck = (nsteps + ckpt_every - 1) / ckpt_every;
  a->rm = rho_mid;
  a->wd = width;
  a->buf = static_cast<char*>(dev_buf);
  a->bytes = bytes;
  a->off_ck = offs[0];
  a->off_seg = offs[1];
  a->off_fin = offs[2];
  a->off_fields = offs[3];
  a->off_grad = offs[4];
  a->off_part = offs[5];
  a->off_out = offs[6];
  a->off_fwd = offs[7];
  const size_t nodes = size_t(c->p.nx) * c->p.ny;
  for (int k = 0; k < kNumFields; ++k)
    a->F.f[k] = reinterpret_cast<double*>(a->buf + a->off_fields + size_t(k) * al(nodes * 8));
  a->g = Geo{c->p.nx, c->p.ny, c->L.pitch, c->L.plane, c->p.precision == LBM_FP32_SHIFTED, c->ph.rho_ref};
  const Tables t = c->tables();
  a->bc = BC{t.tk_b, t.tk_t, t.tv_b, t.tv_t, c->p.t_side_dirichlet, c->p.t_side_val};
  // default priority, like every stream of the library
  hipError_t e = hipStreamCreateWithFlags(&a->replay, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&a->ev_start, &a->ev_replayed[0], &a->ev_replayed[1], &a->ev_reversed[0],
                         &a->ev_reversed[1]})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete a;
    return fail(c, LBM_E_HIP, "adjoint: stream or event creation failed");
  }
  *out = a;
  return LBM_OK;
}

void lbm_adjoint_destroy(lbm_adjoint* a) { delete a; }

}  // extern "C"

template <class S>
static lbm_status adj_forward(lbm_adjoint* a, double* J) {
  lbm_ctx* c = a->c;
  if (!c->initialized) return fail(c, LBM_E_STATE, "adjoint forward before lbm_init_fields");
  const auto t0 = std::chrono::steady_clock::now();
  a->forward_done = false;
  double* out = reinterpret_cast<double*>(a->buf + a->off_out);
  a->start_step = c->step;
  // M_l at the start: stage the current state in checkpoint 0
  for (int k = 0; k < a->nck; ++k) {
    char* ck = a->slot_ptr(a->off_ck, k);
    copy_state<S>(a, ck, false);
    if (k == 0) HIP_TRY(c, liquid_mass<S>(a, ck, out));
    if (k == 0) {
      double m0 = 0;
      HIP_TRY(c, hipMemcpyAsync(&m0, out, 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      a->m0 = m0;
    }
    const int n = std::min(a->ckpt, a->nsteps - k * a->ckpt);
    lbm_status s = lbm_step(c, n);
    if (s != LBM_OK) return s;
  }
  char* fin = a->buf + a->off_fin;
  copy_state<S>(a, fin, false);
  HIP_TRY(c, liquid_mass<S>(a, fin, out));
  double m1 = 0;
  HIP_TRY(c, hipMemcpyAsync(&m1, out, 8, hipMemcpyDeviceToHost, c->stream));
  lbm_status s = lbm_sync(c);
  if (s != LBM_OK) return s;
  if (J) *J = a->m0 - m1;
  a->forward_done = true;
  a->gen = c->generation;
  a->fwd_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return LBM_OK;
}

// one forward step of the fused kernel from the stored state `src` into the
// slot `dst` (same layout as the context's buffers, same launch as lbm_step
// at step index n, so the states are bit-identical to the forward run's);
// without the energy update T is carried over
static hipError_t step_into(lbm_adjoint* a, const char* src, char* dst, int64_t n, hipStream_t st) {
  lbm_ctx* c = a->c;
  LaunchStep L = step_args(c);
  L.fin = src;
  L.fout = dst;
  L.Tin = src + al(a->fbytes);
  L.Tout = dst + al(a->fbytes);
  L.update_T = c->p.thermal && n >= c->p.n_iso;
  L.want_mass = 0;
  hipError_t e = launch_step(L, st);
  if (e == hipSuccess && !L.update_T)
    e = hipMemcpyAsync(dst + al(a->fbytes), src + al(a->fbytes), a->tbytes, hipMemcpyDeviceToDevice, st);
  return e;
}

template <class S>
static lbm_status adj_backward(lbm_adjoint* a, double dJ, double* grad_host) {
  lbm_ctx* c = a->c;
  if (!a->forward_done) return fail(c, LBM_E_STATE, "adjoint backward before forward");
  // the backward replays the recorded trajectory with the lattice's current
  // boundary tables and leaves the lattice at the forward's end state: both
  // are wrong once anything stepped, re-initialised or re-bounded it
  if (c->generation != a->gen)
    return fail(c, LBM_E_STATE,
                "the lattice changed (step, init, boundary, state load or batch run) since the "
                "adjoint forward pass: run the forward pass again");
  const auto t0 = std::chrono::steady_clock::now();
  const Geo& g = a->g;
  const int nodes = g.nx * g.ny;
  const dim3 grid((nodes + kThreads - 1) / kThreads), blk(kThreads);
  double* grad = reinterpret_cast<double*>(a->buf + a->off_grad);
  hipLaunchKernelGGL(k_zero, dim3((g.nx + kThreads - 1) / kThreads), blk, 0, c->stream, grad, g.nx);
  char* fin = a->buf + a->off_fin;
  hipLaunchKernelGGL(k_seed<S>, grid, blk, 0, c->stream, reinterpret_cast<const S*>(fin), g, a->rm, a->wd, dJ,
                     a->F);
  HIP_TRY(c, hipGetLastError());
  // state s of segment k: the checkpoint for s = 0, else slot s of set k & 1
  auto state_of = [&](int k, int s) {
    return s == 0 ? a->slot_ptr(a->off_ck, k) : a->slot_ptr(a->off_seg, (k & 1) * a->ckpt + s);
  };
  auto seg_len = [&](int k) { return std::min(a->ckpt, a->nsteps - k * a->ckpt); };
  // replay segment k with the fused step on the replay stream, each state
  // written straight into its slot, then recompute each step's forward
  // quantities from its state
  auto replay = [&](int k) -> hipError_t {
    const int n0 = k * a->ckpt;
    for (int s = 1; s < seg_len(k); ++s) {
      const hipError_t e = step_into(a, state_of(k, s - 1), state_of(k, s), a->start_step + n0 + s - 1, a->replay);
      if (e != hipSuccess) return e;
    }
    for (int s = 0; s < seg_len(k); ++s) {
      const int64_t n = a->start_step + n0 + s;
      const hipError_t e = recompute_step<S>(a, state_of(k, s), c->p.thermal && n >= c->p.n_iso,
                                             a->fields_at(k, s), a->replay);
      if (e != hipSuccess) return e;
    }
    return hipEventRecord(a->ev_replayed[k & 1], a->replay);
  };
  HIP_TRY(c, hipEventRecord(a->ev_start, c->stream));
  HIP_TRY(c, hipStreamWaitEvent(a->replay, a->ev_start, 0));
  HIP_TRY(c, replay(a->nck - 1));
  for (int k = a->nck - 1; k >= 0; --k) {
    HIP_TRY(c, hipStreamWaitEvent(c->stream, a->ev_replayed[k & 1], 0));
    if (k > 0) {
      // set (k - 1) & 1 was last read by the reversal of segment k + 1
      if (k + 1 < a->nck) HIP_TRY(c, hipStreamWaitEvent(a->replay, a->ev_reversed[(k + 1) & 1], 0));
      HIP_TRY(c, replay(k - 1));
    }
    const int n0 = k * a->ckpt;
    for (int s = seg_len(k) - 1; s >= 0; --s) {
      const int64_t n = a->start_step + n0 + s;
      const bool th = c->p.thermal && n >= c->p.n_iso;
      const char* state = state_of(k, s);
      const Fields F = a->fields_at(k, s);
      HIP_TRY(c, reverse_energy<S>(a, th, F));
      HIP_TRY(c, reverse_step_rest<S>(a, state, th, a->start_step + a->nsteps - 1 - n, F));
    }
    HIP_TRY(c, hipEventRecord(a->ev_reversed[k & 1], c->stream));
  }
  hipLaunchKernelGGL(k_grad_init, dim3((g.nx + kThreads - 1) / kThreads), blk, 0, c->stream, a->F.f[F_THAT], grad,
                     g, a->bc);
  HIP_TRY(c, hipGetLastError());
  // leave the context at the end of the forward run
  copy_state<S>(a, fin, true);
  c->step = a->start_step + a->nsteps;
  if (grad_host) HIP_TRY(c, hipMemcpyAsync(grad_host, grad, size_t(g.nx) * 8, hipMemcpyDeviceToHost, c->stream));
  lbm_status s = lbm_sync(c);
  a->bwd_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

extern "C" {

lbm_status lbm_adjoint_forward(lbm_adjoint* a, double* J) {
  if (!a) return LBM_E_INVAL;
  return a->g.fp32 ? adj_forward<float>(a, J) : adj_forward<double>(a, J);
}

lbm_status lbm_adjoint_backward(lbm_adjoint* a, double dJ, double* grad_t_bottom) {
  if (!a) return LBM_E_INVAL;
  return a->g.fp32 ? adj_backward<float>(a, dJ, grad_t_bottom) : adj_backward<double>(a, dJ, grad_t_bottom);
}

lbm_status lbm_adjoint_timing(const lbm_adjoint* a, double* forward_ms, double* backward_ms) {
  if (!a) return LBM_E_INVAL;
  if (forward_ms) *forward_ms = a->fwd_ms;
  if (backward_ms) *backward_ms = a->bwd_ms;
  return LBM_OK;
}

}  // extern "C"
