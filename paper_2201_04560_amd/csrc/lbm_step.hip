// Fused time step of the pseudopotential LBM with phase change (gfx950).
//
// One workgroup = one wavefront of 64 lanes owns a strip of 58 output
// columns (plus 3 recomputed halo columns each side; 56 and 4 with walls)
// and marches up a segment of rows (3 halo rows each end).  Every row passes through four pipelined stages whose
// inputs are kept in small LDS ring buffers, so each node's populations and
// temperature are read from HBM once and written once per step:
//
//   A(r)    pull the 9 populations of row r (periodic x; periodic y or
//           wet-node walls), moments, T, psi (float64)        Eqs. lbm, psi
//   wall    Zou-He closure of a wall row once its neighbour row has psi
//   B(r-1)  interaction + adhesion + buoyancy force, Q, velocity, Li
//           source S and correction C, MRT collision, store f*
//                               Eqs. shanchen, S, C, Q, collisionMRT
//   C(r-2)  first RK2 stage of the energy equation -> T*   Eq. energy-equation
//   D(r-3)  second RK2 stage -> T^{n+1}, store
//
// Storage S is double (plain step) or float (populations stored as
// g_i = f_i - w_i rho_ref).  C is the type of the collision and energy
// arithmetic.  EOS, psi, forces and Q are float64 in both.
#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

template <class S>
struct StepArgs {
  const S* fin;
  S* fout;
  const S* Tin;
  S* Tout;
  Tables tab;
  const double* part_in;  // previous step's mass partials (known-part densities)
  int npart_in;
  const double* wall_in;  // this step's wall-closure mass corrections
  int nwall_in;
  double* part_out;
  uint32_t* err;
  int nx, ny, pitch;
  long long plane;
  int ty, ntx, nty;
  int halo;  // recomputed columns per side: 3, or 4 with walls (the wall
             // closure reads psi of the neighbour row at x +- 1)
  int walls, update_T, side_dir, want_mass, xcd_remap;
  Phys ph;
  // read-out mode
  double* o_rho;
  double* o_ux;
  double* o_uy;
  double* o_T;
  double* o_f;
  int f_first, f_count;
};

enum { MODE_STEP = 0, MODE_MACRO = 1 };

// tile index for block id: keep runs of consecutive tiles on one XCD
// (workgroups are dispatched round-robin over the 8 XCDs)
__device__ __forceinline__ int tile_of_block(int bid, int nb, int remap) {
  if (!remap || nb < 16) return bid;
  const int q = nb / 8, rem = nb % 8;
  const int xcd = bid % 8, k = bid / 8;
  // XCD j owns tiles [start_j, start_j + q + (j < rem)) in order
  const int start = xcd * q + (xcd < rem ? xcd : rem);
  return start + k;
}

template <class C>
struct Nb9 {  // 3x3 neighbourhood, [dy+1][dx+1]
  C v[3][3];
};

// energy right-hand side K(phi) of Eq. energy-equation at one node, with
// grad / laplacian of the isotropic D2Q9 stencils:
//   grad f = sum W_i f(x + c_i) c_i,  lap f = 6 sum w_i (f(x + c_i) - f(x))
template <class C>
__device__ __forceinline__ C lap9(const C (&f)[3][3]) {
  const C c = f[1][1];
  const C ax = (f[1][2] - c) + (f[2][1] - c) + (f[1][0] - c) + (f[0][1] - c);
  const C dg = (f[2][2] - c) + (f[2][0] - c) + (f[0][0] - c) + (f[0][2] - c);
  return C(6.0) * (ax * C(1.0 / 9.0) + dg * C(1.0 / 36.0));
}
template <class C>
__device__ __forceinline__ C gradx9(const C (&f)[3][3]) {
  return (f[1][2] - f[1][0]) * C(1.0 / 3.0) + (f[2][2] - f[2][0] - f[0][0] + f[0][2]) * C(1.0 / 12.0);
}
template <class C>
__device__ __forceinline__ C grady9(const C (&f)[3][3]) {
  return (f[2][1] - f[0][1]) * C(1.0 / 3.0) + (f[2][2] + f[2][0] - f[0][0] - f[0][2]) * C(1.0 / 12.0);
}

// the phi-independent part of K at one node, computed once in stage C and
// reused by stage D of the same row
template <class C>
struct EnergyCoef {
  C ux, uy, divu, glx, gly, lam_rcv, inv_rcv;
  double rho;
};

template <class C>
__device__ __forceinline__ C energy_rhs(const C (&phi)[3][3], const EnergyCoef<C>& e, const Phys& p) {
  const C gx = gradx9(phi), gy = grady9(phi);
  const C lp = lap9(phi);
  const C T0 = phi[1][1];
  const C dpdt = C(dp_dT(e.rho, double(T0), p));
  return -(e.ux * gx + e.uy * gy) + e.lam_rcv * lp + (e.glx * gx + e.gly * gy) * e.inv_rcv -
         T0 * dpdt * e.divu * e.inv_rcv;
}

template <class S, class C, int MODE>
__global__ __launch_bounds__(kLanes) void lbm_march_kernel(StepArgs<S> A) {
  const int lane = threadIdx.x;
  const int nb = A.ntx * A.nty;
  const int tile = tile_of_block(blockIdx.x, nb, A.xcd_remap);
  const int tx = tile % A.ntx, tyi = tile / A.ntx;
  const int nx = A.nx, ny = A.ny;
  const int halo = A.halo;
  const int x0 = tx * (kLanes - 2 * halo);
  const int y0 = tyi * A.ty;
  const int y1 = min(y0 + A.ty, ny);
  const int xl = x0 - halo + lane;
  const int x = pmod(xl, nx);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const bool outlane = lane >= halo && lane < kLanes - halo && xl < nx;
  const int lm = lane > 0 ? lane - 1 : 0;
  const int lp = lane < kLanes - 1 ? lane + 1 : kLanes - 1;
  const Phys& P = A.ph;
  const double rref = P.rho_ref;
  const long long pl = A.plane;
  const int pitch = A.pitch;
  const bool walls = A.walls != 0;

  __shared__ double s_rho[4][kLanes];
  __shared__ double s_psi[3][kLanes];
  __shared__ C s_T[4][kLanes];
  __shared__ C s_ux[3][kLanes];
  __shared__ C s_uy[3][kLanes];
  __shared__ C s_Ts[3][kLanes];

  // mean density of the previous state (Eq. gravitational_force): the
  // partial sums are summed in the same order by every workgroup
  double rho_bar = 0.0;
  if (P.gy != 0.0) {
    double s = 0.0;
    for (int i = lane; i < A.npart_in; i += kLanes) s += A.part_in[i];
    for (int i = lane; i < A.nwall_in; i += kLanes) s += A.wall_in[i];
    rho_bar = wave_sum(s) / (double(nx) * double(ny));
  }

  uint32_t err = 0;
  double mass_acc = 0.0;
  C gp[9];  // pulled populations of row r-1 (kept for its collision)
#pragma unroll
  for (int i = 0; i < 9; ++i) gp[i] = C(0);
  C jxp = C(0), jyp = C(0);
  double psiw_b = 0.0, psiw_t = 0.0;
  EnergyCoef<C> ec_prev{};  // stage C coefficients of row r-3 (for D)

  const int nit = (y1 - y0) + 6;
  for (int k = 0; k < nit; ++k) {
    const int r = y0 - kHaloY + k;
    // --------------------------------------------------------- stage A(r)
    C g[9];
    C jx = C(0), jy = C(0);
    {
      const bool have = walls ? (r >= 0 && r < ny) : true;
      if (have) {
        const int yr = walls ? r : pmod(r, ny);
        int ydn, yup;  // source rows of populations moving up / down
        bool kdn = true, kup = true;
        if (walls) {
          // rows outside the walls do not exist: clamp the address, drop the value
          kdn = yr >= 1;
          kup = yr + 1 < ny;
          ydn = kdn ? yr - 1 : yr;
          yup = kup ? yr + 1 : yr;
        } else {
          ydn = (yr == 0) ? ny - 1 : yr - 1;
          yup = (yr == ny - 1) ? 0 : yr + 1;
        }
        const S* f = A.fin;
        const long long rc = (long long)yr * pitch, rd = (long long)ydn * pitch,
                        ru = (long long)yup * pitch;
        g[0] = C(f[0 * pl + rc + x]);
        g[1] = C(f[1 * pl + rc + xm]);
        g[3] = C(f[3 * pl + rc + xp]);
        g[2] = kdn ? C(f[2 * pl + rd + x]) : C(0);
        g[5] = kdn ? C(f[5 * pl + rd + xm]) : C(0);
        g[6] = kdn ? C(f[6 * pl + rd + xp]) : C(0);
        g[4] = kup ? C(f[4 * pl + ru + x]) : C(0);
        g[7] = kup ? C(f[7 * pl + ru + xp]) : C(0);
        g[8] = kup ? C(f[8 * pl + ru + xm]) : C(0);
        const double T = double(A.Tin[rc + x]);
        double rho, psi = 0.0;
        if (walls && (yr == 0 || yr == ny - 1)) {
          // known part of the wall density; closed once psi of the
          // neighbour row exists
          const C gk = (yr == 0) ? g[0] + g[1] + g[3] + C(2) * (g[4] + g[7] + g[8])
                                 : g[0] + g[1] + g[3] + C(2) * (g[2] + g[5] + g[6]);
          rho = rref + double(gk);
        } else {
          C sg = g[0];
#pragma unroll
          for (int i = 1; i < 9; ++i) sg += g[i];
          jx = g[1] - g[3] + g[5] - g[6] - g[7] + g[8];
          jy = g[2] - g[4] + g[5] + g[6] - g[7] - g[8];
          rho = rref + double(sg);
          psi = psi_checked(rho, T, P, err);
        }
        s_rho[k & 3][lane] = rho;
        s_psi[k % 3][lane] = psi;
        s_T[k & 3][lane] = C(T);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = C(0);
      }
    }
    __syncthreads();

    // ------------------------------------------------------ wall closures
    if (walls) {
      const bool cb = (r == 1) && (0 >= y0 - kHaloY);
      const bool ct = (r == ny - 1) && (ny - 2 >= y0 - kHaloY);
      if (cb || ct) {
        const int wrow = cb ? 0 : ny - 1, arow = cb ? 1 : ny - 2;
        const int kw = wrow - (y0 - kHaloY), ka = arow - (y0 - kHaloY);
        const double sgn = cb ? 1.0 : -1.0;
        const double K = s_rho[kw & 3][lane];
        const double Tw = double(s_T[kw & 3][lane]);
        const double rw = cb ? A.tab.rho_w_b[x] : A.tab.rho_w_t[x];
        const double psiw = psi_checked(rw, Tw, P, err);
        const double B = wall_coef_B(s_psi[ka % 3][lane], s_psi[ka % 3][lp], s_psi[ka % 3][lm],
                                     psiw, sgn, P);
        const double rwall = wall_density(K, B, Tw, sgn, P);
        s_rho[kw & 3][lane] = rwall;
        s_psi[kw % 3][lane] = psi_checked(rwall, Tw, P, err);
        if (cb) psiw_b = psiw; else psiw_t = psiw;
      }
      if (cb || ct) __syncthreads();
    }

    // ------------------------------------------------------- stage B(r-1)
    if (k >= 2) {
      const int s = r - 1;
      const bool have = walls ? (s >= 0 && s < ny) : true;
      if (have) {
        const int ys = walls ? s : pmod(s, ny);
        const int km = k - 2, kc = k - 1, kq = k;  // ring rows s-1, s, s+1
        const bool wb = walls && ys == 0, wt = walls && ys == ny - 1;
        const double pc = s_psi[kc % 3][lane];
        const double p1 = s_psi[kc % 3][lp], p3 = s_psi[kc % 3][lm];
        double p2, p5, p6, p4, p7, p8;
        if (wt) {
          p2 = p5 = p6 = psiw_t;
        } else {
          p2 = s_psi[kq % 3][lane];
          p5 = s_psi[kq % 3][lp];
          p6 = s_psi[kq % 3][lm];
        }
        if (wb) {
          p4 = p7 = p8 = psiw_b;
        } else {
          p4 = s_psi[km % 3][lane];
          p7 = s_psi[km % 3][lm];
          p8 = s_psi[km % 3][lp];
        }
        const double rho = s_rho[kc & 3][lane];
        const double G = P.G;
        // Eq. shanchen (with psi_w for solid neighbours, Eq. shanchen-walls)
        const double sx = (1.0 / 3.0) * p1 - (1.0 / 3.0) * p3 +
                          (1.0 / 12.0) * p5 - (1.0 / 12.0) * p6 - (1.0 / 12.0) * p7 + (1.0 / 12.0) * p8;
        const double sy = (1.0 / 3.0) * p2 - (1.0 / 3.0) * p4 +
                          (1.0 / 12.0) * p5 + (1.0 / 12.0) * p6 - (1.0 / 12.0) * p7 - (1.0 / 12.0) * p8;
        const double fmx = -G * pc * sx;
        const double fmy = -G * pc * sy;
        const double fx = fmx;
        const double fy = fmy + P.gy * (rho - rho_bar);
        // Eq. Q / Q-psi-based
        const double kq2 = P.kappa * G * 0.5 * pc;
        const double d1 = p1 - pc, d2 = p2 - pc, d3 = p3 - pc, d4 = p4 - pc;
        const double d5 = p5 - pc, d6 = p6 - pc, d7 = p7 - pc, d8 = p8 - pc;
        const double dsum = d5 + d6 + d7 + d8;
        const double qxx = kq2 * ((1.0 / 3.0) * (d1 + d3) + (1.0 / 12.0) * dsum);
        const double qyy = kq2 * ((1.0 / 3.0) * (d2 + d4) + (1.0 / 12.0) * dsum);
        const double qxy = kq2 * ((1.0 / 12.0) * (d5 - d6 + d7 - d8));

        C jxs = jxp, jys = jyp;
        if (wb || wt) {
          // Zou-He reconstruction for the prescribed momentum -F^m/2
          jxs = C(-0.5 * fmx);
          jys = C(-0.5 * fmy);
          if (wb) {
            const C d = C(0.5) * (gp[1] - gp[3]);
            gp[2] = gp[4] + C(2.0 / 3.0) * jys;
            gp[5] = gp[7] - d + C(0.5) * jxs + jys * C(1.0 / 6.0);
            gp[6] = gp[8] + d - C(0.5) * jxs + jys * C(1.0 / 6.0);
          } else {
            const C d = C(0.5) * (gp[1] - gp[3]);
            gp[4] = gp[2] - C(2.0 / 3.0) * jys;
            gp[7] = gp[5] + d - C(0.5) * jxs - jys * C(1.0 / 6.0);
            gp[8] = gp[6] - d + C(0.5) * jxs - jys * C(1.0 / 6.0);
          }
        }
        const double inv_rho = 1.0 / rho;
        const double uxd = (double(jxs) + 0.5 * fx) * inv_rho;
        const double uyd = (double(jys) + 0.5 * fy) * inv_rho;
        s_ux[kc % 3][lane] = C(uxd);
        s_uy[kc % 3][lane] = C(uyd);

        const bool inseg = s >= y0 && s < y1 && outlane;
        if (MODE == MODE_STEP && inseg) {
          // ---- MRT collision in shifted moments n = M g (g = f - w rho_ref)
          const C ux = C(uxd), uy = C(uyd), Fx = C(fx), Fy = C(fy), rc = C(rho);
          const C sg = C(rho - rref);
          const C a4 = gp[1] + gp[2] + gp[3] + gp[4];
          const C d4s = gp[5] + gp[6] + gp[7] + gp[8];
          const C n1 = C(-4) * gp[0] - a4 + C(2) * d4s;
          const C n2 = C(4) * gp[0] - C(2) * a4 + d4s;
          const C n4 = C(-2) * gp[1] + C(2) * gp[3] + gp[5] - gp[6] - gp[7] + gp[8];
          const C n6 = C(-2) * gp[2] + C(2) * gp[4] + gp[5] + gp[6] - gp[7] - gp[8];
          const C n7 = gp[1] - gp[2] + gp[3] - gp[4];
          const C n8 = gp[5] - gp[6] + gp[7] - gp[8];
          const C u2 = ux * ux + uy * uy;
          const C uF = ux * Fx + uy * Fy;
          const double fm2 = fmx * fmx + fmy * fmy;
          const double ps2 = pc * pc;
          const C te = C(P.sig_e * fm2 / ps2), tz = C(P.sig_z * fm2 / ps2);
          const double snud = 1.0 / (3.0 * ((rho - P.rho_v) * P.eta_l + (P.rho_l - rho) * P.eta_v) *
                                         P.inv_drho + 0.5);
          const C snu = C(snud);
          const C se = C(P.s_e), sz = C(P.s_z), sq = C(P.s_q);
          const C qs = C(qxx + qyy), qd = C(qxx - qyy);
          const C m0 = sg;
          const C m1 = n1 - se * (n1 + C(2) * sg - C(3) * rc * u2) + (C(1) - se * C(0.5)) * (C(6) * uF + te) +
                       C(1.5) * se * qs;
          const C m2 = n2 - sz * (n2 - sg + C(3) * rc * u2) + (C(1) - sz * C(0.5)) * (C(-6) * uF - tz) -
                       C(1.5) * sz * qs;
          const C m3 = jxs + Fx;
          const C m4 = n4 - sq * (n4 + rc * ux) - (C(1) - sq * C(0.5)) * Fx;
          const C m5 = jys + Fy;
          const C m6 = n6 - sq * (n6 + rc * uy) - (C(1) - sq * C(0.5)) * Fy;
          const C m7 = n7 - snu * (n7 - rc * (ux * ux - uy * uy)) +
                       (C(1) - snu * C(0.5)) * C(2) * (ux * Fx - uy * Fy) - snu * qd;
          const C m8 = n8 - snu * (n8 - rc * ux * uy) + (C(1) - snu * C(0.5)) * (ux * Fy + uy * Fx) -
                       snu * C(qxy);
          // f* = M^-1 m*
          const C a0 = m0 * C(1.0 / 9.0);
          const C b1 = m1 * C(1.0 / 36.0), b2 = m2 * C(1.0 / 18.0);
          const C e1 = m1 * C(1.0 / 18.0), e2 = m2 * C(1.0 / 36.0);
          const C j3 = m3 * C(1.0 / 6.0), j5 = m5 * C(1.0 / 6.0);
          const C q4 = m4 * C(1.0 / 6.0), q6 = m6 * C(1.0 / 6.0);
          const C q4h = m4 * C(1.0 / 12.0), q6h = m6 * C(1.0 / 12.0);
          const C p7 = m7 * C(0.25), p8 = m8 * C(0.25);
          const C ax0 = a0 - b1 - b2;
          const C dg0 = a0 + e1 + e2;
          C o[9];
          o[0] = a0 - m1 * C(1.0 / 9.0) + m2 * C(1.0 / 9.0);
          o[1] = ax0 + j3 - q4 + p7;
          o[2] = ax0 + j5 - q6 - p7;
          o[3] = ax0 - j3 + q4 + p7;
          o[4] = ax0 - j5 + q6 - p7;
          o[5] = dg0 + j3 + j5 + q4h + q6h + p8;
          o[6] = dg0 - j3 + j5 - q4h + q6h - p8;
          o[7] = dg0 - j3 - j5 - q4h - q6h + p8;
          o[8] = dg0 + j3 - j5 + q4h - q6h - p8;
          const long long base = (long long)ys * pitch + x;
#pragma unroll
          for (int i = 0; i < 9; ++i) A.fout[i * pl + base] = S(o[i]);
          if (A.want_mass) {
            // known-part density of the next step, summed (walls: the
            // populations leaving through a wall are replaced by those the
            // closure will rebuild from the neighbour row)
            double m = rref;
#pragma unroll
            for (int i = 0; i < 9; ++i) m += double(S(o[i]));
            if (walls) {
              const double dn = double(S(o[4])) + double(S(o[7])) + double(S(o[8])) + rref / 6.0;
              const double up = double(S(o[2])) + double(S(o[5])) + double(S(o[6])) + rref / 6.0;
              if (ys == 0) m -= dn;
              if (ys == 1) m += dn;
              if (ys == ny - 2) m += up;
              if (ys == ny - 1) m -= up;
            }
            mass_acc += m;
          }
        }
        if (MODE == MODE_MACRO && inseg) {
          const long long id = (long long)ys * nx + x;
          if (A.o_rho) A.o_rho[id] = rho;
          if (A.o_ux) A.o_ux[id] = uxd;
          if (A.o_uy) A.o_uy[id] = uyd;
          if (A.o_T) A.o_T[id] = double(s_T[kc & 3][lane]);
          if (A.o_f) {
            const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
            const long long N = (long long)nx * ny;
            for (int i = A.f_first; i < A.f_first + A.f_count; ++i)
              A.o_f[(long long)(i - A.f_first) * N + id] = double(gp[i]) + w[i] * rref;
          }
        }
      }
    }
    // carry row r's populations to the next iteration
#pragma unroll
    for (int i = 0; i < 9; ++i) gp[i] = g[i];
    jxp = jx;
    jyp = jy;
    __syncthreads();

    if (MODE == MODE_STEP && A.update_T) {
      EnergyCoef<C> ec_new{};
      // --------------------------------------------------- stage C(r-2)
      if (k >= 4) {
        const int c = r - 2;
        const bool have = walls ? (c >= 0 && c < ny) : true;
        if (have) {
          const int yc = walls ? c : pmod(c, ny);
          double tval;
          const int kind = t_kind(yc, x, nx, ny, A.side_dir, A.tab, tval, P);
          const int km = k - 3, kc = k - 2, kq = k - 1;
          C Ts;
          EnergyCoef<C> ec{};
          if (kind == T_FREE) {
            const int kr[3] = {km, kc, kq};
            C phi[3][3], rr[3][3], uxn[3][3], uyn[3][3];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
              const int s4 = kr[dy] & 3, s3 = kr[dy] % 3;
              phi[dy][0] = s_T[s4][lm];
              phi[dy][1] = s_T[s4][lane];
              phi[dy][2] = s_T[s4][lp];
              rr[dy][0] = C(s_rho[s4][lm]);
              rr[dy][1] = C(s_rho[s4][lane]);
              rr[dy][2] = C(s_rho[s4][lp]);
              uxn[dy][0] = s_ux[s3][lm];
              uxn[dy][1] = s_ux[s3][lane];
              uxn[dy][2] = s_ux[s3][lp];
              uyn[dy][0] = s_uy[s3][lm];
              uyn[dy][1] = s_uy[s3][lane];
              uyn[dy][2] = s_uy[s3][lp];
            }
            const double rho0 = s_rho[kc & 3][lane];
            const C dl = C(P.dlam);
            const double lam0 = (P.lambda_l * (rho0 - P.rho_v) + P.lambda_v * (P.rho_l - rho0)) * P.inv_drho;
            const C inv_rcv = C(1.0 / (rho0 * P.cv));
            ec.ux = uxn[1][1];
            ec.uy = uyn[1][1];
            ec.divu = gradx9(uxn) + grady9(uyn);
            ec.glx = dl * gradx9(rr);
            ec.gly = dl * grady9(rr);
            ec.lam_rcv = C(lam0) * inv_rcv;
            ec.inv_rcv = inv_rcv;
            ec.rho = rho0;
            Ts = phi[1][1] + C(0.5) * energy_rhs(phi, ec, P);
          } else {
            Ts = C(tval);  // ADIABATIC rows are substituted by the reader
          }
          s_Ts[kc % 3][lane] = Ts;
          ec_new = ec;
        }
      }
      __syncthreads();
      // --------------------------------------------------- stage D(r-3)
      if (k >= 6) {
        const int d = r - 3;
        if (d >= y0 && d < y1) {
          const int yd = d;  // inside [0, ny)
          double tval;
          const int kind = t_kind(yd, x, nx, ny, A.side_dir, A.tab, tval, P);
          const int km = k - 4, kc = k - 3, kq = k - 2;
          const long long base = (long long)yd * pitch + x;
          if (kind == T_FREE) {
            const int kr[3] = {km, kc, kq};
            const int yrow[3] = {walls ? yd - 1 : pmod(yd - 1, ny), yd, walls ? yd + 1 : pmod(yd + 1, ny)};
            C phi[3][3];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
              const int s3 = kr[dy] % 3;
              phi[dy][0] = s_Ts[s3][lm];
              phi[dy][1] = s_Ts[s3][lane];
              phi[dy][2] = s_Ts[s3][lp];
            }
            // adiabatic wall rows take the stage value of their neighbour row
            if (yrow[0] == 0 && yd == 1) {
              const int xs[3] = {xm, x, xp};
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                double tv;
                if (t_kind(0, xs[j], nx, ny, A.side_dir, A.tab, tv, P) == T_ADIABATIC) phi[0][j] = phi[1][j];
              }
            }
            if (yrow[2] == ny - 1 && yd == ny - 2) {
              const int xs[3] = {xm, x, xp};
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                double tv;
                if (t_kind(ny - 1, xs[j], nx, ny, A.side_dir, A.tab, tv, P) == T_ADIABATIC)
                  phi[2][j] = phi[1][j];
              }
            }
            const C T0 = s_T[kc & 3][lane];
            const C Tn = T0 + energy_rhs(phi, ec_prev, P);
            if (outlane) {
              A.Tout[base] = S(Tn);
              double tv;
              if (yd == 1 && t_kind(0, x, nx, ny, A.side_dir, A.tab, tv, P) == T_ADIABATIC)
                A.Tout[x] = S(Tn);
              if (yd == ny - 2 && t_kind(ny - 1, x, nx, ny, A.side_dir, A.tab, tv, P) == T_ADIABATIC)
                A.Tout[(long long)(ny - 1) * pitch + x] = S(Tn);
            }
          } else if (kind == T_DIRICHLET) {
            if (outlane) A.Tout[base] = S(tval);
          }
        }
      }
      ec_prev = ec_new;  // row r-2 is stage D's row of the next iteration
      __syncthreads();
    }
  }

  if (MODE == MODE_STEP && A.want_mass) {
    const double tot = wave_sum(mass_acc);
    if (lane == 0) A.part_out[blockIdx.x] = tot;
  }
  const unsigned long long any = __ballot(err != 0);
  if (any) {
    uint32_t e = err;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e |= __shfl_xor(e, off, kLanes);
    if (lane == 0) atomicOr(A.err, e);
  }
}

// ---------------------------------------------------------------------
// initial state: f*_i(y, x) = f_i^eq(rho, u) at (y + c_iy, x + c_ix) so that
// the first pull yields f^eq at every node; T with the Dirichlet values;
// mass partials of the known-part densities for the first step's rho_bar.
// ---------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void lbm_init_kernel(InitArgs<S> A) {
  const long long N = (long long)A.nx * A.ny;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (id < N) {
    const int y = int(id / A.nx), x = int(id % A.nx);
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    double o[9];
    for (int i = 0; i < 9; ++i) {
      int ys = y + cy[i];
      int xs = pmod(x + cx[i], A.nx);
      if (A.walls) {
        if (ys < 0 || ys >= A.ny) ys = y;  // leaves the domain: never pulled
      } else {
        ys = pmod(ys, A.ny);
      }
      const long long j = (long long)ys * A.nx + xs;
      const double rho = A.rho[j], ux = A.ux ? A.ux[j] : 0.0, uy = A.uy ? A.uy[j] : 0.0;
      const double cu = cx[i] * ux + cy[i] * uy;
      const double feq = w[i] * (rho + 3.0 * rho * cu + 4.5 * rho * cu * cu - 1.5 * rho * (ux * ux + uy * uy));
      o[i] = feq - w[i] * A.rho_ref;
      A.f[i * A.plane + (long long)y * A.pitch + x] = S(o[i]);
    }
    double T = A.T[id];
    if (A.thermal) {
      double tv;
      const int kind = t_kind(y, x, A.nx, A.ny, A.side_dir, A.tab, tv, A.ph);
      if (kind == T_DIRICHLET) T = tv;
    }
    A.Tout[(long long)y * A.pitch + x] = S(T);
    // known-part density mass of the first step (same rule as the step kernel)
    m = A.rho_ref;
    for (int i = 0; i < 9; ++i) m += double(S(o[i]));
    if (A.walls) {
      const double dn = double(S(o[4])) + double(S(o[7])) + double(S(o[8])) + A.rho_ref / 6.0;
      const double up = double(S(o[2])) + double(S(o[5])) + double(S(o[6])) + A.rho_ref / 6.0;
      if (y == 0) m -= dn;
      if (y == 1) m += dn;
      if (y == A.ny - 2) m += up;
      if (y == A.ny - 1) m -= up;
    }
  }
  // block partial in fixed order
  __shared__ double red[256 / kLanes];
  const double ws = wave_sum(m);
  if ((threadIdx.x & (kLanes - 1)) == 0) red[threadIdx.x / kLanes] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < int(blockDim.x / kLanes); ++i) t += red[i];
    A.part_out[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------
// wall-closure mass corrections of the coming step: sum over both walls of
// (closed wall density - known part), needed by rho_bar before the step.
// One lane per wall node; same arithmetic as the closure in the step kernel.
// ---------------------------------------------------------------------
template <class S, class C>
__device__ __forceinline__ double pulled_density(const S* f, long long pl, int pitch, int nx, int ny,
                                                 int y, int x, double rref) {
  // interior node: all 9 sources exist
  const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  const long long rc = (long long)y * pitch, rd = (long long)(y - 1) * pitch,
                  ru = (long long)(y + 1) * pitch;
  C g[9];
  g[0] = C(f[0 * pl + rc + x]);
  g[1] = C(f[1 * pl + rc + xm]);
  g[3] = C(f[3 * pl + rc + xp]);
  g[2] = C(f[2 * pl + rd + x]);
  g[5] = C(f[5 * pl + rd + xm]);
  g[6] = C(f[6 * pl + rd + xp]);
  g[4] = C(f[4 * pl + ru + x]);
  g[7] = C(f[7 * pl + ru + xp]);
  g[8] = C(f[8 * pl + ru + xm]);
  C sg = g[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) sg += g[i];
  return rref + double(sg);
}

template <class S, class C>
__global__ __launch_bounds__(256) void lbm_wall_mass_kernel(WallArgs<S> A) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  double dm = 0.0;
  uint32_t err = 0;
  if (id < 2 * A.nx) {
    const bool bot = id < A.nx;
    const int x = bot ? id : id - A.nx;
    const int ny = A.ny, nx = A.nx;
    const int wrow = bot ? 0 : ny - 1, arow = bot ? 1 : ny - 2;
    const double sgn = bot ? 1.0 : -1.0;
    const S* f = A.fin;
    const long long pl = A.plane;
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    // known part of the wall density
    const long long rc = (long long)wrow * A.pitch;
    C g0 = C(f[0 * pl + rc + x]), g1 = C(f[1 * pl + rc + xm]), g3 = C(f[3 * pl + rc + xp]);
    C gk;
    if (bot) {
      const long long ru = (long long)1 * A.pitch;
      const C g4 = C(f[4 * pl + ru + x]), g7 = C(f[7 * pl + ru + xp]), g8 = C(f[8 * pl + ru + xm]);
      gk = g0 + g1 + g3 + C(2) * (g4 + g7 + g8);
    } else {
      const long long rd = (long long)(ny - 2) * A.pitch;
      const C g2 = C(f[2 * pl + rd + x]), g5 = C(f[5 * pl + rd + xm]), g6 = C(f[6 * pl + rd + xp]);
      gk = g0 + g1 + g3 + C(2) * (g2 + g5 + g6);
    }
    const double K = A.ph.rho_ref + double(gk);
    const double Tw = double(C(A.Tin[rc + x]));
    const long long ra = (long long)arow * A.pitch;
    double pa[3];
    const int xs[3] = {x, xp, xm};
    for (int j = 0; j < 3; ++j) {
      const double rho = pulled_density<S, C>(f, pl, A.pitch, nx, ny, arow, xs[j], A.ph.rho_ref);
      const double Ta = double(C(A.Tin[ra + xs[j]]));
      pa[j] = psi_checked(rho, Ta, A.ph, err);
    }
    const double rw = bot ? A.tab.rho_w_b[x] : A.tab.rho_w_t[x];
    const double psiw = psi_checked(rw, Tw, A.ph, err);
    const double B = wall_coef_B(pa[0], pa[1], pa[2], psiw, sgn, A.ph);
    dm = wall_density(K, B, Tw, sgn, A.ph) - K;
  }
  __shared__ double red[256 / kLanes];
  const double ws = wave_sum(dm);
  if ((threadIdx.x & (kLanes - 1)) == 0) red[threadIdx.x / kLanes] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < int(blockDim.x / kLanes); ++i) t += red[i];
    A.wall_out[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------
// diagnostics over the read-out fields (float64 arrays on the device)
// partial layout per block: [mass, sum rho^2, max rho, sum T, sum T^2,
//  max T, max |u|, nonfinite, q_bottom]
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void lbm_norms_kernel(NormArgs A) {
  const long long N = (long long)A.nx * A.ny;
  double v[kNormSlots];
  for (int i = 0; i < kNormSlots; ++i) v[i] = 0.0;
  double mx_r = 0.0, mx_T = 0.0, mx_u = 0.0;
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < N;
       id += (long long)gridDim.x * blockDim.x) {
    const double r = A.rho[id], T = A.T[id], ux = A.ux[id], uy = A.uy[id];
    const bool fin = isfinite(r) && isfinite(T) && isfinite(ux) && isfinite(uy);
    if (!fin) {
      v[7] += 1.0;
      continue;
    }
    v[0] += r;
    v[1] += r * r;
    mx_r = fmax(mx_r, fabs(r));
    v[3] += T;
    v[4] += T * T;
    mx_T = fmax(mx_T, fabs(T));
    mx_u = fmax(mx_u, sqrt(ux * ux + uy * uy));
    if (A.walls && id < A.nx) {
      // lambda dT/dy at y = 0, one-sided second order (Eq. pool-heat-flux)
      const int x = int(id);
      const double dT = (-3.0 * T + 4.0 * A.T[A.nx + x] - A.T[2 * A.nx + x]) * 0.5;
      const double lam = (A.lambda_l * (r - A.rho_v) + A.lambda_v * (A.rho_l - r)) / (A.rho_l - A.rho_v);
      v[8] += lam * dT;
    }
  }
  __shared__ double red[256 / kLanes][kNormSlots];
  const int wid = threadIdx.x / kLanes, ln = threadIdx.x & (kLanes - 1);
  v[2] = mx_r;
  v[5] = mx_T;
  v[6] = mx_u;
  for (int i = 0; i < kNormSlots; ++i) {
    const bool isMax = (i == 2 || i == 5 || i == 6);
    const double s = isMax ? wave_max(v[i]) : wave_sum(v[i]);
    if (ln == 0) red[wid][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < kNormSlots) {
    const int i = threadIdx.x;
    const bool isMax = (i == 2 || i == 5 || i == 6);
    double t = red[0][i];
    for (int w = 1; w < int(blockDim.x / kLanes); ++w) t = isMax ? fmax(t, red[w][i]) : t + red[w][i];
    A.part[(long long)blockIdx.x * kNormSlots + i] = t;
  }
}

// ------------------------------------------------------------- launchers
template <class S, class C>
static hipError_t launch_step_t(const LaunchStep& L, hipStream_t st, int mode) {
  StepArgs<S> a{};
  a.fin = static_cast<const S*>(L.fin);
  a.fout = static_cast<S*>(L.fout);
  a.Tin = static_cast<const S*>(L.Tin);
  a.Tout = static_cast<S*>(L.Tout);
  a.tab = L.tab;
  a.part_in = L.part_in;
  a.npart_in = L.npart_in;
  a.wall_in = L.wall_in;
  a.nwall_in = L.nwall_in;
  a.part_out = L.part_out;
  a.err = L.err;
  a.nx = L.nx;
  a.ny = L.ny;
  a.pitch = L.pitch;
  a.plane = L.plane;
  a.ty = L.ty;
  a.halo = L.halo;
  a.ntx = L.ntx;
  a.nty = L.nty;
  a.walls = L.walls;
  a.update_T = L.update_T;
  a.side_dir = L.side_dir;
  a.want_mass = L.want_mass;
  a.xcd_remap = L.xcd_remap;
  a.ph = L.ph;
  a.o_rho = L.o_rho;
  a.o_ux = L.o_ux;
  a.o_uy = L.o_uy;
  a.o_T = L.o_T;
  a.o_f = L.o_f;
  a.f_first = L.f_first;
  a.f_count = L.f_count;
  const dim3 grid(L.ntx * L.nty), block(kLanes);
  if (mode == MODE_STEP)
    hipLaunchKernelGGL((lbm_march_kernel<S, C, MODE_STEP>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((lbm_march_kernel<S, C, MODE_MACRO>), grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_step(const LaunchStep& L, hipStream_t st) {
  return L.fp32 ? launch_step_t<float, float>(L, st, MODE_STEP)
                : launch_step_t<double, double>(L, st, MODE_STEP);
}

hipError_t launch_macro(const LaunchStep& L, hipStream_t st) {
  return L.fp32 ? launch_step_t<float, float>(L, st, MODE_MACRO)
                : launch_step_t<double, double>(L, st, MODE_MACRO);
}

hipError_t launch_init(const LaunchInit& L, hipStream_t st) {
  const long long N = (long long)L.nx * L.ny;
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (L.fp32) {
    InitArgs<float> a{static_cast<float*>(L.f), static_cast<float*>(L.Tout), L.rho, L.ux, L.uy, L.T,
                      L.part_out, L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane, L.walls, L.thermal,
                      L.side_dir, L.ph.rho_ref};
    hipLaunchKernelGGL(lbm_init_kernel<float>, grid, block, 0, st, a);
  } else {
    InitArgs<double> a{static_cast<double*>(L.f), static_cast<double*>(L.Tout), L.rho, L.ux, L.uy, L.T,
                       L.part_out, L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane, L.walls, L.thermal,
                       L.side_dir, L.ph.rho_ref};
    hipLaunchKernelGGL(lbm_init_kernel<double>, grid, block, 0, st, a);
  }
  return hipGetLastError();
}

int init_blocks(int nx, int ny) { return int(((long long)nx * ny + 255) / 256); }
int wall_blocks(int nx) { return (2 * nx + 255) / 256; }

hipError_t launch_wall_mass(const LaunchWall& L, hipStream_t st) {
  const dim3 grid(wall_blocks(L.nx)), block(256);
  if (L.fp32) {
    WallArgs<float> a{static_cast<const float*>(L.fin), static_cast<const float*>(L.Tin), L.wall_out,
                      L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane};
    hipLaunchKernelGGL((lbm_wall_mass_kernel<float, float>), grid, block, 0, st, a);
  } else {
    WallArgs<double> a{static_cast<const double*>(L.fin), static_cast<const double*>(L.Tin), L.wall_out,
                       L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane};
    hipLaunchKernelGGL((lbm_wall_mass_kernel<double, double>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_norms(const NormArgs& a, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(lbm_norms_kernel, dim3(nblocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace lbm
