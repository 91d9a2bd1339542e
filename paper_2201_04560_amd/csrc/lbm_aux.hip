// Auxiliary kernels of the pseudopotential LBM library (gfx950): initial
// state, the wall-closure mass correction needed by the mean density of
// the buoyancy force, and the float64 diagnostic reductions.
#include <cstring>

#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

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
__device__ __forceinline__ void wall_mass_body(const WallArgs<S>& A, const int bid) {
  const int id = bid * blockDim.x + threadIdx.x;
  double dm = 0.0;
  uint32_t err = 0;
  // rho_bar_k of the closure's buoyancy: the step kernel's fixed-order sum
  // of the known-part partials (fixed_order_sum), its eight accumulators
  // spread over the block's four waves (two each, all loads in flight at
  // once) and combined in the same order, so the result is the step
  // kernel's bit for bit (every thread takes part, before the lanes split)
  __shared__ double s_acc[8][kLanes];
  double rbk = 0.0;
  if (A.ph.gy != 0.0) {
    static_assert(256 / kLanes * 2 == 8, "four waves of two accumulators");
    const double* part = A.part_in;
    const int n = A.npart_in;
    const int w = int(threadIdx.x / kLanes), l = int(threadIdx.x & (kLanes - 1));
    double a0 = 0.0, a1 = 0.0;
    int i = l;
    for (; i + 7 * kLanes < n; i += 8 * kLanes) {
      a0 += part[i + 2 * w * kLanes];
      a1 += part[i + (2 * w + 1) * kLanes];
    }
    if (w == 0)
      for (; i < n; i += kLanes) a0 += part[i];  // fewer than 8 left per lane
    s_acc[2 * w][l] = a0;
    s_acc[2 * w + 1][l] = a1;
    __syncthreads();
    const double t = ((s_acc[0][l] + s_acc[1][l]) + (s_acc[2][l] + s_acc[3][l])) +
                     ((s_acc[4][l] + s_acc[5][l]) + (s_acc[6][l] + s_acc[7][l]));
    rbk = wave_sum(t) / (double(A.nx) * double(A.ny));
  }
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
      // same float64 EOS evaluation as stage A of the step kernel
      const double rho = pulled_density<S, C>(f, pl, A.pitch, nx, ny, arow, xs[j], A.ph.rho_ref);
      const double Ta = double(C(A.Tin[ra + xs[j]]));
      pa[j] = psi_fast(rho, Ta, eos_node(rho, Ta, A.ph), A.ph, err);
    }
    const double rw = bot ? A.tab.rho_w_b[x] : A.tab.rho_w_t[x];  // rho_w, or G_w (modified-psi)
    if (A.ph.wall_mod) {
      const double nbsum = pa[0] / 3.0 + (pa[1] + pa[2]) / 12.0;
      dm = wall_density_mod(K, nbsum, rw, Tw, sgn, A.ph, rbk) - K;
    } else {
      const double psiw = psi_checked(rw, Tw, A.ph, err);
      const double B = wall_coef_B(pa[0], pa[1], pa[2], psiw, sgn, A.ph);
      dm = wall_density(K, B, Tw, sgn, A.ph, rbk) - K;
    }
  }
  __shared__ double red[256 / kLanes];
  const double ws = wave_sum(dm);
  if ((threadIdx.x & (kLanes - 1)) == 0) red[threadIdx.x / kLanes] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < int(blockDim.x / kLanes); ++i) t += red[i];
    A.wall_out[bid] = t;
  }
}

template <class S, class C>
__global__ __launch_bounds__(256) void lbm_wall_mass_kernel(WallArgs<S> A) {
  wall_mass_body<S, C>(A, blockIdx.x);
}

// batched version: workgroups [start[g], start[g+1]) serve lattice g
template <class S, class C>
__global__ __launch_bounds__(256) void lbm_wall_mass_multi_kernel(const WallArgs<S>* __restrict__ desc,
                                                                  const int* __restrict__ start,
                                                                  int ngrid) {
  const int b = blockIdx.x;
  int g = 0;
  while (g + 1 < ngrid && b >= start[g + 1]) ++g;
  wall_mass_body<S, C>(desc[g], b - start[g]);
}

// ---------------------------------------------------------------------
// diagnostics over the read-out fields (float64 arrays on the device)
// partial layout per block: [mass, sum rho^2, max rho, sum |T|, sum T^2,
//  max T, max |u|, nonfinite, wall flux over the bottom nodes that are not
//  adiabatic, flux over the held (Dirichlet) bottom nodes, their number,
//  sum |rho|]
// The flux is lambda dT/dy at y = 0 with the one-sided second-order
// difference of Eq. pool-heat-flux; an adiabatic node carries no flux by
// its condition, so it adds nothing to the wall sum.
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
    v[11] += fabs(r);
    mx_r = fmax(mx_r, fabs(r));
    v[3] += fabs(T);
    v[4] += T * T;
    mx_T = fmax(mx_T, fabs(T));
    mx_u = fmax(mx_u, sqrt(ux * ux + uy * uy));
    if (A.walls && id < A.nx) {
      const int x = int(id);
      const int kind = (A.side_dir && (x == 0 || x == A.nx - 1)) ? T_DIRICHLET : A.tk_b[x];
      if (kind != T_ADIABATIC) {
        const double dT = (-3.0 * T + 4.0 * A.T[A.nx + x] - A.T[2 * A.nx + x]) * 0.5;
        const double lam = (A.lambda_l * (r - A.rho_v) + A.lambda_v * (A.rho_l - r)) / (A.rho_l - A.rho_v);
        v[8] += lam * dT;
        if (kind == T_DIRICHLET) {
          v[9] += lam * dT;
          v[10] += 1.0;
        }
      }
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
                      L.part_in, L.npart_in, L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane};
    hipLaunchKernelGGL((lbm_wall_mass_kernel<float, float>), grid, block, 0, st, a);
  } else {
    WallArgs<double> a{static_cast<const double*>(L.fin), static_cast<const double*>(L.Tin), L.wall_out,
                       L.part_in, L.npart_in, L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane};
    hipLaunchKernelGGL((lbm_wall_mass_kernel<double, double>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_norms(const NormArgs& a, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(lbm_norms_kernel, dim3(nblocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t wall_desc_bytes(int fp32) { return fp32 ? sizeof(WallArgs<float>) : sizeof(WallArgs<double>); }

void fill_wall_desc(const LaunchWall& L, void* out) {
  if (L.fp32) {
    WallArgs<float> a{static_cast<const float*>(L.fin), static_cast<const float*>(L.Tin), L.wall_out,
                      L.part_in, L.npart_in, L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane};
    std::memcpy(out, &a, sizeof a);
  } else {
    WallArgs<double> a{static_cast<const double*>(L.fin), static_cast<const double*>(L.Tin), L.wall_out,
                       L.part_in, L.npart_in, L.tab, L.ph, L.nx, L.ny, L.pitch, L.plane};
    std::memcpy(out, &a, sizeof a);
  }
}

hipError_t launch_wall_multi(int fp32, const void* desc, const int* start, int ngrid, int nblocks,
                             hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL((lbm_wall_mass_multi_kernel<float, float>), dim3(nblocks), dim3(256), 0, st,
                       static_cast<const WallArgs<float>*>(desc), start, ngrid);
  else
    hipLaunchKernelGGL((lbm_wall_mass_multi_kernel<double, double>), dim3(nblocks), dim3(256), 0, st,
                       static_cast<const WallArgs<double>*>(desc), start, ngrid);
  return hipGetLastError();
}

}  // namespace lbm
