// Host runtime and C-ABI of the pseudopotential LBM library: parameter
// validation, carving of the caller's device buffer, launch sequencing,
// read-back, diagnostics and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm_pp.h"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
constexpr uint64_t kStateMagic = 0x324D424C50504E42ull;  // "BNPPLBM2"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Small lattices (fewer than 2048 five-row strips) are bound by one wave's
// per-row latency: their energy step runs two waves per strip (the second
// wave takes the RK2 stages) on 5-row strips.
bool small_lattice(int nx, int ny, int walls) {
  const int ntx = (nx + tile_x(walls) - 1) / tile_x(walls);
  return static_cast<long long>(ntx) * ((ny + 4) / 5) < 2048;
}

int default_tile_y(int nx, int ny, int walls, int fp32) {
  // Before the device is known (buffer sizing): the longest strip that still
  // gives every SIMD about two one-wave workgroups (float64: one and a half);
  // lbm_create replaces it by round_tile_y for the device of the buffer.
  if (small_lattice(nx, ny, walls)) return std::max(2, std::min(5, std::max(ny, 2)));
  const int ntx = (nx + tile_x(walls) - 1) / tile_x(walls);
  const int want = fp32 ? 2048 : 1536;
  static const int cand[] = {64, 48, 32, 24, 16, 12, 8, 6, 5};
  int ty = 5;
  for (int c : cand) {
    if (static_cast<long long>(ntx) * ((ny + c - 1) / c) >= want) {
      ty = c;
      break;
    }
  }
  return std::max(2, std::min(ty, std::max(ny, 2)));
}

// Default strip height once the device is known: the smallest height whose
// launch of one-wave workgroups fits in `per_simd` waves on each SIMD (4 per
// compute unit).  A launch a few waves over a whole round leaves some SIMDs
// one wave more than the rest, and they set its time.  3 waves per SIMD for
// float32 storage and 2 for float64 were the measured optima on MI355X (4096^2
// pool: 100 / 152 rows; 1024 x 2048 pool: 13 / 20 rows).
int round_tile_y(int ntx, int ny, int cus, int per_simd) {
  const int hi = std::max(ny, 2);
  const long long strips = static_cast<long long>(per_simd) * 4 * cus / ntx;
  if (strips < 1) return hi;
  return static_cast<int>(std::min<long long>(hi, std::max<long long>(2, (ny + strips - 1) / strips)));
}

int strip_waves(const lbm_ctx* c) {
  int w = (c->p.strip_waves == 1 || c->p.strip_waves == 2)
              ? c->p.strip_waves
              : (small_lattice(c->p.nx, c->p.ny, c->p.walls) ? 2 : 1);
  // the two-wave march needs 9 population planes below 4 GiB and ny >= 3
  if (w == 2 && !two_wave_fits(c->L.plane, c->L.elem, c->p.ny)) w = 1;
  return w;
}

}  // namespace

void lbm::make_layout(const lbm_params& p, Layout& L) {
  L.elem = p.precision == LBM_FP32_SHIFTED ? 4 : 8;
  L.pitch = int(align_up(size_t(p.nx), 64));
  // plane stride: padded off powers of two so that the 9 loads of a node
  // do not all land in one HBM channel
  const long long cells = (long long)L.pitch * p.ny;
  L.plane = (long long)align_up(size_t(cells), 256) + 192;
  L.ty = p.tile_y > 0 ? p.tile_y : default_tile_y(p.nx, p.ny, p.walls, p.precision == LBM_FP32_SHIFTED);
  L.ntx = (p.nx + tile_x(p.walls) - 1) / tile_x(p.walls);
  L.nty = (p.ny + L.ty - 1) / L.ty;
  L.nblocks = L.ntx * L.nty;
  // partial sums for the shortest allowed strips (tile_y = 2): the tile
  // height can be changed after creation
  L.part_cap = std::max(L.ntx * ((p.ny + 1) / 2) + 8, init_blocks(p.nx, p.ny));
  L.wall_cap = wall_blocks(p.nx);
  size_t o = 0;
  const size_t fbytes = align_up(size_t(9 * L.plane) * L.elem, kAlign);
  const size_t tbytes = align_up(size_t(cells) * L.elem, kAlign);
  for (int i = 0; i < 2; ++i) { L.off_f[i] = o; o += fbytes; }
  for (int i = 0; i < 2; ++i) { L.off_T[i] = o; o += tbytes; }
  L.off_tab = o; o += align_up(size_t(4) * p.nx * sizeof(double), kAlign);
  L.off_tk = o; o += align_up(size_t(2) * p.nx * sizeof(int32_t), kAlign);
  for (int i = 0; i < 2; ++i) { L.off_part[i] = o; o += align_up(size_t(L.part_cap) * 8, kAlign); }
  L.off_wall = o; o += align_up(size_t(L.wall_cap) * 8, kAlign);
  L.off_red = o; o += align_up(size_t(kNormBlocks) * kNormSlots * 8, kAlign);
  L.off_err = o; o += kAlign;
  L.total = o;
}

namespace {

Phys make_phys(const lbm_params& p) {
  Phys h{};
  h.a = p.a;
  h.b = p.b;
  h.R = p.R;
  h.G = p.G;
  h.kw = 0.37464 + 1.54226 * p.omega - 0.2699 * p.omega * p.omega;
  h.Tc = 0.0778 * p.a / (0.45724 * p.b * p.R);
  h.inv_Tc = 1.0 / h.Tc;
  h.inv_sqrtTc = 1.0 / std::sqrt(h.Tc);
  h.akw_isTc = p.a * h.kw * h.inv_sqrtTc;
  h.inv_b = 1.0 / p.b;
  h.sigma = p.sigma;
  h.kappa = p.kappa;
  h.s_e = p.s_e;
  h.s_z = p.s_zeta;
  h.s_j = p.s_j;
  h.s_q = p.s_q;
  h.sig_e = 12.0 * p.sigma / (1.0 / p.s_e - 0.5);
  h.sig_z = 12.0 * p.sigma / (1.0 / p.s_zeta - 0.5);
  h.eta_l = p.eta_l;
  h.eta_v = p.eta_v;
  h.rho_l = p.rho_l;
  h.rho_v = p.rho_v;
  h.inv_drho = 1.0 / (p.rho_l - p.rho_v);
  h.gy = p.gy;
  h.cv = p.cv;
  h.lambda_l = p.lambda_l;
  h.lambda_v = p.lambda_v;
  h.dlam = (p.lambda_l - p.lambda_v) / (p.rho_l - p.rho_v);
  h.t_side_val = p.t_side_val;
  h.rho_ref = p.precision == LBM_FP32_SHIFTED ? p.rho_ref : 0.0;
  h.two_G = 2.0 / p.G;  // exact for G = -1: the same bits as dividing 2 (p - rho / 3) by G
  h.wall_mod = p.wall_model == LBM_WALL_MODIFIED_PSI ? 1 : 0;
  h.outflow_top = p.outflow_top ? 1 : 0;
  return h;
}

std::string g_create_error;

}  // namespace

lbm_status lbm::fail(lbm_ctx* c, lbm_status s, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

extern "C" {

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_E_INVAL: return "invalid argument";
    case LBM_E_NOMEM: return "buffer too small or out of memory";
    case LBM_E_HIP: return "HIP runtime error";
    case LBM_E_STATE: return "call out of order";
    case LBM_E_DOMAIN: return "state left the EOS / pseudopotential domain";
    case LBM_E_UNSUPPORTED: return "unsupported";
    default: break;
  }
  return "unknown status";
}

const char* lbm_last_error(const lbm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

void lbm_default_params(lbm_params* p, int32_t nx, int32_t ny) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->precision = LBM_FP64;
  p->a = 2.0 / 49.0;
  p->b = 2.0 / 21.0;
  p->R = 1.0;
  p->omega = 0.344;
  p->G = -1.0;
  p->sigma = 0.1;
  p->kappa = 0.1;
  p->s_rho = p->s_e = p->s_zeta = p->s_j = p->s_q = 1.25;
  p->eta_l = p->eta_v = 0.1;
  p->rho_l = 6.5;
  p->rho_v = 0.38;
  p->cv = 5.0;
  p->lambda_l = p->lambda_v = 2.0 / 3.0;
  p->xcd_remap = 1;
}

lbm_status lbm_validate(const lbm_params* p) {
  if (!p) return fail(nullptr, LBM_E_INVAL, "null params");
  auto bad = [](const char* m) { return fail(nullptr, LBM_E_INVAL, m); };
  if (p->nx < 1 || p->ny < 1) return bad("nx and ny must be >= 1");
  if ((long long)p->nx * p->ny > (1ll << 31)) return bad("grid larger than 2^31 nodes");
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_SHIFTED) return bad("unknown precision");
  if (p->walls && p->ny < 3) return bad("walls need ny >= 3");
  if (!(p->a > 0) || !(p->b > 0) || !(p->R > 0)) return bad("a, b, R must be > 0");
  if (!(p->G < 0)) return bad("G must be negative (psi of Eq. psi)");
  const double rates[] = {p->s_rho, p->s_e, p->s_zeta, p->s_j, p->s_q};
  for (double s : rates)
    if (!(s > 0 && s < 2)) return bad("relaxation rates must lie in (0, 2)");
  if (!(p->eta_l > 0) || !(p->eta_v > 0)) return bad("viscosities must be > 0");
  if (!(p->rho_l != p->rho_v)) return bad("rho_l must differ from rho_v");
  if (p->thermal) {
    if (!(p->cv > 0)) return bad("cv must be > 0");
    if (!(p->lambda_l >= 0) || !(p->lambda_v >= 0)) return bad("conductivities must be >= 0");
  }
  if (p->n_iso < 0) return bad("n_iso must be >= 0");
  if (p->tile_y < 0 || p->tile_y == 1) return bad("tile_y must be 0 or >= 2");
  if (p->strip_waves < 0 || p->strip_waves > 2) return bad("strip_waves must be 0, 1 or 2");
  if (!std::isfinite(p->rho_ref)) return bad("rho_ref must be finite");
  if (p->wall_model != LBM_WALL_PSI_BASED && p->wall_model != LBM_WALL_MODIFIED_PSI)
    return bad("wall_model must be LBM_WALL_PSI_BASED or LBM_WALL_MODIFIED_PSI");
  if (p->outflow_top != 0 && p->outflow_top != 1) return bad("outflow_top must be 0 or 1");
  if (p->outflow_top && !p->walls) return bad("outflow_top needs walls (a wall at the bottom)");
  if (p->outflow_top && p->gy != 0.0)
    return fail(nullptr, LBM_E_UNSUPPORTED, "outflow_top with gravity is not implemented "
                                            "(the mean density would change with the outflow)");
  return LBM_OK;
}

lbm_status lbm_buffer_bytes(const lbm_params* p, size_t* bytes) {
  lbm_status s = lbm_validate(p);
  if (s != LBM_OK) return s;
  if (!bytes) return fail(nullptr, LBM_E_INVAL, "null bytes");
  Layout L;
  make_layout(*p, L);
  *bytes = L.total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                      lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_E_INVAL, "null out");
  *out = nullptr;
  lbm_status s = lbm_validate(p);
  if (s != LBM_OK) return s;
  if (!dev_buf) return fail(nullptr, LBM_E_INVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign)
    return fail(nullptr, LBM_E_INVAL, "device buffer must be 256-byte aligned");
  Layout L;
  make_layout(*p, L);
  if (bytes < L.total)
    return fail(nullptr, LBM_E_NOMEM, "device buffer smaller than lbm_buffer_bytes()");
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
  c->p = *p;
  c->L = L;
  if (p->tile_y <= 0 && !small_lattice(p->nx, p->ny, p->walls)) {
    hipPointerAttribute_t attr;
    int cus = 0;
    if (hipPointerGetAttributes(&attr, dev_buf) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, attr.device) == hipSuccess &&
        cus > 0) {
      c->L.ty = round_tile_y(L.ntx, p->ny, cus, p->precision == LBM_FP32_SHIFTED ? 3 : 2);
      c->L.nty = (p->ny + c->L.ty - 1) / c->L.ty;
      c->L.nblocks = c->L.ntx * c->L.nty;
    } else {
      (void)hipGetLastError();  // keep the device-independent default
    }
  }
  {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev_buf) == hipSuccess) {
      c->device = attr.device;
    } else {
      (void)hipGetLastError();
      if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    }
  }
  c->ph = make_phys(*p);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->base = static_cast<char*>(dev_buf);
  c->bytes = bytes;
  const int nx = p->nx;
  // psi-based: rho_w = 1; modified-psi: G_w = G (a neutral wall)
  c->rw_b.assign(nx, p->wall_model == LBM_WALL_MODIFIED_PSI ? p->G : 1.0);
  c->rw_t.assign(nx, p->wall_model == LBM_WALL_MODIFIED_PSI ? p->G : 1.0);
  c->tv_b.assign(nx, 0.0);
  c->tv_t.assign(nx, 0.0);
  c->tk_b.assign(nx, LBM_T_FREE);
  c->tk_t.assign(nx, LBM_T_FREE);
  hipError_t e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e == hipSuccess) e = hipMemsetAsync(c->errp(), 0, 4, c->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("lbm_create: ") + hipGetErrorString(e);
    lbm_destroy(c);
    return LBM_E_HIP;
  }
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->kev) (void)hipEventDestroy(e);
  delete c;
}

static lbm_status upload_tables(lbm_ctx* c) {
  const int nx = c->p.nx;
  std::vector<double> d(4 * size_t(nx));
  std::copy(c->rw_b.begin(), c->rw_b.end(), d.begin());
  std::copy(c->rw_t.begin(), c->rw_t.end(), d.begin() + nx);
  std::copy(c->tv_b.begin(), c->tv_b.end(), d.begin() + 2 * nx);
  std::copy(c->tv_t.begin(), c->tv_t.end(), d.begin() + 3 * nx);
  std::vector<int32_t> k(2 * size_t(nx));
  std::copy(c->tk_b.begin(), c->tk_b.end(), k.begin());
  std::copy(c->tk_t.begin(), c->tk_t.end(), k.begin() + nx);
  HIP_TRY(c, hipMemcpyAsync(c->tabd(), d.data(), d.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->tabi(), k.data(), k.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_set_boundary(lbm_ctx* c, const double* rho_w_bottom, const double* rho_w_top,
                            const int32_t* t_bottom_kind, const double* t_bottom_val,
                            const int32_t* t_top_kind, const double* t_top_val) {
  if (!c) return LBM_E_INVAL;
  ++c->generation;  // even a rejected call may leave some tables replaced
  const int nx = c->p.nx;
  auto kind_ok = [&](const int32_t* k) {
    if (!k) return true;
    for (int i = 0; i < nx; ++i)
      if (k[i] < LBM_T_FREE || k[i] > LBM_T_ADIABATIC) return false;
    return true;
  };
  if (!kind_ok(t_bottom_kind) || !kind_ok(t_top_kind))
    return fail(c, LBM_E_INVAL, "temperature kind must be FREE, DIRICHLET or ADIABATIC");
  if (c->p.thermal && c->p.walls) {
    for (int i = 0; i < nx; ++i) {
      if ((t_bottom_kind && t_bottom_kind[i] == LBM_T_FREE) || (t_top_kind && t_top_kind[i] == LBM_T_FREE))
        if (!(c->p.t_side_dirichlet && (i == 0 || i == nx - 1)))
          return fail(c, LBM_E_INVAL, "wall rows need DIRICHLET or ADIABATIC temperature");
    }
  }
  if (c->p.ny < 3) {
    for (int i = 0; i < nx; ++i)
      if ((t_bottom_kind && t_bottom_kind[i] == LBM_T_ADIABATIC) ||
          (t_top_kind && t_top_kind[i] == LBM_T_ADIABATIC))
        return fail(c, LBM_E_INVAL, "ADIABATIC rows need ny >= 3");
  }
  for (const double* w : {rho_w_bottom, rho_w_top})
    if (w)
      for (int i = 0; i < nx; ++i)
        if (!std::isfinite(w[i])) return fail(c, LBM_E_INVAL, "wall tables must be finite");
  if (rho_w_bottom) c->rw_b.assign(rho_w_bottom, rho_w_bottom + nx);
  if (rho_w_top) c->rw_t.assign(rho_w_top, rho_w_top + nx);
  if (t_bottom_kind) c->tk_b.assign(t_bottom_kind, t_bottom_kind + nx);
  if (t_top_kind) c->tk_t.assign(t_top_kind, t_top_kind + nx);
  if (t_bottom_val) c->tv_b.assign(t_bottom_val, t_bottom_val + nx);
  if (t_top_val) c->tv_t.assign(t_top_val, t_top_val + nx);
  return upload_tables(c);
}

static lbm_status check_err(lbm_ctx* c) {
  uint32_t e = 0;
  HIP_TRY(c, hipMemcpyAsync(&e, c->errp(), 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (e) {
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  "domain error (flags 0x%x: 1 rho outside (0,1/b), 2 psi radicand <= 0, 4 T <= 0)", e);
    c->err = buf;
    return LBM_E_DOMAIN;
  }
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
                           const double* T) {
  if (!c) return LBM_E_INVAL;
  if (!rho || !T) return fail(c, LBM_E_INVAL, "rho and T are required");
  const int nx = c->p.nx, ny = c->p.ny;
  const size_t N = size_t(nx) * ny;
  lbm_status s = upload_tables(c);
  if (s != LBM_OK) return s;
  // stage the host fields in the second population buffer
  c->cur = 0;
  c->Tcur = 0;
  c->pcur = 0;
  char* stg = static_cast<char*>(c->f(1));
  double* d_rho = reinterpret_cast<double*>(stg);
  double* d_ux = d_rho + N;
  double* d_uy = d_ux + N;
  double* d_T = d_uy + N;
  HIP_TRY(c, hipMemcpyAsync(d_rho, rho, N * 8, hipMemcpyHostToDevice, c->stream));
  if (ux) HIP_TRY(c, hipMemcpyAsync(d_ux, ux, N * 8, hipMemcpyHostToDevice, c->stream));
  if (uy) HIP_TRY(c, hipMemcpyAsync(d_uy, uy, N * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_T, T, N * 8, hipMemcpyHostToDevice, c->stream));
  LaunchInit L{};
  L.fp32 = c->p.precision == LBM_FP32_SHIFTED;
  L.f = c->f(0);
  L.Tout = c->T(0);
  L.rho = d_rho;
  L.ux = ux ? d_ux : nullptr;
  L.uy = uy ? d_uy : nullptr;
  L.T = d_T;
  L.part_out = c->part(0);
  L.tab = c->tables();
  L.ph = c->ph;
  L.nx = nx;
  L.ny = ny;
  L.pitch = c->L.pitch;
  L.plane = c->L.plane;
  L.walls = c->p.walls;
  L.thermal = c->p.thermal;
  L.side_dir = c->p.t_side_dirichlet;
  HIP_TRY(c, hipMemsetAsync(c->errp(), 0, 4, c->stream));
  HIP_TRY(c, launch_init(L, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->npart = init_blocks(nx, ny);
  c->step = 0;
  ++c->generation;
  c->initialized = true;
  return LBM_OK;
}

}  // extern "C"

LaunchStep lbm::step_args(lbm_ctx* c) {
  LaunchStep L{};
  L.fp32 = c->p.precision == LBM_FP32_SHIFTED;
  L.fin = c->f(c->cur);
  L.fout = c->f(1 - c->cur);
  L.Tin = c->T(c->Tcur);
  L.Tout = c->T(1 - c->Tcur);
  L.tab = c->tables();
  L.part_in = c->part(c->pcur);
  L.npart_in = c->npart;
  L.wall_in = c->wall();
  L.nwall_in = 0;
  L.part_out = c->part(1 - c->pcur);
  L.err = c->errp();
  L.nx = c->p.nx;
  L.ny = c->p.ny;
  L.pitch = c->L.pitch;
  L.plane = c->L.plane;
  L.ty = c->L.ty;
  L.halo = halo_x(c->p.walls);
  L.ntx = c->L.ntx;
  L.nty = c->L.nty;
  L.walls = c->p.walls;
  L.side_dir = c->p.t_side_dirichlet;
  L.xcd_remap = c->p.xcd_remap;
  L.waves = strip_waves(c);
  L.ph = c->ph;
  return L;
}


LaunchWall lbm::wall_args(lbm_ctx* c, const LaunchStep& L) {
  LaunchWall W{};
  W.fp32 = L.fp32;
  W.fin = L.fin;
  W.Tin = L.Tin;
  W.wall_out = c->wall();
  W.part_in = L.part_in;
  W.npart_in = L.npart_in;
  W.tab = L.tab;
  W.ph = c->ph;
  W.nx = c->p.nx;
  W.ny = c->p.ny;
  W.pitch = c->L.pitch;
  W.plane = c->L.plane;
  return W;
}

extern "C" {

lbm_status lbm_set_tile_y(lbm_ctx* c, int32_t tile_y) {
  if (!c) return LBM_E_INVAL;
  if (tile_y < 2) return fail(c, LBM_E_INVAL, "tile_y must be >= 2");
  const int nty = (c->p.ny + tile_y - 1) / tile_y;
  if (c->L.ntx * nty + 8 > c->L.part_cap) return fail(c, LBM_E_INVAL, "tile_y too small for the buffer");
  c->L.ty = tile_y;
  c->L.nty = nty;
  c->L.nblocks = c->L.ntx * nty;
  return LBM_OK;
}

int32_t lbm_get_tile_y(const lbm_ctx* c) { return c ? c->L.ty : -1; }

lbm_status lbm_set_strip_waves(lbm_ctx* c, int32_t waves) {
  if (!c) return LBM_E_INVAL;
  if (waves < 0 || waves > 2) return fail(c, LBM_E_INVAL, "strip_waves must be 0, 1 or 2");
  c->p.strip_waves = waves;
  return LBM_OK;
}

int32_t lbm_get_strip_waves(const lbm_ctx* c) { return c ? strip_waves(c) : -1; }

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) return LBM_E_INVAL;
  if (!c->initialized) return fail(c, LBM_E_STATE, "lbm_step before lbm_init_fields");
  if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps must be >= 0");
  const bool grav = c->ph.gy != 0.0;
  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  for (int64_t n = 0; n < nsteps; ++n) {
    LaunchStep L = step_args(c);
    L.update_T = c->p.thermal && c->step >= c->p.n_iso;
    L.want_mass = grav;
    if (grav && c->p.walls) {
      HIP_TRY(c, launch_wall_mass(wall_args(c, L), c->stream));
      L.nwall_in = wall_blocks(c->p.nx);
    }
    if (c->ktime) {
      if (c->kused + 2 > c->kev.size()) {
        for (int j = 0; j < 2; ++j) {
          hipEvent_t e;
          HIP_TRY(c, hipEventCreate(&e));
          c->kev.push_back(e);
        }
      }
      HIP_TRY(c, hipEventRecord(c->kev[c->kused], c->stream));
    }
    HIP_TRY(c, launch_step(L, c->stream));
    if (c->ktime) {
      HIP_TRY(c, hipEventRecord(c->kev[c->kused + 1], c->stream));
      c->kused += 2;
    }
    c->cur ^= 1;
    if (L.update_T) c->Tcur ^= 1;
    if (grav) {
      c->pcur ^= 1;
      c->npart = c->L.nblocks;
    }
    ++c->step;
    ++c->generation;
  }
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  c->timed = true;
  return LBM_OK;
}

lbm_status lbm_kernel_timing(lbm_ctx* c, int32_t enable) {
  if (!c) return LBM_E_INVAL;
  c->ktime = enable != 0;
  c->kused = 0;
  return LBM_OK;
}

lbm_status lbm_kernel_times(lbm_ctx* c, double* sum_ms, int64_t* count) {
  if (!c || !sum_ms || !count) return LBM_E_INVAL;
  double s = 0.0;
  for (size_t i = 0; i + 1 < c->kused; i += 2) {
    HIP_TRY(c, hipEventSynchronize(c->kev[i + 1]));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->kev[i], c->kev[i + 1]));
    s += ms;
  }
  *sum_ms = s;
  *count = int64_t(c->kused / 2);
  c->kused = 0;
  return LBM_OK;
}

lbm_status lbm_last_step_time(lbm_ctx* c, double* total_ms) {
  if (!c || !total_ms) return LBM_E_INVAL;
  if (!c->timed) return fail(c, LBM_E_STATE, "no lbm_step call yet");
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  *total_ms = ms;
  return LBM_OK;
}

}  // extern "C"

// read-out kernel into the idle population buffer
lbm_status lbm::run_macro(lbm_ctx* c, double* o_rho, double* o_ux, double* o_uy, double* o_T,
                          double* o_f, int f_first, int f_count) {
  LaunchStep L = step_args(c);
  L.fout = nullptr;
  L.Tout = nullptr;
  L.update_T = 0;
  L.want_mass = 0;
  L.o_rho = o_rho;
  L.o_ux = o_ux;
  L.o_uy = o_uy;
  L.o_T = o_T;
  L.o_f = o_f;
  L.f_first = f_first;
  L.f_count = f_count;
  if (c->ph.gy != 0.0 && c->p.walls) {
    HIP_TRY(c, launch_wall_mass(wall_args(c, L), c->stream));
    L.nwall_in = wall_blocks(c->p.nx);
  }
  HIP_TRY(c, launch_macro(L, c->stream));
  return LBM_OK;
}

extern "C" {

lbm_status lbm_read_fields(lbm_ctx* c, double* rho, double* ux, double* uy, double* T) {
  if (!c) return LBM_E_INVAL;
  if (!c->initialized) return fail(c, LBM_E_STATE, "read before init");
  const size_t N = size_t(c->p.nx) * c->p.ny;
  double* stg = static_cast<double*>(c->f(1 - c->cur));
  lbm_status s = run_macro(c, stg, stg + N, stg + 2 * N, stg + 3 * N, nullptr, 0, 0);
  if (s != LBM_OK) return s;
  if (rho) HIP_TRY(c, hipMemcpyAsync(rho, stg, N * 8, hipMemcpyDeviceToHost, c->stream));
  if (ux) HIP_TRY(c, hipMemcpyAsync(ux, stg + N, N * 8, hipMemcpyDeviceToHost, c->stream));
  if (uy) HIP_TRY(c, hipMemcpyAsync(uy, stg + 2 * N, N * 8, hipMemcpyDeviceToHost, c->stream));
  if (T) HIP_TRY(c, hipMemcpyAsync(T, stg + 3 * N, N * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return check_err(c);
}

lbm_status lbm_read_populations(lbm_ctx* c, double* f) {
  if (!c || !f) return LBM_E_INVAL;
  if (!c->initialized) return fail(c, LBM_E_STATE, "read before init");
  const size_t N = size_t(c->p.nx) * c->p.ny;
  double* stg = static_cast<double*>(c->f(1 - c->cur));
  const int per = int(std::min<size_t>(9, c->staging_bytes() / (N * 8)));
  for (int first = 0; first < 9; first += per) {
    const int cnt = std::min(per, 9 - first);
    lbm_status s = run_macro(c, nullptr, nullptr, nullptr, nullptr, stg, first, cnt);
    if (s != LBM_OK) return s;
    HIP_TRY(c, hipMemcpyAsync(f + size_t(first) * N, stg, size_t(cnt) * N * 8, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return check_err(c);
}

}  // extern "C"

NormArgs lbm::norm_args(const lbm_ctx* c, const double* stg, double* part) {
  const size_t N = size_t(c->p.nx) * c->p.ny;
  NormArgs a{};
  a.rho = stg;
  a.ux = stg + N;
  a.uy = stg + 2 * N;
  a.T = stg + 3 * N;
  a.tk_b = c->tabi();
  a.part = part;
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.walls = c->p.walls;
  a.side_dir = c->p.t_side_dirichlet;
  a.lambda_l = c->p.lambda_l;
  a.lambda_v = c->p.lambda_v;
  a.rho_l = c->p.rho_l;
  a.rho_v = c->p.rho_v;
  return a;
}

int lbm::norm_blocks(const lbm_ctx* c) {
  const size_t N = size_t(c->p.nx) * c->p.ny;
  return int(std::min<size_t>(kNormBlocks, (N + 255) / 256));
}

extern "C" {

lbm_status lbm_norms(lbm_ctx* c, lbm_norms_t* out) {
  if (!c || !out) return LBM_E_INVAL;
  if (!c->initialized) return fail(c, LBM_E_STATE, "norms before init");
  const size_t N = size_t(c->p.nx) * c->p.ny;
  double* stg = static_cast<double*>(c->f(1 - c->cur));
  lbm_status s = run_macro(c, stg, stg + N, stg + 2 * N, stg + 3 * N, nullptr, 0, 0);
  if (s != LBM_OK) return s;
  const int nb = norm_blocks(c);
  HIP_TRY(c, launch_norms(norm_args(c, stg, c->red()), nb, c->stream));
  std::vector<double> part(size_t(nb) * kNormSlots);
  HIP_TRY(c, hipMemcpyAsync(part.data(), c->red(), part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double v[kNormSlots] = {0};
  for (int b = 0; b < nb; ++b)
    for (int i = 0; i < kNormSlots; ++i) {
      const double x = part[size_t(b) * kNormSlots + i];
      if (i == 2 || i == 5 || i == 6) v[i] = std::max(v[i], x); else v[i] += x;
    }
  const double n = double(N);
  out->mass = v[0];
  out->rho_mean = v[0] / n;
  out->umax = v[6];
  out->q_bottom = c->p.walls ? v[8] / c->p.nx : 0.0;
  out->q_heater = v[10] > 0.0 ? v[9] / v[10] : 0.0;
  out->n_heater = int64_t(v[10]);
  out->l1_rho = v[11] / n;
  out->l2_rho = std::sqrt(v[1] / n);
  out->linf_rho = v[2];
  out->l1_T = v[3] / n;
  out->l2_T = std::sqrt(v[4] / n);
  out->linf_T = v[5];
  out->nonfinite = int64_t(v[7]);
  out->step = c->step;
  return check_err(c);
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_E_INVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return check_err(c);
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

// ------------------------------------------------------------ checkpoints
struct StateHeader {
  uint64_t magic;
  int64_t step;
  int32_t nx, ny, precision, npart;
  uint64_t fbytes, tbytes, pbytes;
  uint64_t phash;  // hash of the parameters that shape the state (all but the launch choices)
};

// FNV-1a over the parameter block with the launch-only fields (strip height,
// waves per strip, XCD remap) cleared: a state saved under other physics,
// walls or sizes does not load
uint64_t params_hash(const lbm_params& p0) {
  lbm_params p = p0;
  p.tile_y = 0;
  p.strip_waves = 0;
  p.xcd_remap = 0;
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&p);
  for (size_t i = 0; i < sizeof p; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

lbm_status lbm_state_bytes(const lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LBM_E_INVAL;
  const size_t fb = size_t(9 * c->L.plane) * c->L.elem;
  const size_t tb = size_t(c->L.pitch) * c->p.ny * c->L.elem;
  *bytes = sizeof(StateHeader) + fb + tb + size_t(c->L.part_cap) * 8;
  return LBM_OK;
}

lbm_status lbm_save_state(lbm_ctx* c, void* host, size_t bytes) {
  if (!c || !host) return LBM_E_INVAL;
  if (!c->initialized) return fail(c, LBM_E_STATE, "save before init");
  size_t need = 0;
  lbm_state_bytes(c, &need);
  if (bytes < need) return fail(c, LBM_E_NOMEM, "host state buffer too small");
  StateHeader h{};
  h.magic = kStateMagic;
  h.step = c->step;
  h.nx = c->p.nx;
  h.ny = c->p.ny;
  h.precision = c->p.precision;
  h.npart = c->npart;
  h.fbytes = size_t(9 * c->L.plane) * c->L.elem;
  h.tbytes = size_t(c->L.pitch) * c->p.ny * c->L.elem;
  h.pbytes = size_t(c->L.part_cap) * 8;
  h.phash = params_hash(c->p);
  char* o = static_cast<char*>(host);
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  HIP_TRY(c, hipMemcpyAsync(o, c->f(c->cur), h.fbytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(o + h.fbytes, c->T(c->Tcur), h.tbytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(o + h.fbytes + h.tbytes, c->part(c->pcur), h.pbytes, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return check_err(c);
}

lbm_status lbm_load_state(lbm_ctx* c, const void* host, size_t bytes) {
  if (!c || !host) return LBM_E_INVAL;
  size_t need = 0;
  lbm_state_bytes(c, &need);
  if (bytes < need) return fail(c, LBM_E_INVAL, "state buffer too small");
  StateHeader h;
  std::memcpy(&h, host, sizeof h);
  if (h.magic != kStateMagic || h.nx != c->p.nx || h.ny != c->p.ny || h.precision != c->p.precision ||
      h.fbytes != size_t(9 * c->L.plane) * c->L.elem ||
      h.tbytes != size_t(c->L.pitch) * c->p.ny * c->L.elem || h.pbytes != size_t(c->L.part_cap) * 8 ||
      h.npart < 0 || h.npart > c->L.part_cap || h.phash != params_hash(c->p))
    return fail(c, LBM_E_INVAL, "state does not match this context (size, storage or parameters)");
  lbm_status s = upload_tables(c);
  if (s != LBM_OK) return s;
  const char* i = static_cast<const char*>(host) + sizeof h;
  c->cur = 0;
  c->Tcur = 0;
  c->pcur = 0;
  HIP_TRY(c, hipMemcpyAsync(c->f(0), i, h.fbytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->T(0), i + h.fbytes, h.tbytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->part(0), i + h.fbytes + h.tbytes, h.pbytes, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemsetAsync(c->errp(), 0, 4, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->npart = h.npart;
  c->step = h.step;
  c->initialized = true;
  ++c->generation;
  return LBM_OK;
}

}  // extern "C"
