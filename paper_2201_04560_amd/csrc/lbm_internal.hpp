// Internal state of a lattice context, shared by the runtime sources.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbm_pp.h"
#include "lbm_kernels.hpp"

namespace lbm {

struct Layout {
  int pitch = 0;
  long long plane = 0;  // elements between population planes
  int elem = 8;         // bytes per stored value
  int ty = 0, ntx = 0, nty = 0, nblocks = 0;
  int part_cap = 0, wall_cap = 0;
  size_t off_f[2] = {0, 0}, off_T[2] = {0, 0};
  size_t off_tab = 0, off_tk = 0, off_part[2] = {0, 0}, off_wall = 0, off_red = 0, off_err = 0;
  size_t total = 0;
};

}  // namespace lbm

struct lbm_ctx {
  lbm_params p{};
  lbm::Layout L;
  lbm::Phys ph{};
  hipStream_t stream = nullptr;
  char* base = nullptr;
  size_t bytes = 0;
  int device = -1;  // the GPU that holds the buffer
  int cur = 0, Tcur = 0, pcur = 0, npart = 0;
  int64_t step = 0;
  // bumped by every call that changes the state or the boundary tables
  // (step, init, boundary, state load, batch run): an adjoint backward
  // checks that nothing changed since its forward pass
  uint64_t generation = 0;
  bool initialized = false;
  std::vector<double> rw_b, rw_t, tv_b, tv_t;
  std::vector<int32_t> tk_b, tk_t;
  std::string err;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  // optional per-launch timing of the step kernel (event pairs on the stream)
  bool ktime = false;
  std::vector<hipEvent_t> kev;
  size_t kused = 0;

  void* f(int i) const { return base + L.off_f[i]; }
  void* T(int i) const { return base + L.off_T[i]; }
  double* part(int i) const { return reinterpret_cast<double*>(base + L.off_part[i]); }
  double* wall() const { return reinterpret_cast<double*>(base + L.off_wall); }
  double* red() const { return reinterpret_cast<double*>(base + L.off_red); }
  uint32_t* errp() const { return reinterpret_cast<uint32_t*>(base + L.off_err); }
  double* tabd() const { return reinterpret_cast<double*>(base + L.off_tab); }
  int32_t* tabi() const { return reinterpret_cast<int32_t*>(base + L.off_tk); }
  lbm::Tables tables() const {
    lbm::Tables t;
    const int nx = p.nx;
    t.rho_w_b = tabd();
    t.rho_w_t = tabd() + nx;
    t.tv_b = tabd() + 2 * nx;
    t.tv_t = tabd() + 3 * nx;
    t.tk_b = tabi();
    t.tk_t = tabi() + nx;
    return t;
  }
  size_t staging_bytes() const { return size_t(9 * L.plane) * L.elem; }
};

#define HIP_TRY(ctx, expr)                                                     \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);          \
      return LBM_E_HIP;                                                        \
    }                                                                          \
  } while (0)


namespace lbm {
// workgroups of the diagnostics reduction (grid-stride over the lattice)
constexpr int kNormBlocks = 512;

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& msg);
// read-out kernel: rho, u, T (and/or populations) of the current step into
// the given device arrays (the idle population buffer serves as staging)
lbm_status run_macro(lbm_ctx* c, double* o_rho, double* o_ux, double* o_uy, double* o_T, double* o_f,
                     int f_first, int f_count);
// arguments of the diagnostics kernel over the fields staged at stg, its
// per-workgroup partial sums going to part; and its workgroup count
NormArgs norm_args(const lbm_ctx* c, const double* stg, double* part);
int norm_blocks(const lbm_ctx* c);
LaunchStep step_args(lbm_ctx* c);
LaunchWall wall_args(lbm_ctx* c, const LaunchStep& L);
void make_layout(const lbm_params& p, Layout& L);
}  // namespace lbm
