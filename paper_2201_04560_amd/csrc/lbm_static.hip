// lbm_norms_device: the diagnostics of lbm_norms for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).  Nothing here allocates, on the host or the device:
// the per-workgroup partial sums live in a file-scope device array of fixed
// size, one copy per GPU, and the final fixed-order sum runs on the device,
// so the call neither synchronises nor copies to the host.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/lbm_pp.h"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

// one partial per slot and workgroup of the diagnostics reduction: 512 x 12
// float64 = 48 KiB per GPU, held until the process ends
constexpr int kScratchDoubles = kNormBlocks * kNormSlots;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of the GPU's own copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side handle, never a device address.
lbm_status scratch_for(lbm_ctx* c, double** out) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(c, LBM_E_UNSUPPORTED, "lbm_norms_device: device index outside 0..63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[c->device]) {
    int prev = 0;
    HIP_TRY(c, hipGetDevice(&prev));
    HIP_TRY(c, hipSetDevice(c->device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(prev);
    HIP_TRY(c, e);
    HIP_TRY(c, e2);
    if (!p) return fail(c, LBM_E_HIP, "lbm_norms_device: no device address for the scratch array");
    g_scratch[c->device] = static_cast<double*>(p);
  }
  *out = g_scratch[c->device];
  return LBM_OK;
}

// Final pass: slot i summed (or maximised) over the workgroups in workgroup
// order, the same order and operations as the host sum of lbm_norms, then
// the derived fields.
__global__ __launch_bounds__(64) void norms_final_kernel(const double* __restrict__ part, int nb, double n,
                                                         int nx, int walls, int64_t step,
                                                         lbm_norms_t* __restrict__ out) {
  __shared__ double v[kNormSlots];
  const int i = threadIdx.x;
  if (i < kNormSlots) {
    const bool is_max = (i == 2 || i == 5 || i == 6);
    double t = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double x = part[b * kNormSlots + i];
      t = is_max ? (t < x ? x : t) : t + x;
    }
    v[i] = t;
  }
  __syncthreads();
  if (i == 0) {
    out->mass = v[0];
    out->rho_mean = v[0] / n;
    out->umax = v[6];
    out->q_bottom = walls ? v[8] / double(nx) : 0.0;
    out->q_heater = v[10] > 0.0 ? v[9] / v[10] : 0.0;
    out->l1_rho = v[11] / n;
    out->l2_rho = sqrt(v[1] / n);
    out->linf_rho = v[2];
    out->l1_T = v[3] / n;
    out->l2_T = sqrt(v[4] / n);
    out->linf_T = v[5];
    out->nonfinite = int64_t(v[7]);
    out->n_heater = int64_t(v[10]);
    out->step = step;
  }
}

}  // namespace

extern "C" lbm_status lbm_norms_device(lbm_ctx* c, lbm_norms_t* dev_out) {
  if (!c || !dev_out) return LBM_E_INVAL;
  if (reinterpret_cast<uintptr_t>(dev_out) % alignof(lbm_norms_t))
    return fail(c, LBM_E_INVAL, "lbm_norms_device: output must be 8-byte aligned");
  if (!c->initialized) return fail(c, LBM_E_STATE, "norms before init");
  const int nb = norm_blocks(c);
  if (size_t(nb) * kNormSlots > size_t(kScratchDoubles))
    return fail(c, LBM_E_INVAL, "lbm_norms_device: more partial sums than the 48 KiB scratch array holds");
  double* part = nullptr;
  lbm_status s = scratch_for(c, &part);
  if (s != LBM_OK) return s;
  const size_t N = size_t(c->p.nx) * c->p.ny;
  double* stg = static_cast<double*>(c->f(1 - c->cur));
  s = run_macro(c, stg, stg + N, stg + 2 * N, stg + 3 * N, nullptr, 0, 0);
  if (s != LBM_OK) return s;
  HIP_TRY(c, launch_norms(norm_args(c, stg, part), nb, c->stream));
  hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(64), 0, c->stream, part, nb, double(N), c->p.nx,
                     c->p.walls, int64_t(c->step), dev_out);
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}
