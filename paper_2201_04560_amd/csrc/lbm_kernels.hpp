// Host-side interface to the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm {

constexpr int kNormSlots = 12;

// The two-wave march addresses a row's 9 population planes with 32-bit
// per-lane byte offsets, usable while the 9 planes span less than 4 GiB, and
// wraps periodic rows with one correction, which needs ny >= 3.
inline bool two_wave_fits(long long plane, int elem, int ny) {
  return 9ll * plane * elem < (1ll << 32) && ny >= 3;
}
// the 9 population planes (and so the temperature plane) below 4 GiB: byte
// offsets into them fit 32 bits (buffer accesses of the one-wave step)
inline bool arrays_fit_32bit(long long plane, int elem) { return 9ll * plane * elem < (1ll << 32); }

struct LaunchStep {
  int fp32;
  const void* fin;
  void* fout;
  const void* Tin;
  void* Tout;
  Tables tab;
  const double* part_in;
  int npart_in;
  const double* wall_in;
  int nwall_in;
  double* part_out;
  uint32_t* err;
  int nx, ny, pitch;
  long long plane;
  int ty, ntx, nty, halo;
  int walls, update_T, side_dir, want_mass, xcd_remap;
  int waves;  // 2: energy step marched by two waves per strip
  Phys ph;
  double* o_rho;
  double* o_ux;
  double* o_uy;
  double* o_T;
  double* o_f;
  int f_first, f_count;
};

template <class S>
struct InitArgs {
  S* f;
  S* Tout;
  const double* rho;
  const double* ux;
  const double* uy;
  const double* T;
  double* part_out;
  Tables tab;
  Phys ph;
  int nx, ny, pitch;
  long long plane;
  int walls, thermal, side_dir;
  double rho_ref;
};

struct LaunchInit {
  int fp32;
  void* f;
  void* Tout;
  const double* rho;
  const double* ux;
  const double* uy;
  const double* T;
  double* part_out;
  Tables tab;
  Phys ph;
  int nx, ny, pitch;
  long long plane;
  int walls, thermal, side_dir;
};

template <class S>
struct WallArgs {
  const S* fin;
  const S* Tin;
  double* wall_out;
  const double* part_in;  // known-part density partials of the step (rho_bar_k)
  int npart_in;
  Tables tab;
  Phys ph;
  int nx, ny, pitch;
  long long plane;
};

struct LaunchWall {
  int fp32;
  const void* fin;
  const void* Tin;
  double* wall_out;
  const double* part_in;
  int npart_in;
  Tables tab;
  Phys ph;
  int nx, ny, pitch;
  long long plane;
};

struct NormArgs {
  const double* rho;
  const double* ux;
  const double* uy;
  const double* T;
  const int32_t* tk_b;  // temperature kinds of the bottom row (per column)
  double* part;
  int nx, ny, walls, side_dir;
  double lambda_l, lambda_v, rho_l, rho_v;
};

hipError_t launch_step(const LaunchStep& L, hipStream_t st);
hipError_t launch_macro(const LaunchStep& L, hipStream_t st);
hipError_t launch_init(const LaunchInit& L, hipStream_t st);
hipError_t launch_wall_mass(const LaunchWall& L, hipStream_t st);
hipError_t launch_norms(const NormArgs& a, int nblocks, hipStream_t st);
int init_blocks(int nx, int ny);
int wall_blocks(int nx);

// batched launches over several lattices: per-lattice argument blocks are
// filled on the host, copied to device memory and indexed by workgroup range
size_t step_desc_bytes(int fp32);
void fill_step_desc(const LaunchStep& L, void* out);
// wall_mode: 0 periodic, 1 psi-based walls, 2 some lattice has modified-psi
// walls or an outflow top
// waves = 2 (energy-update launches only): two waves per strip; every
// lattice of the launch must satisfy two_wave_fits()
hipError_t launch_step_multi(int fp32, int wall_mode, int thermal, int waves, const void* desc,
                             const int* start, int ngrid, int nblocks, hipStream_t st);
size_t wall_desc_bytes(int fp32);
void fill_wall_desc(const LaunchWall& L, void* out);
hipError_t launch_wall_multi(int fp32, const void* desc, const int* start, int ngrid, int nblocks,
                             hipStream_t st);

}  // namespace lbm
