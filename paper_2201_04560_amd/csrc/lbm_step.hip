// Fused time step of the pseudopotential LBM with phase change (gfx950).
//
// One workgroup = one wavefront of 64 lanes owns a strip of 58 output
// columns (3 recomputed halo columns each side; 56 and 4 with walls) and
// marches up a segment of rows (3 halo rows at each end).  Every row passes
// through four pipelined stages whose inputs live in small LDS ring
// buffers, so each node's populations and temperature are read from HBM
// once and written once per step:
//
//   A(r)    pull the 9 populations of row r (prefetched one row ahead),
//           moments, T, EOS terms and psi in float64    Eqs. lbm, psi,
//                                                       peng-robinson
//   wall    Zou-He closure of a wall row once its neighbour row has psi
//   B(r-1)  interaction + adhesion + buoyancy force, Q, velocity, Li
//           source S and correction C, MRT collision, store f*
//                               Eqs. shanchen, S, C, Q, collisionMRT
//   C(r-2)  first RK2 stage of the energy equation -> T*   Eq. energy-equation
//   D(r-3)  second RK2 stage -> T^{n+1}, store
//
// In the one-wave march the workgroup is a single wavefront, and LDS
// operations of one wavefront complete in program order, so the stages are
// separated by compiler-only barriers: no s_barrier / memory fence that
// would also drain the prefetched global loads.  The two-wave march (the
// energy step on small lattices) gives C and D to a second wave one row
// behind, with one workgroup barrier per row.  Each kernel is instantiated
// for three wall modes: periodic in y, psi-based Zou-He walls, and walls
// with the modified-psi model or the zero-gradient outflow top.
//
// Storage S is double (plain step) or float (populations stored as
// g_i = f_i - w_i rho_ref).  C is the type of the collision, energy,
// force and Q arithmetic.  The EOS and psi (and the wall closure's Newton
// solve) are float64 in both: psi near the spinodal needs its digits,
// while the forces and Q, weighted sums of psi differences between
// neighbours, feed the float32 collision (on the 4 x 512^2 vaporisation:
// step 25.7 -> 25.3 us, density deviation from float64 after 20,000 steps
// 1.21e-3 -> 1.22e-3, against float64 forces and Q, MI355X).
#include <cstring>
#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

template <class S, class C>
struct StepArgs {
  const S* fin;
  S* fout;
  const S* Tin;
  S* Tout;
  const double* tabd;     // rho_w bottom, rho_w top, T value bottom, T value top
  const int32_t* tabk;    // T kind bottom, T kind top
  const double* part_in;  // previous step's mass partials (known-part densities)
  const double* wall_in;  // this step's wall-closure mass corrections
  double* part_out;
  uint32_t* err;
  long long plane;
  int nx, ny, pitch, npart_in, nwall_in;
  int ty, ntx, nty, halo;
  int side_dir, want_mass, xcd_remap;
  Phys ph;
  PhysC<C> pc;
};

struct MacroOut {
  double* rho;
  double* ux;
  double* uy;
  double* T;
  double* f;
  int f_first, f_count;
};

enum { MODE_STEP = 0, MODE_MACRO = 1 };

// compiler-level barrier between pipeline stages of the single wavefront
__device__ __forceinline__ void stage_barrier() { __builtin_amdgcn_wave_barrier(); }

// tile index for block id: keep runs of consecutive tiles on one XCD
// (workgroups are dispatched round-robin over the 8 XCDs)
__device__ __forceinline__ int tile_of_block(int bid, int nb, int remap) {
  if (!remap || nb < 16) return bid;
  const int q = nb / 8, rem = nb % 8;
  const int xcd = bid % 8, k = bid / 8;
  const int start = xcd * q + (xcd < rem ? xcd : rem);
  return start + k;
}

// Sum of the mean-density partials of the previous step (and the wall
// closure's corrections), the same fixed order in every workgroup: lane l
// accumulates entries l, l + 64, ... into eight interleaved partial sums so
// that eight loads are in flight (the loop of one dependent load at a time
// cost about 24 us per 4096^2 step), then the sums and the lanes combine.
// global-memory load and store through a generic pointer.  The batched
// kernels read their lattices' pointers from a device table, where the
// compiler cannot infer the address space and issues flat accesses; those
// also count against the LDS wait counter, so every LDS wait of a row would
// wait for the prefetched next row as well.  GA = false: a plain access
// (the single-lattice kernels, whose pointers are kernel arguments).
template <bool GA, class T>
__device__ __forceinline__ T gld(const T* p) {
  if constexpr (GA)
    return *(const __attribute__((address_space(1))) T*)p;
  else
    return *p;
}
template <bool GA, class T>
__device__ __forceinline__ void gst(T* p, const T v) {
  if constexpr (GA)
    *(__attribute__((address_space(1))) T*)p = v;
  else
    *p = v;
}

// Raw buffer access (two-wave march, whose arrays are below 4 GiB): the
// array is one buffer resource, the row's byte offset an SGPR and the lane's
// offset a 32-bit VGPR, so that no per-access 64-bit address is formed (with
// plain pointers the compiler kept 64-bit lane offsets and added them to
// each row's base: 19 64-bit adds per row of wave 0).  num_records is the
// array's size in bytes.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 family: 32-bit data format, no swizzle
template <class T>
__device__ __forceinline__ rsrc_t make_rsrc(const T* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, int(bytes), kRsrcWord3);
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float bload(float*, rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double bload(double*, rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}


// isotropic D2Q9 stencils on a 3x3 neighbourhood [dy+1][dx+1]:
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

// T-independent part of the energy right-hand side at one node (computed
// in stage C, reused by stage D of the same row)
template <class C>
struct EnergyCoef {
  C ux, uy, divu, glx, gly, lam_rcv, inv_rcv;
  C dpdt_s;  // (dp/dT)_rho at the stage temperature T*, for stage D
};

// K(phi) of Eq. energy-equation with (dp/dT)_rho given
template <class C>
__device__ __forceinline__ C energy_rhs(const C (&phi)[3][3], const EnergyCoef<C>& e, C dpdt) {
  const C gx = gradx9(phi), gy = grady9(phi);
  return -(e.ux * gx + e.uy * gy) + e.lam_rcv * lap9(phi) + (e.glx * gx + e.gly * gy) * e.inv_rcv -
         phi[1][1] * dpdt * e.divu * e.inv_rcv;
}

// (dp/dT)_rho = A1 + a kw A2 (1 + kw (1 - sqrt(T/T_c))) / sqrt(T T_c)
template <class C>
__device__ __forceinline__ C dpdt_at(C A1, C A2, C T, const PhysC<C>& q) {
  const C rs = rsq_c(T);
  const C sa = C(1) + q.kw * (C(1) - T * rs * q.inv_sqrtTc);
  return A1 + q.akw_isTc * A2 * sa * rs;
}

// target waves per SIMD: the float32-storage kernels fit 3 without spills
template <class S>
struct WavesPerEU {
  static constexpr int value = sizeof(S) == 4 ? 3 : 2;
};

// compile-time loop: f(integral_constant<int, j>) for j = 0 .. N-1
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int N>
using Ph = std::integral_constant<int, N>;

// A wave's loads and stores share one completion counter, and with both in
// flight a wait for a load also waits for every store issued before it.
// The one-wave float64 march with walls therefore issues a row's stores only
// after the next wait for its prefetched row (one iteration later), so that
// wait finds them done: 5 % faster on the 4096^2 pool on MI355X.  Elsewhere
// it measured no faster (the two-wave march) or slower (float32: the held
// values spill at three waves per SIMD; periodic float64 at 512^2).
constexpr bool kDeferStores = true;

// wait until every vector memory operation of the wave has completed
// (s_waitcnt vmcnt(0), the other counters left free)
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// one strip of one lattice; bid is the workgroup's index within its lattice.
// RPI rows enter the pipeline per iteration.  The code is written for any
// RPI; 1 is instantiated: with 2 (two independent row chains per wave) the
// step ran 3-6 % slower on 512^2 and up to 60 % slower on 4096^2 on MI355X
// (more registers, no gain in overlap).
// WS (energy step only): the strip is marched by two waves of one
// workgroup, wave 0 through stages A and B, wave 1 through C and D one row
// later; they exchange rows through LDS rings of 8 rows and meet at one
// workgroup barrier per row.  Handing the collision to wave 1 as well (21
// values per node through LDS) measured slower on MI355X.
// WM: 0 periodic in y, 1 Zou-He walls (psi-based), 2 walls with the modified-
// psi model and/or the zero-gradient outflow top (runtime flags of Phys);
// lattices without those features run the WM = 1 code, which does not carry
// their branches.
// GA: global-memory accesses name their address space (batched kernels,
// see gld); the batched two-wave float32 step on 4 x 512^2 27.8 -> 27.3 us
// on MI355X.
// BUF1: the one-wave march accesses its arrays through buffer resources
// (float32 storage, 9 planes below 4 GiB; chosen by the launcher).
template <class S, class C, int WM, bool THERMAL, int MODE, int RPI, bool WS, bool GA, bool BUF1 = false>
__device__ __forceinline__ void march_body(const StepArgs<S, C>& A, const MacroOut& O, const int bid) {
  constexpr bool WALLS = WM != 0;
  // Newton steps of the float64 reciprocals and square roots: one is below
  // float32 storage's rounding by orders of magnitude
  constexpr int kNR = sizeof(S) == 4 ? 1 : 2;
  constexpr bool WX = WM == 2;
  constexpr bool DEFER = kDeferStores && !WS && WALLS && sizeof(S) == 8;
  const bool wall_mod = WX && A.ph.wall_mod;
  const bool outflow = WX && A.ph.outflow_top;
  static_assert(!WS || (MODE == MODE_STEP && THERMAL && RPI == 1), "two-wave march: energy step only");
  const int lane = WS ? int(threadIdx.x & (kLanes - 1)) : int(threadIdx.x);
  const int wave = WS ? __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)) : 0;
  const int nb = A.ntx * A.nty;
  if (bid >= nb) return;  // padding workgroup of a batched launch
  const int tile = tile_of_block(bid, nb, A.xcd_remap);
  const int tx = tile % A.ntx, tyi = tile / A.ntx;
  const int nx = A.nx, ny = A.ny;
  constexpr int halo = WALLS ? 4 : 3;
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
  const bool side_col = A.side_dir && (x == 0 || x == nx - 1);
  const Phys& P = A.ph;
  const PhysC<C>& Q = A.pc;
  const double rref = P.rho_ref;
  // byte offsets of the lane's column and its two neighbours; row and plane
  // offsets are uniform, so loads and stores take an SGPR base address
  const uint32_t ox = uint32_t(x) * sizeof(S), oxm = uint32_t(xm) * sizeof(S),
                 oxp = uint32_t(xp) * sizeof(S);
  const size_t plane_b = size_t(A.plane) * sizeof(S), row_b = size_t(A.pitch) * sizeof(S);
  const char* fin = reinterpret_cast<const char*>(A.fin);
  char* fout = reinterpret_cast<char*>(A.fout);
  const char* Tin = reinterpret_cast<const char*>(A.Tin);
  char* Tout = reinterpret_cast<char*>(A.Tout);
  auto ld = [](const char* base, uint32_t off) { return gld<GA>(reinterpret_cast<const S*>(base + off)); };
  auto st = [](char* base, uint32_t off, S v) { gst<GA>(reinterpret_cast<S*>(base + off), v); };
  // OFF32 (two-wave march): the plane offsets are folded into per-lane 32-bit
  // offsets computed once, so a row's loads and stores share one 64-bit row
  // address instead of one per plane (fewer scalar instructions on the
  // wave's chain; 512^2 float32 14.3 -> 13.2 us on MI355X).  Needs 9 planes
  // below 4 GiB, which the launcher checks.
  constexpr bool OFF32 = WS;
  // TRIM: wave 0 keeps its rows in a register ring and the loop is unrolled
  // by the ring length (periodic lattices); with walls the unrolled closure
  // code pushed the kernel into scratch memory, so there the loop keeps
  // runtime ring slots and copies each row once
  constexpr bool TRIM = WS && !WALLS;
  const uint32_t pb32 = uint32_t(plane_b);
  const uint32_t lo[9] = {ox,           oxm + pb32,     ox + 2 * pb32, oxp + 3 * pb32, ox + 4 * pb32,
                          oxm + 5 * pb32, oxp + 6 * pb32, oxp + 7 * pb32, oxm + 8 * pb32};
  const uint32_t so[9] = {ox,           ox + pb32,     ox + 2 * pb32, ox + 3 * pb32, ox + 4 * pb32,
                          ox + 5 * pb32, ox + 6 * pb32, ox + 7 * pb32, ox + 8 * pb32};
  // byte offset of row y >= 0 (OFF32: one 32-bit multiply)
  const uint32_t rb32 = uint32_t(row_b);
  // BUF (float32 storage, two-wave march, or BUF1): the four arrays as
  // buffer resources (9 planes, and the temperature's pitch x ny, below 4
  // GiB: checked by the launcher).  On MI355X: two-wave 4 x 512^2 float32
  // 26.3 -> 25.5 us per step, one-wave 4096^2 pool float32 429 -> 402 us;
  // float64 measured no faster (single lattice 1 % slower), nor did the
  // one-wave batched kernel (finest ladder mesh 214 -> 222 us)
  static_assert(!BUF1 || (!WS && sizeof(S) == 4), "one-wave float32 buffer accesses only");
  constexpr bool BUF = (OFF32 && sizeof(S) == 4) || BUF1;
  const uint32_t fbytes32 = uint32_t(9 * plane_b), tbytes32 = uint32_t(size_t(ny) * row_b);
  const rsrc_t rs_fin = make_rsrc(A.fin, fbytes32), rs_fout = make_rsrc(A.fout, fbytes32);
  const rsrc_t rs_Tin = make_rsrc(A.Tin, tbytes32), rs_Tout = make_rsrc(A.Tout, tbytes32);
  auto bld = [](rsrc_t r, uint32_t voff, uint32_t soff) { return bload(static_cast<S*>(nullptr), r, voff, soff); };
  // a row index in [-3, ny + 3) wrapped onto the periodic lattice; the
  // two-wave march runs only with ny >= 3, where one correction suffices
  auto wrapy = [&](const int a) {
    if constexpr (WS)
      return a < 0 ? a + ny : (a >= ny ? a - ny : a);
    else
      return wrap3(a, ny);
  };
  auto roff = [&](const int y) -> size_t {
    if constexpr (OFF32)
      return size_t(uint32_t(y) * rb32);
    else
      return size_t(y) * row_b;
  };

  // rings of R rows indexed by (row - first row) & (R - 1)
  constexpr int R = WS ? 8 : 4 * RPI;  // ring rows
  __shared__ double s_rho[R][kLanes];
  __shared__ C s_psi[R][kLanes];
  __shared__ C s_T[R][kLanes];
  __shared__ C s_ux[R][kLanes];
  __shared__ C s_uy[R][kLanes];
  __shared__ C s_Ts[R][kLanes];
  // density in the compute type for the energy stencils (float32 path only;
  // the float64 path reads s_rho)
  constexpr bool kRhoC = sizeof(C) < sizeof(double);
  __shared__ C s_rc[kRhoC ? R : 1][kLanes];
  // two-wave march: EOS terms and 1/rho handed from wave 0 to wave 1
  __shared__ C s_a1[WS ? R : 1][kLanes];
  __shared__ C s_a2[WS ? R : 1][kLanes];
  __shared__ C s_ir[WS ? R : 1][kLanes];
  constexpr int kColl = 21;  // collision inputs of a node

  // mean density of the current state (Eq. gravitational_force), and for
  // the wall closure the mean with every wall node at its known part: the
  // partials (known-part densities of every node) and the closure's
  // corrections are summed in the same order by every workgroup
  double rho_bar = 0.0, rho_bar_k = 0.0;
  if (P.gy != 0.0) {
    const double* part = A.part_in;
    const double* wall = A.wall_in;
    const double sp = fixed_order_sum([&](int i) { return gld<GA>(part + i); }, A.npart_in, lane);
    const double sw = fixed_order_sum([&](int i) { return gld<GA>(wall + i); }, A.nwall_in, lane);
    const double n = double(nx) * double(ny);
    rho_bar_k = sp / n;
    rho_bar = (sp + sw) / n;
  }

  // issue the loads of row r into (gn, Tn)
  auto load_row = [&](int r, C (&gn)[9], C& Tn) {
    const bool have = WALLS ? (r >= 0 && r < ny) : true;
    if (!have) return;
    const int yr = __builtin_amdgcn_readfirstlane(WALLS ? r : wrapy(r));
    int ydn, yup;
    bool kdn = true, kup = true;
    if (WALLS) {
      // rows outside the walls do not exist: clamp the address, drop the value
      kdn = yr >= 1;
      kup = yr + 1 < ny;
      ydn = kdn ? yr - 1 : yr;
      yup = kup ? yr + 1 : yr;
    } else {
      ydn = (yr == 0) ? ny - 1 : yr - 1;
      yup = (yr == ny - 1) ? 0 : yr + 1;
    }
    const char* rc = fin + roff(yr);
    const char* rd = fin + roff(ydn);
    const char* ru = fin + roff(yup);
    C v2, v5, v6, v4, v7, v8;
    const uint32_t oc = uint32_t(yr) * rb32;
    if constexpr (BUF && !OFF32) {
      // one-wave march: the plane offsets go into the SGPR offset
      const uint32_t od = uint32_t(ydn) * rb32, ou = uint32_t(yup) * rb32;
      gn[0] = C(bld(rs_fin, ox, oc));
      gn[1] = C(bld(rs_fin, oxm, oc + pb32));
      gn[3] = C(bld(rs_fin, oxp, oc + 3 * pb32));
      v2 = C(bld(rs_fin, ox, od + 2 * pb32));
      v5 = C(bld(rs_fin, oxm, od + 5 * pb32));
      v6 = C(bld(rs_fin, oxp, od + 6 * pb32));
      v4 = C(bld(rs_fin, ox, ou + 4 * pb32));
      v7 = C(bld(rs_fin, oxp, ou + 7 * pb32));
      v8 = C(bld(rs_fin, oxm, ou + 8 * pb32));
    } else if constexpr (BUF) {
      const uint32_t od = uint32_t(ydn) * rb32, ou = uint32_t(yup) * rb32;
      gn[0] = C(bld(rs_fin, lo[0], oc));
      gn[1] = C(bld(rs_fin, lo[1], oc));
      gn[3] = C(bld(rs_fin, lo[3], oc));
      v2 = C(bld(rs_fin, lo[2], od));
      v5 = C(bld(rs_fin, lo[5], od));
      v6 = C(bld(rs_fin, lo[6], od));
      v4 = C(bld(rs_fin, lo[4], ou));
      v7 = C(bld(rs_fin, lo[7], ou));
      v8 = C(bld(rs_fin, lo[8], ou));
    } else if constexpr (OFF32) {
      gn[0] = C(ld(rc, lo[0]));
      gn[1] = C(ld(rc, lo[1]));
      gn[3] = C(ld(rc, lo[3]));
      v2 = C(ld(rd, lo[2]));
      v5 = C(ld(rd, lo[5]));
      v6 = C(ld(rd, lo[6]));
      v4 = C(ld(ru, lo[4]));
      v7 = C(ld(ru, lo[7]));
      v8 = C(ld(ru, lo[8]));
    } else {
      gn[0] = C(ld(rc, ox));
      gn[1] = C(ld(rc + plane_b, oxm));
      gn[3] = C(ld(rc + 3 * plane_b, oxp));
      v2 = C(ld(rd + 2 * plane_b, ox));
      v5 = C(ld(rd + 5 * plane_b, oxm));
      v6 = C(ld(rd + 6 * plane_b, oxp));
      v4 = C(ld(ru + 4 * plane_b, ox));
      v7 = C(ld(ru + 7 * plane_b, oxp));
      v8 = C(ld(ru + 8 * plane_b, oxm));
    }
    // beyond a wall the values are dropped by wall_mask where the row is
    // consumed; the zero-gradient outflow keeps the top row's (the clamped
    // address: its populations from above are pulled from its own row)
    gn[2] = v2;
    gn[5] = v5;
    gn[6] = v6;
    gn[4] = v4;
    gn[7] = v7;
    gn[8] = v8;
    if constexpr (BUF)
      Tn = C(bld(rs_Tin, ox, oc));
    else
      Tn = C(ld(Tin + roff(yr), ox));
  };

  // populations pulled from beyond a wall do not exist.  They are zeroed
  // where the row is consumed, not where its loads are issued: a select
  // next to the loads made the wave wait for its prefetched row at once
  // (walled one-wave march, 4096^2 pool float32 on MI355X)
  auto wall_mask = [&](const int r, C (&g)[9]) {
    if constexpr (WALLS) {
      if (r < 1) g[2] = g[5] = g[6] = C(0);
      if (r + 1 >= ny && !outflow) g[4] = g[7] = g[8] = C(0);
    }
  };

  uint32_t err = 0;
  double mass_acc = 0.0;
  const int rbase = y0 - kHaloY;                 // first row of stage A
  const int nit = (y1 - y0) + 2 * kHaloY;        // rows through stage A
  const int rend = rbase + nit;                  // one past the last of them
  // ring slot of a row: (row - rbase) & (R - 1); in iteration k the j-th
  // row has slot (RPI k + j) & (R - 1), a constant once k & 3 is fixed
  C gn[RPI][9], Tn[RPI];
#pragma unroll
  for (int j = 0; j < RPI; ++j) {
    Tn[j] = C(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) gn[j][i] = C(0);
    if (!TRIM && rbase + j < rend) load_row(rbase + j, gn[j], Tn[j]);
  }
  // two-wave march, wave 0: register ring of pulled rows, slot (row - rbase)
  // & 3 (a constant in the unrolled loop): row r is read from its slot, r + 1
  // is loaded into the next once stage A has read row r (so the wait for row
  // r does not wait for the new loads too) and r - 1 is still in the previous
  // one, so no row is copied between registers (with the one-correction row
  // wrap: 512^2 12.7 -> 12.3 us float32, 15.7 -> 15.2 us float64 on MI355X)
  C gq[TRIM ? 4 : 1][9], Tq[TRIM ? 4 : 1];
#pragma unroll
  for (int j = 0; j < (TRIM ? 4 : 1); ++j) {
    Tq[j] = C(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) gq[j][i] = C(0);
  }
  if (TRIM && wave == 0 && rbase < rend) load_row(rbase, gq[0], Tq[0]);
  // carries from the previous iteration's last row (its pulled populations
  // and moments feed the next row's collision)
  C gprev[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) gprev[i] = C(0);
  C jxprev = C(0), jyprev = C(0);
  double psiw_b = 0.0, psiw_t = 0.0;
  // rolling per-row carries: EOS terms of the last two stage-A rows (for
  // stage C two rows later), 1/rho of the last stage-B row and the energy
  // coefficients of the last stage-C row (each read one row later)
  C a1h[2] = {C(0), C(0)}, a2h[2] = {C(0), C(0)}, irprev = C(0);
  EnergyCoef<C> ecprev{};

  // kind of the temperature condition at (y, x') for the lane's column x'
  // (xs = 0, 1, 2 for x - 1, x, x + 1); only evaluated on rows 0 / ny - 1
  auto row_kind = [&](int y, int xs, double& val) {
    const int xx = xs == 0 ? xm : (xs == 1 ? x : xp);
    if (A.side_dir && (xx == 0 || xx == nx - 1)) {
      val = P.t_side_val;
      return int(T_DIRICHLET);
    }
    const int top = (y == ny - 1) ? 1 : 0;
    val = gld<GA>(A.tabd + (2 + top) * nx + xx);
    return int(gld<GA>(A.tabk + top * nx + xx));
  };
  auto node_kind = [&](int y, double& val) {
    if (side_col) {
      val = P.t_side_val;
      return int(T_DIRICHLET);
    }
    if (y == 0 || y == ny - 1) return row_kind(y, 1, val);
    val = 0.0;
    return int(T_FREE);
  };
  // the same as a select (no divergent branch), for the two-wave march
  auto node_kind_sel = [&](int y, double& val) {
    int k = T_FREE;
    val = 0.0;
    if (y == 0 || y == ny - 1) k = row_kind(y, 1, val);  // uniform over the wave
    if (side_col) {
      val = P.t_side_val;
      k = T_DIRICHLET;
    }
    return k;
  };

  // ------------------------------------------------------------ stage A(r)
  // moments, EOS and psi of row r (slot SA); wall rows keep the known part
  // of their density until the closure
  auto stageA = [&](auto sa, const int r, C (&g)[9], const C Tr, C& jx, C& jy, C& a1, C& a2) {
    const int SA = int(sa);
    jx = C(0);
    jy = C(0);
    a1 = C(0);
    a2 = C(0);
    const bool have = WALLS ? (r >= 0 && r < ny) : true;
    if (have) {
      const int yr = WALLS ? r : wrapy(r);
      const double T = double(Tr);
      double rho, psi = 0.0;
      if (WALLS && (yr == 0 || (yr == ny - 1 && !outflow))) {
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
        const EosNode e = eos_node<kNR>(rho, T, P);
        psi = psi_fast<kNR>(rho, T, e, P, err);
        a1 = C(e.A1);
        a2 = C(e.A2);
      }
      s_rho[SA][lane] = rho;
      if constexpr (kRhoC) s_rc[SA][lane] = C(rho);
      s_psi[SA][lane] = C(psi);
      s_T[SA][lane] = Tr;
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = C(0);
    }
  };

  // ---------------------------------------------------------- wall closures
  // wall row in slot SW, its interior neighbour row in slot SN
  auto closure = [&](auto swc, auto snc, const bool bottom) {
    const int SW = int(swc), SN = int(snc);
    const double sgn = bottom ? 1.0 : -1.0;
    const double K = s_rho[SW][lane];
    const double Tw = double(s_T[SW][lane]);
    const double rw = gld<GA>(A.tabd + (bottom ? 0 : 1) * nx + x);  // rho_w, or G_w (modified-psi)
    double psiw, rwall, psiwall;
    if (wall_mod) {
      const double nbsum = double(s_psi[SN][lane]) / 3.0 + (double(s_psi[SN][lp]) + double(s_psi[SN][lm])) / 12.0;
      rwall = wall_density_mod(K, nbsum, rw, Tw, sgn, P, rho_bar_k);
      psiwall = psi_checked(rwall, Tw, P, err);
      // solid neighbours seen by F^m: G psi psi_s = G_w psi^2
      psiw = rw / P.G * psiwall;
    } else {
      psiw = psi_checked(rw, Tw, P, err);
      const double B = wall_coef_B(double(s_psi[SN][lane]), double(s_psi[SN][lp]), double(s_psi[SN][lm]), psiw, sgn, P);
      rwall = wall_density(K, B, Tw, sgn, P, rho_bar_k);
      psiwall = psi_checked(rwall, Tw, P, err);
    }
    s_rho[SW][lane] = rwall;
    if constexpr (kRhoC) s_rc[SW][lane] = C(rwall);
    s_psi[SW][lane] = C(psiwall);
    if (bottom) psiw_b = psiw; else psiw_t = psiw;
  };

  // deferred stores (DEFER): the last collided row's populations and
  // the last row's new temperature, issued by flush_stores()
  S dq_f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) dq_f[i] = S(0);
  bool dq_fon = false, dq_Ton = false;
  int dq_frow = 0, dq_Trow = 0;
  S dq_T = S(0);
  auto flush_stores = [&]() {
    if (dq_fon) {
      char* orow = fout + size_t(__builtin_amdgcn_readfirstlane(dq_frow)) * row_b;
#pragma unroll
      for (int i = 0; i < 9; ++i) st(orow + i * plane_b, ox, dq_f[i]);
    }
    if (dq_Ton) st(Tout + size_t(__builtin_amdgcn_readfirstlane(dq_Trow)) * row_b, ox, dq_T);
    dq_fon = false;
    dq_Ton = false;
  };

  // MRT collision of one row from its inputs ci (pulled populations, jx, jy,
  // ux, uy, Fx, Fy, rho, rho - rho_ref, |F^m|^2/psi^2, Qxx + Qyy, Qxx - Qyy,
  // Qxy) in shifted moments n = M g (g = f - w rho_ref); stores the row
  auto collide_store = [&](const int ys, const C (&ci)[kColl], const double rho_node) {
    const C* gp = ci;
    const C jxs = ci[9], jys = ci[10], ux = ci[11], uy = ci[12], Fx = ci[13], Fy = ci[14];
    const C rc = ci[15], sg = ci[16], fm2_ps2 = ci[17], qs = ci[18], qd = ci[19], qxyc = ci[20];
    const C a4 = (gp[1] + gp[2]) + (gp[3] + gp[4]);
    const C d4s = (gp[5] + gp[6]) + (gp[7] + gp[8]);
    const C n1 = C(-4) * gp[0] - a4 + C(2) * d4s;
    const C n2 = C(4) * gp[0] - C(2) * a4 + d4s;
    const C n4 = C(2) * (gp[3] - gp[1]) + (gp[5] - gp[7]) + (gp[8] - gp[6]);
    const C n6 = C(2) * (gp[4] - gp[2]) + (gp[5] - gp[7]) + (gp[6] - gp[8]);
    const C n7 = (gp[1] + gp[3]) - (gp[2] + gp[4]);
    const C n8 = (gp[5] + gp[7]) - (gp[6] + gp[8]);
    const C u2 = ux * ux + uy * uy;
    const C uF = ux * Fx + uy * Fy;
    const C te = C(P.sig_e) * fm2_ps2, tz = C(P.sig_z) * fm2_ps2;
    C snu = Q.snu_const;
    if (Q.snu_varies) {
      const C eta = Q.eta_v + (Q.eta_l - Q.eta_v) * (rc - Q.rho_v) * Q.inv_drho;
      snu = rcp_c(C(3) * eta + C(0.5));
    }
    const C se = Q.s_e, sz = Q.s_z, sq = Q.s_q;
    const C r3u2 = C(3) * rc * u2;
    const C m0 = sg;
    const C m1 = n1 - se * (n1 + C(2) * sg - r3u2) + (C(1) - se * C(0.5)) * (C(6) * uF + te) +
                 C(1.5) * se * qs;
    const C m2 = n2 - sz * (n2 - sg + r3u2) - (C(1) - sz * C(0.5)) * (C(6) * uF + tz) -
                 C(1.5) * sz * qs;
    const C m3 = jxs + Fx;
    const C m4 = n4 - sq * (n4 + rc * ux) - (C(1) - sq * C(0.5)) * Fx;
    const C m5 = jys + Fy;
    const C m6 = n6 - sq * (n6 + rc * uy) - (C(1) - sq * C(0.5)) * Fy;
    const C hnu = C(1) - snu * C(0.5);
    const C m7 = n7 - snu * (n7 - rc * (ux * ux - uy * uy)) + hnu * C(2) * (ux * Fx - uy * Fy) -
                 snu * qd;
    const C m8 = n8 - snu * (n8 - rc * ux * uy) + hnu * (ux * Fy + uy * Fx) - snu * qxyc;
    // f* = M^-1 m*
    const C a0 = m0 * C(1.0 / 9.0);
    const C ax0 = a0 - m1 * C(1.0 / 36.0) - m2 * C(1.0 / 18.0);
    const C dg0 = a0 + m1 * C(1.0 / 18.0) + m2 * C(1.0 / 36.0);
    const C j3 = m3 * C(1.0 / 6.0), j5 = m5 * C(1.0 / 6.0);
    const C q4 = m4 * C(1.0 / 6.0), q6 = m6 * C(1.0 / 6.0);
    const C q4h = m4 * C(1.0 / 12.0), q6h = m6 * C(1.0 / 12.0);
    const C p7c = m7 * C(0.25), p8c = m8 * C(0.25);
    C o[9];
    o[0] = a0 + (m2 - m1) * C(1.0 / 9.0);
    o[1] = ax0 + j3 - q4 + p7c;
    o[2] = ax0 + j5 - q6 - p7c;
    o[3] = ax0 - j3 + q4 + p7c;
    o[4] = ax0 - j5 + q6 - p7c;
    o[5] = dg0 + j3 + j5 + q4h + q6h + p8c;
    o[6] = dg0 - j3 + j5 - q4h + q6h - p8c;
    o[7] = dg0 - j3 - j5 - q4h - q6h + p8c;
    o[8] = dg0 + j3 - j5 + q4h - q6h - p8c;
    if constexpr (DEFER) {
#pragma unroll
      for (int i = 0; i < 9; ++i) dq_f[i] = S(o[i]);
      dq_fon = true;
      dq_frow = ys;
    } else {
      const int ysu = __builtin_amdgcn_readfirstlane(ys);
      char* orow = fout + roff(ysu);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if constexpr (BUF && !OFF32)
          bstore(rs_fout, ox, uint32_t(ysu) * rb32 + uint32_t(i) * pb32, S(o[i]));
        else if constexpr (BUF)
          bstore(rs_fout, so[i], uint32_t(ysu) * rb32, S(o[i]));
        else if constexpr (OFF32)
          st(orow, so[i], S(o[i]));
        else
          st(orow + i * plane_b, ox, S(o[i]));
      }
    }
    if (A.want_mass) {
      // known-part density of the next step: the collision conserves mass
      // (the populations leaving the node sum to its density up to the
      // rounding of the stored values); at walls the populations leaving
      // through the wall are replaced by those the closure will rebuild
      // from the neighbour row
      double m = rho_node;
      if (WALLS && (ys <= 1 || ys >= ny - 2)) {
        const double dn = double(S(o[4])) + double(S(o[7])) + double(S(o[8])) + rref / 6.0;
        const double up = double(S(o[2])) + double(S(o[5])) + double(S(o[6])) + rref / 6.0;
        if (ys == 0) m -= dn;
        if (ys == 1) m += dn;
        if (ys == ny - 2) m += up;
        if (ys == ny - 1) m -= up;
      }
      mass_acc += m;
    }
  };

  // ------------------------------------------------------------ stage B(s)
  // forces, velocity and collision of row s (slot SB); gp are its pulled
  // populations, (jxs, jys) its momentum
  auto stageB = [&](auto sbc, const int s, const C (&gin)[9], C jxs, C jys, C& irho_out) {
    const int SB = int(sbc);
    const int km = (SB + R - 1) & (R - 1), kc = SB, kq = (SB + 1) & (R - 1);  // rows s-1, s, s+1
    const bool have = WALLS ? (s >= 0 && s < ny) : true;
    if (!have) return;
    C gp[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) gp[i] = gin[i];
    const int ys = WALLS ? s : wrapy(s);
    const bool wb = WALLS && ys == 0;
    const bool wt = WALLS && ys == ny - 1 && !outflow;
    const bool ot = WALLS && ys == ny - 1 && outflow;
    const C pc = s_psi[kc][lane];
    const C p1 = s_psi[kc][lp], p3 = s_psi[kc][lm];
    C p2, p5, p6, p4, p7, p8;
    if (wt) {
      p2 = p5 = p6 = C(psiw_t);
    } else if (ot) {
      // zero-gradient outflow: psi above the top row is the top row's own
      p2 = pc;
      p5 = p1;
      p6 = p3;
    } else {
      p2 = s_psi[kq][lane];
      p5 = s_psi[kq][lp];
      p6 = s_psi[kq][lm];
    }
    if (wb) {
      p4 = p7 = p8 = C(psiw_b);
    } else {
      p4 = s_psi[km][lane];
      p7 = s_psi[km][lm];
      p8 = s_psi[km][lp];
    }
    const double rho = s_rho[kc][lane];
    const C G = C(P.G);
    // Eq. shanchen (psi_w for solid neighbours: Eq. shanchen-walls)
    C d1 = p1 - pc, d2 = p2 - pc, d3 = p3 - pc, d4 = p4 - pc;
    C d5 = p5 - pc, d6 = p6 - pc, d7 = p7 - pc, d8 = p8 - pc;
    if (WALLS && wall_mod) {
      // Eq. Q-mod-psi-based: solid neighbours drop out of Q
      if (wb) d4 = d7 = d8 = C(0);
      if (wt) d2 = d5 = d6 = C(0);
    }
    const C sx = C(1.0 / 3.0) * (p1 - p3) + C(1.0 / 12.0) * ((p5 - p7) + (p8 - p6));
    const C sy = C(1.0 / 3.0) * (p2 - p4) + C(1.0 / 12.0) * ((p5 - p7) + (p6 - p8));
    const C fmx = -G * pc * sx;
    const C fmy = -G * pc * sy;
    const C fx = fmx;
    const C fy = fmy + C(P.gy * (rho - rho_bar));
    // Eq. Q / Q-psi-based
    const C kq2 = C(P.kappa * P.G * 0.5) * pc;
    const C dsum = (d5 + d6) + (d7 + d8);
    const C qxx = kq2 * (C(1.0 / 3.0) * (d1 + d3) + C(1.0 / 12.0) * dsum);
    const C qyy = kq2 * (C(1.0 / 3.0) * (d2 + d4) + C(1.0 / 12.0) * dsum);
    const C qxy = kq2 * (C(1.0 / 12.0) * ((d5 + d7) - (d6 + d8)));

    if (wb || wt) {
      // Zou-He reconstruction for the prescribed momentum -(F^m + F^b)/2,
      // the closure's buoyancy taken with rho_bar_k
      jxs = C(-0.5) * fmx;
      jys = C(-0.5) * (fmy + C(P.gy * (rho - rho_bar_k)));
      const C d = C(0.5) * (gp[1] - gp[3]);
      if (wb) {
        gp[2] = gp[4] + C(2.0 / 3.0) * jys;
        gp[5] = gp[7] - d + C(0.5) * jxs + jys * C(1.0 / 6.0);
        gp[6] = gp[8] + d - C(0.5) * jxs + jys * C(1.0 / 6.0);
      } else {
        gp[4] = gp[2] - C(2.0 / 3.0) * jys;
        gp[7] = gp[5] + d - C(0.5) * jxs - jys * C(1.0 / 6.0);
        gp[8] = gp[6] - d + C(0.5) * jxs - jys * C(1.0 / 6.0);
      }
    }
    const C inv_rho = rcp_c(C(rho));
    irho_out = inv_rho;
    const C uxd = (jxs + C(0.5) * fx) * inv_rho;
    const C uyd = (jys + C(0.5) * fy) * inv_rho;
    s_ux[kc][lane] = C(uxd);
    s_uy[kc][lane] = C(uyd);

    const bool inseg = s >= y0 && s < y1 && outlane;
    if (MODE == MODE_STEP && inseg) {
      // collision inputs in the compute type
      C ci[kColl];
#pragma unroll
      for (int i = 0; i < 9; ++i) ci[i] = gp[i];
      ci[9] = jxs;
      ci[10] = jys;
      ci[11] = C(uxd);
      ci[12] = C(uyd);
      ci[13] = C(fx);
      ci[14] = C(fy);
      ci[15] = C(rho);
      ci[16] = C(rho - rref);
      // sigma term 12 sigma |F^m|^2 / (psi^2 (tau - 1/2)) without the constant
      ci[17] = (fmx * fmx + fmy * fmy) * rcp_c(pc * pc);
      ci[18] = C(qxx + qyy);
      ci[19] = C(qxx - qyy);
      ci[20] = C(qxy);
      collide_store(ys, ci, rho);
    }
    if (MODE == MODE_MACRO && inseg) {
      const long long id = (long long)ys * nx + x;
      if (O.rho) O.rho[id] = rho;
      if (O.ux) O.ux[id] = uxd;
      if (O.uy) O.uy[id] = uyd;
      if (O.T) O.T[id] = double(s_T[kc][lane]);
      if (O.f) {
        const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        const long long N = (long long)nx * ny;
        for (int i = O.f_first; i < O.f_first + O.f_count; ++i)
          O.f[(long long)(i - O.f_first) * N + id] = double(gp[i]) + w[i] * rref;
      }
    }
  };

  // ------------------------------------------------------------ stage C(c)
  // RK2 stage temperature T* of a free node of the row in slot kc (rows in
  // slots km, kc, kq); fills the energy coefficients that stage D reuses
  auto stageC_core = [&](const int km, const int kc, const int kq, const C a1, const C a2,
                         const C irho, EnergyCoef<C>& ec) {
    const int kr[3] = {km, kc, kq};
    C phi[3][3], rr[3][3], uxn[3][3], uyn[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int sr = kr[dy];
      phi[dy][0] = s_T[sr][lm];
      phi[dy][1] = s_T[sr][lane];
      phi[dy][2] = s_T[sr][lp];
      if constexpr (kRhoC) {
        rr[dy][0] = s_rc[sr][lm];
        rr[dy][1] = s_rc[sr][lane];
        rr[dy][2] = s_rc[sr][lp];
      } else {
        rr[dy][0] = C(s_rho[sr][lm]);
        rr[dy][1] = C(s_rho[sr][lane]);
        rr[dy][2] = C(s_rho[sr][lp]);
      }
      uxn[dy][0] = s_ux[sr][lm];
      uxn[dy][1] = s_ux[sr][lane];
      uxn[dy][2] = s_ux[sr][lp];
      uyn[dy][0] = s_uy[sr][lm];
      uyn[dy][1] = s_uy[sr][lane];
      uyn[dy][2] = s_uy[sr][lp];
    }
    const C inv_rcv = irho * Q.inv_cv;
    const C lam0 = Q.lambda_v + Q.dlam * (rr[1][1] - Q.rho_v);
    ec.ux = uxn[1][1];
    ec.uy = uyn[1][1];
    ec.divu = gradx9(uxn) + grady9(uyn);
    ec.glx = Q.dlam * gradx9(rr);
    ec.gly = Q.dlam * grady9(rr);
    ec.lam_rcv = lam0 * inv_rcv;
    ec.inv_rcv = inv_rcv;
    const C dpdt_n = dpdt_at(a1, a2, phi[1][1], Q);
    const C Ts = phi[1][1] + C(0.5) * energy_rhs(phi, ec, dpdt_n);
    ec.dpdt_s = dpdt_at(a1, a2, Ts, Q);
    return Ts;
  };
  // stage C of row c (slot SC).  SEL (two-wave march): the free-node update
  // is evaluated on every lane and kept by a select, with no divergent
  // branch (512^2: float32 15.1 -> 14.2 us, float64 17.6 -> 16.6 us per step
  // on MI355X; in the one-wave march the select measured up to 2 % slower
  // on the 4096^2 pool, so it branches)
  auto stageC = [&](auto scc, auto selc, const int c, const C a1, const C a2, const C irho,
                    EnergyCoef<C>& ec_out) {
    constexpr bool SEL = decltype(selc)::value;
    const int SC = int(scc);
    const int km = (SC + R - 1) & (R - 1), kc = SC, kq = (SC + 1) & (R - 1);
    const bool have = WALLS ? (c >= 0 && c < ny) : true;
    if (!have) return;
    const int yc = WALLS ? c : wrapy(c);
    double tval;
    // ADIABATIC rows get tval here and are substituted by the reader
    if constexpr (SEL) {
      const int kind = node_kind_sel(yc, tval);
      EnergyCoef<C> ec;
      const C Tf = stageC_core(km, kc, kq, a1, a2, irho, ec);
      ec_out = ec;
      s_Ts[kc][lane] = kind == T_FREE ? Tf : C(tval);
    } else {
      const int kind = node_kind(yc, tval);
      C Ts;
      if (kind == T_FREE) {
        EnergyCoef<C> ec;
        Ts = stageC_core(km, kc, kq, a1, a2, irho, ec);
        ec_out = ec;
      } else {
        Ts = C(tval);
      }
      s_Ts[kc][lane] = Ts;
    }
  };

  // ------------------------------------------------------------ stage D(d)
  // new temperature of a free node of the row in slot kc (row index yd)
  auto stageD_core = [&](const int km, const int kc, const int kq, const int yd,
                         const EnergyCoef<C>& ec) {
    C phi[3][3];
    phi[0][0] = s_Ts[km][lm];
    phi[0][1] = s_Ts[km][lane];
    phi[0][2] = s_Ts[km][lp];
    phi[1][0] = s_Ts[kc][lm];
    phi[1][1] = s_Ts[kc][lane];
    phi[1][2] = s_Ts[kc][lp];
    phi[2][0] = s_Ts[kq][lm];
    phi[2][1] = s_Ts[kq][lane];
    phi[2][2] = s_Ts[kq][lp];
    // adiabatic rows 0 / ny-1 take the stage value of their neighbour row
    if (yd == 1) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double tv;
        if (row_kind(0, j, tv) == T_ADIABATIC) phi[0][j] = phi[1][j];
      }
    }
    if (yd == ny - 2) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double tv;
        if (row_kind(ny - 1, j, tv) == T_ADIABATIC) phi[2][j] = phi[1][j];
      }
    }
    const C T0 = s_T[kc][lane];
    return T0 + energy_rhs(phi, ec, ec.dpdt_s);
  };
  // store of a node's new temperature (deferred or not)
  auto store_T = [&](char* trow, const int yd, const S v) {
    if constexpr (DEFER) {
      dq_T = v;
      dq_Ton = true;
      dq_Trow = yd;
    } else {
      if constexpr (BUF)
        bstore(rs_Tout, ox, uint32_t(__builtin_amdgcn_readfirstlane(yd)) * rb32, v);
      else
        st(trow, ox, v);
    }
  };
  // adiabatic boundary rows copy the new value of their neighbour row
  auto adiabatic_copies = [&](const int yd, const S v) {
    double tv;
    if (yd == 1 && row_kind(0, 1, tv) == T_ADIABATIC) {
      if constexpr (BUF)
        bstore(rs_Tout, ox, 0u, v);
      else
        st(Tout, ox, v);
    }
    if (yd == ny - 2 && row_kind(ny - 1, 1, tv) == T_ADIABATIC) {
      if constexpr (BUF)
        bstore(rs_Tout, ox, uint32_t(ny - 1) * rb32, v);
      else
        st(Tout + size_t(ny - 1) * row_b, ox, v);
    }
  };
  // stage D of row d (slot SD), d inside the strip; SEL as in stage C.
  // DIRICHLET nodes store their value, ADIABATIC ones nothing.
  auto stageD = [&](auto sdc, auto selc, const int d, const EnergyCoef<C>& ec) {
    constexpr bool SEL = decltype(selc)::value;
    const int SD = int(sdc);
    const int km = (SD + R - 1) & (R - 1), kc = SD, kq = (SD + 1) & (R - 1);
    const int yd = d;
    char* trow = Tout + roff(__builtin_amdgcn_readfirstlane(yd));
    double tval;
    if constexpr (SEL) {
      const int kind = node_kind_sel(yd, tval);
      const bool fr = kind == T_FREE;
      const C Tnew = stageD_core(km, kc, kq, yd, ec);
      if (outlane && kind != T_ADIABATIC) {
        store_T(trow, yd, fr ? S(Tnew) : S(tval));
        if (fr) adiabatic_copies(yd, S(Tnew));
      }
    } else {
      const int kind = node_kind(yd, tval);
      if (kind == T_FREE) {
        const C Tnew = stageD_core(km, kc, kq, yd, ec);
        if (outlane) {
          store_T(trow, yd, S(Tnew));
          adiabatic_copies(yd, S(Tnew));
        }
      } else if (kind == T_DIRICHLET) {
        if (outlane) store_T(trow, yd, S(tval));
      }
    }
  };

  // one iteration: rows r_j = rbase + RPI k + j through stage A, then the
  // rows one, two and three behind through stages B, C and D
  auto body = [&](auto phc, const int k) {
    constexpr int PH = decltype(phc)::value;
    const int r0 = rbase + RPI * k;
    C g[RPI][9], Tr[RPI], jxc[RPI], jyc[RPI], a1c[RPI], a2c[RPI], irc[RPI];
    EnergyCoef<C> ecc[RPI];
#pragma unroll
    for (int j = 0; j < RPI; ++j) {
      Tr[j] = Tn[j];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[j][i] = gn[j][i];
      wall_mask(r0 + j, g[j]);
    }
    if constexpr (DEFER) {
      wait_vmem();
      flush_stores();
    }
#pragma unroll
    for (int j = 0; j < RPI; ++j)
      if (r0 + RPI + j < rend) load_row(r0 + RPI + j, gn[j], Tn[j]);
    static_for<RPI>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int S0 = (RPI * PH + j) & (R - 1);
      jxc[j] = jyc[j] = a1c[j] = a2c[j] = irc[j] = C(0);
      ecc[j] = EnergyCoef<C>{};
      if (r0 + j < rend) stageA(Ph<S0>{}, r0 + j, g[j], Tr[j], jxc[j], jyc[j], a1c[j], a2c[j]);
    });
    stage_barrier();
    if (WALLS) {
      static_for<RPI>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int S0 = (RPI * PH + j) & (R - 1), S1 = (S0 + R - 1) & (R - 1);
        const int r = r0 + j;
        if (r < rend) {
          if (r == 1 && 0 >= rbase) closure(Ph<S1>{}, Ph<S0>{}, true);
          if (r == ny - 1 && ny - 2 >= rbase && !outflow) closure(Ph<S0>{}, Ph<S1>{}, false);
        }
      });
      stage_barrier();
    }
    static_for<RPI>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int SB = (RPI * PH + j + R - 1) & (R - 1);
      const int s = r0 + j - 1;
      if (s >= rbase + 1 && s <= rend - 2) {
        if constexpr (j == 0)
          stageB(Ph<SB>{}, s, gprev, jxprev, jyprev, irc[j]);
        else
          stageB(Ph<SB>{}, s, g[j > 0 ? j - 1 : 0], jxc[j > 0 ? j - 1 : 0], jyc[j > 0 ? j - 1 : 0], irc[j]);
      }
    });
#pragma unroll
    for (int i = 0; i < 9; ++i) gprev[i] = g[RPI - 1][i];
    jxprev = jxc[RPI - 1];
    jyprev = jyc[RPI - 1];
    stage_barrier();
    if (MODE == MODE_STEP && THERMAL) {
      static_for<RPI>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int SC = (RPI * PH + j + R - 2) & (R - 1);
        const int c = r0 + j - 2;
        // EOS terms of row c: stage A two rows back; 1/rho: stage B one row back
        const C a1 = a1h[RPI == 2 ? j : 0], a2 = a2h[RPI == 2 ? j : 0];
        const C ir = j == 0 ? irprev : irc[j > 0 ? j - 1 : 0];
        if (c >= rbase + 2 && c <= rend - 3)
          stageC(Ph<SC>{}, std::false_type{}, c, a1, a2, ir, ecc[j]);
      });
      stage_barrier();
      static_for<RPI>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int SD = (RPI * PH + j + R - 3) & (R - 1);
        const int d = r0 + j - 3;
        if (d >= y0 && d < y1)
          stageD(Ph<SD>{}, std::false_type{}, d, j == 0 ? ecprev : ecc[j > 0 ? j - 1 : 0]);
      });
      stage_barrier();
    }
    // shift the rolling carries by RPI rows
    if constexpr (RPI == 2) {
      a1h[0] = a1c[0];
      a1h[1] = a1c[1];
      a2h[0] = a2c[0];
      a2h[1] = a2c[1];
    } else {
      a1h[0] = a1h[1];
      a1h[1] = a1c[0];
      a2h[0] = a2h[1];
      a2h[1] = a2c[0];
    }
    irprev = irc[RPI - 1];
    ecprev = ecc[RPI - 1];
  };

  if constexpr (!WS) {
    // the row loop, unrolled by 4 iterations so that every ring slot is a constant
    const int niter = (nit + RPI - 1) / RPI;
    for (int kb = 0; kb < niter; kb += 4) {
      body(Ph<0>{}, kb);
      if (kb + 1 < niter) body(Ph<1>{}, kb + 1);
      if (kb + 2 < niter) body(Ph<2>{}, kb + 2);
      if (kb + 3 < niter) body(Ph<3>{}, kb + 3);
    }
  } else {
    // two waves, one barrier per iteration; iteration k: wave 0 takes row
    // r = rbase + k through A and r - 1 through B; wave 1 takes r - 3 through
    // C and r - 4 through D, all of whose inputs wave 0 wrote in earlier
    // iterations.  Ring slot of row q: (q - rbase) & 7; in iteration k wave
    // 0 writes rows r, r - 1 while wave 1 reads rows >= r - 5.
    const int niter = nit + 1;
    // the loop is unrolled by the ring length, so that every ring slot is a
    // constant (LDS addresses become immediate offsets; 16.0 -> 15.1 us per
    // float32 step at 512^2 on MI355X, float64 18.6 -> 17.6 us)
    if constexpr (!TRIM) {
      // runtime ring slots (walls)
      if (wave == 0) {
        __builtin_amdgcn_s_setprio(2);
        for (int k = 0; k < niter; ++k) {
          const int r = rbase + k;
          const int sr = k & (R - 1), sr1 = (k + R - 1) & (R - 1);
          if (k < nit) {
            C g[9], jx, jy, a1, a2;
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = gn[0][i];
            wall_mask(r, g);
            const C Tr = Tn[0];
            if (r + 1 < rend) load_row(r + 1, gn[0], Tn[0]);
            stageA(sr, r, g, Tr, jx, jy, a1, a2);
            s_a1[sr][lane] = a1;
            s_a2[sr][lane] = a2;
            stage_barrier();
            if (WALLS) {
              if (r == 1 && 0 >= rbase) closure(sr1, sr, true);
              if (r == ny - 1 && ny - 2 >= rbase && !outflow) closure(sr, sr1, false);
              stage_barrier();
            }
            const int sB = r - 1;
            if (sB >= rbase + 1 && sB <= rend - 2) {
              C ir = C(0);
              stageB(sr1, sB, gprev, jxprev, jyprev, ir);
              s_ir[sr1][lane] = ir;
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) gprev[i] = g[i];
            jxprev = jx;
            jyprev = jy;
          }
          __syncthreads();
        }
      } else {
        EnergyCoef<C> ecw{};
        for (int k = 0; k < niter; ++k) {
          const int r = rbase + k;
          const int c = r - 3, d = r - 4;
          EnergyCoef<C> ecn{};
          if (c >= rbase + 2 && c <= rend - 3) {
            const int sc = (k + R - 3) & (R - 1);
            stageC(sc, std::true_type{}, c, s_a1[sc][lane], s_a2[sc][lane], s_ir[sc][lane], ecn);
          }
          stage_barrier();
          if (d >= y0 && d < y1) stageD((k + R - 4) & (R - 1), std::true_type{}, d, ecw);
          ecw = ecn;
          __syncthreads();
        }
      }
    } else if (wave == 0) {
      // wave 0 carries the longer chain (pull, EOS, forces, collision): it
      // goes first when waves of its SIMD compete for an issue slot (on
      // MI355X: float64 512^2 19.5 -> 18.6 us per step; batched 4 x 512^2
      // float32 26.7 -> 25.5 us; priority 3 measured the same as 2)
      __builtin_amdgcn_s_setprio(2);
      auto w0 = [&](auto phc, const int k) {
        constexpr int PH = decltype(phc)::value;
        constexpr int SR = PH, SR1 = (PH + R - 1) & (R - 1);
        constexpr int Q0 = PH & 3, Q1 = (PH + 1) & 3, QP = (PH + 3) & 3;  // rows r, r + 1, r - 1
        const int r = rbase + k;
        if (k < nit) {
          C jx, jy, a1, a2;
          stageA(Ph<SR>{}, r, gq[Q0], Tq[Q0], jx, jy, a1, a2);
          if (r + 1 < rend) load_row(r + 1, gq[Q1], Tq[Q1]);
          s_a1[SR][lane] = a1;
          s_a2[SR][lane] = a2;
          stage_barrier();
          if (WALLS) {
            if (r == 1 && 0 >= rbase) closure(Ph<SR1>{}, Ph<SR>{}, true);
            if (r == ny - 1 && ny - 2 >= rbase && !outflow) closure(Ph<SR>{}, Ph<SR1>{}, false);
            stage_barrier();
          }
          const int sB = r - 1;
          if (sB >= rbase + 1 && sB <= rend - 2) {
            C ir = C(0);
            stageB(Ph<SR1>{}, sB, gq[QP], jxprev, jyprev, ir);
            s_ir[SR1][lane] = ir;
          }
          jxprev = jx;
          jyprev = jy;
        }
        __syncthreads();
      };
      for (int kb = 0; kb < niter; kb += 8) {
        w0(Ph<0>{}, kb);
        if (kb + 1 < niter) w0(Ph<1>{}, kb + 1);
        if (kb + 2 < niter) w0(Ph<2>{}, kb + 2);
        if (kb + 3 < niter) w0(Ph<3>{}, kb + 3);
        if (kb + 4 < niter) w0(Ph<4>{}, kb + 4);
        if (kb + 5 < niter) w0(Ph<5>{}, kb + 5);
        if (kb + 6 < niter) w0(Ph<6>{}, kb + 6);
        if (kb + 7 < niter) w0(Ph<7>{}, kb + 7);
      }
    } else {
      EnergyCoef<C> ecw{};
      auto w1 = [&](auto phc, const int k) {
        constexpr int PH = decltype(phc)::value;
        constexpr int SC = (PH + R - 3) & (R - 1), SD = (PH + R - 4) & (R - 1);
        const int r = rbase + k;
        const int c = r - 3, d = r - 4;
        EnergyCoef<C> ecn{};
        if (c >= rbase + 2 && c <= rend - 3)
          stageC(Ph<SC>{}, std::true_type{}, c, s_a1[SC][lane], s_a2[SC][lane], s_ir[SC][lane], ecn);
        stage_barrier();
        if (d >= y0 && d < y1) stageD(Ph<SD>{}, std::true_type{}, d, ecw);
        ecw = ecn;
        __syncthreads();
      };
      for (int kb = 0; kb < niter; kb += 8) {
        w1(Ph<0>{}, kb);
        if (kb + 1 < niter) w1(Ph<1>{}, kb + 1);
        if (kb + 2 < niter) w1(Ph<2>{}, kb + 2);
        if (kb + 3 < niter) w1(Ph<3>{}, kb + 3);
        if (kb + 4 < niter) w1(Ph<4>{}, kb + 4);
        if (kb + 5 < niter) w1(Ph<5>{}, kb + 5);
        if (kb + 6 < niter) w1(Ph<6>{}, kb + 6);
        if (kb + 7 < niter) w1(Ph<7>{}, kb + 7);
      }
    }
  }

  if constexpr (DEFER) flush_stores();
  if (MODE == MODE_STEP && A.want_mass) {
    const double tot = wave_sum(mass_acc);
    if (lane == 0 && wave == 0) gst<GA>(A.part_out + bid, tot);
  }
  const unsigned long long any = __ballot(err != 0);
  if (any) {
    uint32_t e = err;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e |= __shfl_xor(e, off, kLanes);
    if (lane == 0) atomicOr(A.err, e);
  }
}

template <class S, class C, int WM, bool THERMAL, int MODE, bool BUF1>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(WavesPerEU<S>::value, 8)))
void lbm_march_kernel(StepArgs<S, C> A, MacroOut O) {
  march_body<S, C, WM, THERMAL, MODE, 1, false, false, BUF1>(A, O, blockIdx.x);
}

// the energy step with two waves per strip (see march_body)
template <class S, class C, int WM>
__global__ __launch_bounds__(2 * kLanes) __attribute__((amdgpu_waves_per_eu(WavesPerEU<S>::value, 8)))
void lbm_march2_kernel(StepArgs<S, C> A) {
  const MacroOut O{};
  march_body<S, C, WM, true, MODE_STEP, 1, true, false>(A, O, blockIdx.x);
}

// Batched launch over several lattices of one kind (same storage, walls and
// energy flags): workgroups [start[g], start[g+1]) serve lattice g, whose
// arguments are read from the descriptor table in device memory.  Each
// lattice's workgroup count is padded to a multiple of 8 so that the XCD of
// a workgroup is the same as in a single-lattice launch.
template <class S, class C, int WM, bool THERMAL>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(WavesPerEU<S>::value, 8)))
void lbm_march_multi_kernel(const StepArgs<S, C>* __restrict__ desc, const int* __restrict__ start,
                            int ngrid) {
  const int b = blockIdx.x;
  int g = 0;
  while (g + 1 < ngrid && b >= start[g + 1]) ++g;
  const MacroOut O{};
  // arguments read through the table and plain (flat) accesses: unlike the
  // two-wave kernel, this one ran slower with a local copy of the arguments
  // and with global-address accesses (finest mesh of the pool ladder, 4 x
  // 1024 x 2048 float32, 52-row strips: 213 us per step, 227 with the
  // global accesses, 241 with the copy as well, on MI355X)
  march_body<S, C, WM, THERMAL, MODE_STEP, 1, false, false>(desc[g], O, b - start[g]);
}

// the batched launch with two waves per strip (energy step; see march_body)
template <class S, class C, int WM>
__global__ __launch_bounds__(2 * kLanes) __attribute__((amdgpu_waves_per_eu(WavesPerEU<S>::value, 8)))
void lbm_march2_multi_kernel(const StepArgs<S, C>* __restrict__ desc, const int* __restrict__ start,
                             int ngrid) {
  const int b = blockIdx.x;
  int g = 0;
  while (g + 1 < ngrid && b >= start[g + 1]) ++g;
  const MacroOut O{};
  // a copy of the lattice's arguments: read through desc they were loaded
  // again at their uses inside the row loop (322 scalar loads, each with a
  // wait that also drains the LDS queue; 22 with the copy): 4 x 512^2
  // float32 27.5 -> 26.9 us per step on MI355X
  const StepArgs<S, C> a = desc[g];
  march_body<S, C, WM, true, MODE_STEP, 1, true, true>(a, O, b - start[g]);
}

// ------------------------------------------------------------- launchers
template <class C>
static PhysC<C> phys_c(const Phys& p) {
  PhysC<C> q{};
  q.s_e = C(p.s_e);
  q.s_z = C(p.s_z);
  q.s_q = C(p.s_q);
  q.snu_const = C(1.0 / (3.0 * p.eta_v + 0.5));
  q.eta_l = C(p.eta_l);
  q.eta_v = C(p.eta_v);
  q.rho_v = C(p.rho_v);
  q.inv_drho = C(p.inv_drho);
  q.lambda_v = C(p.lambda_v);
  q.dlam = C(p.dlam);
  q.inv_cv = C(1.0 / p.cv);
  q.kw = C(p.kw);
  q.inv_sqrtTc = C(p.inv_sqrtTc);
  q.akw_isTc = C(p.akw_isTc);
  q.snu_varies = p.eta_l != p.eta_v;
  return q;
}

template <class S, class C, int WM, bool THERMAL, int MODE>
static void launch_one(const StepArgs<S, C>& a, const MacroOut& o, int nblocks, bool buf,
                       hipStream_t st) {
  // (the energy step only: the isothermal kernel with walls needed more
  // registers with buffers, 121 -> 130 VGPRs, one wave per SIMD fewer)
  if constexpr (sizeof(S) == 4 && MODE == MODE_STEP && THERMAL) {
    if (buf) {
      hipLaunchKernelGGL((lbm_march_kernel<S, C, WM, THERMAL, MODE, true>), dim3(nblocks), dim3(kLanes), 0,
                         st, a, o);
      return;
    }
  }
  hipLaunchKernelGGL((lbm_march_kernel<S, C, WM, THERMAL, MODE, false>), dim3(nblocks), dim3(kLanes), 0,
                     st, a, o);
}

// wall mode of a lattice: 0 periodic, 1 psi-based walls, 2 walls with the
// modified-psi model or the outflow top
static int wall_mode(int walls, const Phys& ph) {
  return walls ? ((ph.wall_mod || ph.outflow_top) ? 2 : 1) : 0;
}

template <class S, class C, bool THERMAL, int MODE>
static void launch_wm(int wm, const StepArgs<S, C>& a, const MacroOut& o, int nblocks, bool buf,
                      hipStream_t st) {
  if (wm == 2) launch_one<S, C, 2, THERMAL, MODE>(a, o, nblocks, buf, st);
  else if (wm == 1) launch_one<S, C, 1, THERMAL, MODE>(a, o, nblocks, buf, st);
  else launch_one<S, C, 0, THERMAL, MODE>(a, o, nblocks, buf, st);
}

template <class S, class C>
static StepArgs<S, C> make_args(const LaunchStep& L) {
  StepArgs<S, C> a{};
  a.fin = static_cast<const S*>(L.fin);
  a.fout = static_cast<S*>(L.fout);
  a.Tin = static_cast<const S*>(L.Tin);
  a.Tout = static_cast<S*>(L.Tout);
  a.tabd = L.tab.rho_w_b;
  a.tabk = L.tab.tk_b;
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
  a.ntx = L.ntx;
  a.nty = L.nty;
  a.halo = L.halo;
  a.side_dir = L.side_dir;
  a.want_mass = L.want_mass;
  a.xcd_remap = L.xcd_remap;
  a.ph = L.ph;
  a.pc = phys_c<C>(L.ph);
  return a;
}

template <class S, class C>
static hipError_t launch_step_t(const LaunchStep& L, hipStream_t st, int mode) {
  const StepArgs<S, C> a = make_args<S, C>(L);
  MacroOut o{L.o_rho, L.o_ux, L.o_uy, L.o_T, L.o_f, L.f_first, L.f_count};
  const int nb = L.ntx * L.nty;
  const int wm = wall_mode(L.walls, L.ph);
  // one-wave float32 step: buffer accesses where the 9 planes fit 4 GiB
  const bool buf = L.fp32 && arrays_fit_32bit(L.plane, 4);
  if (mode == MODE_MACRO) {
    launch_wm<S, C, false, MODE_MACRO>(wm, a, o, nb, false, st);
  } else if (L.update_T && L.waves == 2 && two_wave_fits(L.plane, L.fp32 ? 4 : 8, L.ny)) {
    if (wm == 2)
      hipLaunchKernelGGL((lbm_march2_kernel<S, C, 2>), dim3(nb), dim3(2 * kLanes), 0, st, a);
    else if (wm == 1)
      hipLaunchKernelGGL((lbm_march2_kernel<S, C, 1>), dim3(nb), dim3(2 * kLanes), 0, st, a);
    else
      hipLaunchKernelGGL((lbm_march2_kernel<S, C, 0>), dim3(nb), dim3(2 * kLanes), 0, st, a);
  } else if (L.update_T) {
    launch_wm<S, C, true, MODE_STEP>(wm, a, o, nb, buf, st);
  } else {
    launch_wm<S, C, false, MODE_STEP>(wm, a, o, nb, false, st);
  }
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

size_t step_desc_bytes(int fp32) {
  return fp32 ? sizeof(StepArgs<float, float>) : sizeof(StepArgs<double, double>);
}

void fill_step_desc(const LaunchStep& L, void* out) {
  if (L.fp32) {
    const StepArgs<float, float> a = make_args<float, float>(L);
    std::memcpy(out, &a, sizeof a);
  } else {
    const StepArgs<double, double> a = make_args<double, double>(L);
    std::memcpy(out, &a, sizeof a);
  }
}

template <class S, class C, int WM, bool THERMAL>
static void launch_multi_t(const void* desc, const int* start, int ngrid, int nblocks, int waves,
                           hipStream_t st) {
  if (THERMAL && waves == 2)
    hipLaunchKernelGGL((lbm_march2_multi_kernel<S, C, WM>), dim3(nblocks), dim3(2 * kLanes), 0, st,
                       static_cast<const StepArgs<S, C>*>(desc), start, ngrid);
  else
    hipLaunchKernelGGL((lbm_march_multi_kernel<S, C, WM, THERMAL>), dim3(nblocks), dim3(kLanes), 0, st,
                       static_cast<const StepArgs<S, C>*>(desc), start, ngrid);
}

template <class S, class C>
static void launch_multi_s(int wm, int thermal, const void* desc, const int* start, int ngrid,
                           int nblocks, int waves, hipStream_t st) {
  if (wm == 2) {
    if (thermal) launch_multi_t<S, C, 2, true>(desc, start, ngrid, nblocks, waves, st);
    else launch_multi_t<S, C, 2, false>(desc, start, ngrid, nblocks, waves, st);
  } else if (wm == 1) {
    if (thermal) launch_multi_t<S, C, 1, true>(desc, start, ngrid, nblocks, waves, st);
    else launch_multi_t<S, C, 1, false>(desc, start, ngrid, nblocks, waves, st);
  } else {
    if (thermal) launch_multi_t<S, C, 0, true>(desc, start, ngrid, nblocks, waves, st);
    else launch_multi_t<S, C, 0, false>(desc, start, ngrid, nblocks, waves, st);
  }
}

hipError_t launch_step_multi(int fp32, int wall_mode, int thermal, int waves, const void* desc,
                             const int* start, int ngrid, int nblocks, hipStream_t st) {
  if (fp32) launch_multi_s<float, float>(wall_mode, thermal, desc, start, ngrid, nblocks, waves, st);
  else launch_multi_s<double, double>(wall_mode, thermal, desc, start, ngrid, nblocks, waves, st);
  return hipGetLastError();
}

}  // namespace lbm
