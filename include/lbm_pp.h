/*
 * lbm_pp.h -- C-ABI of the MI355X (gfx950) library that advances the
 * pseudopotential lattice-Boltzmann model of liquid-vapour phase change of
 * Jaramillo, Mapelli & Cabezas-Gomez, "Pseudopotential Lattice Boltzmann
 * Method for boiling heat transfer: a mesh refinement procedure".
 *
 * One time step (Sec. 2 of the paper) on an nx x ny D2Q9 lattice:
 *   moments (Eq. DensityAndVelocityRelationToF), Peng-Robinson EOS and
 *   pseudopotential (Eqs. peng-robinson, psi), interaction, adhesion and
 *   buoyancy forces (Eqs. shanchen, psi-based-formula, shanchen-walls,
 *   gravitational_force), the Li forcing and surface-tension terms S, C, Q
 *   (Eqs. li_source_terms, S, C, Q, Q-psi-based), MRT collision
 *   (Eq. collisionMRT), streaming with wet-node Zou-He walls (Sec. 2.2),
 *   and the explicit RK2 update of the energy equation (Eq. energy-equation).
 * Host helpers cover the mesh-refinement parameter rules of Sec. 3
 * (Eq. a-deltax, Eq. integral_coexistence_curve, Eq. surface_tension).
 *
 * Conventions
 *  - Every function returns lbm_status; nothing aborts or throws across the
 *    ABI.  A failing call leaves the context usable unless stated.
 *  - Device memory is owned by the caller: lbm_buffer_bytes() gives the size
 *    of ONE device allocation that lbm_create() borrows until lbm_destroy().
 *    The library itself allocates no device memory.
 *  - All device work is enqueued on the HIP stream given to lbm_create()
 *    (NULL = the default stream).  lbm_step() is asynchronous; calls that
 *    return host data synchronise that stream.  Device-side domain errors
 *    (density outside (0, 1/b), psi radicand <= 0, T <= 0, NaN) are sticky
 *    and reported as LBM_E_DOMAIN by the next synchronising call.
 *  - Host arrays are row-major [ny][nx] (x fastest), y = 0 is the bottom
 *    row, and are float64 whatever the storage precision.  They are only
 *    read or written during the call.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_PP_H
#define LBM_PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVAL = 1,       /* bad argument or parameter set */
  LBM_E_NOMEM = 2,       /* caller buffer too small, host allocation failed */
  LBM_E_HIP = 3,         /* HIP runtime error (text in lbm_last_error) */
  LBM_E_STATE = 4,       /* call out of order (e.g. step before init) */
  LBM_E_DOMAIN = 5,      /* state left the EOS / pseudopotential domain */
  LBM_E_UNSUPPORTED = 6, /* valid request the library does not implement */
  /* range sentinels, never returned: every int32 value is an lbm_status, so
   * lbm_status_string() may be given any code a caller holds */
  LBM_STATUS_MIN_ = -0x7fffffff - 1,
  LBM_STATUS_MAX_ = 0x7fffffff
} lbm_status;

enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1 };          /* storage precision */
enum { LBM_T_FREE = 0, LBM_T_DIRICHLET = 1, LBM_T_ADIABATIC = 2 };
/* contact-angle model of the walls (Sec. 2.2) */
enum { LBM_WALL_PSI_BASED = 0, LBM_WALL_MODIFIED_PSI = 1 };

/* All quantities in lattice units.  lbm_default_params() fills the values
 * used by the paper's droplet runs (Sec. 4.1) on the ladder EOS a = 2/49. */
typedef struct lbm_params {
  int32_t nx, ny;
  int32_t precision;   /* LBM_FP64 or LBM_FP32_SHIFTED (populations stored
                          as f_i - w_i rho_ref, collision in float32, EOS,
                          psi and forces in float64) */
  int32_t walls;       /* 0: periodic in y; 1: wet-node Zou-He walls on rows
                          0 and ny-1 (x is always periodic) */
  int32_t thermal;     /* 1: solve the energy equation */
  int32_t n_iso;       /* the first n_iso steps keep T frozen (Sec. 4.1) */
  int32_t t_side_dirichlet; /* 1: columns 0 and nx-1 held at t_side_val */
  int32_t tile_y;      /* rows per workgroup strip; 0 = library default: 5 on
                          small lattices, else the smallest height whose launch
                          fits 3 (float32) / 2 (float64) waves per SIMD of the
                          buffer's device */
  double a, b, R, omega, G;      /* Eq. peng-robinson, Eq. psi (G = -1) */
  double sigma, kappa;           /* Eqs. S and Q */
  double s_rho, s_e, s_zeta, s_j, s_q;   /* MRT rates; s_nu from eta(rho) */
  double eta_l, eta_v;           /* Eq. eta-rho: viscosities of both phases */
  double rho_l, rho_v;           /* phase densities used by eta(rho), lambda(rho) */
  double gy;                     /* gravity along +y (Eq. gravitational_force) */
  double cv, lambda_l, lambda_v; /* Sec. 2.3 */
  double t_side_val;
  double rho_ref;                /* shift of the float32 storage */
  int32_t xcd_remap;             /* 1: keep neighbouring tiles on one XCD */
  int32_t strip_waves;           /* waves per strip of the energy step: 1, 2, or 0 = by lattice
                                    size (2 on lattices with fewer than 2048 five-row strips) */
  int32_t wall_model;            /* LBM_WALL_PSI_BASED: adhesion of Eq. psi-based-formula with
                                    the per-column wall densities rho_w, Q of Eq. Q-psi-based;
                                    LBM_WALL_MODIFIED_PSI: adhesion of Eq. mod-psi-based-formula
                                    with per-column strengths G_w, Q of Eq. Q-mod-psi-based.
                                    Either way the Zou-He closure imposes zero fluid velocity
                                    with the chosen F^m and the buoyancy F^b taken with the
                                    mean density whose wall nodes are at their known parts
                                    (wall density from a Newton solve) */
  int32_t outflow_top;           /* 1: row ny-1 is a zero-gradient outflow (the open end of the
                                    1-D boiling problem, Sec. 4.2) instead of a wall: its
                                    populations entering from above are those of row ny-2, psi
                                    above it is its own, its temperature kind must be ADIABATIC
                                    or DIRICHLET; needs walls = 1 and gy = 0
                                    (LBM_E_UNSUPPORTED otherwise) */
  int32_t reserved_i[4];
  double reserved_d[8];
} lbm_params;

typedef struct lbm_norms_t {
  double mass;        /* sum of rho over all nodes */
  double rho_mean;
  double umax;        /* max |u| */
  double q_bottom;    /* wall heat flux of Eq. pool-heat-flux: (1/nx) sum_x
                         lambda(rho) dT/dy at y = 0 with the one-sided
                         second-order difference (-3 T0 + 4 T1 - T2)/2;
                         ADIABATIC bottom nodes carry no flux and add 0;
                         0 unless walls */
  double q_heater;    /* mean of lambda dT/dy over the held (DIRICHLET)
                         bottom nodes, the side columns included when they
                         are held: the heater flux of a heated strip whose
                         surroundings are adiabatic; 0 if there are none */
  double l1_rho, l2_rho, linf_rho;   /* discrete norms of rho: mean |rho|,
                                        rms, max |rho| */
  double l1_T, l2_T, linf_T;         /* the same for T */
  int64_t nonfinite;  /* nodes whose rho, u or T is not finite (left out of
                         every other field) */
  int64_t n_heater;   /* number of nodes averaged in q_heater */
  int64_t step;
} lbm_norms_t;

const char* lbm_status_string(lbm_status s);
/* Text of the last error on this context (or of the last failed create when
 * ctx is NULL).  Valid until the next call on the same context. */
const char* lbm_last_error(const lbm_ctx* ctx);

void lbm_default_params(lbm_params* p, int32_t nx, int32_t ny);
/* Check a parameter set without touching the GPU.  LBM_E_INVAL if nx or ny
 * < 1, walls with ny < 3, a, b <= 0, a rate outside (0, 2), thermal with
 * cv <= 0 or negative conductivities, rho_l == rho_v, or an unknown precision. */
lbm_status lbm_validate(const lbm_params* p);
/* Size in bytes of the device buffer lbm_create() needs for p. */
lbm_status lbm_buffer_bytes(const lbm_params* p, size_t* bytes);

/* Borrow dev_buf (>= lbm_buffer_bytes, any alignment >= 256 B) on hip_stream
 * (a hipStream_t, may be NULL).  The device must be current.  On success
 * *out owns host state only; lbm_destroy() releases it. */
lbm_status lbm_create(const lbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                      lbm_ctx** out);
void lbm_destroy(lbm_ctx* ctx);

/* Per-column boundary tables, host arrays of nx entries; NULL keeps the
 * current table (defaults: rho_w = 1 or G_w = G, T kinds FREE, values 0).
 * rho_w_*: the wall tables of rows 0 and ny-1: with LBM_WALL_PSI_BASED the
 * wall densities rho_w(x) of Eq. psi-based-formula (inside the EOS domain,
 * else the next step reports LBM_E_DOMAIN), with LBM_WALL_MODIFIED_PSI the
 * adhesion strengths G_w(x) of Eq. mod-psi-based-formula; non-finite
 * entries are rejected with LBM_E_INVAL.  t_*_kind / t_*_val: temperature
 * condition of rows 0 and ny-1 (FREE, DIRICHLET value, or ADIABATIC = copy
 * of the adjacent row after each RK stage).  Must precede lbm_init_fields()
 * to take effect at init. */
lbm_status lbm_set_boundary(lbm_ctx* ctx, const double* rho_w_bottom, const double* rho_w_top,
                            const int32_t* t_bottom_kind, const double* t_bottom_val,
                            const int32_t* t_top_kind, const double* t_top_val);

/* Initial state: f_i = f_i^eq(rho, u) (Eq. EquilibriumDistribution) and T
 * as given, then (thermal runs) the DIRICHLET values of the boundary tables
 * applied.  rho and T are required; ux, uy may be NULL (zero).  Resets the
 * step counter.  Synchronises. */
lbm_status lbm_init_fields(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy,
                           const double* T);

/* Advance nsteps >= 0 time steps; asynchronous on the context stream. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* rho, u = (sum f c + F/2)/rho and T at the current step (any pointer may
 * be NULL).  Synchronises. */
lbm_status lbm_read_fields(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* T);
/* Populations f_i at the current step after the wall closure, host array
 * [9][ny][nx] in the paper's velocity order.  Synchronises. */
lbm_status lbm_read_populations(lbm_ctx* ctx, double* f);
/* Global diagnostics (fixed-order float64 reductions).  Synchronises. */
lbm_status lbm_norms(lbm_ctx* ctx, lbm_norms_t* out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the diagnostics of
 * lbm_norms() written as one lbm_norms_t into device memory (dev_out,
 * 8-byte aligned, caller-owned), enqueued on the context stream without
 * synchronising and without any host or device allocation.  Its reduction
 * keeps the per-workgroup partial sums in a fixed library array of 48 KiB
 * per GPU (512 workgroups x 12 sums; the reduction never uses more, so every
 * lattice size fits), held until the process ends; the read-out stages
 * rho, u, T in the context's idle population buffer, as lbm_norms() does.
 * The values equal lbm_norms()'s (same partial sums, same final order);
 * `step` is the host's count when the call is enqueued.  Calls that overlap
 * on one GPU (contexts on different streams) share that array and race:
 * order them on one stream or by events.  Device errors stay sticky and are
 * reported by the next synchronising call. */
lbm_status lbm_norms_device(lbm_ctx* ctx, lbm_norms_t* dev_out);

/* Checkpoint: raw storage of the populations, T and the step counter. */
lbm_status lbm_state_bytes(const lbm_ctx* ctx, size_t* bytes);
lbm_status lbm_save_state(lbm_ctx* ctx, void* host, size_t bytes);
lbm_status lbm_load_state(lbm_ctx* ctx, const void* host, size_t bytes);

/* Rows per workgroup strip of the step kernel (>= 2).  The result of a step
 * does not depend on it (bitwise without gravity; rho_bar's summation order
 * changes with it otherwise). */
lbm_status lbm_set_tile_y(lbm_ctx* ctx, int32_t tile_y);
int32_t lbm_get_tile_y(const lbm_ctx* ctx);
/* Waves marching each strip in the energy step: 1 (one wave, all stages),
 * 2 (a second wave takes the RK2 stages one row behind), 0 = by lattice
 * size.  Identical results; a performance choice.  2 applies while the 9
 * population planes span less than 4 GiB and ny >= 3 (other lattices run
 * one wave).
 * get returns the effective value. */
lbm_status lbm_set_strip_waves(lbm_ctx* ctx, int32_t waves);
int32_t lbm_get_strip_waves(const lbm_ctx* ctx);

/* Wait for the context stream; report sticky device errors. */
lbm_status lbm_sync(lbm_ctx* ctx);
int64_t lbm_step_count(const lbm_ctx* ctx);

/* Device time (milliseconds) of the last lbm_step() call, measured with HIP
 * events recorded on the context stream around its launches.  Waits for the
 * second event. */
lbm_status lbm_last_step_time(lbm_ctx* ctx, double* total_ms);
/* Per-launch timing of the step kernel: while enabled, every step-kernel
 * launch of lbm_step() is bracketed by a pair of HIP events on the context
 * stream (the event pool grows on the host as needed).  lbm_kernel_times()
 * waits for the recorded events, returns the sum of the kernel spans (ms)
 * and their number, and clears the record.  Enabling also clears it. */
lbm_status lbm_kernel_timing(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_kernel_times(lbm_ctx* ctx, double* sum_ms, int64_t* count);

/* ---- batches of lattices: the mesh-refinement ladder (Sec. 3) ----------- */
typedef struct lbm_batch lbm_batch;
/* Device bytes of the argument tables of a batch (up to 64 lattices and 64
 * distinct launch configurations per run). */
lbm_status lbm_batch_bytes(int32_t precision, size_t* bytes);
/* Group n (1..64) created and initialised contexts of one precision and one
 * wall setting.  The contexts keep their buffers and stay usable on their
 * own; dev_buf (>= lbm_batch_bytes, 256-byte aligned, caller-owned) holds the
 * argument tables.  Work is ordered after / before the caller's hip_stream by
 * events; the batch captures graphs on a stream of its own. */
lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, void* dev_buf, size_t bytes,
                            void* hip_stream, lbm_batch** out);
void lbm_batch_destroy(lbm_batch* b);
const char* lbm_batch_last_error(const lbm_batch* b);
/* Advance lattice g by steps[g] time steps: launch t advances every lattice
 * with t < steps[g] in one multi-lattice kernel launch (the coarse levels run
 * beside the fine ones).  use_graph != 0: repeated launch pairs are captured
 * into a hipGraph once and replayed.  The result equals lbm_step() on each
 * context (same kernels, same arithmetic).  Asynchronous. */
lbm_status lbm_batch_run(lbm_batch* b, const int64_t* steps, int32_t use_graph);
/* Plan the schedule lbm_batch_run(b, steps, use_graph) would run from the
 * lattices' current states, upload its argument tables and capture (and
 * instantiate) its graphs, without launching anything or advancing a
 * lattice: the run that follows replays them at once.  A batch keeps its
 * instantiated graphs until lbm_batch_destroy() and re-uploads only tables
 * whose content changed, so repeated runs of one schedule need neither. */
lbm_status lbm_batch_prepare(lbm_batch* b, const int64_t* steps, int32_t use_graph);
/* Device time of the last run (HIP events), number of step launches it
 * covered and of graph launches used.  Waits for the run. */
lbm_status lbm_batch_last_time(lbm_batch* b, double* ms, int64_t* kernel_launches,
                               int64_t* graph_launches);

/* Tile-height autotuner: times `steps` steps (after 2 warm-up steps) for each
 * candidate tile_y with HIP events and keeps the fastest.  Advances the
 * context's state by n * (steps + 2) steps, so run it on a throwaway context
 * initialised like the real one. */
lbm_status lbm_autotune_tile_y(lbm_ctx* ctx, const int32_t* candidates, int32_t n, int32_t steps,
                               int32_t* best_tile_y, double* best_ms_per_step);
/* Strip heights that fill whole rounds of wave slots on the context's GPU:
 * for m = 1..16 waves per SIMD (4 SIMDs per compute unit), the smallest
 * tile_y whose launch of column tiles x strips x waves (waves per strip;
 * 0 = the context's current setting) fits in m x 4 x compute units.  A
 * launch just under such a multiple leaves no SIMD with one wave more than
 * the others.  Ascending, distinct, each in [2, max(ny, 2)].  Writes
 * min(count, cap) heights to out (out may be NULL with cap 0) and the count
 * to *count.  LBM_E_INVAL for a null ctx or count, waves outside 0..2 or a
 * negative cap; LBM_E_HIP if the device cannot be queried.  Host only; no
 * GPU work. */
lbm_status lbm_tile_candidates(const lbm_ctx* ctx, int32_t waves, int32_t* out, int32_t cap,
                               int32_t* count);

/* ---- host parameter pipeline (Sec. 3); float64, no GPU ----------------- */
/* T_c of Eq. peng-robinson's a = 0.45724 R^2 T_c^2/p_c, b = 0.0778 R T_c/p_c */
double lbm_pr_critical_temperature(double a, double b, double R);
/* Maxwell coexistence of the EOS at temperature T. */
lbm_status lbm_pr_maxwell(double a, double b, double R, double omega, double T,
                          double* rho_v, double* rho_l, double* p_sat);
/* sigma solving Eq. integral_coexistence_curve at the Maxwell densities
 * (secant from -16 G sigma_0 = 2). */
lbm_status lbm_fit_sigma(double a, double b, double R, double omega, double G, double T,
                         double* sigma);
/* Planar surface tension of Eq. surface_tension for kappa = 0 from the
 * continuum profile of the normal balance. */
lbm_status lbm_planar_gamma(double a, double b, double R, double omega, double G, double T,
                            double sigma, double* gamma0);
/* Latent heat of vaporisation h_fg of the EOS at temperature T (Sec. 4.2,
 * the h_fg of Eq. stefan-analytical and of the Jakob number Ja =
 * c_v (T_w - T_sat) / h_fg): the integral of T (dp/dT)_rho / rho^2 over
 * [rho_v, rho_l], evaluated in closed form for Eq. peng-robinson.  rho_v,
 * rho_l: the coexistence densities at T (lbm_pr_maxwell).  LBM_E_INVAL for
 * non-positive a, b, R or T, T >= T_c, rho_l <= rho_v <= 0, b rho_l >= 1, a
 * null h_fg or a non-finite result. */
lbm_status lbm_pr_latent_heat(double a, double b, double R, double omega, double T, double rho_v,
                              double rho_l, double* h_fg);
/* beta of Eq. stefan-analytical: the root of
 * sqrt(pi) beta exp(beta^2) erf(beta) = Ja (Ja = c_v (T_w - T_sat) / h_fg >= 0),
 * by bisection to the last bits.  LBM_E_INVAL for a negative or non-finite
 * Ja or a null beta. */
lbm_status lbm_stefan_beta(double ja, double* beta);

/* ---- reverse mode: heater-profile gradient (Sec. 2 step, Sec. 4) --------
 * Objective: evaporated liquid mass J = M_l(start) - M_l(end) over nsteps
 * steps, M_l = sum_x rho H(rho), H(rho) = (1 + tanh((rho - rho_mid)/width))/2,
 * rho the density a step reads (pull-streamed populations, Eq.
 * DensityAndVelocityRelationToF).  Gradient with respect to the bottom-row
 * Dirichlet temperatures t_bottom_val[x] (entries overridden by the side
 * columns or not DIRICHLET get 0).
 * Scope: periodic lattices (walls = 0) without gravity (gy = 0) with the
 * energy equation on (thermal = 1); otherwise LBM_E_UNSUPPORTED.
 * The forward pass runs the fused step on the context and stores a
 * checkpoint every ckpt_every steps in dev_buf (caller-owned, 256-byte
 * aligned, >= lbm_adjoint_bytes; it also holds two sets of ckpt_every
 * recomputed states with 13 float64 forward fields per node and step, and
 * the float64 adjoint fields).  The backward pass recomputes each segment with
 * the same kernel (identical trajectory) and each step's forward quantities
 * from its state, the next segment on a stream of the adjoint's own while the
 * current one is reversed step by step on the context stream; it leaves the
 * context at the end state of the forward pass. */
typedef struct lbm_adjoint lbm_adjoint;
lbm_status lbm_adjoint_bytes(const lbm_params* p, int32_t nsteps, int32_t ckpt_every, size_t* bytes);
lbm_status lbm_adjoint_create(lbm_ctx* ctx, int32_t nsteps, int32_t ckpt_every, double rho_mid, double width,
                              void* dev_buf, size_t bytes, lbm_adjoint** out);
void lbm_adjoint_destroy(lbm_adjoint* a);
/* Advance ctx (initialised) by nsteps from its current state; J on the host. */
lbm_status lbm_adjoint_forward(lbm_adjoint* a, double* J);
/* grad_t_bottom (host, nx doubles) = dJ * dJ/dt_bottom_val.  Needs a
 * forward pass first; may be called again for another dJ.  LBM_E_STATE if
 * the context was stepped, re-initialised, given new boundary tables, loaded
 * from a saved state or run in a batch since that forward pass (the gradient
 * would belong to another trajectory). */
lbm_status lbm_adjoint_backward(lbm_adjoint* a, double dJ, double* grad_t_bottom);
/* Host wall-clock milliseconds of the last forward and backward passes. */
lbm_status lbm_adjoint_timing(const lbm_adjoint* a, double* forward_ms, double* backward_ms);

/* One mesh of the refinement procedure (Sec. 3) relative to the base mesh
 * (dx = dx_mesh / dx_base, e.g. 1/2 for a twice finer mesh):
 *   a = a_base dx^2 (Eq. a-deltax), T = Tr T_c(a), Maxwell densities,
 *   sigma from Eq. integral_coexistence_curve,
 *   kappa from Eq. gamma-meshes-relation with gamma = (1 - kappa) gamma_0
 *   (Eq. surface_tension, continuum planar profile), base kappa = kappa0,
 *   g = gy0 dx^3 (Table 1), steps = steps0 / dx^2 (viscous regime). */
typedef struct lbm_level {
  double dx, a, Tc, T, rho_v, rho_l, p_sat, sigma, kappa, gamma, gy;
  int64_t steps;
} lbm_level;
lbm_status lbm_refinement_level(double a_base, double dx, double Tr, double b, double R, double omega,
                                double G, double kappa0, double gy0, int64_t steps0, lbm_level* out);

#ifdef __cplusplus
}
#endif
#endif /* LBM_PP_H */
