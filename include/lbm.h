/*
 * lbm.h -- C ABI of the MI355X (gfx950) conservative phase-field lattice
 * Boltzmann library (arXiv 2505.12205).
 *
 * The library advances two population sets on D2Q9 or D3Q19:
 *   h -- phase-field populations of the conservative Allen-Cahn equation
 *        (the paper's "LBE for interface tracking", Eqs. lbe_interface,
 *        forcing_term, equilibrium_with_force, equilibrium_function);
 *   g -- pressure/velocity populations with the weighted-MRT collision
 *        (the paper's "LBE for hydrodynamics", Eqs. lbe_standard,
 *        equilibrium_modified, equilibrium, force_term, total_force,
 *        pressure_force, viscous_force_wmrt, mrt_collision, appendix A),
 * coupled through the isotropic finite differences of phi (Eqs. gradient_phi,
 * laplacian_phi), the chemical potential and surface tension (Eqs.
 * chemical_potential, beta_kappa_relation, surface_tension_force) and the
 * boundary treatments of appendix B.  One step is [macroscopic update ->
 * collision -> streaming -> boundary conditions].
 *
 * Conventions
 *   - Every pointer named *_dev is a device pointer on the current HIP device;
 *     every other pointer is a host pointer.
 *   - Field layout: x fastest, node = x + nx*(y + ny*z); vector fields are
 *     planar, u[d*N + node] (d = 0..2; the z plane is present and zero in 2D).
 *   - Population layout of exported/imported states: pop[a*N + node] with the
 *     velocity order of appendix A.
 *   - All launches go to the stream given at init; no call allocates or
 *     synchronises unless documented.  A handle must be used by one host
 *     thread at a time.
 *   - Return value: LBM_OK (0) or a negative LBM_E* code; lbm_last_error()
 *     then holds a message (thread-local).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)      /* bad argument or parameter set */
#define LBM_ENOMEM (-2)      /* state buffer too small / library scratch allocation failed */
#define LBM_EDEVICE (-3)     /* a HIP call failed; message holds hipGetErrorString */
#define LBM_EUNSTABLE (-4)   /* a reduction found a non-finite value */
#define LBM_EUNSUPPORTED (-5)/* valid but not implemented combination */

typedef enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19 } lbm_lattice;

/* Face boundary types (appendix B).  Faces are indexed -x,+x,-y,+y,-z,+z.
 * PERIODIC must be paired on both faces of an axis.  VELOCITY_INLET is
 * supported on the -z face of D3Q19 domains and the -y face of D2Q9 domains;
 * CONVECTIVE_OUTLET on the opposite face. */
typedef enum {
  LBM_BC_PERIODIC = 0,
  LBM_BC_NOSLIP = 1,            /* halfway bounce-back, both sets */
  LBM_BC_FREESLIP = 2,          /* halfway specular reflection, both sets */
  LBM_BC_VELOCITY_INLET = 3,    /* circular plug nozzle, non-equilibrium bounce-back */
  LBM_BC_CONVECTIVE_OUTLET = 4  /* first-order implicit convective outflow */
} lbm_bc;

/* Population storage.  FP32 stores populations as they are.  The 16-bit
 * forms store deviations from the lattice-weight rest value, decoded to FP32
 * in registers: g_a / w_a, and (h_a - w_a phi_ref) / w_a with phi_ref the
 * phase field, at the step the value was written, of the node that reads it
 * (the node it streams into). */
typedef enum { LBM_FP32 = 0, LBM_FP16_DEV = 1, LBM_BF16_DEV = 2 } lbm_storage;

/* Body force: rho g (Poiseuille channel) or (rho - rho_L) g (jets). */
typedef enum { LBM_FB_RHO_G = 0, LBM_FB_RHO_MINUS_RHOL_G = 1 } lbm_body_force;

/* Characteristic velocity of the convective outlet (appendix B options). */
typedef enum { LBM_OUTLET_LOCAL = 0, LBM_OUTLET_MAX = 1, LBM_OUTLET_AVERAGE = 2 } lbm_outlet_mode;

/* variant_flags: clamp phi to [0,1] inside rho(phi) and tau(phi) only */
#define LBM_VF_CLAMP_PHI 1u
/* variant_flags: the hydrodynamic set relaxes with the single-relaxation BGK
 * operator (Eq. bgk_collision, rate 1/(tau + 1/2)) and the viscous force
 * takes its BGK form (Eq. viscous_force_bgk), in place of the WMRT operator
 * and Eq. viscous_force_wmrt.  The phase-field set is unchanged.  All domains
 * of a batch must agree (LBM_EINVAL otherwise). */
#define LBM_VF_BGK 2u

/* Problem statement in lattice units (dx = dt = 1, cs^2 = 1/3). */
typedef struct {
  int lattice;           /* lbm_lattice */
  int nx, ny, nz;        /* nz = 1 for D2Q9 */
  double rho_h, rho_l;   /* densities at phi = 1 (heavy) and phi = 0 (light), Eq. density_interpolation */
  double tau_h, tau_l;   /* relaxation times, nu = tau cs^2 (Eq. kinematic_viscosity), tau linear in phi (Eq. relaxation_time) */
  double sigma, xi;      /* surface tension and interface width: beta = 12 sigma/xi, kappa = 3 sigma xi/2 */
  double mobility;       /* M = tau_phi cs^2 (Eq. mobility_relation) */
  double gravity[3];
  int body_force;        /* lbm_body_force */
  int bc[6];             /* lbm_bc per face -x,+x,-y,+y,-z,+z */
  double inlet_center[2];/* nozzle centre in the inlet face's tangential axes (x,y for z faces) */
  double inlet_radius;   /* nozzle radius R: phi_in = u_in/u_j = 1/2 [1 + tanh(2 (R - r)/xi)] */
  double inlet_u;        /* plug speed u_j along the inward normal */
  int outlet_mode;       /* lbm_outlet_mode: the convective velocity U of the outflow
                            (appendix B): the node's own outward velocity at the layer
                            next to the outlet (LOCAL), or its maximum (MAX) or average
                            (AVERAGE) over that layer; clipped at zero */
  int storage;           /* lbm_storage */
  unsigned variant_flags;/* LBM_VF_* */
} lbm_params;

typedef struct lbm_sim lbm_sim;

/* Bytes of the caller-owned device state buffer for these parameters
 * (populations, phase field(s), velocity, outlet plane).  Returns LBM_EINVAL
 * for an invalid parameter set (bad lattice or size, tau <= -1/2, xi <= 0,
 * rho_l <= 0, unpaired periodic faces, unsupported inlet/outlet placement). */
int lbm_state_bytes(const lbm_params* p, size_t* bytes);

/* Create a simulation on the caller's buffer and stream.
 *   phi0_dev  initial phase field [N] (required)
 *   u0_dev    initial velocity [3N] or NULL for rest (D2Q9: the third
 *             component is ignored)
 *   state_dev caller-allocated device buffer of at least lbm_state_bytes();
 *             it must outlive the handle and is not freed by the library
 *   stream    hipStream_t (NULL = default stream)
 * Initial populations: h_a = phi0 Gamma_a(u0) - F^phi_a/2, g_a = f^eq_a(p* = 0, u0),
 * u^{-1} = u0.  Launches on the stream and returns without synchronising. */
int lbm_init(const lbm_params* p, const float* phi0_dev, const float* u0_dev, void* state_dev,
             size_t state_bytes, void* stream, lbm_sim** out);

/* Advance n >= 0 steps (asynchronous).  Pairs of steps replay hipGraphs that
 * lbm_init and every change of launch shape (lbm_set_tile, lbm_set_store_hint,
 * lbm_set_blocks_per_cu, lbm_autotune) capture; lbm_step itself only launches
 * (an odd remaining step goes eagerly). */
int lbm_step(lbm_sim* s, int n);

/* Steps taken since init or the last import/load. */
long long lbm_steps_done(const lbm_sim* s);

/* Macroscopic fields of the current state into caller device buffers; mask
 * bit 0 phi[N], bit 1 u[3N] (the velocity of the latest macroscopic update),
 * bit 2 p[N] = p* rho cs^2 (Eq. equilibrium's normalised pressure). */
#define LBM_FIELD_PHI 1u
#define LBM_FIELD_U 2u
#define LBM_FIELD_P 4u
int lbm_fields(lbm_sim* s, unsigned mask, float* phi_dev, float* u_dev, float* p_dev);

/* Sum of phi and kinetic energy 0.5 sum rho |u|^2 over all nodes, accumulated
 * in FP64 on the GPU: per-thread strided sums, wavefront (64-lane) reductions,
 * one partial per block of 256 threads, then a fixed-order final pass
 * (deterministic).  Synchronises the stream.  Returns LBM_EUNSTABLE if either
 * is not finite. */
int lbm_reduce(lbm_sim* s, double* mass, double* kinetic);

/* Canonical FP32 copy of the state (post-stream populations at the current
 * time, h[qN], g[qN], and the stored velocity u[3N]) into caller device buffers. */
int lbm_export_state(lbm_sim* s, float* h_dev, float* g_dev, float* u_dev);

/* Replace the state from canonical FP32 device arrays (same layout as export). */
int lbm_import_state(lbm_sim* s, const float* h_dev, const float* g_dev, const float* u_dev);

/* Checkpoint: raw copy of the state buffer plus the step counter into host
 * memory (synchronises).  lbm_checkpoint_bytes gives the size needed. */
int lbm_checkpoint_bytes(const lbm_sim* s, size_t* bytes);
int lbm_save(lbm_sim* s, void* host_buf, size_t bytes);
int lbm_load(lbm_sim* s, const void* host_buf, size_t bytes);

/* Launch shape of the fused kernel: threads per block along x and y
 * (bx a multiple of 16, bx * by a multiple of 64 up to 512). */
int lbm_set_tile(lbm_sim* s, int bx, int by);
int lbm_get_tile(const lbm_sim* s, int* bx, int* by);

/* D3Q19 interior kernel: planes per z-marching task (the tile's phase field
 * and its halo staged in an LDS ring of planes), or 0 (the default) for the
 * tiled kernel that reads the stencil from global memory.  Both give the same
 * result bit for bit; the autotuners try both. */
int lbm_set_zchunk(lbm_sim* s, int planes);
int lbm_get_zchunk(const lbm_sim* s, int* planes);

/* Non-temporal hint (nonzero) on the population stores of the fused kernel. */
int lbm_set_store_hint(lbm_sim* s, int nontemporal);

/* Resident blocks per compute unit of the persistent launches (1..64): the
 * interior kernels run as about CUs x blocks_per_cu blocks, each walking a
 * contiguous chunk of tiles.  0: one block per tile (per z-chunk task of the
 * marching kernel), refilled by the hardware dispatcher. */
int lbm_set_blocks_per_cu(lbm_sim* s, int blocks_per_cu);
int lbm_get_blocks_per_cu(const lbm_sim* s, int* blocks_per_cu);

/* Autotuner: times trial_steps eager steps for each candidate tile shape,
 * blocks per compute unit, store hint and (D3Q19) z-marching chunk (0 or 32
 * planes) and keeps the fastest; results are cached per (lattice, storage,
 * grid, boundary set) for the life of the process, so later simulations of
 * the same shape take the cached choice without trials.  The state advances
 * by the trial steps.  Synchronises.  Outputs (nullable): chosen bx, by,
 * hint, and its mean ms per step. */
int lbm_autotune(lbm_sim* s, int trial_steps, int* bx, int* by, int* nontemporal, double* ms_per_step);

/* Time the step's kernels over n eager steps with HIP events on the
 * simulation's stream; out_ms[0] = mean phase-field pass, out_ms[1] = mean
 * fused collide-stream kernel, out_ms[2] = mean boundary-plane kernels (0 if
 * none).  Synchronises.  The state advances by n steps. */
int lbm_kernel_times(lbm_sim* s, int n, double* out_ms);

void lbm_destroy(lbm_sim* s);
const char* lbm_last_error(void);
const char* lbm_version(void);

/* ------------------------------------------------------------------------
 * Batched form: ndom independent domains (each with its own lbm_params and
 * initial fields; all share the lattice and the storage form) advanced by
 * the same kernel launches.  Per step: one persistent launch walks the
 * interior tiles of all domains in contiguous chunks for the phase-field
 * pass, one for the fused step, plus one launch over the face layers of all
 * domains for each, and one over all outlet planes.  Pairs of steps replay a
 * captured hipGraph.  Every domain's arithmetic is the single-domain
 * arithmetic, node for node.
 * ---------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* Bytes of the caller-owned arena for all domains (each slice 256-B aligned). */
int lbm_batch_state_bytes(int ndom, const lbm_params* per_domain, size_t* bytes);

/* phi0_dev[d] (required) and u0_dev[d] (u0_dev or its entries may be NULL)
 * are device pointers to each domain's initial fields, read before return
 * of the init kernels on `stream` (keep them alive until the stream has run
 * them).  state_dev: caller-allocated arena of lbm_batch_state_bytes(). */
int lbm_batch_init(int ndom, const lbm_params* per_domain, const float* const* phi0_dev,
                   const float* const* u0_dev, void* state_dev, size_t state_bytes, void* stream,
                   lbm_batch** out);
int lbm_batch_step(lbm_batch* b, int n);
long long lbm_batch_steps_done(const lbm_batch* b);
/* mass[ndom], kinetic[ndom] (host); FP64, fixed order, the same arithmetic
 * as lbm_reduce with the partials of all domains in one launch; synchronises
 * once.  Every entry is written; LBM_EUNSTABLE if any domain's value is not
 * finite. */
int lbm_batch_reduce(lbm_batch* b, double* mass, double* kinetic);
/* As lbm_set_zchunk, for every domain of the batch. */
int lbm_batch_set_zchunk(lbm_batch* b, int planes);
/* Allocation-free variant of lbm_batch_reduce, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  out_dev: caller-owned device buffer of 2 * ndom doubles;
 * out_dev[2d] = sum phi and out_dev[2d + 1] = kinetic energy of domain d,
 * bitwise the values lbm_batch_reduce returns.  Launches on the batch's
 * stream and returns without synchronising or copying to the host; nothing
 * is allocated or freed.  The partial sums live in a static device array of
 * 16384 pairs of doubles (256 KiB on each GPU, held until the process ends),
 * so ndom > 16384 is rejected with LBM_EINVAL.  All calls on one GPU share
 * that array: calls that overlap on one GPU (on different streams) race.
 * Non-finite values are returned as they are. */
int lbm_batch_reduce_noalloc(lbm_batch* b, double* out_dev);
int lbm_batch_fields(lbm_batch* b, int dom, unsigned mask, float* phi_dev, float* u_dev, float* p_dev);
int lbm_batch_export_state(lbm_batch* b, int dom, float* h_dev, float* g_dev, float* u_dev);
/* Intact liquid length of each domain, length[ndom] (host), in nodes along
 * the streamwise axis: the first layer from the inlet with no node above
 * `threshold` (the layer count if none).  Synchronises. */
int lbm_batch_intact_length(lbm_batch* b, float threshold, int* length);
/* launch shape: threads per block bx*by (as lbm_set_tile), resident blocks
 * per compute unit of the persistent launches (0: one block per tile, as
 * lbm_set_blocks_per_cu), non-temporal stores */
int lbm_batch_set_launch(lbm_batch* b, int bx, int by, int blocks_per_cu, int nontemporal);
/* autotuner over tile shape x blocks per CU x store hint; cached per batch
 * shape for the process; advances the state by the trials; synchronises */
int lbm_batch_autotune(lbm_batch* b, int trial_steps, int* bx, int* by, int* blocks_per_cu,
                       int* nontemporal, double* ms_per_step);
/* mean ms of (phase-field launches, fused-step launches, outlet launch) */
int lbm_batch_kernel_times(lbm_batch* b, int n, double* out_ms);
void lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
