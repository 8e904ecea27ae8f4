/*
 * ora.h -- plain FP64 CPU oracle of the conservative phase-field lattice
 * Boltzmann step (arXiv 2505.12205, "Methodology" and appendices A/B).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * implementation.
 *
 * Naming: h = phase-field populations (the paper's g, Eq. lbe_interface),
 *         g = hydrodynamic pressure/velocity populations (the paper's f,
 *             Eq. lbe_standard).
 *
 * Layout of every population array: pop[a * N + node], node = x + nx*(y + ny*z).
 * Velocity arrays: u[d * N + node], d = 0..2 (the z component is zero in 2D).
 */
#ifndef ORA_H
#define ORA_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_PERIODIC = 0, ORA_NOSLIP = 1, ORA_FREESLIP = 2, ORA_INLET = 3, ORA_OUTLET = 4 };

typedef struct {
  int q;                 /* 9 -> D2Q9 (nz must be 1), 19 -> D3Q19 */
  int nx, ny, nz;
  double rho_h, rho_l;   /* heavy fluid at phi = 1, light fluid at phi = 0 */
  double tau_h, tau_l;   /* relaxation times; nu = tau * cs^2 */
  double sigma, xi, mobility;
  double gravity[3];
  int body_force;        /* 0: F_b = rho g ; 1: F_b = (rho - rho_l) g */
  int bc[6];             /* faces -x,+x,-y,+y,-z,+z : ORA_* */
  double inlet_center[2];/* in the face's two tangential axes (x,y for z faces) */
  double inlet_radius;
  double inlet_u;        /* plug speed along the inward normal */
  int outlet_mode;       /* 0 local, 1 plane maximum, 2 plane average */
  int flags;             /* bit 0: clamp phi to [0,1] inside rho(phi), tau(phi);
                            bit 1: BGK collision and viscous force for g (else WMRT) */
} ora_params;

typedef struct ora_sim ora_sim;

/* lattice tables (for tests): e[q*3], w[q], opp[q], M[q*q], Minv[q*q], srel[q] (1 = relaxed by s_nu) */
int ora_lattice(int q, int* e, double* w, int* opp, double* M, double* Minv, int* srel);

ora_sim* ora_create(const ora_params* p);
void ora_destroy(ora_sim* s);
/* initial state from phi0[N] and (nullable) u0[3N] */
int ora_init(ora_sim* s, const double* phi0, const double* u0);
/* overwrite the state (canonical post-stream populations at time n, u^{n-1}) */
int ora_set_state(ora_sim* s, const double* h, const double* g, const double* u);
int ora_get_state(const ora_sim* s, double* h, double* g, double* u);
int ora_step(ora_sim* s, int nsteps);
/* nsteps steps of the phase-field set alone under the prescribed velocity
 * scale[k] * u_field[3N] at step k; the hydrodynamic set is not advanced.
 * Periodic, no-slip and free-slip faces only (returns -1 otherwise). */
int ora_step_h_prescribed(ora_sim* s, const double* u_field, const double* scale, int nsteps);
/* macroscopic fields of the current state: phi[N], u[3N] (last computed u^n), p[N] = p* rho cs^2 */
int ora_fields(ora_sim* s, double* phi, double* u, double* p);
/* sum of phi and kinetic energy 0.5 sum rho |u|^2, in FP64 with compensated sums */
int ora_reduce(ora_sim* s, double* mass, double* kinetic);

/* One step evaluated only at the listed nodes, from a full-grid FP32 state
 * (canonical populations h[q*N], g[q*N], velocity u^{n-1}[3N]).  Outputs the
 * post-step populations and u^n at each listed node: h_out[k*q + a] etc. */
int ora_step_nodes_f32(const ora_params* p, const float* h, const float* g, const float* u,
                       long nnodes, const long* nodes,
                       double* h_out, double* g_out, double* u_out);

/* ---- single-node building blocks, exposed for the unit pins ---- */
void ora_feq(int q, double pstar, const double* u, double* feq);
void ora_heq(int q, double phi, const double* u, double* heq);
void ora_grad_lap(int q, const double* phin, double* grad, double* lap);
double ora_chem_potential(double phi, double lap, double sigma, double xi);
/* op: collision operator of the hydrodynamic set */
#define ORA_OP_WMRT 0
#define ORA_OP_BGK 1
void ora_viscous_force(int q, int op, const double* g, const double* feq, double tau,
                       const double* gradrho, double* fmu);
void ora_collide_g(int q, int op, const double* g, const double* feq, const double* force,
                   double rho, double tau, double* gplus);
void ora_phase_forcing(int q, double phi, const double* gradphi, double xi, double* fphi);
void ora_collide_h(int q, const double* h, double phi, const double* u, const double* gradphi,
                   double xi, double mobility, double* hplus);
/* whole node update from its neighbourhood: phin[a] = phi(x + e_a) */
void ora_collide_node(const ora_params* p, const double* h, const double* g,
                      const double* u_prev, const double* phin,
                      double* hplus, double* gplus, double* u_new);

#ifdef __cplusplus
}
#endif
#endif
