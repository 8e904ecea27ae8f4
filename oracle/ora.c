/*
 * ora.c -- plain FP64 CPU oracle of the conservative phase-field lattice
 * Boltzmann step of arXiv 2505.12205.  TEST INFRASTRUCTURE ONLY: it is used by
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark,
 * never by the product path, and it shares no code with the HIP kernels.
 *
 * Written for readability against the paper, not for speed:
 *   - every formula is evaluated in the form the paper prints it (Gamma_a with
 *     the 1/cs^2 factors, the moment matrix M and its numerically inverted
 *     M^{-1}, the literal M^{-1} S M products of the collision and the viscous
 *     force), in double precision, with moment sums in index order a = 0..q-1;
 *   - streaming is a pull from a second population array (two-lattice), not
 *     an in-place scheme;
 *   - one time step is [macroscopic update -> collision -> streaming ->
 *     boundary conditions], the paper's cycle (section "Algorithm") rotated so
 *     that the first macroscopic update acts on the initial state.
 *
 * Readings of points where the paper is silent or inconsistent are marked
 * "reading:" below.
 */
#include "ora.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19
static const double CS2 = 1.0 / 3.0; /* lattice speed of sound squared, c = 1 */

/* ------------------------------------------------------------------------ */
/* Lattices.  Velocity order and moment matrices follow appendix A.          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int q, d;
  int e[QMAX][3];
  double w[QMAX];
  int opp[QMAX];
  double M[QMAX][QMAX];
  double Minv[QMAX][QMAX];
  int srel[QMAX]; /* 1 where the diagonal of S is s_nu, 0 where it is 1 */
} lattice_t;

/* D2Q9: velocities in the column order of the D2Q9 matrix of appendix A
 * (its momentum rows fix e_x and e_y).  Weights 4/9, 1/9, 1/36 (reading: the
 * paper does not print them; these are the isotropic D2Q9 weights). */
static const int D2Q9_E[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                 {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
static const double D2Q9_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},         {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},     {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},      {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},      {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* D3Q19: velocities in the column order of the weighted D3Q19 matrix of
 * appendix A (rows 1-3 are e_x, e_y, e_z); weights from Eq. weights. */
static const int D3Q19_E[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double D3Q19_M[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {-1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, -2, 2, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, -2, 2, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, -2, 2, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1},
    {1, -2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, -1, -1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0}};

/* Gauss-Jordan inverse with partial pivoting (plain textbook routine). */
static int invert(int n, const double A[QMAX][QMAX], double B[QMAX][QMAX]) {
  double W[QMAX][2 * QMAX];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) W[i][j] = (j < n) ? A[i][j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
    if (fabs(W[piv][c]) < 1e-300) return -1;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) {
        double t = W[c][j];
        W[c][j] = W[piv][j];
        W[piv][j] = t;
      }
    double inv = 1.0 / W[c][c];
    for (int j = 0; j < 2 * n; ++j) W[c][j] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = W[r][c];
      if (f != 0.0)
        for (int j = 0; j < 2 * n; ++j) W[r][j] -= f * W[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[i][j] = W[i][j + n];
  return 0;
}

static lattice_t LAT9, LAT19;
static int lat_ready = 0;

static void build_lattices(void) {
  if (lat_ready) return;
  memset(&LAT9, 0, sizeof LAT9);
  memset(&LAT19, 0, sizeof LAT19);
  LAT9.q = 9;
  LAT9.d = 2;
  for (int a = 0; a < 9; ++a) {
    LAT9.e[a][0] = D2Q9_E[a][0];
    LAT9.e[a][1] = D2Q9_E[a][1];
    LAT9.e[a][2] = 0;
    int s = abs(D2Q9_E[a][0]) + abs(D2Q9_E[a][1]);
    LAT9.w[a] = s == 0 ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    for (int k = 0; k < 9; ++k) LAT9.M[a][k] = D2Q9_M[a][k];
  }
  /* reading: the relaxation matrix is printed for D3Q19 only; for D2Q9 the
   * two stress rows (p_xx, p_xy: rows 7 and 8) relax with s_nu, all other
   * rows with 1, as in the D3Q19 matrix. */
  LAT9.srel[7] = LAT9.srel[8] = 1;
  LAT19.q = 19;
  LAT19.d = 3;
  for (int a = 0; a < 19; ++a) {
    for (int d = 0; d < 3; ++d) LAT19.e[a][d] = D3Q19_E[a][d];
    int s = abs(D3Q19_E[a][0]) + abs(D3Q19_E[a][1]) + abs(D3Q19_E[a][2]);
    LAT19.w[a] = s == 0 ? 12.0 / 36.0 : (s == 1 ? 2.0 / 36.0 : 1.0 / 36.0);
    for (int k = 0; k < 19; ++k) LAT19.M[a][k] = D3Q19_M[a][k];
  }
  /* S = diag(1,1,1,1,s,s,s,s,s,1,...,1) (Eq. 23 of the paper's numbering). */
  for (int k = 4; k <= 8; ++k) LAT19.srel[k] = 1;
  lattice_t* Ls[2] = {&LAT9, &LAT19};
  for (int l = 0; l < 2; ++l) {
    lattice_t* L = Ls[l];
    for (int a = 0; a < L->q; ++a)
      for (int b = 0; b < L->q; ++b)
        if (L->e[a][0] == -L->e[b][0] && L->e[a][1] == -L->e[b][1] && L->e[a][2] == -L->e[b][2])
          L->opp[a] = b;
    invert(L->q, L->M, L->Minv);
  }
  lat_ready = 1;
}

static const lattice_t* lattice_of(int q) {
  build_lattices();
  return q == 9 ? &LAT9 : (q == 19 ? &LAT19 : NULL);
}

int ora_lattice(int q, int* e, double* w, int* opp, double* M, double* Minv, int* srel) {
  const lattice_t* L = lattice_of(q);
  if (!L) return -1;
  for (int a = 0; a < q; ++a) {
    for (int d = 0; d < 3; ++d) e[a * 3 + d] = L->e[a][d];
    w[a] = L->w[a];
    opp[a] = L->opp[a];
    srel[a] = L->srel[a];
    for (int b = 0; b < q; ++b) {
      M[a * q + b] = L->M[a][b];
      Minv[a * q + b] = L->Minv[a][b];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-node formulas                                                      */
/* ------------------------------------------------------------------------ */

/* Eq. dimensionless_distribution: Gamma_a(u) */
static void gamma_fn(const lattice_t* L, const double* u, double* G) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int a = 0; a < L->q; ++a) {
    double eu = L->e[a][0] * u[0] + L->e[a][1] * u[1] + L->e[a][2] * u[2];
    G[a] = L->w[a] * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Eq. equilibrium: f_a^eq = p* w_a + (Gamma_a - w_a) */
static void feq_fn(const lattice_t* L, double pstar, const double* u, double* feq) {
  double G[QMAX];
  gamma_fn(L, u, G);
  for (int a = 0; a < L->q; ++a) feq[a] = pstar * L->w[a] + (G[a] - L->w[a]);
}

void ora_feq(int q, double pstar, const double* u, double* feq) {
  feq_fn(lattice_of(q), pstar, u, feq);
}

/* Eq. equilibrium_function: h_a^eq = phi Gamma_a */
static void heq_fn(const lattice_t* L, double phi, const double* u, double* heq) {
  double G[QMAX];
  gamma_fn(L, u, G);
  for (int a = 0; a < L->q; ++a) heq[a] = phi * G[a];
}

void ora_heq(int q, double phi, const double* u, double* heq) { heq_fn(lattice_of(q), phi, u, heq); }

/* Eqs. gradient_phi and laplacian_phi with c = dx = dt = 1 */
static void grad_lap_fn(const lattice_t* L, const double* phin, double* grad, double* lap) {
  grad[0] = grad[1] = grad[2] = 0.0;
  double l = 0.0;
  for (int a = 0; a < L->q; ++a) {
    for (int d = 0; d < 3; ++d) grad[d] += L->e[a][d] * L->w[a] * phin[a];
    l += L->w[a] * (phin[a] - phin[0]);
  }
  for (int d = 0; d < 3; ++d) grad[d] /= CS2;
  *lap = 2.0 * l / CS2;
}

void ora_grad_lap(int q, const double* phin, double* grad, double* lap) {
  grad_lap_fn(lattice_of(q), phin, grad, lap);
}

/* Eq. chemical_potential with beta, kappa from Eq. beta_kappa_relation.
 * reading: the bulk term is taken as 4 beta phi (phi - 1)(phi - 1/2); with the
 * printed factor (1 - phi) the potential does not vanish on the equilibrium
 * profile of Eq. kernel_function for these beta and kappa. */
double ora_chem_potential(double phi, double lap, double sigma, double xi) {
  double beta = 12.0 * sigma / xi;
  double kappa = 3.0 * sigma * xi / 2.0;
  return 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap;
}

/* (M^{-1} S M) x, literally: moments, relax, back-transform */
static void mrt_apply(const lattice_t* L, double s_nu, const double* x, double* y) {
  double m[QMAX];
  for (int k = 0; k < L->q; ++k) {
    double acc = 0.0;
    for (int a = 0; a < L->q; ++a) acc += L->M[k][a] * x[a];
    m[k] = acc * (L->srel[k] ? s_nu : 1.0);
  }
  for (int b = 0; b < L->q; ++b) {
    double acc = 0.0;
    for (int k = 0; k < L->q; ++k) acc += L->Minv[b][k] * m[k];
    y[b] = acc;
  }
}

/* reading: s_nu = 1/(tau + 1/2), so that S = s_nu I reproduces the BGK
 * operator of Eq. bgk_collision. */
static double s_nu_of(double tau) { return 1.0 / (tau + 0.5); }

/* Eq. viscous_force_wmrt: F_mu,i = -(nu/(cs^2 dt)) [sum_b e_bi e_bj (M^-1 S M (f - f^eq))_b] d_j rho,
 * with nu = tau cs^2 (Eq. kinematic_viscosity).
 * op = ORA_OP_BGK: Eq. viscous_force_bgk, the same sum with (f - f^eq)/(tau + 1/2). */
static void viscous_fn(const lattice_t* L, int op, const double* g, const double* feq, double tau,
                       const double* gradrho, double* fmu) {
  double x[QMAX], y[QMAX];
  for (int a = 0; a < L->q; ++a) x[a] = g[a] - feq[a];
  if (op == ORA_OP_BGK)
    for (int a = 0; a < L->q; ++a) y[a] = x[a] / (tau + 0.5);
  else
    mrt_apply(L, s_nu_of(tau), x, y);
  double nu = tau * CS2;
  for (int i = 0; i < 3; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 3; ++j) {
      double T = 0.0;
      for (int b = 0; b < L->q; ++b) T += L->e[b][i] * L->e[b][j] * y[b];
      acc += T * gradrho[j];
    }
    fmu[i] = -(nu / CS2) * acc;
  }
}

void ora_viscous_force(int q, int op, const double* g, const double* feq, double tau,
                       const double* gradrho, double* fmu) {
  viscous_fn(lattice_of(q), op, g, feq, tau, gradrho, fmu);
}

/* Eqs. force_term, equilibrium_modified, mrt_collision, lbe_standard (collision part);
 * op = ORA_OP_BGK: Eq. bgk_collision in place of Eq. mrt_collision. */
static void collide_g_fn(const lattice_t* L, int op, const double* g, const double* feq, const double* F,
                         double rho, double tau, double* gplus) {
  double Fa[QMAX], y[QMAX] = {0}, om[QMAX];
  for (int a = 0; a < L->q; ++a) {
    double eF = L->e[a][0] * F[0] + L->e[a][1] * F[1] + L->e[a][2] * F[2];
    Fa[a] = L->w[a] * eF / (rho * CS2);
    double fbar = feq[a] - 0.5 * Fa[a];
    y[a] = g[a] - fbar;
  }
  if (op == ORA_OP_BGK)
    for (int a = 0; a < L->q; ++a) om[a] = y[a] / (tau + 0.5);
  else
    mrt_apply(L, s_nu_of(tau), y, om);
  for (int a = 0; a < L->q; ++a) gplus[a] = g[a] - om[a] + Fa[a];
}

void ora_collide_g(int q, int op, const double* g, const double* feq, const double* force, double rho,
                   double tau, double* gplus) {
  collide_g_fn(lattice_of(q), op, g, feq, force, rho, tau, gplus);
}

/* Eq. forcing_term.  reading: the unit normal is regularised as
 * grad phi / sqrt(|grad phi|^2 + 1e-24) so that it is defined where the
 * gradient vanishes (there the prefactor vanishes too in the bulk). */
static void phase_forcing_fn(const lattice_t* L, double phi, const double* gradphi, double xi,
                             double* fphi) {
  double theta = (1.0 - 4.0 * (phi - 0.5) * (phi - 0.5)) / xi;
  double norm = sqrt(gradphi[0] * gradphi[0] + gradphi[1] * gradphi[1] +
                     gradphi[2] * gradphi[2] + 1e-24);
  for (int a = 0; a < L->q; ++a) {
    double en = (L->e[a][0] * gradphi[0] + L->e[a][1] * gradphi[1] + L->e[a][2] * gradphi[2]) / norm;
    fphi[a] = theta * L->w[a] * en;
  }
}

void ora_phase_forcing(int q, double phi, const double* gradphi, double xi, double* fphi) {
  phase_forcing_fn(lattice_of(q), phi, gradphi, xi, fphi);
}

/* Eqs. lbe_interface (collision part), equilibrium_with_force,
 * equilibrium_function, mobility_relation */
static void collide_h_fn(const lattice_t* L, const double* h, double phi, const double* u,
                         const double* gradphi, double xi, double mobility, double* hplus) {
  double heq[QMAX], fphi[QMAX];
  heq_fn(L, phi, u, heq);
  phase_forcing_fn(L, phi, gradphi, xi, fphi);
  double tau_phi = mobility / CS2;
  for (int a = 0; a < L->q; ++a) {
    double hbar = heq[a] - 0.5 * fphi[a];
    hplus[a] = h[a] - (h[a] - hbar) / (tau_phi + 0.5) + fphi[a];
  }
}

void ora_collide_h(int q, const double* h, double phi, const double* u, const double* gradphi,
                   double xi, double mobility, double* hplus) {
  collide_h_fn(lattice_of(q), h, phi, u, gradphi, xi, mobility, hplus);
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Body force.  reading: F_b = rho g for the Poiseuille channel, F_b =
 * (rho - rho_L) g for the jets (and the Rayleigh-Taylor case), as selected. */
static void body_force_fn(const ora_params* P, double rho, double* Fb) {
  double r = P->body_force == 1 ? rho - P->rho_l : rho;
  for (int d = 0; d < 3; ++d) Fb[d] = r * P->gravity[d];
}

/* Whole node: the macroscopic update followed by both collisions.
 *   phin[a] = phi(x + e_a), phin[0] = phi(x).
 * 1) phi, rho (Eq. density_interpolation); grad/laplacian of phi; chemical
 *    potential; surface tension F_s = mu grad phi; grad rho = (rho_H - rho_L) grad phi.
 * 2) p* = sum g (Eq. normalized_pressure); tau (Eq. relaxation_time).
 * 3) u^n = sum g e + F/(2 rho) (Eq. velocity_update), with the viscous force
 *    evaluated from f^eq(p*, u^{n-1}) as in the macroscopic procedure (Alg. 3).
 * 4) phase-field collision with u^n (Alg. 1, first procedure).
 * 5) hydrodynamic collision with f^eq(p*, u^n) and the viscous force
 *    re-evaluated from it (Alg. 1, second procedure).
 * reading: the printed algorithms evaluate the viscous force twice, once with
 * the stored velocity (macroscopic update) and once with the updated one
 * (collision); both are kept.
 * flags bit 1 selects the BGK operator and its viscous force for the
 * hydrodynamic set (the phase-field set is single-relaxation either way). */
void ora_collide_node(const ora_params* P, const double* h, const double* g,
                      const double* u_prev, const double* phin,
                      double* hplus, double* gplus, double* u_new) {
  const lattice_t* L = lattice_of(P->q);
  const int op = (P->flags & 2) ? ORA_OP_BGK : ORA_OP_WMRT;
  const double phi = phin[0];
  const double phi_c = (P->flags & 1) ? clamp01(phi) : phi;
  const double rho = P->rho_l + phi_c * (P->rho_h - P->rho_l); /* phi_L = 0 */
  double gradphi[3], lap;
  grad_lap_fn(L, phin, gradphi, &lap);
  const double mu = ora_chem_potential(phi, lap, P->sigma, P->xi);
  double Fs[3], gradrho[3], Fb[3];
  for (int d = 0; d < 3; ++d) {
    Fs[d] = mu * gradphi[d];                     /* Eq. surface_tension_force */
    gradrho[d] = (P->rho_h - P->rho_l) * gradphi[d]; /* Eq. density_gradient_phase_field */
  }
  body_force_fn(P, rho, Fb);

  double pstar = 0.0;
  for (int a = 0; a < L->q; ++a) pstar += g[a];
  const double tau = P->tau_l + phi_c * (P->tau_h - P->tau_l);

  /* macroscopic update: viscous force from the stored velocity */
  double feq_old[QMAX], fmu[3], F[3];
  feq_fn(L, pstar, u_prev, feq_old);
  viscous_fn(L, op, g, feq_old, tau, gradrho, fmu);
  for (int d = 0; d < 3; ++d) {
    double Fp = -pstar * CS2 * gradrho[d]; /* Eq. pressure_force */
    F[d] = Fs[d] + Fb[d] + Fp + fmu[d];    /* Eq. total_force */
  }
  double j[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < L->q; ++a)
    for (int d = 0; d < 3; ++d) j[d] += g[a] * L->e[a][d];
  for (int d = 0; d < 3; ++d) u_new[d] = j[d] + F[d] / (2.0 * rho);

  /* phase-field collision */
  collide_h_fn(L, h, phi, u_new, gradphi, P->xi, P->mobility, hplus);

  /* hydrodynamic collision */
  double feq_new[QMAX], fmu2[3], F2[3];
  feq_fn(L, pstar, u_new, feq_new);
  viscous_fn(L, op, g, feq_new, tau, gradrho, fmu2);
  for (int d = 0; d < 3; ++d) {
    double Fp = -pstar * CS2 * gradrho[d];
    F2[d] = Fs[d] + Fb[d] + Fp + fmu2[d];
  }
  collide_g_fn(L, op, g, feq_new, F2, rho, tau, gplus);
}

/* ------------------------------------------------------------------------ */
/* Grid, ghosts and boundary conditions (appendix B)                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  const ora_params* P;
  const lattice_t* L;
  int n[3];
  long N;
  /* state at time n: either double or float arrays */
  const double *hd, *gd, *ud;
  const float *hf, *gf, *uf;
  const double* phi; /* precomputed phi = sum h (full-grid mode) or NULL */
  /* post-collision values (full-grid mode) */
  const double *hpost, *gpost, *unew;
  /* sampled mode: one-node cache of the last collision */
  long cnode;
  double ch[QMAX], cg[QMAX], cu[3];
} ctx_t;

static inline long node_of(const ctx_t* c, const int* x) {
  return x[0] + (long)c->n[0] * (x[1] + (long)c->n[1] * x[2]);
}
static inline double HV(const ctx_t* c, int a, long i) {
  return c->hd ? c->hd[a * c->N + i] : (double)c->hf[a * c->N + i];
}
static inline double GV(const ctx_t* c, int a, long i) {
  return c->gd ? c->gd[a * c->N + i] : (double)c->gf[a * c->N + i];
}
static inline double UV(const ctx_t* c, int d, long i) {
  return c->ud ? c->ud[d * c->N + i] : (double)c->uf[d * c->N + i];
}
static double phi_node(const ctx_t* c, long i) {
  if (c->phi) return c->phi[i];
  double s = 0.0;
  for (int a = 0; a < c->L->q; ++a) s += HV(c, a, i);
  return s;
}

/* tangential axes of a face's normal axis */
static void tangential_axes(int axis, int* t1, int* t2) {
  if (axis == 0) { *t1 = 1; *t2 = 2; }
  else if (axis == 1) { *t1 = 0; *t2 = 2; }
  else { *t1 = 0; *t2 = 1; }
}

/* Inlet profile.  reading: the nozzle is a circular disc with a uniform
 * (plug) profile smoothed by the equilibrium kernel:
 *   psi(r) = 1/2 [1 + tanh(2 (R - r)/xi)],  phi_in = psi,  u_in = u_j psi n. */
static double inlet_psi(const ora_params* P, int face, const int* x) {
  int t1, t2;
  tangential_axes(face / 2, &t1, &t2);
  double d1 = x[t1] - P->inlet_center[0], d2 = x[t2] - P->inlet_center[1];
  double r = sqrt(d1 * d1 + d2 * d2);
  return 0.5 * (1.0 + tanh(2.0 * (P->inlet_radius - r) / P->xi));
}

static void inward_normal(int face, double* n) {
  n[0] = n[1] = n[2] = 0.0;
  n[face / 2] = (face % 2 == 0) ? 1.0 : -1.0;
}

/* phi at x + e_a with the ghost rules.  Periodic faces wrap (Eq. periodic_phi).
 * reading: at walls and at the outlet the ghost takes the value of the
 * adjacent fluid node (zero normal gradient); at the inlet it takes phi_in. */
static double phi_neighbour(const ctx_t* c, const int* x, int a) {
  int y[3];
  int inlet_face = -1;
  for (int d = 0; d < 3; ++d) {
    y[d] = x[d] + c->L->e[a][d];
    int face = -1;
    if (y[d] < 0) face = 2 * d;
    else if (y[d] >= c->n[d]) face = 2 * d + 1;
    if (face < 0) continue;
    int bc = c->P->bc[face];
    if (bc == ORA_PERIODIC) y[d] = (y[d] + c->n[d]) % c->n[d];
    else {
      y[d] = y[d] < 0 ? 0 : c->n[d] - 1;
      if (bc == ORA_INLET) inlet_face = face;
    }
  }
  if (inlet_face >= 0) return inlet_psi(c->P, inlet_face, y);
  return phi_node(c, node_of(c, y));
}

/* Full collision at one node from the state held by the context. */
static void collide_at(const ctx_t* c, const int* x, double* hp, double* gp, double* un) {
  const lattice_t* L = c->L;
  long i = node_of(c, x);
  double h[QMAX], g[QMAX], up[3], phin[QMAX];
  for (int a = 0; a < L->q; ++a) {
    h[a] = HV(c, a, i);
    g[a] = GV(c, a, i);
  }
  for (int d = 0; d < 3; ++d) up[d] = UV(c, d, i);
  phin[0] = phi_node(c, i);
  for (int a = 1; a < L->q; ++a) phin[a] = phi_neighbour(c, x, a);
  ora_collide_node(c->P, h, g, up, phin, hp, gp, un);
}

/* post-collision population a of set `which` (0 = h, 1 = g) at node x */
static double post_val(ctx_t* c, const int* x, int which, int a) {
  long i = node_of(c, x);
  if (c->hpost) return which == 0 ? c->hpost[a * c->N + i] : c->gpost[a * c->N + i];
  if (c->cnode != i) {
    collide_at(c, x, c->ch, c->cg, c->cu);
    c->cnode = i;
  }
  return which == 0 ? c->ch[a] : c->cg[a];
}

static void unew_at(ctx_t* c, const int* x, double* u) {
  long i = node_of(c, x);
  if (c->unew) {
    for (int d = 0; d < 3; ++d) u[d] = c->unew[d * c->N + i];
    return;
  }
  if (c->cnode != i) {
    collide_at(c, x, c->ch, c->cg, c->cu);
    c->cnode = i;
  }
  for (int d = 0; d < 3; ++d) u[d] = c->cu[d];
}

/* Pull streaming of one population into node x (Eqs. streaming_f/g), with
 *  - periodic wrap (Eqs. periodic_f/g),
 *  - halfway bounce-back at no-slip walls (Eqs. no_slip_f/g),
 *  - halfway specular reflection at free-slip walls (Eqs. free_slip_f/g).
 *    reading: a population leaving node y towards the wall keeps its
 *    tangential velocity and has its normal component reversed, landing on
 *    y + e_t; in pull form population a at x comes from population
 *    reflect(a) at x - e_{a,t}.
 * Returns 0 when the source lies beyond an inlet or outlet face (the value is
 * then set by that boundary condition).  Where no-slip and free-slip faces
 * meet, bounce-back is used. */
static int pull_one(ctx_t* c, const int* x, int which, int a, double* val) {
  const lattice_t* L = c->L;
  int s[3], crossed[3] = {0, 0, 0};
  int any = 0, noslip = 0;
  for (int d = 0; d < 3; ++d) {
    s[d] = x[d] - L->e[a][d];
    int face = -1;
    if (s[d] < 0) face = 2 * d;
    else if (s[d] >= c->n[d]) face = 2 * d + 1;
    if (face < 0) continue;
    int bc = c->P->bc[face];
    if (bc == ORA_PERIODIC) {
      s[d] = (s[d] + c->n[d]) % c->n[d];
      continue;
    }
    if (bc == ORA_INLET || bc == ORA_OUTLET) return 0;
    crossed[d] = 1;
    any = 1;
    if (bc == ORA_NOSLIP) noslip = 1;
  }
  if (!any) {
    *val = post_val(c, s, which, a);
    return 1;
  }
  if (noslip) {
    *val = post_val(c, x, which, L->opp[a]);
    return 1;
  }
  int er[3], src[3];
  for (int d = 0; d < 3; ++d) {
    er[d] = crossed[d] ? -L->e[a][d] : L->e[a][d];
    src[d] = crossed[d] ? x[d] : s[d];
  }
  int ar = -1;
  for (int b = 0; b < L->q; ++b)
    if (L->e[b][0] == er[0] && L->e[b][1] == er[1] && L->e[b][2] == er[2]) ar = b;
  *val = post_val(c, src, which, ar);
  return 1;
}

static int inlet_face_of(const ctx_t* c, const int* x) {
  for (int f = 0; f < 6; ++f) {
    if (c->P->bc[f] != ORA_INLET) continue;
    int d = f / 2;
    if ((f % 2 == 0 && x[d] == 0) || (f % 2 == 1 && x[d] == c->n[d] - 1)) return f;
  }
  return -1;
}
static int outlet_face_of(const ctx_t* c, const int* x) {
  for (int f = 0; f < 6; ++f) {
    if (c->P->bc[f] != ORA_OUTLET) continue;
    int d = f / 2;
    if ((f % 2 == 0 && x[d] == 0) || (f % 2 == 1 && x[d] == c->n[d] - 1)) return f;
  }
  return -1;
}

/* Velocity inlet (appendix B, "Velocity Boundary") applied to the populations
 * streamed into inlet node x; unknown[a] marks those whose source lies beyond
 * the inlet.
 * Hydrodynamic set, with f' = g + F_a/2:
 *   f'_a = f'_abar + (f^eq_a - f^eq_abar) - (1/N_g) e_a . M,
 *   M = sum_{e_b . n = 0} e_b (f'_b - f^eq_b).
 *   reading: the force in f' is the body force at phi_in (the inlet carries a
 *   single phase, so the interfacial forces vanish there); N_g = 2 for both
 *   lattices, the count that makes sum_a e_a f'_a equal u_in exactly (the
 *   printed N = 4 for D3Q19 removes only half of the tangential excess).
 *   Because e_b . u_in = 0 on the tangential set, the p* part of f^eq drops
 *   out of M and of f^eq_a - f^eq_abar; p* = 0 is used there.
 * Phase-field set:
 *   h_a = h^eq_a - h^neq_abar - [e_a has a tangential component] theta / N_h,
 *   theta = sum_{e_b . n = 0} h^neq_b,   N_h = 2 (D2Q9) or 4 (D3Q19)
 *   as printed, which makes sum_a h_a = phi_in exactly. */
static void apply_inlet(ctx_t* c, const int* x, int face, double* hn, double* gn,
                        const int* unknown) {
  const lattice_t* L = c->L;
  const ora_params* P = c->P;
  double n[3], uin[3];
  inward_normal(face, n);
  double psi = inlet_psi(P, face, x);
  for (int d = 0; d < 3; ++d) uin[d] = P->inlet_u * psi * n[d];
  double phi_in = psi;
  double rho_in = P->rho_l + phi_in * (P->rho_h - P->rho_l);
  double Fb[3];
  body_force_fn(P, rho_in, Fb);
  double feq[QMAX], heq[QMAX], Fa[QMAX];
  feq_fn(L, 0.0, uin, feq);
  heq_fn(L, phi_in, uin, heq);
  for (int a = 0; a < L->q; ++a) {
    double eF = L->e[a][0] * Fb[0] + L->e[a][1] * Fb[1] + L->e[a][2] * Fb[2];
    Fa[a] = L->w[a] * eF / (rho_in * CS2);
  }
  double Mx[3] = {0, 0, 0}, theta = 0.0;
  int nh = 0;
  for (int a = 0; a < L->q; ++a) {
    double en = L->e[a][0] * n[0] + L->e[a][1] * n[1] + L->e[a][2] * n[2];
    if (en == 0.0) {
      double fp = gn[a] + 0.5 * Fa[a];
      for (int d = 0; d < 3; ++d) Mx[d] += L->e[a][d] * (fp - feq[a]);
      theta += hn[a] - heq[a];
    }
    if (unknown[a]) {
      int tang = 0;
      for (int d = 0; d < 3; ++d)
        if (n[d] == 0.0 && L->e[a][d] != 0) tang = 1;
      nh += tang;
    }
  }
  const double Ng = 2.0;
  for (int a = 0; a < L->q; ++a) {
    if (!unknown[a]) continue;
    int b = L->opp[a];
    double fpb = gn[b] + 0.5 * Fa[b];
    double eM = L->e[a][0] * Mx[0] + L->e[a][1] * Mx[1] + L->e[a][2] * Mx[2];
    double fpa = fpb + (feq[a] - feq[b]) - eM / Ng;
    gn[a] = fpa - 0.5 * Fa[a];
    int tang = 0;
    for (int d = 0; d < 3; ++d)
      if (n[d] == 0.0 && L->e[a][d] != 0) tang = 1;
    hn[a] = heq[a] - (hn[b] - heq[b]) - (tang ? theta / nh : 0.0);
  }
}

/* streaming + wall rules + inlet for one node; returns 0 if the node lies on
 * an outlet face (completed by apply_outlet). */
static int stream_node(ctx_t* c, const int* x, double* hn, double* gn) {
  const lattice_t* L = c->L;
  int unknown[QMAX];
  int nunk = 0;
  for (int a = 0; a < L->q; ++a) {
    int ok = pull_one(c, x, 0, a, &hn[a]);
    pull_one(c, x, 1, a, &gn[a]);
    unknown[a] = !ok;
    if (!ok) {
      hn[a] = gn[a] = 0.0;
      nunk++;
    }
  }
  if (outlet_face_of(c, x) >= 0) return 0;
  int f = inlet_face_of(c, x);
  if (f >= 0 && nunk) apply_inlet(c, x, f, hn, gn, unknown);
  return 1;
}

/* Convective outflow (appendix B, "Convective Boundary"): first-order
 * implicit Orlanski update of every population of both sets,
 *   chi(N, t+1) = (chi(N, t) + lambda chi(N-1, t+1)) / (1 + lambda),
 * lambda = U dt/dy.  reading: U is the outward normal velocity u^n at the
 * layer N-1 from the latest macroscopic update, clipped at zero (local), or
 * its maximum / average over that layer; chi(N, t) is the outlet layer of the
 * state at time t. */
static double outlet_lambda(ctx_t* c, const int* x, int face) {
  int d = face / 2;
  double sgn = (face % 2 == 1) ? 1.0 : -1.0; /* outward normal sign */
  int mode = c->P->outlet_mode;
  double u[3];
  int y[3] = {x[0], x[1], x[2]};
  y[d] = (face % 2 == 1) ? c->n[d] - 2 : 1;
  if (mode == 0) {
    unew_at(c, y, u);
    double U = sgn * u[d];
    return U > 0.0 ? U : 0.0;
  }
  int t1, t2;
  tangential_axes(d, &t1, &t2);
  double mx = -1e300, sum = 0.0;
  long cnt = 0;
  for (int i2 = 0; i2 < c->n[t2]; ++i2)
    for (int i1 = 0; i1 < c->n[t1]; ++i1) {
      int z[3];
      z[d] = y[d];
      z[t1] = i1;
      z[t2] = i2;
      unew_at(c, z, u);
      double U = sgn * u[d];
      if (U > mx) mx = U;
      sum += U;
      cnt++;
    }
  double U = (mode == 1) ? mx : sum / (double)cnt;
  return U > 0.0 ? U : 0.0;
}

static void outlet_node(ctx_t* c, const int* x, int face, double* hn, double* gn) {
  const lattice_t* L = c->L;
  int d = face / 2;
  int y[3] = {x[0], x[1], x[2]};
  y[d] = (face % 2 == 1) ? c->n[d] - 2 : 1;
  double hy[QMAX], gy[QMAX];
  stream_node(c, y, hy, gy);
  double lam = outlet_lambda(c, x, face);
  long i = node_of(c, x);
  for (int a = 0; a < L->q; ++a) {
    hn[a] = (HV(c, a, i) + lam * hy[a]) / (1.0 + lam);
    gn[a] = (GV(c, a, i) + lam * gy[a]) / (1.0 + lam);
  }
}

/* ------------------------------------------------------------------------ */
/* Full-grid simulation                                                      */
/* ------------------------------------------------------------------------ */

struct ora_sim {
  ora_params P;
  const lattice_t* L;
  long N;
  double *h, *g, *u;       /* state: populations at time n, u^{n-1} */
  double *hn, *gn, *un;    /* work: post-collision / next populations, u^n */
  double *hp, *gp;         /* post-collision */
  double* phi;
};

static int valid_params(const ora_params* p) {
  if (!p || (p->q != 9 && p->q != 19)) return 0;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
  if (p->q == 9 && p->nz != 1) return 0;
  if (p->tau_h <= -0.5 || p->tau_l <= -0.5 || p->xi <= 0.0 || p->rho_l <= 0.0) return 0;
  return 1;
}

ora_sim* ora_create(const ora_params* p) {
  if (!valid_params(p)) return NULL;
  ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
  s->P = *p;
  s->L = lattice_of(p->q);
  s->N = (long)p->nx * p->ny * p->nz;
  size_t q = (size_t)p->q, N = (size_t)s->N;
  s->h = calloc(q * N, sizeof(double));
  s->g = calloc(q * N, sizeof(double));
  s->hn = calloc(q * N, sizeof(double));
  s->gn = calloc(q * N, sizeof(double));
  s->hp = calloc(q * N, sizeof(double));
  s->gp = calloc(q * N, sizeof(double));
  s->u = calloc(3 * N, sizeof(double));
  s->un = calloc(3 * N, sizeof(double));
  s->phi = calloc(N, sizeof(double));
  if (!s->h || !s->g || !s->hn || !s->gn || !s->hp || !s->gp || !s->u || !s->un || !s->phi) {
    ora_destroy(s);
    return NULL;
  }
  return s;
}

void ora_destroy(ora_sim* s) {
  if (!s) return;
  free(s->h); free(s->g); free(s->hn); free(s->gn); free(s->hp); free(s->gp);
  free(s->u); free(s->un); free(s->phi);
  free(s);
}

static void ctx_full(const ora_sim* s, ctx_t* c) {
  memset(c, 0, sizeof *c);
  c->P = &s->P;
  c->L = s->L;
  c->n[0] = s->P.nx;
  c->n[1] = s->P.ny;
  c->n[2] = s->P.nz;
  c->N = s->N;
  c->hd = s->h;
  c->gd = s->g;
  c->ud = s->u;
  c->cnode = -1;
}

static void coords(const ora_params* P, long i, int* x) {
  x[0] = (int)(i % P->nx);
  x[1] = (int)((i / P->nx) % P->ny);
  x[2] = (int)(i / ((long)P->nx * P->ny));
}

static void compute_phi(ora_sim* s) {
  const int q = s->L->q;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < s->N; ++i) {
    double acc = 0.0;
    for (int a = 0; a < q; ++a) acc += s->h[a * s->N + i]; /* Eq. phase_field_variable */
    s->phi[i] = acc;
  }
}

/* reading (initial populations; the paper gives none): u^{-1} = u0,
 * h_a = h^eq_a(phi0, u0) - F^phi_a / 2 (so that sum_a h_a = phi0 exactly) and
 * g_a = f^eq_a(p* = 0, u0).  The initial state is a post-boundary state: at
 * velocity-inlet nodes the populations entering from beyond the inlet are
 * set by the inlet condition from the others, as after every streaming. */
int ora_init(ora_sim* s, const double* phi0, const double* u0) {
  const lattice_t* L = s->L;
  const long N = s->N;
  ctx_t c;
  ctx_full(s, &c);
  memcpy(s->phi, phi0, sizeof(double) * N);
  c.phi = s->phi;
  /* the D2Q9 velocity set (appendix A) has no z component: a third
     component of the initial velocity is dropped in 2D */
  const long nu = (L->q == 9) ? 2 * N : 3 * N;
  for (long i = 0; i < 3 * N; ++i) s->u[i] = (u0 && i < nu) ? u0[i] : 0.0;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    int x[3];
    coords(&s->P, i, x);
    double phin[QMAX], grad[3], lap, u[3], heq[QMAX], fphi[QMAX], feq[QMAX];
    phin[0] = phi0[i];
    for (int a = 1; a < L->q; ++a) phin[a] = phi_neighbour(&c, x, a);
    grad_lap_fn(L, phin, grad, &lap);
    for (int d = 0; d < 3; ++d) u[d] = s->u[d * N + i];
    heq_fn(L, phi0[i], u, heq);
    phase_forcing_fn(L, phi0[i], grad, s->P.xi, fphi);
    feq_fn(L, 0.0, u, feq);
    for (int a = 0; a < L->q; ++a) {
      s->h[a * N + i] = heq[a] - 0.5 * fphi[a];
      s->g[a * N + i] = feq[a];
    }
  }
  for (long i = 0; i < N; ++i) {
    int x[3];
    coords(&s->P, i, x);
    int f = inlet_face_of(&c, x);
    if (f < 0) continue;
    double hn[QMAX], gn[QMAX], n[3];
    int unknown[QMAX];
    inward_normal(f, n);
    for (int a = 0; a < L->q; ++a) {
      hn[a] = s->h[a * N + i];
      gn[a] = s->g[a * N + i];
      unknown[a] = (L->e[a][0] * n[0] + L->e[a][1] * n[1] + L->e[a][2] * n[2]) > 0.0;
    }
    apply_inlet(&c, x, f, hn, gn, unknown);
    for (int a = 0; a < L->q; ++a) {
      s->h[a * N + i] = hn[a];
      s->g[a * N + i] = gn[a];
    }
  }
  return 0;
}

int ora_set_state(ora_sim* s, const double* h, const double* g, const double* u) {
  size_t qN = (size_t)s->L->q * s->N;
  memcpy(s->h, h, qN * sizeof(double));
  memcpy(s->g, g, qN * sizeof(double));
  memcpy(s->u, u, 3 * (size_t)s->N * sizeof(double));
  return 0;
}

int ora_get_state(const ora_sim* s, double* h, double* g, double* u) {
  size_t qN = (size_t)s->L->q * s->N;
  if (h) memcpy(h, s->h, qN * sizeof(double));
  if (g) memcpy(g, s->g, qN * sizeof(double));
  if (u) memcpy(u, s->u, 3 * (size_t)s->N * sizeof(double));
  return 0;
}

int ora_step(ora_sim* s, int nsteps) {
  const lattice_t* L = s->L;
  const long N = s->N;
  const int q = L->q;
  for (int it = 0; it < nsteps; ++it) {
    compute_phi(s);
    /* macroscopic update + collision at every node */
#pragma omp parallel
    {
      ctx_t c;
      ctx_full(s, &c);
      c.phi = s->phi;
#pragma omp for schedule(static)
      for (long i = 0; i < N; ++i) {
        int x[3];
        coords(&s->P, i, x);
        double hp[QMAX], gp[QMAX], un[3];
        collide_at(&c, x, hp, gp, un);
        for (int a = 0; a < q; ++a) {
          s->hp[a * N + i] = hp[a];
          s->gp[a * N + i] = gp[a];
        }
        for (int d = 0; d < 3; ++d) s->un[d * N + i] = un[d];
      }
    }
    /* streaming + boundary conditions */
#pragma omp parallel
    {
      ctx_t c;
      ctx_full(s, &c);
      c.phi = s->phi;
      c.hpost = s->hp;
      c.gpost = s->gp;
      c.unew = s->un;
#pragma omp for schedule(static)
      for (long i = 0; i < N; ++i) {
        int x[3];
        coords(&s->P, i, x);
        double hn[QMAX], gn[QMAX];
        if (!stream_node(&c, x, hn, gn)) {
          int f = outlet_face_of(&c, x);
          outlet_node(&c, x, f, hn, gn);
        }
        for (int a = 0; a < q; ++a) {
          s->hn[a * N + i] = hn[a];
          s->gn[a * N + i] = gn[a];
        }
      }
    }
    double* t;
    t = s->h; s->h = s->hn; s->hn = t;
    t = s->g; s->g = s->gn; s->gn = t;
    t = s->u; s->u = s->un; s->un = t;
  }
  return 0;
}

/* Phase-field transport alone under a prescribed velocity (section
 * "Circular Interface in a Shear Flow": the velocity is imposed and only the
 * phase field evolves).  Each of the nsteps steps is
 *   phi = sum h;  h+ = collision of Eq. lbe_interface with u = scale[k] u_field
 *   (the gradient of phi and the forcing term as in the full step);
 *   pull streaming of h with the wall and periodic rules of the full step.
 * The hydrodynamic set and the stored velocity are left untouched.  Faces
 * with a velocity inlet or a convective outlet are rejected (returns -1). */
int ora_step_h_prescribed(ora_sim* s, const double* u_field, const double* scale, int nsteps) {
  const lattice_t* L = s->L;
  const long N = s->N;
  const int q = L->q;
  for (int f = 0; f < 6; ++f)
    if (s->P.bc[f] == ORA_INLET || s->P.bc[f] == ORA_OUTLET) return -1;
  for (int it = 0; it < nsteps; ++it) {
    compute_phi(s);
    const double sc = scale[it];
#pragma omp parallel
    {
      ctx_t c;
      ctx_full(s, &c);
      c.phi = s->phi;
#pragma omp for schedule(static)
      for (long i = 0; i < N; ++i) {
        int x[3];
        coords(&s->P, i, x);
        double h[QMAX], phin[QMAX], grad[3], lap, u[3], hp[QMAX];
        for (int a = 0; a < q; ++a) h[a] = s->h[a * N + i];
        phin[0] = s->phi[i];
        for (int a = 1; a < q; ++a) phin[a] = phi_neighbour(&c, x, a);
        grad_lap_fn(L, phin, grad, &lap);
        for (int d = 0; d < 3; ++d) u[d] = sc * u_field[d * N + i];
        collide_h_fn(L, h, phin[0], u, grad, s->P.xi, s->P.mobility, hp);
        for (int a = 0; a < q; ++a) s->hp[a * N + i] = hp[a];
      }
    }
#pragma omp parallel
    {
      ctx_t c;
      ctx_full(s, &c);
      c.phi = s->phi;
      c.hpost = s->hp;
      c.gpost = s->g; /* not read: only the phase-field set is streamed */
      c.unew = s->u;
#pragma omp for schedule(static)
      for (long i = 0; i < N; ++i) {
        int x[3];
        coords(&s->P, i, x);
        for (int a = 0; a < q; ++a) pull_one(&c, x, 0, a, &s->hn[a * N + i]);
      }
    }
    double* t = s->h;
    s->h = s->hn;
    s->hn = t;
  }
  return 0;
}

int ora_fields(ora_sim* s, double* phi, double* u, double* p) {
  const long N = s->N;
  const int q = s->L->q;
  for (long i = 0; i < N; ++i) {
    double ph = 0.0, ps = 0.0;
    for (int a = 0; a < q; ++a) {
      ph += s->h[a * N + i];
      ps += s->g[a * N + i];
    }
    if (phi) phi[i] = ph;
    double phc = (s->P.flags & 1) ? clamp01(ph) : ph;
    double rho = s->P.rho_l + phc * (s->P.rho_h - s->P.rho_l);
    if (p) p[i] = ps * rho * CS2; /* p* = p / (rho cs^2) */
  }
  if (u) memcpy(u, s->u, 3 * (size_t)N * sizeof(double));
  return 0;
}

/* Neumaier-compensated FP64 sums of phi and 0.5 rho |u|^2 */
int ora_reduce(ora_sim* s, double* mass, double* kinetic) {
  const long N = s->N;
  const int q = s->L->q;
  double sm = 0.0, cm = 0.0, sk = 0.0, ck = 0.0;
  for (long i = 0; i < N; ++i) {
    double ph = 0.0;
    for (int a = 0; a < q; ++a) ph += s->h[a * N + i];
    double phc = (s->P.flags & 1) ? clamp01(ph) : ph;
    double rho = s->P.rho_l + phc * (s->P.rho_h - s->P.rho_l);
    double uu = 0.0;
    for (int d = 0; d < 3; ++d) uu += s->u[d * N + i] * s->u[d * N + i];
    double k = 0.5 * rho * uu;
    double t = sm + ph;
    cm += fabs(sm) >= fabs(ph) ? (sm - t) + ph : (ph - t) + sm;
    sm = t;
    t = sk + k;
    ck += fabs(sk) >= fabs(k) ? (sk - t) + k : (k - t) + sk;
    sk = t;
  }
  *mass = sm + cm;
  *kinetic = sk + ck;
  return 0;
}

int ora_step_nodes_f32(const ora_params* p, const float* h, const float* g, const float* u,
                       long nnodes, const long* nodes, double* h_out, double* g_out,
                       double* u_out) {
  if (!valid_params(p)) return -1;
  const lattice_t* L = lattice_of(p->q);
  const long N = (long)p->nx * p->ny * p->nz;
#pragma omp parallel
  {
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.P = p;
    c.L = L;
    c.n[0] = p->nx;
    c.n[1] = p->ny;
    c.n[2] = p->nz;
    c.N = N;
    c.hf = h;
    c.gf = g;
    c.uf = u;
    c.cnode = -1;
#pragma omp for schedule(dynamic, 4)
    for (long k = 0; k < nnodes; ++k) {
      int x[3];
      coords(p, nodes[k], x);
      double hn[QMAX], gn[QMAX], un[3];
      if (!stream_node(&c, x, hn, gn)) outlet_node(&c, x, outlet_face_of(&c, x), hn, gn);
      unew_at(&c, x, un);
      for (int a = 0; a < L->q; ++a) {
        h_out[k * L->q + a] = hn[a];
        g_out[k * L->q + a] = gn[a];
      }
      for (int d = 0; d < 3; ++d) u_out[k * 3 + d] = un[d];
    }
  }
  return 0;
}
