/* CPU FP64 oracle for the Asynchrony-Tolerant (AT) compressible Navier-Stokes step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this code;
 * only the test-suite, the smoke check and the CPU leg of the benchmark do.  It is written
 * from the paper (Kumari & Donzis, "Direct Numerical Simulations of turbulent flows using
 * high-order Asynchrony-Tolerant schemes: accuracy and performance") and shares no code,
 * header, table or constant with the GPU path.
 *
 * What it computes (each function in atns_oracle.c cites the passage it follows):
 *   * compressible NS right-hand side in total-energy flux form (Sec. 2, Eqs. cont, mome, ie
 *     recast so that mass, momentum and total energy telescope, Sec. 2.1 Eqs. convf-ts4);
 *   * 4th-order central first derivatives, with AT ghost values at every face of every
 *     virtual processing element (Sec. 2.1 Eq. at; Appendix B Table atschemes, (1,4) rows), or
 *     6th-order ones with the (1,6) rows (Sec. 4.1.2; Appendix B);
 *   * delays per (step, PE, face) from the periodic (CAA, Sec. 3.1.2 Alg. CAA) or random
 *     (SAA, Sec. 3.1.1 Alg. SAA) rules, or from an explicit table;
 *   * low-storage third-order Runge-Kutta (Williamson's 2N scheme) with a fixed time step
 *     (Sec. 2.2 fixes the step size; the paper's own integrator is AB2);
 *   * FP64 diagnostics: K, <eps>, enstrophy, M_t (Sec. 4), conserved totals.
 *
 * Parity status per function is listed in the oracle section of the design notes; functions
 * without a closed-form or paper pin say "parity unpinned" there.
 */
#ifndef ATNS_ORACLE_H
#define ATNS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OK = 0, ORA_E_INVAL = -1, ORA_E_SCHEDULE = -3, ORA_E_STATE = -5, ORA_E_NOMEM = -6 };
enum { ORA_SYNC = 0, ORA_CAA = 1, ORA_SAA = 2, ORA_EXPLICIT = 3 };

typedef struct {
  int32_t n[3];          /* grid points per direction (x, y, z) on [0, 2 pi)^3            */
  int32_t p[3];          /* virtual PEs per direction; n[d] % p[d] == 0, n[d]/p[d] >= 4    */
  int32_t max_delay;     /* largest delay any face may use; ring keeps max_delay + t_l levels */
  int32_t forcing;       /* 0 / 1                                                          */
  int32_t order;         /* spatial order: 4 ((1,4) AT rows, t_l = 3 levels, M = 2 layers) or */
                         /* 6 ((1,6) AT rows, t_l = 4 levels, M = 3 layers)                   */
  double gamma, prandtl, gas_r, mu_ref, t_ref, mu_exp, dt;
  int32_t form;          /* 0: total-energy flux form (conserved E, D1 o D1 viscous fluxes);      */
                         /* 1: the paper's own discretisation (Sec. 2, Eqs. cont, mome, ie): the  */
                         /*    fifth variable is rho e, viscous and conduction terms expanded with */
                         /*    (2,4) AT second derivatives and 3-step mixed derivatives (order 4) */
  int32_t visc;          /* viscosity law: 0 mu_ref (T/t_ref)^mu_exp; 1 Sutherland (form 1 only):  */
                         /* mu_ref (T/t_ref)^(3/2) (t_ref + S) / (T + S)                           */
  double suth_s;         /* Sutherland's constant S (same units as T)                              */
} ora_config;

/* stats vector layout (all doubles) */
enum {
  ORA_ST_STEP = 0, ORA_ST_TIME, ORA_ST_MASS, ORA_ST_MOMX, ORA_ST_MOMY, ORA_ST_MOMZ, ORA_ST_ENERGY,
  ORA_ST_MASS_RK, ORA_ST_MOMX_RK, ORA_ST_MOMY_RK, ORA_ST_MOMZ_RK, ORA_ST_ENERGY_RK,
  ORA_ST_K, ORA_ST_EPS, ORA_ST_ENS, ORA_ST_MT, ORA_ST_UMAX, ORA_ST_NONFINITE, ORA_ST_COUNT
};

typedef struct ora_sim ora_sim;

int ora_create(const ora_config* cfg, ora_sim** out);
void ora_destroy(ora_sim* s);
/* q: [nlev][5][nz][ny][nx], oldest level first; the last level is the current state. */
int ora_init_field(ora_sim* s, const double* q, int32_t nlev);
int ora_set_schedule(ora_sim* s, int32_t mode, int32_t L, int32_t c_r, uint64_t seed,
                     const int8_t* table, int64_t n_steps);
int ora_get_schedule(const ora_sim* s, int8_t* out, int64_t n_steps);
int ora_set_forcing(ora_sim* s, const double* fhat, int64_t n_steps);
int ora_rhs(ora_sim* s, double* out);            /* [5][N] at the current state, c = 0 */
int ora_rk_step(ora_sim* s, int32_t nsteps);
/* nsteps second-order Adams-Bashforth steps (Sec. 2.2, Eq. time_ab); the first with no stored
 * f^{n-1} (after initialisation or Runge-Kutta steps) is forward Euler. */
int ora_ab2_step(ora_sim* s, int32_t nsteps);
int ora_stats(ora_sim* s, double* out);          /* ORA_ST_COUNT doubles */
int ora_get_field(const ora_sim* s, double* q);  /* [5][N] */
int64_t ora_step(const ora_sim* s);

/* test hooks */
int ora_rhs_periodic_standard(const ora_config* cfg, const double* q, double* out);
double ora_at_weight(int32_t l, double kappa);          /* (1,4): quadratic, l = 0..2 */
double ora_at_weight6(int32_t l, double kappa);         /* (1,6): cubic, l = 0..3     */
int64_t ora_count_at_points(const ora_config* cfg);
int ora_forcing_field(const ora_config* cfg, const double* fhat_step, double* out /*[3][N]*/);
uint64_t ora_splitmix64(uint64_t seed, uint64_t counter);
int ora_get_flux(const ora_sim* s, double* out);   /* [3][5][N] from the last RHS evaluation */
/* [7][N]: u, v, w, p, du/dx, sigma_ij du_i/dx_j, |curl u|^2 with synchronous periodic derivatives */
int ora_diag_fields(const ora_config* cfg, const double* q, double* out);
/* The derivative along a line of e points of one PE that uses only those points (the second
 * step of the paper's mixed derivatives): central (1,4) where the stencil stays inside, the
 * standard one-sided and biased fourth-order stencils at the two points next to each end. */
int ora_pe_derivative(const double* g, int32_t e, double h, double* out);
/* mu(T) and dmu/dT of the configured viscosity law. */
double ora_viscosity(const ora_config* cfg, double T, double* dmu_dT);

#ifdef __cplusplus
}
#endif
#endif
