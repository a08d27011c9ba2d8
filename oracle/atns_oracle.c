/* CPU FP64 oracle for the Asynchrony-Tolerant compressible Navier-Stokes step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU leg of the
 * benchmark, never by the product library.  Written from the paper; shares nothing with the
 * GPU path.  Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fused multiply-add,
 * so every expression rounds as written).
 *
 * Deliberately plain: full-field arrays, one pass per step of the method, no blocking or fusion.
 */
#include "atns_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NQ 5          /* conserved: rho, rho u, rho v, rho w, E                        */
#define NPUB 4        /* published primitives per ghost point: u, v, w, T              */
#define NG 12         /* G_ij = d u_i / d x_j at 3 i + j (9), then d T / d x_j (3)      */
/* M, the points a central stencil reaches on each side (2 for the 4th-order, 3 for the 6th-order
 * scheme), is also the number of boundary layers each PE publishes per face (Sec. 3, Eq. NB), and
 * t_l = M + 1 the number of past levels an AT extrapolation combines (Appendix B). */
#define MAXLAYER 3
#define NFORCE 40

static const double TWO_PI = 6.283185307179586476925286766559;

/* Williamson's low-storage third-order Runge-Kutta (2N form): dQ <- A_s dQ + dt R(Q),
 * Q <- Q + B_s dQ; stage s approximates time t_n + C_s dt. */
static const double RK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
static const double RK_C[3] = {0.0, 1.0 / 3.0, 3.0 / 4.0};

struct ora_sim {
  ora_config c;
  int M;                 /* layers per face: order / 2 */
  int tl;                /* levels per AT extrapolation: M + 1 */
  int e[3];              /* tile edge per direction */
  int64_t npts;
  double h[3];
  double cv, cp;
  int R;                 /* ring levels kept = max_delay + t_l (L + t_l levels, Sec. 3.1) */
  double* q;             /* [5][N] */
  double* dq;            /* [5][N] */
  double* prim;          /* [5][N]: rho, u, v, w, T */
  double* grad;          /* [12][N] */
  double* flux;          /* [3][5][N]: flux in direction j of conserved variable c */
  double* rhs;           /* [5][N] */
  int64_t slab[3];       /* points in one published slab set of direction d */
  double* ring_pub[3];   /* [R][4][slab[d]] primitives published on faces normal to d */
  double* ring_flux[3];  /* [R][5][slab[d]] flux F_d published on faces normal to d    */
  double* ring_q[3];     /* form 1: [R][5][slab[d]] conserved variables on faces normal to d */
  int64_t* slot_level;   /* [R] level held by each ring slot, -1 = empty */
  int8_t* sched;         /* [sched_steps][ntiles][6] */
  int64_t sched_steps;
  double* fhat;          /* [force_steps][40][3][2] */
  int64_t force_steps;
  int32_t kf[NFORCE][3];
  int64_t step;
  double tot_rk[NQ];
  int ab2_prev;          /* dq holds dt f^{n-1} from an Adams-Bashforth step */
  int initialised;
  int err;
};

/* ------------------------------------------------------------------ helpers */

static int64_t idx3(const ora_config* c, int x, int y, int z) {
  return ((int64_t)z * c->n[1] + y) * c->n[0] + x;
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static int tile_index(const ora_sim* s, const int p[3]) {
  int tx = p[0] / s->e[0], ty = p[1] / s->e[1], tz = p[2] / s->e[2];
  return (tz * s->c.p[1] + ty) * s->c.p[0] + tx;
}

static int ntiles(const ora_config* c) { return c->p[0] * c->p[1] * c->p[2]; }

static int layers_of(const ora_config* c) { return c->order == 6 ? 3 : 2; }

static int check_config(const ora_config* c) {
  if (c->order != 4 && c->order != 6) return ORA_E_INVAL;
  for (int d = 0; d < 3; d++) {
    if (c->n[d] <= 0 || c->p[d] <= 0) return ORA_E_INVAL;
    if (c->n[d] % c->p[d] != 0) return ORA_E_INVAL;
    if (c->n[d] / c->p[d] < 2 * layers_of(c)) return ORA_E_INVAL;
  }
  if (c->max_delay < 0 || c->max_delay > 16) return ORA_E_INVAL;
  if (!(c->gamma > 1.0) || !(c->gas_r > 0.0) || !(c->prandtl > 0.0) || !(c->t_ref > 0.0))
    return ORA_E_INVAL;
  if (!(c->mu_ref >= 0.0) || !(c->dt > 0.0)) return ORA_E_INVAL;
  if (c->form != 0 && c->form != 1) return ORA_E_INVAL;
  if (c->visc != 0 && c->visc != 1) return ORA_E_INVAL;
  if (c->visc == 1 && (c->form != 1 || !(c->suth_s > 0.0))) return ORA_E_INVAL;
  if (c->form == 1) {
    if (c->order != 4) return ORA_E_INVAL;
    /* the one-sided stencils of the mixed derivatives take five points of one PE */
    for (int d = 0; d < 3; d++)
      if (c->n[d] / c->p[d] < 5) return ORA_E_INVAL;
  }
  return ORA_OK;
}

static void set_err(ora_sim* s, int code) {
#pragma omp atomic write
  s->err = code;
}

/* ------------------------------------------------------------------ AT weights
 * Quadratic Lagrange extrapolation in time from levels n-k, n-k-1, n-k-2 to the time
 * t_n + c dt, kappa = k + c.  At c = 0 these are exactly the Appendix B polynomials
 * (k^2+3k+2)/2, -(k^2+2k), (k^2+k)/2 of the (1,4) and (2,4) AT schemes, which reduce to the
 * standard scheme at k = 0 (Sec. 2.1, remark after Eq. at22). */
double ora_at_weight(int32_t l, double kappa) {
  if (l == 0) return (kappa + 1.0) * (kappa + 2.0) / 2.0;
  if (l == 1) return -kappa * (kappa + 2.0);
  if (l == 2) return kappa * (kappa + 1.0) / 2.0;
  return 0.0;
}

/* Cubic extrapolation from levels n-k .. n-k-3 to t_n + c dt, kappa = k + c: at c = 0 the
 * Appendix B polynomials of the (1,6) and (2,6) schemes, (k^3+6k^2+11k+6)/6, -(k^3+5k^2+6k)/2,
 * (k^3+4k^2+3k)/2, -(k^3+3k^2+2k)/6, written here in their factored form. */
double ora_at_weight6(int32_t l, double kappa) {
  if (l == 0) return (kappa + 1.0) * (kappa + 2.0) * (kappa + 3.0) / 6.0;
  if (l == 1) return -kappa * (kappa + 2.0) * (kappa + 3.0) / 2.0;
  if (l == 2) return kappa * (kappa + 1.0) * (kappa + 3.0) / 2.0;
  if (l == 3) return -kappa * (kappa + 1.0) * (kappa + 2.0) / 6.0;
  return 0.0;
}

static double at_weight(const ora_sim* s, int l, double kappa) {
  return s->tl == 4 ? ora_at_weight6(l, kappa) : ora_at_weight(l, kappa);
}

/* ------------------------------------------------------------------ schedule
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output number `counter + 1` of the generator
 * seeded with `seed`. */
uint64_t ora_splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Draw of a uniform integer in {0..L} for (step n, PE t, face f): the high 32 bits of the
 * SplitMix64 output scaled by L + 1 (multiply-shift). */
static int saa_draw(uint64_t seed, int64_t n, int t, int f, int nt, int L) {
  uint64_t ctr = ((uint64_t)n * (uint64_t)nt + (uint64_t)t) * 6u + (uint64_t)f;
  uint64_t z = ora_splitmix64(seed, ctr);
  return (int)(((z >> 32) * (uint64_t)(L + 1)) >> 32);
}

/* Delay schedules (Sec. 3.1).  CAA (Alg. CAA): PEs exchange every c_r steps, so the delay
 * cycles 0, 1, ..., c_r - 1 with L = c_r - 1; the first max(c_r, t_l) steps run synchronously
 * (enough levels for one extrapolation exist from step t_l - 1 on).
 * SAA (Alg. SAA): one exchange per step, delays random and bounded by L; the first L + t_l
 * steps (t_l = 3 levels for the 4th-order scheme, 4 for the 6th-order one) run synchronously. */
int ora_set_schedule(ora_sim* s, int32_t mode, int32_t L, int32_t c_r, uint64_t seed,
                     const int8_t* table, int64_t n_steps) {
  if (!s || n_steps < 0) return ORA_E_INVAL;
  const int nt = ntiles(&s->c);
  int8_t* t = (int8_t*)calloc((size_t)(n_steps > 0 ? n_steps : 1) * nt * 6, 1);
  if (!t) return ORA_E_NOMEM;
  if (mode == ORA_SYNC) {
    /* all zero */
  } else if (mode == ORA_CAA) {
    if (c_r < 1 || L != c_r - 1) { free(t); return ORA_E_INVAL; }
    const int warm = c_r > s->tl ? c_r : s->tl;
    for (int64_t n = 0; n < n_steps; n++) {
      int k = (n < warm) ? 0 : (int)(n % c_r);
      for (int i = 0; i < nt * 6; i++) t[n * nt * 6 + i] = (int8_t)k;
    }
  } else if (mode == ORA_SAA) {
    if (L < 0) { free(t); return ORA_E_INVAL; }
    for (int64_t n = 0; n < n_steps; n++)
      for (int ti = 0; ti < nt; ti++)
        for (int f = 0; f < 6; f++)
          t[(n * nt + ti) * 6 + f] = (int8_t)((n < L + s->tl) ? 0 : saa_draw(seed, n, ti, f, nt, L));
  } else if (mode == ORA_EXPLICIT) {
    if (!table) { free(t); return ORA_E_INVAL; }
    memcpy(t, table, (size_t)n_steps * nt * 6);
  } else {
    free(t);
    return ORA_E_INVAL;
  }
  /* every delayed read needs levels n-k .. n-k-(t_l-1) >= 0 and still in the ring */
  for (int64_t n = 0; n < n_steps; n++)
    for (int i = 0; i < nt * 6; i++) {
      int k = t[n * nt * 6 + i];
      if (k < 0 || k > s->c.max_delay || (k > 0 && n - k - (s->tl - 1) < 0)) { free(t); return ORA_E_SCHEDULE; }
    }
  free(s->sched);
  s->sched = t;
  s->sched_steps = n_steps;
  return ORA_OK;
}

int ora_get_schedule(const ora_sim* s, int8_t* out, int64_t n_steps) {
  if (!s || !out || n_steps > s->sched_steps) return ORA_E_INVAL;
  memcpy(out, s->sched, (size_t)n_steps * ntiles(&s->c) * 6);
  return ORA_OK;
}

static int delay_of(const ora_sim* s, int tile, int face) {
  return s->sched[(s->step * ntiles(&s->c) + tile) * 6 + face];
}

/* ------------------------------------------------------------------ ring of published data
 * Each PE publishes, on each of its faces, the M own layers next to that face (the boundary
 * points N_B of Sec. 3).  Layer j in {0 .. 2M-1} of tile t along d holds local index
 * {0 .. M-1, e-M .. e-1}. */
static int64_t slab_index(const ora_sim* s, int d, const int r[3]) {
  const int e = s->e[d];
  const int l = r[d] % e;
  const int M = s->M;
  int j;
  if (l < M) j = l;
  else if (l >= e - M) j = l - e + 2 * M;
  else return -1;
  const int plane = (r[d] / e) * 2 * M + j;
  const int a = (d == 0) ? 1 : 0;          /* faster transverse direction */
  const int b = (d == 2) ? 1 : 2;          /* slower transverse direction */
  return ((int64_t)plane * s->c.n[b] + r[b]) * s->c.n[a] + r[a];
}

static double ring_read(ora_sim* s, int kind, int d, int comp, int64_t level, const int r[3]) {
  const int slot = (int)(level % s->R);
  if (level < 0 || s->slot_level[slot] != level) { set_err(s, ORA_E_SCHEDULE); return NAN; }
  const int64_t j = slab_index(s, d, r);
  if (j < 0) { set_err(s, ORA_E_STATE); return NAN; }
  if (kind == 0) return s->ring_pub[d][((int64_t)slot * NPUB + comp) * s->slab[d] + j];
  if (kind == 2) return s->ring_q[d][((int64_t)slot * NQ + comp) * s->slab[d] + j];
  return s->ring_flux[d][((int64_t)slot * NQ + comp) * s->slab[d] + j];
}

/* ------------------------------------------------------------------ derivatives
 * Value at r = p + m e_d of a quantity, as the PE that owns p sees it (Sec. 2.1, Eq. at):
 * inside the PE -> current value; outside (a buffer point across face f) with delay k:
 * k = 0 -> the neighbour's current value; k >= 1 -> sum_l w_l(k + c_s) * published(n-k-l). */
static double seen(ora_sim* s, int kind, int comp, const double* cur, int d, const int p[3],
                   int m, int stage) {
  const int e = s->e[d];
  const int lr = p[d] % e + m;
  int r[3] = {p[0], p[1], p[2]};
  r[d] = wrap(p[d] + m, s->c.n[d]);
  const int64_t ir = idx3(&s->c, r[0], r[1], r[2]);
  if (lr >= 0 && lr < e) return cur[ir];
  const int face = 2 * d + (lr < 0 ? 0 : 1);
  const int k = delay_of(s, tile_index(s, p), face);
  if (k == 0) return cur[ir];
  const double kap = (double)k + RK_C[stage];
  double v = 0.0;
  for (int l = 0; l < s->tl; l++)
    v += at_weight(s, l, kap) * ring_read(s, kind, d, comp, s->step - k - l, r);
  return v;
}

/* Central first derivatives, the k = 0 rows of the Appendix B schemes:
 * (1,4): (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 h);
 * (1,6): (-f_{i-3} + 9 f_{i-2} - 45 f_{i-1} + 45 f_{i+1} - 9 f_{i+2} + f_{i+3}) / (60 h);
 * v[] holds f at offsets -M .. -1, +1 .. +M. */
static double d1_central(int order, const double* v, double h) {
  if (order == 6) return (-v[0] + 9.0 * v[1] - 45.0 * v[2] + 45.0 * v[3] - 9.0 * v[4] + v[5]) / (60.0 * h);
  return (v[0] - 8.0 * v[1] + 8.0 * v[2] - v[3]) / (12.0 * h);
}

/* The central derivative with AT ghost values substituted. */
static double d1_at(ora_sim* s, int kind, int comp, const double* cur, int d, const int p[3],
                    int stage) {
  double v[2 * MAXLAYER];
  int i = 0;
  for (int m = -s->M; m <= s->M; m++)
    if (m != 0) v[i++] = seen(s, kind, comp, cur, d, p, m, stage);
  return d1_central(s->c.order, v, s->h[d]);
}

/* The same stencil on the periodic grid with every point current (standard FD, Eq. du). */
static double d1_periodic(const ora_config* c, const double* f, int d, const int p[3], double h) {
  double v[2 * MAXLAYER];
  const int M = layers_of(c);
  int i = 0;
  for (int m = -M; m <= M; m++) {
    if (m == 0) continue;
    int r[3] = {p[0], p[1], p[2]};
    r[d] = wrap(p[d] + m, c->n[d]);
    v[i++] = f[idx3(c, r[0], r[1], r[2])];
  }
  return d1_central(c->order, v, h);
}

/* ------------------------------------------------------------------ physics (Sec. 2)
 * Ideal gas p = rho R T, e = c_v T; mu = mu_ref (T / T_ref)^mu_exp; k = mu c_p / Pr;
 * sigma_ij = mu (du_i/dx_j + du_j/dx_i - 2/3 delta_ij du_k/dx_k). */
static void primitives(const ora_config* c, double cv, const double* q, int64_t npts, int64_t i,
                       double* pr) {
  const double rho = q[i];
  const double u = q[npts + i] / rho, v = q[2 * npts + i] / rho, w = q[3 * npts + i] / rho;
  pr[0] = rho; pr[1] = u; pr[2] = v; pr[3] = w;
  if (c->form == 1) {
    pr[4] = q[4 * npts + i] / rho / cv;               /* rho e = rho c_v T (Eq. ie) */
  } else {
    const double ke = 0.5 * (u * u + v * v + w * w);
    pr[4] = (q[4 * npts + i] / rho - ke) / cv;        /* E = rho (c_v T + |u|^2 / 2) */
  }
}

/* Viscosity laws: the power law, and Sutherland's law named in Sec. 2,
 * mu = mu_ref (T / T_ref)^(3/2) (T_ref + S) / (T + S); with dmu/dT for the expanded viscous
 * terms of the paper's form. */
static double viscosity(const ora_config* c, double T, double* dmu) {
  if (c->visc == 1) {
    const double mu = c->mu_ref * pow(T / c->t_ref, 1.5) * (c->t_ref + c->suth_s) / (T + c->suth_s);
    if (dmu) *dmu = mu * (1.5 / T - 1.0 / (T + c->suth_s));
    return mu;
  }
  const double mu = c->mu_ref * pow(T / c->t_ref, c->mu_exp);
  if (dmu) *dmu = c->mu_exp * mu / T;
  return mu;
}

double ora_viscosity(const ora_config* cfg, double T, double* dmu_dT) { return viscosity(cfg, T, dmu_dT); }

static void stress(const ora_config* c, double T, const double* G, double sig[9], double* kappa_t,
                   double cp) {
  const double mu = viscosity(c, T, NULL);
  const double theta = G[0] + G[4] + G[8];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double sij = mu * (G[3 * i + j] + G[3 * j + i]);
      if (i == j) sij -= (2.0 / 3.0) * mu * theta;
      sig[3 * i + j] = sij;
    }
  *kappa_t = mu * cp / c->prandtl;
}

/* Total flux in direction j of (rho, rho u_i, E) - the total-energy form of Eqs. cont, mome,
 * ie: (m_j, m_i u_j + p delta_ij - sigma_ij, (E + p) u_j - u_i sigma_ij - k dT/dx_j). */
static void flux_point(const ora_config* c, double cp, const double* qv, const double* pr,
                       const double* G, double F[3][NQ]) {
  double sig[9], kt;
  stress(c, pr[4], G, sig, &kt, cp);
  const double p = pr[0] * c->gas_r * pr[4];
  for (int j = 0; j < 3; j++) {
    F[j][0] = qv[1 + j];
    for (int i = 0; i < 3; i++) F[j][1 + i] = qv[1 + i] * pr[1 + j] + (i == j ? p : 0.0) - sig[3 * i + j];
    F[j][4] = (qv[4] + p) * pr[1 + j]
              - (pr[1] * sig[0 * 3 + j] + pr[2] * sig[1 * 3 + j] + pr[3] * sig[2 * 3 + j])
              - kt * G[9 + j];
  }
}

/* ------------------------------------------------------------------ forcing (Sec. 4.2)
 * f(x) = sum over the 40 half-space wavevectors 0 < |k|^2 <= 6 of 2 Re(fhat_k e^{i k.x}),
 * ordered by ascending kz, then ky, then kx (each -2..2). */
static void forcing_list(int32_t kf[NFORCE][3]) {
  int nk = 0;
  for (int kz = -2; kz <= 2; kz++)
    for (int ky = -2; ky <= 2; ky++)
      for (int kx = -2; kx <= 2; kx++) {
        int k2 = kx * kx + ky * ky + kz * kz;
        if (k2 == 0 || k2 > 6) continue;
        int half = kz > 0 || (kz == 0 && ky > 0) || (kz == 0 && ky == 0 && kx > 0);
        if (!half) continue;
        kf[nk][0] = kx; kf[nk][1] = ky; kf[nk][2] = kz;
        nk++;
      }
}

static void force_at(const ora_config* c, const int32_t kf[NFORCE][3], const double* fh,
                     const int p[3], double f[3]) {
  const double x = TWO_PI * p[0] / c->n[0], y = TWO_PI * p[1] / c->n[1], z = TWO_PI * p[2] / c->n[2];
  f[0] = f[1] = f[2] = 0.0;
  for (int k = 0; k < NFORCE; k++) {
    const double ph = kf[k][0] * x + kf[k][1] * y + kf[k][2] * z;
    const double cs = cos(ph), sn = sin(ph);
    for (int a = 0; a < 3; a++)
      f[a] += 2.0 * (fh[(k * 3 + a) * 2] * cs - fh[(k * 3 + a) * 2 + 1] * sn);
  }
}

int ora_forcing_field(const ora_config* cfg, const double* fhat_step, double* out) {
  int32_t kf[NFORCE][3];
  forcing_list(kf);
  const int64_t npts = (int64_t)cfg->n[0] * cfg->n[1] * cfg->n[2];
#pragma omp parallel for schedule(static)
  for (int z = 0; z < cfg->n[2]; z++)
    for (int y = 0; y < cfg->n[1]; y++)
      for (int x = 0; x < cfg->n[0]; x++) {
        int p[3] = {x, y, z};
        double f[3];
        force_at(cfg, kf, fhat_step, p, f);
        for (int a = 0; a < 3; a++) out[a * npts + idx3(cfg, x, y, z)] = f[a];
      }
  return ORA_OK;
}

/* ------------------------------------------------------------------ lifecycle */

int ora_create(const ora_config* cfg, ora_sim** out) {
  if (!cfg || !out) return ORA_E_INVAL;
  int rc = check_config(cfg);
  if (rc) return rc;
  ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
  if (!s) return ORA_E_NOMEM;
  s->c = *cfg;
  s->M = layers_of(cfg);
  s->tl = s->M + 1;
  s->npts = (int64_t)cfg->n[0] * cfg->n[1] * cfg->n[2];
  for (int d = 0; d < 3; d++) {
    s->e[d] = cfg->n[d] / cfg->p[d];
    s->h[d] = TWO_PI / cfg->n[d];
  }
  s->cv = cfg->gas_r / (cfg->gamma - 1.0);
  s->cp = cfg->gamma * cfg->gas_r / (cfg->gamma - 1.0);
  s->R = cfg->max_delay + s->tl;
  const int64_t N = s->npts;
  s->q = (double*)calloc((size_t)NQ * N, sizeof(double));
  s->dq = (double*)calloc((size_t)NQ * N, sizeof(double));
  s->prim = (double*)calloc((size_t)5 * N, sizeof(double));
  s->grad = (double*)calloc((size_t)NG * N, sizeof(double));
  s->flux = (double*)calloc((size_t)3 * NQ * N, sizeof(double));
  s->rhs = (double*)calloc((size_t)NQ * N, sizeof(double));
  s->slot_level = (int64_t*)malloc(sizeof(int64_t) * s->R);
  int ok = s->q && s->dq && s->prim && s->grad && s->flux && s->rhs && s->slot_level;
  for (int d = 0; d < 3; d++) {
    const int a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
    s->slab[d] = (int64_t)2 * s->M * cfg->p[d] * cfg->n[a] * cfg->n[b];
    s->ring_pub[d] = (double*)malloc(sizeof(double) * s->R * NPUB * s->slab[d]);
    s->ring_flux[d] = (double*)malloc(sizeof(double) * s->R * NQ * s->slab[d]);
    ok = ok && s->ring_pub[d] && s->ring_flux[d];
    if (cfg->form == 1) {
      s->ring_q[d] = (double*)malloc(sizeof(double) * s->R * NQ * s->slab[d]);
      ok = ok && s->ring_q[d];
    }
  }
  if (!ok) { ora_destroy(s); return ORA_E_NOMEM; }
  for (int i = 0; i < s->R; i++) s->slot_level[i] = -1;
  forcing_list(s->kf);
  *out = s;
  return ORA_OK;
}

void ora_destroy(ora_sim* s) {
  if (!s) return;
  free(s->q); free(s->dq); free(s->prim); free(s->grad); free(s->flux); free(s->rhs);
  free(s->slot_level); free(s->sched); free(s->fhat);
  for (int d = 0; d < 3; d++) { free(s->ring_pub[d]); free(s->ring_flux[d]); free(s->ring_q[d]); }
  free(s);
}

int ora_set_forcing(ora_sim* s, const double* fhat, int64_t n_steps) {
  if (!s || !fhat || n_steps < 0) return ORA_E_INVAL;
  double* t = (double*)malloc(sizeof(double) * (size_t)(n_steps > 0 ? n_steps : 1) * NFORCE * 6);
  if (!t) return ORA_E_NOMEM;
  memcpy(t, fhat, sizeof(double) * (size_t)n_steps * NFORCE * 6);
  free(s->fhat);
  s->fhat = t;
  s->force_steps = n_steps;
  return ORA_OK;
}

/* ------------------------------------------------------------------ RHS passes */

static void compute_primitives(ora_sim* s, const double* q) {
  const int64_t N = s->npts;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; i++) {
    double pr[5];
    primitives(&s->c, s->cv, q, N, i, pr);
    for (int c = 0; c < 5; c++) s->prim[c * N + i] = pr[c];
  }
}

/* Publication at stage 1 of step n (the send buffer of Algs. SAA / CAA): the two own layers
 * next to each face of every PE, for the primitives (kind 0) or the face-normal flux (kind 1). */
static void publish(ora_sim* s, int kind, int slot) {
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
  for (int d = 0; d < 3; d++) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->n[2]; z++)
      for (int y = 0; y < c->n[1]; y++)
        for (int x = 0; x < c->n[0]; x++) {
          const int r[3] = {x, y, z};
          const int64_t j = slab_index(s, d, r);
          if (j < 0) continue;
          const int64_t i = idx3(c, x, y, z);
          if (kind == 0) {
            for (int cc = 0; cc < NPUB; cc++)
              s->ring_pub[d][((int64_t)slot * NPUB + cc) * s->slab[d] + j] = s->prim[(1 + cc) * N + i];
          } else {
            for (int cc = 0; cc < NQ; cc++)
              s->ring_flux[d][((int64_t)slot * NQ + cc) * s->slab[d] + j] = s->flux[(d * NQ + cc) * N + i];
          }
        }
  }
}

/* Velocity and temperature gradients with AT ghosts (kind 0 data). */
static void compute_gradients(ora_sim* s, int stage, int sync) {
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->n[2]; z++)
    for (int y = 0; y < c->n[1]; y++)
      for (int x = 0; x < c->n[0]; x++) {
        const int p[3] = {x, y, z};
        const int64_t i = idx3(c, x, y, z);
        for (int a = 0; a < 4; a++) {          /* u, v, w, T */
          const double* f = s->prim + (int64_t)(1 + a) * N;
          for (int d = 0; d < 3; d++) {
            const double g = sync ? d1_periodic(c, f, d, p, s->h[d]) : d1_at(s, 0, a, f, d, p, stage);
            const int gi = (a < 3) ? 3 * a + d : 9 + d;
            s->grad[(int64_t)gi * N + i] = g;
          }
        }
      }
}

static void compute_fluxes(ora_sim* s, const double* q) {
  const int64_t N = s->npts;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; i++) {
    double qv[NQ], pr[5], G[NG], F[3][NQ];
    for (int c = 0; c < NQ; c++) qv[c] = q[c * N + i];
    for (int c = 0; c < 5; c++) pr[c] = s->prim[c * N + i];
    for (int g = 0; g < NG; g++) G[g] = s->grad[(int64_t)g * N + i];
    flux_point(&s->c, s->cp, qv, pr, G, F);
    for (int j = 0; j < 3; j++)
      for (int c = 0; c < NQ; c++) s->flux[(j * NQ + c) * N + i] = F[j][c];
  }
}

/* RHS = -sum_j D_j^{AT} F_j + S with S = (0, rho f, rho f . u) (Eq. mome forcing term). */
static void compute_divergence(ora_sim* s, const double* q, int stage, int sync, double* out) {
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
  const double* fh = (c->forcing && s->fhat) ? s->fhat + s->step * NFORCE * 6 : NULL;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->n[2]; z++)
    for (int y = 0; y < c->n[1]; y++)
      for (int x = 0; x < c->n[0]; x++) {
        const int p[3] = {x, y, z};
        const int64_t i = idx3(c, x, y, z);
        double src[NQ] = {0, 0, 0, 0, 0};
        if (fh) {
          double f[3];
          force_at(c, s->kf, fh, p, f);
          const double rho = q[i];
          for (int a = 0; a < 3; a++) src[1 + a] = rho * f[a];
          src[4] = q[N + i] * f[0] + q[2 * N + i] * f[1] + q[3 * N + i] * f[2];
        }
        for (int cc = 0; cc < NQ; cc++) {
          double div = 0.0;
          for (int d = 0; d < 3; d++) {
            const double* F = s->flux + (int64_t)(d * NQ + cc) * N;
            div += sync ? d1_periodic(c, F, d, p, s->h[d]) : d1_at(s, 1, cc, F, d, p, stage);
          }
          out[cc * N + i] = -div + src[cc];
        }
      }
}

/* ------------------------------------------------------------------ the paper's own form (form 1)
 * Sec. 2, Eqs. cont, mome, ie with (rho, rho u_i, rho e) as the variables (Sec. 3.1: the five
 * variables each PE stores and sends):
 *   d rho / dt    = - d(rho u_j)/dx_j
 *   d rho u_i /dt = - d(rho u_i u_j)/dx_j - dp/dx_i + d sigma_ij / dx_j + rho f_i
 *   d rho e / dt  = - d(rho e u_j)/dx_j - p du_j/dx_j + d(k dT/dx_j)/dx_j + sigma_ij S_ij
 * with the viscous and conduction terms expanded as the paper computes them (Sec. 2.1):
 *   d sigma_ij/dx_j = mu (d2 u_i/dx_j dx_j + 1/3 d/dx_i (du_k/dx_k))
 *                     + mu'(T) dT/dx_j (du_i/dx_j + du_j/dx_i - 2/3 delta_ij du_k/dx_k),
 *   d(k dT/dx_j)/dx_j = k d2T/dx_j dx_j + k'(T) (dT/dx_j)^2,  k = mu c_p / Pr.
 * First derivatives: the (1,4) AT scheme; pure second derivatives: the (2,4) AT scheme (Appendix
 * B); both take the value of the differentiated function at a ghost point across a delayed face
 * from the delayed levels of the published conserved variables, f(q^{n-k-l}) extrapolated with the
 * weights of Eq. at.  Mixed derivatives d2 f / dx_a dx_b: the AT first derivatives along b and
 * along a at every point, then a derivative of each along the other direction that uses only the
 * PE's own points (central where it fits, the standard one-sided fourth-order stencils at the two
 * points next to a face), and the average of the two (Sec. 2.1, three steps). */

/* Functions of the conserved variables that the form differentiates. */
enum { FN_U = 0, FN_T = 3, FN_P = 4, FN_M = 5, FN_UU = 8, FN_EU = 17 };

static double fn_of(const ora_sim* s, int fn, const double q[NQ]) {
  const double rho = q[0];
  if (fn < 3) return q[1 + fn] / rho;
  if (fn == FN_T) return q[4] / rho / s->cv;
  if (fn == FN_P) return rho * s->c.gas_r * (q[4] / rho / s->cv);
  if (fn < FN_UU) return q[1 + (fn - FN_M)];
  if (fn < FN_EU) { const int ij = fn - FN_UU; return q[1 + ij / 3] * q[1 + ij % 3] / rho; }
  return q[4] * q[1 + (fn - FN_EU)] / rho;
}

static void publish_q(ora_sim* s, const double* q, int slot) {
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
  for (int d = 0; d < 3; d++) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->n[2]; z++)
      for (int y = 0; y < c->n[1]; y++)
        for (int x = 0; x < c->n[0]; x++) {
          const int r[3] = {x, y, z};
          const int64_t j = slab_index(s, d, r);
          if (j < 0) continue;
          const int64_t i = idx3(c, x, y, z);
          for (int cc = 0; cc < NQ; cc++) s->ring_q[d][((int64_t)slot * NQ + cc) * s->slab[d] + j] = q[cc * N + i];
        }
  }
}

/* f at r = p + m e_d as the PE owning p sees it: inside or across a face with k = 0, f of the
 * current state; across a face with delay k >= 1, sum_l w_l(k + c_s) f(q^{n-k-l}). */
static double seen_fn(ora_sim* s, int fn, const double* q, int d, const int p[3], int m, int stage) {
  const int e = s->e[d];
  const int lr = p[d] % e + m;
  int r[3] = {p[0], p[1], p[2]};
  r[d] = wrap(p[d] + m, s->c.n[d]);
  const int64_t ir = idx3(&s->c, r[0], r[1], r[2]);
  double qv[NQ];
  int k = 0;
  if (lr < 0 || lr >= e) k = delay_of(s, tile_index(s, p), 2 * d + (lr < 0 ? 0 : 1));
  if (k == 0) {
    for (int cc = 0; cc < NQ; cc++) qv[cc] = q[cc * s->npts + ir];
    return fn_of(s, fn, qv);
  }
  const double kap = (double)k + RK_C[stage];
  double v = 0.0;
  for (int l = 0; l < s->tl; l++) {
    for (int cc = 0; cc < NQ; cc++) qv[cc] = ring_read(s, 2, d, cc, s->step - k - l, r);
    v += at_weight(s, l, kap) * fn_of(s, fn, qv);
  }
  return v;
}

/* (1,4) AT first derivative and (2,4) AT second derivative of f along d at p (Appendix B: the
 * delayed side's values replaced by their extrapolations, the stencils otherwise standard,
 * (-f_{-2} + 16 f_{-1} - 30 f_0 + 16 f_{+1} - f_{+2}) / (12 h^2) for the second derivative). */
static double d1_fn(ora_sim* s, int fn, const double* q, int d, const int p[3], int stage) {
  double v[4];
  int i = 0;
  for (int m = -2; m <= 2; m++)
    if (m != 0) v[i++] = seen_fn(s, fn, q, d, p, m, stage);
  return d1_central(4, v, s->h[d]);
}

static double d2_fn(ora_sim* s, int fn, const double* q, int d, const int p[3], int stage) {
  double v[5];
  for (int m = -2; m <= 2; m++) v[m + 2] = seen_fn(s, fn, q, d, p, m, stage);
  const double h = s->h[d];
  return (-v[0] + 16.0 * v[1] - 30.0 * v[2] + 16.0 * v[3] - v[4]) / (12.0 * h * h);
}

/* Derivative at local index l of a line g[0 .. e-1] of one PE using only those points. */
static double pe_d1(const double* g, int e, int l, double h) {
  if (l >= 2 && l <= e - 3) return (g[l - 2] - 8.0 * g[l - 1] + 8.0 * g[l + 1] - g[l + 2]) / (12.0 * h);
  if (l == 0) return (-25.0 * g[0] + 48.0 * g[1] - 36.0 * g[2] + 16.0 * g[3] - 3.0 * g[4]) / (12.0 * h);
  if (l == 1) return (-3.0 * g[0] - 10.0 * g[1] + 18.0 * g[2] - 6.0 * g[3] + g[4]) / (12.0 * h);
  if (l == e - 2)
    return (3.0 * g[e - 1] + 10.0 * g[e - 2] - 18.0 * g[e - 3] + 6.0 * g[e - 4] - g[e - 5]) / (12.0 * h);
  return (25.0 * g[e - 1] - 48.0 * g[e - 2] + 36.0 * g[e - 3] - 16.0 * g[e - 4] + 3.0 * g[e - 5]) / (12.0 * h);
}

int ora_pe_derivative(const double* g, int32_t e, double h, double* out) {
  if (!g || !out || e < 5) return ORA_E_INVAL;
  for (int l = 0; l < e; l++) out[l] = pe_d1(g, e, l, h);
  return ORA_OK;
}

/* That derivative along a at p of the gradient component gi (s->grad), within p's PE. */
static double pe_d1_grad(const ora_sim* s, int gi, int a, const int p[3]) {
  const int e = s->e[a];
  const int l = p[a] % e;
  double line[e];
  int r[3] = {p[0], p[1], p[2]};
  for (int j = 0; j < e; j++) {
    r[a] = p[a] - l + j;
    line[j] = s->grad[(int64_t)gi * s->npts + idx3(&s->c, r[0], r[1], r[2])];
  }
  return pe_d1(line, e, l, s->h[a]);
}

/* d2 u_k / dx_a dx_b, a != b: the average of the two PE-local derivatives of the AT gradients. */
static double mixed_u(const ora_sim* s, int k, int a, int b, const int p[3]) {
  return 0.5 * (pe_d1_grad(s, 3 * k + b, a, p) + pe_d1_grad(s, 3 * k + a, b, p));
}

/* AT gradients of u, v, w, T (G_ij = du_i/dx_j, then dT/dx_j) from the conserved state. */
static void gradients_paper(ora_sim* s, const double* q, int stage) {
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->n[2]; z++)
    for (int y = 0; y < c->n[1]; y++)
      for (int x = 0; x < c->n[0]; x++) {
        const int p[3] = {x, y, z};
        const int64_t i = idx3(c, x, y, z);
        for (int a = 0; a < 4; a++)
          for (int d = 0; d < 3; d++) {
            const int fn = a < 3 ? FN_U + a : FN_T;
            s->grad[(int64_t)((a < 3) ? 3 * a + d : 9 + d) * N + i] = d1_fn(s, fn, q, d, p, stage);
          }
      }
}

static void rhs_paper(ora_sim* s, const double* q, int stage, double* out) {
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
  const double* fh = (c->forcing && s->fhat) ? s->fhat + s->step * NFORCE * 6 : NULL;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->n[2]; z++)
    for (int y = 0; y < c->n[1]; y++)
      for (int x = 0; x < c->n[0]; x++) {
        const int p[3] = {x, y, z};
        const int64_t i = idx3(c, x, y, z);
        double G[NG];
        for (int g = 0; g < NG; g++) G[g] = s->grad[(int64_t)g * N + i];
        const double rho = s->prim[i], T = s->prim[4 * N + i];
        const double pres = rho * c->gas_r * T;
        double dmu;
        const double mu = viscosity(c, T, &dmu);
        const double kt = mu * s->cp / c->prandtl, dkt = dmu * s->cp / c->prandtl;
        const double th = G[0] + G[4] + G[8];
        double f[3] = {0.0, 0.0, 0.0};
        if (fh) force_at(c, s->kf, fh, p, f);
        /* continuity */
        double div = 0.0;
        for (int j = 0; j < 3; j++) div += d1_fn(s, FN_M + j, q, j, p, stage);
        out[i] = -div;
        /* momentum */
        for (int a = 0; a < 3; a++) {
          double conv = 0.0, lap = 0.0;
          for (int j = 0; j < 3; j++) {
            conv += d1_fn(s, FN_UU + 3 * a + j, q, j, p, stage);
            lap += d2_fn(s, FN_U + a, q, j, p, stage);
          }
          double gdiv = d2_fn(s, FN_U + a, q, a, p, stage);      /* d/dx_a (du_a/dx_a) */
          for (int k = 0; k < 3; k++)
            if (k != a) gdiv += mixed_u(s, k, a, k, p);          /* d/dx_a (du_k/dx_k) */
          double visc = mu * (lap + gdiv / 3.0);
          for (int j = 0; j < 3; j++)
            visc += dmu * G[9 + j] * (G[3 * a + j] + G[3 * j + a] - (a == j ? 2.0 / 3.0 * th : 0.0));
          out[(1 + a) * N + i] = -conv - d1_fn(s, FN_P, q, a, p, stage) + visc + rho * f[a];
        }
        /* internal energy */
        double conv = 0.0, lapT = 0.0, grT = 0.0;
        for (int j = 0; j < 3; j++) {
          conv += d1_fn(s, FN_EU + j, q, j, p, stage);
          lapT += d2_fn(s, FN_T, q, j, p, stage);
          grT += G[9 + j] * G[9 + j];
        }
        double sig[9], kdummy;
        stress(c, T, G, sig, &kdummy, s->cp);
        double diss = 0.0;
        for (int g = 0; g < 9; g++) diss += sig[g] * G[g];
        out[4 * N + i] = -conv - pres * th + kt * lapT + dkt * grT + diss;
      }
}

/* One RHS evaluation at step s->step, RK stage `stage`; publishes at stage 0 when asked. */
static int eval_rhs(ora_sim* s, const double* q, int stage, int do_publish, double* out) {
  if (!s->sched || s->step >= s->sched_steps) return ORA_E_SCHEDULE;
  if (s->c.forcing && (!s->fhat || s->step >= s->force_steps)) return ORA_E_STATE;
  s->err = 0;
  const int slot = (int)(s->step % s->R);
  compute_primitives(s, q);
  if (s->c.form == 1) {
    if (do_publish) {
      s->slot_level[slot] = s->step;
      publish_q(s, q, slot);
    }
    gradients_paper(s, q, stage);
    if (s->err) return s->err;
    rhs_paper(s, q, stage, out);
    return s->err;
  }
  if (do_publish) {
    s->slot_level[slot] = s->step;
    publish(s, 0, slot);
  }
  compute_gradients(s, stage, 0);
  if (s->err) return s->err;
  compute_fluxes(s, q);
  if (do_publish) publish(s, 1, slot);
  compute_divergence(s, q, stage, 0, out);
  return s->err;
}

/* History levels are published with synchronous (k = 0) gradients and fluxes. */
int ora_init_field(ora_sim* s, const double* q, int32_t nlev) {
  if (!s || !q || nlev < 1 || nlev > s->R) return ORA_E_INVAL;
  const int64_t N = s->npts;
  for (int i = 0; i < s->R; i++) s->slot_level[i] = -1;
  for (int lev = 0; lev < nlev - 1; lev++) {
    const double* ql = q + (int64_t)lev * NQ * N;
    const int slot = lev % s->R;
    if (s->c.form == 1) {
      s->slot_level[slot] = lev;
      publish_q(s, ql, slot);
      continue;
    }
    compute_primitives(s, ql);
    s->slot_level[slot] = lev;
    publish(s, 0, slot);
    compute_gradients(s, 0, 1);
    compute_fluxes(s, ql);
    publish(s, 1, slot);
  }
  memcpy(s->q, q + (int64_t)(nlev - 1) * NQ * N, sizeof(double) * NQ * N);
  memset(s->dq, 0, sizeof(double) * NQ * N);
  s->ab2_prev = 0;
  s->step = nlev - 1;
  const double vol = s->h[0] * s->h[1] * s->h[2];
  for (int c = 0; c < NQ; c++) {
    double t = 0.0;
    for (int64_t i = 0; i < N; i++) t += s->q[c * N + i];
    s->tot_rk[c] = t * vol;
  }
  s->initialised = 1;
  return ORA_OK;
}

int ora_rhs(ora_sim* s, double* out) {
  if (!s || !out) return ORA_E_INVAL;
  if (!s->initialised) return ORA_E_STATE;
  return eval_rhs(s, s->q, 0, 0, out);
}

int ora_rk_step(ora_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return ORA_E_INVAL;
  if (!s->initialised) return ORA_E_STATE;
  const int64_t N = s->npts;
  const double dt = s->c.dt;
  const double vol = s->h[0] * s->h[1] * s->h[2];
  for (int it = 0; it < nsteps; it++) {
    for (int st = 0; st < 3; st++) {
      int rc = eval_rhs(s, s->q, st, st == 0, s->rhs);
      if (rc) return rc;
      const double A = RK_A[st], B = RK_B[st];
      for (int c = 0; c < NQ; c++) {
        double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
        for (int64_t i = 0; i < N; i++) {
          const int64_t j = c * N + i;
          const double d = (st == 0) ? dt * s->rhs[j] : A * s->dq[j] + dt * s->rhs[j];
          s->dq[j] = d;
          s->q[j] = s->q[j] + B * d;
          acc += d;
        }
        s->tot_rk[c] += B * acc * vol;
      }
    }
    s->step++;
  }
  s->ab2_prev = 0;
  return ORA_OK;
}

/* Second-order Adams-Bashforth (Sec. 2.2, Eq. time_ab with T = 2, beta_0 = 3/2, beta_1 = -1/2):
 * Q^{n+1} = Q^n + dt (3/2 f^n - 1/2 f^{n-1}).  f^n is evaluated once per step at t_n (AT
 * extrapolation at kappa = k, i.e. c_s = 0), publishing level n; f^{n-1} is kept from the previous
 * step (dq holds dt f^{n-1}).  A step with no stored f^{n-1} (the first after initialisation or
 * after Runge-Kutta steps) is forward Euler. */
int ora_ab2_step(ora_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return ORA_E_INVAL;
  if (!s->initialised) return ORA_E_STATE;
  const int64_t N = s->npts;
  const double dt = s->c.dt;
  const double vol = s->h[0] * s->h[1] * s->h[2];
  for (int it = 0; it < nsteps; it++) {
    int rc = eval_rhs(s, s->q, 0, 1, s->rhs);
    if (rc) return rc;
    const int prev = s->ab2_prev;
    for (int c = 0; c < NQ; c++) {
      double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
      for (int64_t i = 0; i < N; i++) {
        const int64_t j = c * N + i;
        const double d = dt * s->rhs[j];
        const double inc = prev ? 1.5 * d - 0.5 * s->dq[j] : d;
        s->dq[j] = d;
        s->q[j] = s->q[j] + inc;
        acc += inc;
      }
      s->tot_rk[c] += acc * vol;
    }
    s->ab2_prev = 1;
    s->step++;
  }
  return ORA_OK;
}

/* Diagnostics at the current state with synchronous periodic derivatives (global reductions
 * are the I/O-time operations of Sec. 3.1): K = <rho |u|^2 / 2>, <eps> = <sigma_ij du_i/dx_j>,
 * Omega = <|curl u|^2>, M_t = <|u|^2>^{1/2} / (gamma R <T>)^{1/2} (Sec. 4). */
int ora_stats(ora_sim* s, double* out) {
  if (!s || !out) return ORA_E_INVAL;
  if (!s->initialised) return ORA_E_STATE;
  const ora_config* c = &s->c;
  const int64_t N = s->npts;
  compute_primitives(s, s->q);
  compute_gradients(s, 0, 1);
  double sm[NQ] = {0, 0, 0, 0, 0}, ke = 0, eps = 0, ens = 0, u2 = 0, tsum = 0, umax = 0;
  int nonfinite = 0;
  for (int64_t i = 0; i < N; i++) {
    double G[NG], sig[9], kt;
    for (int g = 0; g < NG; g++) G[g] = s->grad[(int64_t)g * N + i];
    const double rho = s->prim[i], u = s->prim[N + i], v = s->prim[2 * N + i], w = s->prim[3 * N + i];
    const double T = s->prim[4 * N + i];
    for (int cc = 0; cc < NQ; cc++) {
      const double qv = s->q[cc * N + i];
      if (!isfinite(qv)) nonfinite = 1;
      sm[cc] += qv;
    }
    const double uu = u * u + v * v + w * w;
    ke += 0.5 * rho * uu;
    u2 += uu;
    tsum += T;
    if (sqrt(uu) > umax) umax = sqrt(uu);
    stress(c, T, G, sig, &kt, s->cp);
    double e = 0.0;
    for (int a = 0; a < 9; a++) e += sig[a] * G[a];
    eps += e;
    const double ox = G[7] - G[5], oy = G[2] - G[6], oz = G[3] - G[1];
    ens += ox * ox + oy * oy + oz * oz;
  }
  const double vol = s->h[0] * s->h[1] * s->h[2];
  memset(out, 0, sizeof(double) * ORA_ST_COUNT);
  out[ORA_ST_STEP] = (double)s->step;
  out[ORA_ST_TIME] = (double)s->step * c->dt;
  out[ORA_ST_MASS] = sm[0] * vol;
  out[ORA_ST_MOMX] = sm[1] * vol;
  out[ORA_ST_MOMY] = sm[2] * vol;
  out[ORA_ST_MOMZ] = sm[3] * vol;
  out[ORA_ST_ENERGY] = sm[4] * vol;
  for (int cc = 0; cc < NQ; cc++) out[ORA_ST_MASS_RK + cc] = s->tot_rk[cc];
  out[ORA_ST_K] = ke / N;
  out[ORA_ST_EPS] = eps / N;
  out[ORA_ST_ENS] = ens / N;
  out[ORA_ST_MT] = sqrt(u2 / N) / sqrt(c->gamma * c->gas_r * (tsum / N));
  out[ORA_ST_UMAX] = umax;
  out[ORA_ST_NONFINITE] = nonfinite;
  return ORA_OK;
}

int ora_get_field(const ora_sim* s, double* q) {
  if (!s || !q) return ORA_E_INVAL;
  memcpy(q, s->q, sizeof(double) * NQ * s->npts);
  return ORA_OK;
}

int ora_get_flux(const ora_sim* s, double* out) {
  if (!s || !out) return ORA_E_INVAL;
  memcpy(out, s->flux, sizeof(double) * 3 * NQ * s->npts);
  return ORA_OK;
}

int64_t ora_step(const ora_sim* s) { return s ? s->step : -1; }

/* ------------------------------------------------------------------ test hooks */

/* Standard synchronous FD on the periodic grid, no PEs (Eq. du with the 4th-order stencil). */
int ora_rhs_periodic_standard(const ora_config* cfg, const double* q, double* out) {
  ora_config c = *cfg;
  c.p[0] = c.p[1] = c.p[2] = 1;
  c.forcing = 0;
  ora_sim* s;
  int rc = ora_create(&c, &s);
  if (rc) return rc;
  memcpy(s->q, q, sizeof(double) * NQ * s->npts);
  compute_primitives(s, s->q);
  compute_gradients(s, 0, 1);
  compute_fluxes(s, s->q);
  compute_divergence(s, s->q, 0, 1, out);
  ora_destroy(s);
  return ORA_OK;
}

/* Point fields behind the turbulence statistics of Sec. 4.1, with the synchronous central
 * derivatives of the run's order on the periodic grid (the derivatives ora_stats uses): out
 * [7][N] = u, v, w, p = rho R T, du/dx, the dissipation sigma_ij du_i/dx_j and |curl u|^2 --
 * the per-point terms whose means are <eps> and Omega in ora_stats. */
int ora_diag_fields(const ora_config* cfg, const double* q, double* out) {
  if (!cfg || !q || !out) return ORA_E_INVAL;
  ora_config c = *cfg;
  c.p[0] = c.p[1] = c.p[2] = 1;
  c.forcing = 0;
  ora_sim* s;
  int rc = ora_create(&c, &s);
  if (rc) return rc;
  const int64_t N = s->npts;
  compute_primitives(s, q);
  compute_gradients(s, 0, 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; i++) {
    double G[NG], sig[9], kt;
    for (int g = 0; g < NG; g++) G[g] = s->grad[(int64_t)g * N + i];
    const double rho = s->prim[i], T = s->prim[4 * N + i];
    for (int a = 0; a < 3; a++) out[a * N + i] = s->prim[(1 + a) * N + i];
    out[3 * N + i] = rho * c.gas_r * T;
    out[4 * N + i] = G[0];
    stress(&s->c, T, G, sig, &kt, s->cp);
    double e = 0.0;
    for (int a = 0; a < 9; a++) e += sig[a] * G[a];
    out[5 * N + i] = e;
    const double ox = G[7] - G[5], oy = G[2] - G[6], oz = G[3] - G[1];
    out[6 * N + i] = ox * ox + oy * oy + oz * oz;
  }
  ora_destroy(s);
  return ORA_OK;
}

/* Number of points whose stencil in some direction reaches across a PE face (N_B, Eq. NB),
 * counted by walking each point's stencil. */
int64_t ora_count_at_points(const ora_config* cfg) {
  if (check_config(cfg)) return -1;
  int e[3];
  for (int d = 0; d < 3; d++) e[d] = cfg->n[d] / cfg->p[d];
  const int M = layers_of(cfg);
  int64_t cnt = 0;
  for (int z = 0; z < cfg->n[2]; z++)
    for (int y = 0; y < cfg->n[1]; y++)
      for (int x = 0; x < cfg->n[0]; x++) {
        const int p[3] = {x, y, z};
        int ghost = 0;
        for (int d = 0; d < 3 && !ghost; d++)
          for (int m = -M; m <= M; m++) {
            const int l = p[d] % e[d] + m;
            if (l < 0 || l >= e[d]) ghost = 1;
          }
        cnt += ghost;
      }
  return cnt;
}
