// Host-side internals shared by the single-run C ABI (atns_host.hip) and the batched / served
// paths (batch.hip): the run handle, its workspace layout, error reporting and stage arguments.
#pragma once

#include <string>
#include <vector>

#include "atns_internal.h"

namespace atns {

// Records the message of the failing call (thread-local, read by at_last_error) and returns code.
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return ::atns::fail(AT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Williamson (1980) low-storage RK3 coefficients.
constexpr double kRkA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
constexpr double kRkB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
constexpr double kRkC[3] = {0.0, 1.0 / 3.0, 3.0 / 4.0};

inline size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Byte offsets of the workspace regions of one run.
struct Layout {
  size_t q[2], dq, ring, gv, flux, grad, tot_part, stat_part, stat_out, force_table, phase_x, phase_y, phase_z, total;
  int64_t ntot;  // FP64 total-accumulator slots (an upper bound on fused-stage workgroups)
};

struct EventTimer;

}  // namespace atns

struct at_batch;

struct at_sim {
  at_config cfg;
  atns::Geom g;
  atns::Layout L;
  hipStream_t stream;
  int device;
  uint8_t* ws;
  int8_t* d_sched = nullptr;
  int64_t sched_steps = 0;
  std::vector<uint8_t> step_delayed;  // per step: does any face read a delayed level
  int8_t* d_zero = nullptr;
  double* d_fhat = nullptr;
  std::vector<double> h_fhat;         // host copy of the forcing table (batched launches stage it)
  int64_t force_steps = 0;
  int* d_wv = nullptr;  // [2][40] kx and pair id of each wavevector, then [16][2] ky, kz per pair
  int npair = 0;
  int pair_ky[atns::kMaxPairs], pair_kz[atns::kMaxPairs];
  double* d_staging = nullptr;  // 5 N doubles
  int64_t step = 0;
  int initialised = 0;
  int qcur = 0;                 // which state buffer holds the current state
  int tile = 1;                 // fused-stage launch shape (index into tile_shape) and z chunk of
  int zchunk = 64;              // the stages that read no delayed level
  int tile_d = 1;               // the same for the stages that read delayed levels
  int zchunk_d = 64;
  int64_t tot_used = 0;               // FP64 total slots written by stage launches so far
  int ab2_prev = 0;                   // the RK register holds dt f^{n-1} of an Adams-Bashforth step
  atns::EventTimer* timer = nullptr;  // non-null while kernel timing is enabled
  at_batch* batch = nullptr;          // the batch this run is a member of, if any
};

namespace atns {

// Schedule and forcing tables must cover steps [first, first + count).
int check_step_tables(at_sim* s, int64_t first, int64_t count);

// Configuration checks of at_create (AT_OK or the error, with its message recorded).
int validate(const at_config* c);
// Grid, PE and ring geometry of a valid configuration.
Geom make_geom(const at_config* c);

// Removes a run from its batch (called when the run is destroyed).
void batch_forget(at_batch* b, at_sim* s);

template <typename T>
Coef<T> coef_of(const at_config& c) {
  Coef<T> cf{};
  for (int d = 0; d < 3; ++d) {
    cf.inv12h[d] = (T)(1.0 / (12.0 * (kTwoPi / c.n[d])));
    cf.inv60h[d] = (T)(1.0 / (60.0 * (kTwoPi / c.n[d])));
  }
  const double cv = c.gas_r / (c.gamma - 1.0);
  const double cp = c.gamma * c.gas_r / (c.gamma - 1.0);
  cf.gas_r = (T)c.gas_r;
  cf.inv_cv = (T)(1.0 / cv);
  cf.cp_over_pr = (T)(cp / c.prandtl);
  cf.mu_ref = (T)c.mu_ref;
  cf.inv_tref = (T)(1.0 / c.t_ref);
  cf.mu_exp = (T)c.mu_exp;
  cf.suth_s = (T)c.sutherland_s;
  cf.visc = c.visc_law;
  cf.form = c.form;
  return cf;
}

template <typename T>
Coef<T> make_coef(const at_sim* s) {
  return coef_of<T>(s->cfg);
}

// Stage arguments of run s at its current state (q = current buffer, q_out = the other).
template <typename T>
StageArgs<T> base_args(at_sim* s) {
  StageArgs<T> a{};
  a.g = s->g;
  a.cf = make_coef<T>(s);
  a.q = (T*)(s->ws + s->L.q[s->qcur]);
  a.q_out = (T*)(s->ws + s->L.q[1 - s->qcur]);
  a.dq = (T*)(s->ws + s->L.dq);
  a.ring = (T*)(s->ws + s->L.ring);
  a.gv_out = (T*)(s->ws + s->L.gv);
  a.gv = a.gv_out;
  a.at_ghost = tile_aligned(s->g, s->tile_d) ? 1 : 0;
  a.tot_part = (double*)(s->ws + s->L.tot_part);
  a.vol = (kTwoPi / s->cfg.n[0]) * (kTwoPi / s->cfg.n[1]) * (kTwoPi / s->cfg.n[2]);
  a.dt = (T)s->cfg.dt;
  a.force.table = nullptr;
  a.force.phase_y = (const T*)(s->ws + s->L.phase_y);
  a.force.phase_z = (const T*)(s->ws + s->L.phase_z);
  a.force.npair = s->npair;
  a.force.pair_kyz = s->d_wv + 2 * kNForce;
  return a;
}

}  // namespace atns
