// Host side of the C ABI (include/atns.h): validation, workspace layout, schedules, forcing
// tables, and the stage loop of the low-storage RK3 step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sim_internal.h"

using namespace atns;

namespace atns {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int check_step_tables(at_sim* s, int64_t first, int64_t count) {
  if (!s->d_sched || first + count > s->sched_steps)
    return fail(AT_E_SCHEDULE, "delay schedule does not cover the requested steps");
  if (s->cfg.forcing && (!s->d_fhat || first + count > s->force_steps))
    return fail(AT_E_SCHEDULE, "forcing table does not cover the requested steps");
  return AT_OK;
}

int validate(const at_config* c) {
  if (!c) return fail(AT_E_INVAL, "config is NULL");
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 4 || c->p[d] < 1) return fail(AT_E_INVAL, "n[d] >= 4 and p[d] >= 1 required");
    if (c->n[d] % c->p[d]) return fail(AT_E_INVAL, "n[d] must be a multiple of p[d]");
    if (c->n[d] > (1 << 14)) return fail(AT_E_INVAL, "n[d] too large");
  }
  if (c->order != 4 && c->order != 6) return fail(AT_E_INVAL, "order must be 4 or 6");
  const int M = c->order / 2;
  for (int d = 0; d < 3; ++d)
    if (c->n[d] / c->p[d] < 2 * M) return fail(AT_E_INVAL, "PE edge n[d]/p[d] must be >= order");
  if (c->order == 6 && c->forcing) return fail(AT_E_INVAL, "forcing is not implemented for the sixth-order scheme");
  if (c->form != 0 && c->form != 1) return fail(AT_E_INVAL, "form must be 0 or 1");
  if (c->visc_law != 0 && c->visc_law != 1) return fail(AT_E_INVAL, "visc_law must be 0 or 1");
  if (c->visc_law == 1 && (c->form != 1 || !(c->sutherland_s > 0.0) || !std::isfinite(c->sutherland_s)))
    return fail(AT_E_INVAL, "Sutherland's law needs form 1 and a positive constant");
  if (c->form == 1) {
    if (c->order != 4) return fail(AT_E_INVAL, "the paper's form is built with the fourth-order rows");
    if (c->forcing) return fail(AT_E_INVAL, "forcing is not implemented for the paper's form");
    for (int d = 0; d < 3; ++d)
      if (c->n[d] / c->p[d] < 5)
        return fail(AT_E_INVAL, "the paper's form needs PE edges >= 5 (one-sided mixed-derivative stencils)");
    if (12.0 * c->n[0] * c->n[1] * c->n[2] >= 4294967296.0)
      return fail(AT_E_INVAL, "grid too large for one handle (element offsets must stay below 2^32)");
  }
  if (c->max_delay < 0 || c->max_delay > kMaxDelay) return fail(AT_E_INVAL, "max_delay out of 0..8");
  if (c->precision != AT_FP64 && c->precision != AT_FP32) return fail(AT_E_INVAL, "bad precision");
  if (c->forcing != 0 && c->forcing != 1) return fail(AT_E_INVAL, "forcing must be 0 or 1");
  {
    // the stage kernel indexes fields and the ring with 32-bit element offsets
    const double npts = (double)c->n[0] * c->n[1] * c->n[2];
    double slab = 0.0;
    for (int d = 0; d < 3; ++d) slab += 2.0 * M * c->p[d] * npts / c->n[d];
    if ((c->order == 6 ? 3 * kNQ : kNQ) * npts >= 4294967296.0 ||
        (c->max_delay + M + 1) * kNRing * slab >= 4294967296.0)
      return fail(AT_E_INVAL, "grid too large for one handle (element offsets must stay below 2^32)");
  }
  if (!(c->gamma > 1.0) || !(c->gas_r > 0.0) || !(c->prandtl > 0.0) || !(c->t_ref > 0.0) ||
      !(c->mu_ref >= 0.0) || !(c->dt > 0.0) || !std::isfinite(c->mu_exp))
    return fail(AT_E_INVAL, "bad physical parameter");
  return AT_OK;
}

Geom make_geom(const at_config* c) {
  Geom g{};
  g.form = c->form;
  g.order = c->order;
  g.M = c->order / 2;
  g.tl = g.M + 1;
  g.npts = 1;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c->n[d];
    g.p[d] = c->p[d];
    g.e[d] = c->n[d] / c->p[d];
    g.npts *= c->n[d];
  }
  g.slab[0] = (int64_t)2 * g.M * c->p[0] * c->n[1] * c->n[2];
  g.slab[1] = (int64_t)2 * g.M * c->p[1] * c->n[0] * c->n[2];
  g.slab[2] = (int64_t)2 * g.M * c->p[2] * c->n[0] * c->n[1];
  // components per published point: u, v, w, T and the face-normal flux, or the five conserved
  // variables of the paper's form
  const int ncomp = c->form == 1 ? kNQ : kNRing;
  g.ring_dir_off[0] = 0;
  g.ring_dir_off[1] = ncomp * g.slab[0];
  g.ring_dir_off[2] = ncomp * (g.slab[0] + g.slab[1]);
  g.ring_slot = ncomp * (g.slab[0] + g.slab[1] + g.slab[2]);
  g.R = c->max_delay + g.tl;
  g.ntiles = c->p[0] * c->p[1] * c->p[2];
  return g;
}

}  // namespace atns

namespace {


Layout make_layout(const at_config* c, const Geom& g) {
  const size_t w = c->precision == AT_FP32 ? 4 : 8;
  const size_t N = (size_t)g.npts;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.q[0] = take(kNQ * N * w);
  L.q[1] = take(kNQ * N * w);
  L.dq = take(kNQ * N * w);
  L.ring = take((size_t)g.R * g.ring_slot * w);
  // per stage of a step, in ring-slot layout: the AT sums (fourth order) or the extrapolated face
  // values (sixth order); the flux buffer (sixth order)
  L.gv = take(c->form == 0 ? (size_t)3 * g.ring_slot * w : 0);
  L.flux = take(c->order == 6 ? (size_t)3 * kNQ * N * w : 0);
  L.grad = take(c->form == 1 ? (size_t)kNGrad * N * w : 0);
  // smallest tile (16 x 4) and smallest z chunk (4) bound the workgroup count of any stage launch
  L.ntot = (int64_t)((c->n[0] + 15) / 16) * ((c->n[1] + 3) / 4) * ((c->n[2] + 3) / 4);
  if (c->order == 6) L.ntot = std::max<int64_t>(L.ntot, blocks6(g));
  if (c->form == 1) L.ntot = std::max<int64_t>(L.ntot, paper_blocks(g));
  L.tot_part = take((size_t)L.ntot * kNQ * 8);
  L.stat_part = take((size_t)stats_blocks(g) * kNStat * 8);
  L.stat_out = take(kStatOutBytes);
  L.force_table = take((size_t)kMaxPairs * c->n[0] * 6 * w);
  L.phase_x = take((size_t)5 * c->n[0] * 2 * w);
  L.phase_y = take((size_t)5 * c->n[1] * 2 * w);
  L.phase_z = take((size_t)3 * c->n[2] * 2 * w);
  L.total = off;
  return L;
}

}  // namespace

// HIP events around each launch; pairs are harvested when timings are queried.
struct atns::EventTimer final : LaunchHook {
  struct Pending {
    int id;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  hipEvent_t open_ev = nullptr;
  double total_ms[kKCount] = {};
  int64_t launches[kKCount] = {};
  bool failed = false;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) failed = true;
    return e;
  }
  void before(int, hipStream_t s) override {
    open_ev = get();
    if (open_ev && hipEventRecord(open_ev, s) != hipSuccess) failed = true;
  }
  void after(int id, hipStream_t s) override {
    hipEvent_t e = get();
    if (e && hipEventRecord(e, s) != hipSuccess) failed = true;
    pending.push_back({id, open_ev, e});
    open_ev = nullptr;
  }
  hipError_t harvest(hipStream_t s) {
    hipError_t err = hipStreamSynchronize(s);
    if (err != hipSuccess) return err;
    for (const Pending& p : pending) {
      float ms = 0.f;
      if (p.a && p.b && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        total_ms[p.id] += ms;
        launches[p.id] += 1;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return hipSuccess;
  }
  void reset() {
    for (int i = 0; i < kKCount; ++i) {
      total_ms[i] = 0.0;
      launches[i] = 0;
    }
  }
  ~EventTimer() override {
    for (hipEvent_t e : pool)
      if (e) (void)hipEventDestroy(e);
    for (const Pending& p : pending) {
      if (p.a) (void)hipEventDestroy(p.a);
      if (p.b) (void)hipEventDestroy(p.b);
    }
  }
};

namespace {



// Forcing wavevectors in the documented order, and the (ky, kz) pair of each.
void forcing_lists(int kx[kNForce], int pair[kNForce], int pky[kMaxPairs], int pkz[kMaxPairs],
                   int* npair) {
  int nk = 0, np = 0;
  for (int kz = -2; kz <= 2; ++kz)
    for (int ky = -2; ky <= 2; ++ky)
      for (int x = -2; x <= 2; ++x) {
        const int k2 = x * x + ky * ky + kz * kz;
        if (k2 == 0 || k2 > 6) continue;
        if (!(kz > 0 || (kz == 0 && ky > 0) || (kz == 0 && ky == 0 && x > 0))) continue;
        int pid = -1;
        for (int j = 0; j < np; ++j)
          if (pky[j] == ky && pkz[j] == kz) pid = j;
        if (pid < 0) {
          pid = np++;
          pky[pid] = ky;
          pkz[pid] = kz;
        }
        kx[nk] = x;
        pair[nk] = pid;
        ++nk;
      }
  *npair = np;
}

template <typename T>
int upload_phases(at_sim* s) {
  auto table = [&](int n, int m0, int nm, size_t off) -> int {
    std::vector<T> h((size_t)nm * n * 2);
    for (int m = 0; m < nm; ++m)
      for (int j = 0; j < n; ++j) {
        const double ph = (double)(m0 + m) * kTwoPi * j / n;
        h[((size_t)m * n + j) * 2] = (T)std::cos(ph);
        h[((size_t)m * n + j) * 2 + 1] = (T)std::sin(ph);
      }
    HIP_TRY(hipMemcpyAsync(s->ws + off, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return AT_OK;
  };
  int rc = table(s->cfg.n[0], -2, 5, s->L.phase_x);
  if (!rc) rc = table(s->cfg.n[1], -2, 5, s->L.phase_y);
  if (!rc) rc = table(s->cfg.n[2], 0, 3, s->L.phase_z);
  return rc;
}

uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
hipError_t launch_hooked(at_sim* s, const StageArgs<T>& a, int mode, bool at) {
  const int id = mode == kModeStepH ? kKStage : (mode == kModeRhsH ? kKRhs : kKPublish);
  if (s->timer) s->timer->before(id, s->stream);
  hipError_t e = launch_fused<T>(a, at ? s->tile_d : s->tile, at ? s->zchunk_d : s->zchunk, mode, at, s->stream);
  if (s->timer) s->timer->after(id, s->stream);
  return e;
}

// Sixth-order stage arguments of run s at its current state and step.
template <typename T>
Stage6Args<T> base6(at_sim* s) {
  Stage6Args<T> a{};
  a.g = s->g;
  a.cf = make_coef<T>(s);
  for (int d = 0; d < 3; ++d) a.i60h[d] = a.cf.inv60h[d];
  a.q = (T*)(s->ws + s->L.q[s->qcur]);
  a.q_out = (T*)(s->ws + s->L.q[1 - s->qcur]);
  a.dq = (T*)(s->ws + s->L.dq);
  a.flux = (T*)(s->ws + s->L.flux);
  a.ring = (T*)(s->ws + s->L.ring);
  a.gv = (T*)(s->ws + s->L.gv);
  a.tot_part = (double*)(s->ws + s->L.tot_part);
  tile6_of(s->g, &a.bx, &a.by);
  a.delays = s->d_sched ? s->d_sched + (size_t)s->step * s->g.ntiles * 6 : s->d_zero;
  a.step_mod_r = (int)(s->step % s->g.R);
  a.mode = kModeStepH;
  a.dt = (T)s->cfg.dt;
  a.vol = (kTwoPi / s->cfg.n[0]) * (kTwoPi / s->cfg.n[1]) * (kTwoPi / s->cfg.n[2]);
  return a;
}

// The two launches of one sixth-order stage (the second left out when only publishing).
template <typename T>
hipError_t launch6_hooked(at_sim* s, const Stage6Args<T>& a, bool div) {
  if (s->timer) s->timer->before(kK6Grad, s->stream);
  hipError_t e = launch_stage6<T>(a, true, s->stream);
  if (s->timer) s->timer->after(kK6Grad, s->stream);
  if (e != hipSuccess || !div) return e;
  if (s->timer) s->timer->before(kK6Div, s->stream);
  e = launch_stage6<T>(a, false, s->stream);
  if (s->timer) s->timer->after(kK6Div, s->stream);
  return e;
}

// The sixth-order extrapolated face values of the current step for its nst stages (c_s = kRkC[st],
// or 0 for one Adams-Bashforth or RHS stage), once per step that reads delayed levels.
template <typename T>
hipError_t launch_ghosts6_hooked(at_sim* s, int nst) {
  if (!s->d_sched || !s->step_delayed[(size_t)s->step]) return hipSuccess;
  Stage6Args<T> a = base6<T>(s);
  a.nst = nst;
  for (int st = 0; st < 3; ++st) a.cs3[st] = nst == 3 ? (T)kRkC[st] : T(0);
  if (s->timer) s->timer->before(kK6Ghost, s->stream);
  hipError_t e = launch_ghosts6<T>(a, s->stream);
  if (s->timer) s->timer->after(kK6Ghost, s->stream);
  return e;
}

template <typename T>
hipError_t launch_views(at_sim* s, const StageArgs<T>& a, int nst = 3) {
  if (s->timer) s->timer->before(kKGhost, s->stream);
  hipError_t e = launch_at_sums<T>(a, kRkC, s->stream, nst);
  if (s->timer) s->timer->after(kKGhost, s->stream);
  return e;
}

// Arguments of the paper's form (form 1) at the current state and step.
template <typename T>
StagePArgs<T> basep(at_sim* s) {
  StagePArgs<T> a{};
  a.g = s->g;
  a.cf = make_coef<T>(s);
  a.q = (T*)(s->ws + s->L.q[s->qcur]);
  a.q_out = (T*)(s->ws + s->L.q[1 - s->qcur]);
  a.dq = (T*)(s->ws + s->L.dq);
  a.grad = (T*)(s->ws + s->L.grad);
  a.ring = (T*)(s->ws + s->L.ring);
  a.tot_part = (double*)(s->ws + s->L.tot_part);
  a.delays = s->d_sched ? s->d_sched + (size_t)s->step * s->g.ntiles * 6 : s->d_zero;
  a.step_mod_r = (int)(s->step % s->g.R);
  a.slot = a.step_mod_r;
  a.mode = kModeStepH;
  a.dt = (T)s->cfg.dt;
  a.vol = (kTwoPi / s->cfg.n[0]) * (kTwoPi / s->cfg.n[1]) * (kTwoPi / s->cfg.n[2]);
  return a;
}

template <typename T>
hipError_t launchp_hooked(at_sim* s, const StagePArgs<T>& a, int which) {
  const int id = which == kPPublish ? kKPPublish : (which == kPRhs ? kKPRhs : kKPGrad);
  if (s->timer) s->timer->before(id, s->stream);
  hipError_t e = launch_stagep<T>(a, which, s->stream);
  if (s->timer) s->timer->after(id, s->stream);
  return e;
}

// One RHS evaluation of the paper's form (its gradients, publishing level n at stage 1 of a step
// when asked, then every term and the update).
template <typename T>
hipError_t stagep(at_sim* s, const StagePArgs<T>& a, bool publish = false) {
  hipError_t e = launchp_hooked<T>(s, a, publish ? kPGradPublish : kPGrad);
  if (e != hipSuccess) return e;
  return launchp_hooked<T>(s, a, kPRhs);
}

template <typename T>
int do_stats(at_sim* s, double* host_out) {
  const Coef<T> cf = make_coef<T>(s);
  double* part = (double*)(s->ws + s->L.stat_part);
  double* out = (double*)(s->ws + s->L.stat_out);
  HIP_TRY(launch_stats<T>(s->g, cf, (const T*)(s->ws + s->L.q[s->qcur]), part, out,
                          (const double*)(s->ws + s->L.tot_part), s->tot_used, s->cfg.gamma,
                          s->stream, s->timer));
  if (host_out) {
    // the statistics, the RK totals and the initial totals (kStatInit) in one copy
    HIP_TRY(hipMemcpyAsync(host_out, out, (kStatInit + kNQ) * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return AT_OK;
}

template <typename T>
int do_init(at_sim* s, const double* q_host, int nlev) {
  const int64_t N = s->g.npts;
  s->qcur = 0;
  T* q = (T*)(s->ws + s->L.q[0]);
  for (int lev = 0; lev < nlev; ++lev) {
    HIP_TRY(hipMemcpyAsync(s->d_staging, q_host + (size_t)lev * kNQ * N, sizeof(double) * kNQ * N,
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_convert<T>(s->d_staging, q, kNQ * N, s->stream));
    if (lev < nlev - 1 && s->g.form == 1) {
      StagePArgs<T> a = basep<T>(s);
      a.slot = (int)(lev % s->g.R);
      HIP_TRY(launchp_hooked<T>(s, a, kPPublish));
    } else if (lev < nlev - 1 && s->g.order == 6) {
      Stage6Args<T> a = base6<T>(s);
      a.delays = s->d_zero;
      a.step_mod_r = (int)(lev % s->g.R);
      a.publish = 1;
      HIP_TRY(launch6_hooked<T>(s, a, false));
    } else if (lev < nlev - 1) {
      // publish the history level with synchronous derivatives (all delays zero)
      StageArgs<T> a = base_args<T>(s);
      a.delays = s->d_zero;
      a.step = lev;
      a.step_mod_r = (int)(lev % s->g.R);
      a.publish = 1;
      HIP_TRY(launch_hooked<T>(s, a, kModePublishH, false));
    }
  }
  HIP_TRY(hipMemsetAsync(s->ws + s->L.dq, 0, sizeof(T) * kNQ * N, s->stream));
  HIP_TRY(hipMemsetAsync(s->ws + s->L.tot_part, 0, sizeof(double) * kNQ * s->L.ntot, s->stream));
  s->tot_used = 0;
  // the initial totals stay on the device (read with the statistics): no synchronisation here
  int rc = do_stats<T>(s, nullptr);
  if (rc) return rc;
  double* out = (double*)(s->ws + s->L.stat_out);
  HIP_TRY(hipMemcpyAsync(out + kStatInit, out, kNQ * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
  s->step = nlev - 1;
  s->ab2_prev = 0;
  s->initialised = 1;
  return AT_OK;
}


// Sixth-order RK3 steps: per stage the gradient / flux launch (publishing at stage 1) and the
// divergence / update launch; delayed faces extrapolate to t_n + c_s dt.
template <typename T>
int do_steps6(at_sim* s, int nsteps) {
  if (nsteps > 0) s->tot_used = std::max(s->tot_used, blocks6(s->g));
  for (int it = 0; it < nsteps; ++it) {
    HIP_TRY(launch_ghosts6_hooked<T>(s, 3));
    for (int st = 0; st < 3; ++st) {
      Stage6Args<T> a = base6<T>(s);
      a.gv += (size_t)st * s->g.ring_slot;
      a.cs = (T)kRkC[st];
      a.rk_a = (T)kRkA[st];
      a.rk_b = (T)kRkB[st];
      a.publish = st == 0;
      a.store_dq = st < 2;
      HIP_TRY(launch6_hooked<T>(s, a, true));
      s->qcur = 1 - s->qcur;
    }
    s->step++;
  }
  return AT_OK;
}

// The paper's form: publication at the start of each step, then per stage the gradients and the
// right-hand side with the update (RK3), or one such stage per step (AB2, c_s = 0).
template <typename T>
int do_stepsp(at_sim* s, int nsteps, bool ab2) {
  if (nsteps > 0) s->tot_used = std::max(s->tot_used, paper_blocks(s->g));
  for (int it = 0; it < nsteps; ++it) {
    for (int st = 0; st < (ab2 ? 1 : 3); ++st) {
      StagePArgs<T> a = basep<T>(s);
      if (ab2) {
        a.rk_b = s->ab2_prev ? T(1.5) : T(1);
        a.c_prev = s->ab2_prev ? T(-0.5) : T(0);
        a.store_dq = 1;
      } else {
        a.cs = (T)kRkC[st];
        a.rk_a = (T)kRkA[st];
        a.rk_b = (T)kRkB[st];
        a.store_dq = st < 2;
      }
      HIP_TRY(stagep<T>(s, a, st == 0));
      s->qcur = 1 - s->qcur;
    }
    s->ab2_prev = ab2 ? 1 : 0;
    s->step++;
  }
  return AT_OK;
}

template <typename T>
int do_steps(at_sim* s, int nsteps) {
  if (s->g.form == 1) return do_stepsp<T>(s, nsteps, false);
  if (s->g.order == 6) return do_steps6<T>(s, nsteps);
  const size_t row = (size_t)s->g.ntiles * 6;
  if (nsteps > 0)
    s->tot_used = std::max({s->tot_used, fused_blocks(s->g, s->tile, s->zchunk), fused_blocks(s->g, s->tile_d, s->zchunk_d)});
  for (int it = 0; it < nsteps; ++it) {
    StageArgs<T> a = base_args<T>(s);
    a.delays = s->d_sched + (size_t)s->step * row;
    a.step = s->step;
    a.step_mod_r = (int)(s->step % s->g.R);
    if (s->cfg.forcing) {
      T* tab = (T*)(s->ws + s->L.force_table);
      HIP_TRY(launch_force_table<T>(s->g, s->d_fhat + (size_t)s->step * kNForce * 6, s->d_wv,
                                    s->d_wv + kNForce, s->npair, tab,
                                    (const T*)(s->ws + s->L.phase_x), s->stream, s->timer));
      a.force.table = tab;
    }
    for (int st = 0; st < 3; ++st) {
      a.q = (T*)(s->ws + s->L.q[s->qcur]);
      a.q_out = (T*)(s->ws + s->L.q[1 - s->qcur]);
      a.gv = a.gv_out + (size_t)st * s->g.ring_slot;
      a.rk_a = (T)kRkA[st];
      a.rk_b = (T)kRkB[st];
      a.publish = st == 0;
      a.store_dq = st < 2;
      // the AT sums of all three stages, once per step that reads delayed levels
      if (st == 0 && s->step_delayed[(size_t)s->step]) HIP_TRY(launch_views<T>(s, a));
      HIP_TRY(launch_hooked<T>(s, a, kModeStepH, s->step_delayed[(size_t)s->step] != 0));
      s->qcur = 1 - s->qcur;
    }
    s->step++;
  }
  return AT_OK;
}

// Second-order Adams-Bashforth steps (Sec. 2.2, Eq. time_ab, beta = 3/2, -1/2): one stage per
// step at t_n (the AT sums of c_s = 0, the first of the three regions), publishing level n; the
// register keeps dt f^n for the next step.  Without a stored dt f^{n-1} the step is forward Euler
// (the Runge-Kutta update with A = 0, B = 1).
template <typename T>
int do_ab2_steps(at_sim* s, int nsteps) {
  if (s->g.form == 1) return do_stepsp<T>(s, nsteps, true);
  if (s->g.order == 6) {
    if (nsteps > 0) s->tot_used = std::max(s->tot_used, blocks6(s->g));
    for (int it = 0; it < nsteps; ++it) {
      HIP_TRY(launch_ghosts6_hooked<T>(s, 1));
      Stage6Args<T> a = base6<T>(s);
      a.rk_b = s->ab2_prev ? T(1.5) : T(1);
      a.c_prev = s->ab2_prev ? T(-0.5) : T(0);
      a.publish = 1;
      a.store_dq = 1;
      HIP_TRY(launch6_hooked<T>(s, a, true));
      s->qcur = 1 - s->qcur;
      s->ab2_prev = 1;
      s->step++;
    }
    return AT_OK;
  }
  const size_t row = (size_t)s->g.ntiles * 6;
  if (nsteps > 0)
    s->tot_used = std::max({s->tot_used, fused_blocks(s->g, s->tile, s->zchunk), fused_blocks(s->g, s->tile_d, s->zchunk_d)});
  for (int it = 0; it < nsteps; ++it) {
    StageArgs<T> a = base_args<T>(s);
    a.delays = s->d_sched + (size_t)s->step * row;
    a.step = s->step;
    a.step_mod_r = (int)(s->step % s->g.R);
    if (s->cfg.forcing) {
      T* tab = (T*)(s->ws + s->L.force_table);
      HIP_TRY(launch_force_table<T>(s->g, s->d_fhat + (size_t)s->step * kNForce * 6, s->d_wv,
                                    s->d_wv + kNForce, s->npair, tab,
                                    (const T*)(s->ws + s->L.phase_x), s->stream, s->timer));
      a.force.table = tab;
    }
    a.gv = a.gv_out;
    a.rk_a = T(0);
    a.rk_b = s->ab2_prev ? T(1.5) : T(1);
    a.c_prev = s->ab2_prev ? T(-0.5) : T(0);
    a.publish = 1;
    a.store_dq = 1;
    if (s->step_delayed[(size_t)s->step]) HIP_TRY(launch_views<T>(s, a, 1));  // the c_s = 0 sums only
    HIP_TRY(launch_hooked<T>(s, a, kModeStepH, s->step_delayed[(size_t)s->step] != 0));
    s->qcur = 1 - s->qcur;
    s->ab2_prev = 1;
    s->step++;
  }
  return AT_OK;
}

template <typename T>
int do_rhs(at_sim* s, void* out) {
  if (s->g.form == 1) {
    StagePArgs<T> a = basep<T>(s);
    a.mode = kModeRhsH;
    a.rhs_out = (T*)out;
    HIP_TRY(stagep<T>(s, a));
    return AT_OK;
  }
  if (s->g.order == 6) {
    HIP_TRY(launch_ghosts6_hooked<T>(s, 1));
    Stage6Args<T> a = base6<T>(s);
    a.mode = kModeRhsH;
    a.rhs_out = (T*)out;
    HIP_TRY(launch6_hooked<T>(s, a, true));
    return AT_OK;
  }
  StageArgs<T> a = base_args<T>(s);
  a.delays = s->d_sched + (size_t)s->step * s->g.ntiles * 6;
  a.step = s->step;
  a.step_mod_r = (int)(s->step % s->g.R);
  a.rk_a = T(0);
  a.rk_b = T(0);
  a.publish = 0;
  a.rhs_out = (T*)out;
  if (s->cfg.forcing) {
    T* tab = (T*)(s->ws + s->L.force_table);
    HIP_TRY(launch_force_table<T>(s->g, s->d_fhat + (size_t)s->step * kNForce * 6, s->d_wv,
                                  s->d_wv + kNForce, s->npair, tab, (const T*)(s->ws + s->L.phase_x),
                                  s->stream, s->timer));
    a.force.table = tab;
  }
  if (s->step_delayed[(size_t)s->step]) HIP_TRY(launch_views<T>(s, a));
  HIP_TRY(launch_hooked<T>(s, a, kModeRhsH, s->step_delayed[(size_t)s->step] != 0));
  return AT_OK;
}

template <typename T>
int do_get_field(at_sim* s, double* q_host) {
  const int64_t N = s->g.npts;
  HIP_TRY(launch_to_double<T>((const T*)(s->ws + s->L.q[s->qcur]), s->d_staging, kNQ * N, s->stream));
  HIP_TRY(hipMemcpyAsync(q_host, s->d_staging, sizeof(double) * kNQ * N, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return AT_OK;
}

}  // namespace

extern "C" {

const char* at_version(void) { return "atns 0.1 (gfx950)"; }

const char* at_last_error(void) { return g_last_error.c_str(); }

size_t at_workspace_bytes(const at_config* cfg) {
  if (validate(cfg)) return 0;
  const Geom g = make_geom(cfg);
  return make_layout(cfg, g).total;
}

int at_create(const at_config* cfg, void* ws, size_t ws_bytes, void* stream, at_sim** out) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!out) return fail(AT_E_INVAL, "out is NULL");
  const Geom g = make_geom(cfg);
  const Layout L = make_layout(cfg, g);
  if (!ws || ((uintptr_t)ws & 255)) return fail(AT_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (ws_bytes < L.total) return fail(AT_E_WORKSPACE, "workspace smaller than at_workspace_bytes");
  at_sim* s = new (std::nothrow) at_sim();
  if (!s) return fail(AT_E_INVAL, "out of host memory");
  s->cfg = *cfg;
  s->g = g;
  s->L = L;
  s->stream = (hipStream_t)stream;
  s->ws = (uint8_t*)ws;
  // default launch shape: 32 x 8 columns if it fits the LDS at this precision, else 16 x 8
  s->tile = fused_lds_bytes(1, cfg->precision == AT_FP32 ? 4 : 8, cfg->forcing != 0) <= kLdsBytes ? 1 : 5;
  s->zchunk = cfg->n[2] / cfg->p[2] >= 16 ? cfg->n[2] / cfg->p[2] : cfg->n[2];
  if (s->zchunk > 128) s->zchunk = 128;
  s->tile_d = s->tile;
  s->zchunk_d = s->zchunk;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc(&s->d_zero, (size_t)g.ntiles * 6);
  if (e == hipSuccess) e = hipMemsetAsync(s->d_zero, 0, (size_t)g.ntiles * 6, s->stream);
  if (e == hipSuccess) e = hipMalloc(&s->d_staging, sizeof(double) * kNQ * g.npts);
  if (e == hipSuccess) e = hipMalloc(&s->d_wv, sizeof(int) * (2 * kNForce + 2 * kMaxPairs));
  if (e != hipSuccess) {
    at_destroy(s);
    return fail(AT_E_HIP, std::string("allocation: ") + hipGetErrorString(e));
  }
  int wv[2 * kNForce + 2 * kMaxPairs] = {};
  forcing_lists(wv, wv + kNForce, s->pair_ky, s->pair_kz, &s->npair);
  for (int i = 0; i < s->npair; ++i) {
    wv[2 * kNForce + 2 * i] = s->pair_ky[i];
    wv[2 * kNForce + 2 * i + 1] = s->pair_kz[i];
  }
  e = hipMemcpyAsync(s->d_wv, wv, sizeof(wv), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    at_destroy(s);
    return fail(AT_E_HIP, std::string("upload: ") + hipGetErrorString(e));
  }
  rc = cfg->precision == AT_FP32 ? upload_phases<float>(s) : upload_phases<double>(s);
  if (rc) {
    at_destroy(s);
    return rc;
  }
  *out = s;
  return AT_OK;
}

int at_init_field(at_sim* s, const double* q_host, int32_t n_levels) {
  if (!s || !q_host) return fail(AT_E_INVAL, "NULL argument");
  if (n_levels < 1 || n_levels > s->g.R) return fail(AT_E_INVAL, "n_levels must be in 1 .. max_delay + t_l");
  return s->cfg.precision == AT_FP32 ? do_init<float>(s, q_host, n_levels) : do_init<double>(s, q_host, n_levels);
}

int at_set_delay_schedule(at_sim* s, int32_t mode, int32_t L, int32_t c_r, uint64_t seed,
                          const int8_t* table, int64_t n_steps) {
  if (!s) return fail(AT_E_INVAL, "NULL handle");
  if (n_steps < 1 || n_steps > (int64_t)1 << 24) return fail(AT_E_INVAL, "n_steps out of range");
  const int nt = s->g.ntiles;
  std::vector<int8_t> t((size_t)n_steps * nt * 6, 0);
  switch (mode) {
    case AT_SYNC:
      break;
    case AT_CAA:
      // synchronous for the first max(c_r, t_l) steps (the levels one extrapolation needs)
      if (c_r < 1 || L != c_r - 1) return fail(AT_E_INVAL, "CAA needs c_r >= 1 and L = c_r - 1");
      for (int64_t n = std::max(c_r, s->g.tl); n < n_steps; ++n)
        std::memset(&t[(size_t)n * nt * 6], (int)(n % c_r), (size_t)nt * 6);
      break;
    case AT_SAA:
      // synchronous for the first L + t_l steps (Alg. SAA)
      if (L < 0) return fail(AT_E_INVAL, "SAA needs L >= 0");
      for (int64_t n = L + s->g.tl; n < n_steps; ++n)
        for (int ti = 0; ti < nt; ++ti)
          for (int f = 0; f < 6; ++f) {
            const uint64_t ctr = ((uint64_t)n * nt + ti) * 6u + f;
            const uint64_t z = splitmix64(seed, ctr);
            t[((size_t)n * nt + ti) * 6 + f] = (int8_t)(((z >> 32) * (uint64_t)(L + 1)) >> 32);
          }
      break;
    case AT_EXPLICIT:
      if (!table) return fail(AT_E_INVAL, "EXPLICIT needs a table");
      std::memcpy(t.data(), table, t.size());
      break;
    default:
      return fail(AT_E_INVAL, "unknown delay mode");
  }
  for (int64_t n = 0; n < n_steps; ++n)
    for (int i = 0; i < nt * 6; ++i) {
      const int k = t[(size_t)n * nt * 6 + i];
      if (k < 0 || k > s->cfg.max_delay || (k > 0 && n - k - (s->g.tl - 1) < 0))
        return fail(AT_E_SCHEDULE, "schedule entry out of range or reads a level before 0");
    }
  if (s->d_sched) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipFree(s->d_sched));
    s->d_sched = nullptr;
  }
  s->step_delayed.assign((size_t)n_steps, 0);
  for (int64_t n = 0; n < n_steps; ++n)
    for (int i = 0; i < nt * 6; ++i)
      if (t[(size_t)n * nt * 6 + i] > 0) s->step_delayed[(size_t)n] = 1;
  HIP_TRY(hipMalloc(&s->d_sched, t.size()));
  HIP_TRY(hipMemcpyAsync(s->d_sched, t.data(), t.size(), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->sched_steps = n_steps;
  return AT_OK;
}

int at_set_forcing(at_sim* s, const double* fhat, int64_t n_steps) {
  if (!s || !fhat) return fail(AT_E_INVAL, "NULL argument");
  if (!s->cfg.forcing) return fail(AT_E_INVAL, "forcing is disabled in the config");
  if (n_steps < 1) return fail(AT_E_INVAL, "n_steps < 1");
  const size_t bytes = sizeof(double) * (size_t)n_steps * kNForce * 6;
  if (s->d_fhat) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipFree(s->d_fhat));
    s->d_fhat = nullptr;
  }
  HIP_TRY(hipMalloc(&s->d_fhat, bytes));
  HIP_TRY(hipMemcpyAsync(s->d_fhat, fhat, bytes, hipMemcpyHostToDevice, s->stream));
  s->h_fhat.assign(fhat, fhat + (size_t)n_steps * kNForce * 6);
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->force_steps = n_steps;
  return AT_OK;
}

int at_rhs(at_sim* s, void* out) {
  if (!s || !out) return fail(AT_E_INVAL, "NULL argument");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field first");
  int rc = check_step_tables(s, s->step, 1);
  if (rc) return rc;
  return s->cfg.precision == AT_FP32 ? do_rhs<float>(s, out) : do_rhs<double>(s, out);
}

int at_rk_step(at_sim* s, int32_t n_steps) {
  if (!s) return fail(AT_E_INVAL, "NULL handle");
  if (n_steps < 0) return fail(AT_E_INVAL, "n_steps < 0");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field first");
  int rc = check_step_tables(s, s->step, n_steps);
  if (rc) return rc;
  s->ab2_prev = 0;  // the register now holds the Runge-Kutta one
  return s->cfg.precision == AT_FP32 ? do_steps<float>(s, n_steps) : do_steps<double>(s, n_steps);
}

int at_ab2_step(at_sim* s, int32_t n_steps) {
  if (!s) return fail(AT_E_INVAL, "NULL handle");
  if (n_steps < 0) return fail(AT_E_INVAL, "n_steps < 0");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field first");
  int rc = check_step_tables(s, s->step, n_steps);
  if (rc) return rc;
  return s->cfg.precision == AT_FP32 ? do_ab2_steps<float>(s, n_steps) : do_ab2_steps<double>(s, n_steps);
}

int at_stats(at_sim* s, at_stats_t* out) {
  if (!s || !out) return fail(AT_E_INVAL, "NULL argument");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field first");
  double st[kStatInit + kNQ];
  int rc = s->cfg.precision == AT_FP32 ? do_stats<float>(s, st) : do_stats<double>(s, st);
  if (rc) return rc;
  const double N = (double)s->g.npts;
  const double vol = (kTwoPi / s->cfg.n[0]) * (kTwoPi / s->cfg.n[1]) * (kTwoPi / s->cfg.n[2]);
  double tot_init[kNQ];
  for (int c = 0; c < kNQ; ++c) tot_init[c] = st[kStatInit + c] * vol;
  std::memset(out, 0, sizeof(*out));
  out->step = s->step;
  out->time = (double)s->step * s->cfg.dt;
  out->mass = st[0] * vol;
  for (int a = 0; a < 3; ++a) out->mom[a] = st[1 + a] * vol;
  out->energy = st[4] * vol;
  out->mass_rk = tot_init[0] + st[kNStat + 0];
  for (int a = 0; a < 3; ++a) out->mom_rk[a] = tot_init[1 + a] + st[kNStat + 1 + a];
  out->energy_rk = tot_init[4] + st[kNStat + 4];
  out->K = st[5] / N;
  out->eps = st[6] / N;
  out->enstrophy = st[7] / N;
  out->Mt = std::sqrt(st[8] / N) / std::sqrt(s->cfg.gamma * s->cfg.gas_r * (st[9] / N));
  out->umax = st[10];
  out->nonfinite = st[11] != 0.0;
  return AT_OK;
}

int at_get_field(at_sim* s, double* q_host) {
  if (!s || !q_host) return fail(AT_E_INVAL, "NULL argument");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field first");
  return s->cfg.precision == AT_FP32 ? do_get_field<float>(s, q_host) : do_get_field<double>(s, q_host);
}

int at_field_device(at_sim* s, void** ptr) {
  if (!s || !ptr) return fail(AT_E_INVAL, "NULL argument");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field first");
  *ptr = s->ws + s->L.q[s->qcur];
  return AT_OK;
}

namespace {
int check_shape(const at_sim* s, int32_t tile, int32_t zchunk) {
  if (tile < 0 || tile >= kTileCount) return fail(AT_E_INVAL, "unknown tile shape");
  if (zchunk < 4) return fail(AT_E_INVAL, "z chunk must be >= 4");
  const size_t word = s->cfg.precision == AT_FP32 ? 4 : 8;
  if (fused_lds_bytes(tile, word, s->cfg.forcing != 0) > kLdsBytes)
    return fail(AT_E_INVAL, "tile shape needs more LDS than a compute unit has at this precision");
  return AT_OK;
}
}  // namespace

int at_set_stage_tuning(at_sim* s, int32_t tile_sync, int32_t zchunk_sync, int32_t tile_delayed,
                        int32_t zchunk_delayed) {
  if (!s) return fail(AT_E_INVAL, "NULL handle");
  int rc = check_shape(s, tile_sync, zchunk_sync);
  if (!rc) rc = check_shape(s, tile_delayed, zchunk_delayed);
  if (rc) return rc;
  s->tile = tile_sync;
  s->zchunk = std::min(zchunk_sync, s->cfg.n[2]);
  s->tile_d = tile_delayed;
  s->zchunk_d = std::min(zchunk_delayed, s->cfg.n[2]);
  return AT_OK;
}

int at_get_stage_tuning(at_sim* s, int32_t* tile_sync, int32_t* zchunk_sync, int32_t* tile_delayed,
                        int32_t* zchunk_delayed) {
  if (!s || !tile_sync || !zchunk_sync || !tile_delayed || !zchunk_delayed) return fail(AT_E_INVAL, "NULL argument");
  *tile_sync = s->tile;
  *zchunk_sync = s->zchunk;
  *tile_delayed = s->tile_d;
  *zchunk_delayed = s->zchunk_d;
  return AT_OK;
}

int at_set_tuning(at_sim* s, int32_t tile, int32_t zchunk) {
  return at_set_stage_tuning(s, tile, zchunk, tile, zchunk);
}

int at_get_tuning(at_sim* s, int32_t* tile, int32_t* zchunk) {
  if (!s || !tile || !zchunk) return fail(AT_E_INVAL, "NULL argument");
  *tile = s->tile;
  *zchunk = s->zchunk;
  return AT_OK;
}

int at_set_kernel_timing(at_sim* s, int32_t enable) {
  if (!s) return fail(AT_E_INVAL, "NULL handle");
  if (enable && !s->timer) {
    s->timer = new (std::nothrow) EventTimer();
    if (!s->timer) return fail(AT_E_INVAL, "out of host memory");
  } else if (!enable && s->timer) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    delete s->timer;
    s->timer = nullptr;
  } else if (enable && s->timer) {
    HIP_TRY(s->timer->harvest(s->stream));
    s->timer->reset();
  }
  return AT_OK;
}

int at_kernel_timing(at_sim* s, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches || kernel < 0 || kernel >= kKCount) return fail(AT_E_INVAL, "bad argument");
  if (!s->timer) {
    *total_ms = 0.0;
    *launches = 0;
    return AT_OK;
  }
  HIP_TRY(s->timer->harvest(s->stream));
  if (s->timer->failed) return fail(AT_E_HIP, "event creation or record failed");
  *total_ms = s->timer->total_ms[kernel];
  *launches = s->timer->launches[kernel];
  return AT_OK;
}

const char* at_kernel_name(int32_t kernel) { return kernel_name(kernel); }

int at_destroy(at_sim* s) {
  if (!s) return AT_OK;
  (void)hipStreamSynchronize(s->stream);
  if (s->batch) batch_forget(s->batch, s);
  delete s->timer;
  if (s->d_sched) (void)hipFree(s->d_sched);
  if (s->d_zero) (void)hipFree(s->d_zero);
  if (s->d_fhat) (void)hipFree(s->d_fhat);
  if (s->d_wv) (void)hipFree(s->d_wv);
  if (s->d_staging) (void)hipFree(s->d_staging);
  delete s;
  return AT_OK;
}

}  // extern "C"
