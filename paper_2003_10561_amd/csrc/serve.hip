// Served runs: a request trace (arrival time, grid, PE grid, steps, delays, initial field) is
// served by one batch with continuous batching.  Requests are admitted first come first served
// when a slot is free and their device footprint fits the HBM budget and the free device memory;
// admitted runs join the batch at the next step boundary, every loop iteration advances all
// members by one RK step (one launch per kernel per stage, replayed from a HIP graph while
// membership is unchanged), and a run leaves at the boundary where it has done its steps, after
// its final statistics (and optionally its field) are read back.  Each iteration advances the batch
// by the fewest steps any active run has left, at most kMaxChunk (fewer host round trips; no run
// overshoots, and admission waits at most that many steps).  The server owns the workspaces it
// allocates for admitted requests and frees them when they leave.
#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "sim_internal.h"

using namespace atns;

namespace {

using Clock = std::chrono::steady_clock;
constexpr int64_t kMaxChunk = 8;

struct Active {
  int req;
  at_sim* sim;
  void* ws;
  size_t bytes;
  int64_t end_step;
};

at_config request_config(const at_serve_config* sc, const at_request* r) {
  at_config c{};
  for (int d = 0; d < 3; ++d) {
    c.n[d] = r->n;
    c.p[d] = r->p;
  }
  c.order = 4;
  c.max_delay = r->L > 0 ? r->L : 0;
  c.precision = sc->precision;
  c.forcing = 0;
  c.gamma = 1.4;
  c.prandtl = 0.7;
  c.gas_r = 1.0;
  c.mu_ref = r->mu_ref;
  c.t_ref = 1.0;
  c.mu_exp = 0.76;
  c.dt = r->dt;
  return c;
}

// Device bytes a request holds while admitted: its workspace, the library's staging buffer and
// its schedule table.
size_t footprint(const at_config& c, int steps) {
  const size_t ws = at_workspace_bytes(&c);
  if (!ws) return 0;
  const size_t N = (size_t)c.n[0] * c.n[1] * c.n[2];
  const size_t P = (size_t)c.p[0] * c.p[1] * c.p[2];
  return ws + sizeof(double) * kNQ * N + (size_t)(steps + 1) * P * 6 + 4096;
}

int admit(const at_serve_config* sc, const at_request* r, int idx, hipStream_t stream, at_batch* batch,
          Active* out) {
  const at_config c = request_config(sc, r);
  const size_t ws_bytes = at_workspace_bytes(&c);
  if (!ws_bytes) return AT_E_INVAL;
  void* ws = nullptr;
  HIP_TRY(hipMalloc(&ws, ws_bytes));
  at_sim* s = nullptr;
  int rc = at_create(&c, ws, ws_bytes, stream, &s);
  if (!rc) rc = at_init_field(s, r->q0, 1);
  if (!rc) {
    const int64_t n_steps = (int64_t)r->steps + 1;
    if (r->mode == AT_CAA)
      rc = at_set_delay_schedule(s, AT_CAA, r->L, r->L + 1, 0, nullptr, n_steps);
    else if (r->mode == AT_SAA)
      rc = at_set_delay_schedule(s, AT_SAA, r->L, 0, r->seed, nullptr, n_steps);
    else
      rc = at_set_delay_schedule(s, AT_SYNC, 0, 0, 0, nullptr, n_steps);
  }
  if (!rc) rc = at_batch_add(batch, s);
  if (rc) {
    if (s) at_destroy(s);
    (void)hipFree(ws);
    return rc;
  }
  out->req = idx;
  out->sim = s;
  out->ws = ws;
  out->bytes = footprint(c, r->steps);
  out->end_step = s->step + r->steps;
  return AT_OK;
}

int retire(const at_request* r, Active& a, at_batch* batch, at_result* res) {
  int rc = at_stats(a.sim, &res->stats);  // synchronises the stream
  if (!rc && r->q_final) rc = at_get_field(a.sim, r->q_final);
  const int rc2 = at_batch_remove(batch, a.sim);
  at_destroy(a.sim);
  const hipError_t e = hipFree(a.ws);
  if (!rc) rc = rc2;
  if (!rc && e != hipSuccess) rc = fail(AT_E_HIP, std::string("hipFree: ") + hipGetErrorString(e));
  return rc;
}

}  // namespace

extern "C" int at_serve(const at_serve_config* sc, const at_request* reqs, int32_t nreq, void* hip_stream,
                        at_result* results, double* makespan_s) {
  if (!sc || (!reqs && nreq) || (!results && nreq) || nreq < 0) return fail(AT_E_INVAL, "bad argument");
  if (sc->precision != AT_FP32 && sc->precision != AT_FP64) return fail(AT_E_INVAL, "bad precision");
  if (sc->max_active < 1 || !(sc->hbm_budget_bytes > 0)) return fail(AT_E_INVAL, "bad server limits");
  for (int i = 0; i < nreq; ++i) {
    const at_request& r = reqs[i];
    if (i && r.arrival_s < reqs[i - 1].arrival_s) return fail(AT_E_INVAL, "requests must be sorted by arrival");
    if (!r.q0 || r.steps < 1 || r.n < 4 || r.p < 1 || r.L < 0 ||
        (r.mode != AT_SYNC && r.mode != AT_CAA && r.mode != AT_SAA))
      return fail(AT_E_INVAL, "bad request " + std::to_string(i));
    const at_config c = request_config(sc, &r);
    if (!at_workspace_bytes(&c)) return fail(AT_E_INVAL, "request " + std::to_string(i) + ": " + at_last_error());
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  at_batch* batch = nullptr;
  int rc = at_batch_create(sc->precision, hip_stream, &batch);
  if (rc) return rc;
  if (sc->tile >= 0) {
    rc = sc->tile_delayed >= 0
             ? at_batch_set_stage_tuning(batch, sc->tile, sc->zchunk, sc->tile_delayed, sc->zchunk_delayed)
             : at_batch_set_tuning(batch, sc->tile, sc->zchunk);
    if (rc) {
      at_batch_destroy(batch);
      return rc;
    }
  }
  for (int i = 0; i < nreq; ++i) {
    results[i] = at_result{};
    results[i].status = 1;  // pending
  }
  std::deque<int> queue;
  std::vector<Active> active;
  size_t used = 0;
  int next = 0, done = 0;
  const Clock::time_point t0 = Clock::now();
  auto now = [&] { return std::chrono::duration<double>(Clock::now() - t0).count(); };
  while (done < nreq && !rc) {
    const double t = now();
    while (next < nreq && reqs[next].arrival_s <= t) queue.push_back(next++);
    // admission at this step boundary
    while (!queue.empty() && (int)active.size() < sc->max_active) {
      const int i = queue.front();
      const at_config c = request_config(sc, &reqs[i]);
      const size_t need = footprint(c, reqs[i].steps);
      if (need > sc->hbm_budget_bytes) {  // can never be admitted
        results[i].status = AT_E_WORKSPACE;
        queue.pop_front();
        ++done;
        continue;
      }
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
      if (used + need > sc->hbm_budget_bytes || need + ((size_t)1 << 30) > free_b) break;
      Active a{};
      const int arc = admit(sc, &reqs[i], i, stream, batch, &a);
      queue.pop_front();
      if (arc) {
        results[i].status = arc;
        ++done;
        continue;
      }
      results[i].admit_s = now();
      used += a.bytes;
      active.push_back(a);
    }
    if (active.empty() && !queue.empty()) {
      // the head request does not fit the free device memory even with the server empty
      results[queue.front()].status = fail(AT_E_WORKSPACE, "request does not fit the free device memory");
      queue.pop_front();
      ++done;
      continue;
    }
    if (active.empty()) {
      if (next < nreq) {
        const double wait = reqs[next].arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait < 1e-3 ? wait : 1e-3));
      }
      continue;
    }
    int64_t chunk = kMaxChunk;
    for (const Active& a : active) chunk = std::min(chunk, a.end_step - a.sim->step);
    rc = at_batch_step(batch, (int32_t)std::max<int64_t>(chunk, 1));
    if (rc) break;
    for (size_t k = 0; k < active.size();) {
      Active& a = active[k];
      if (a.sim->step < a.end_step) {
        ++k;
        continue;
      }
      const int i = a.req;
      const int rrc = retire(&reqs[i], a, batch, &results[i]);
      results[i].done_s = now();
      results[i].status = rrc;
      used -= a.bytes;
      ++done;
      active.erase(active.begin() + (long)k);
      if (rrc) rc = rrc;
    }
  }
  if (makespan_s) *makespan_s = now();
  for (Active& a : active) {  // only after an error
    at_batch_remove(batch, a.sim);
    at_destroy(a.sim);
    (void)hipFree(a.ws);
  }
  at_batch_destroy(batch);
  return rc;
}
