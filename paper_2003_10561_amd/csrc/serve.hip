// Served runs: a request trace (arrival time, grid, PE grid, steps, delays, initial field) is
// served by one batch with continuous batching.  Requests are admitted first come first served
// when a slot is free and their device footprint fits the HBM budget and the free device memory;
// admitted runs join the batch at the next step boundary, every loop iteration advances all
// members by one chunk of RK steps (one launch per kernel per stage, replayed from a HIP graph
// while membership is unchanged), and a run leaves at the boundary where it has done its steps,
// after its final statistics (and optionally its field) are read back.  Each chunk is the fewest
// steps any active run has left, at most kMaxChunk (fewer host round trips; no run overshoots).
//
// The host work of an admission stays off the GPU's critical path: while a chunk runs, the next
// queued requests are prepared on a second stream (their handles created, fields copied and
// converted, schedules uploaded), and they join at the following boundary behind an event.  At a
// boundary the device is idle anyway (the chunk has been waited for), so that is where finished
// runs are read back and released.  Workspaces of finished runs go to a pool and are reused by later
// admissions; the server frees them at the end.
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
  size_t ws_bytes;  // the workspace block (from the pool, possibly larger than needed)
  size_t bytes;     // the footprint the request is charged against the budget
  int64_t end_step;
  hipEvent_t ready;  // prepared runs: their set-up work on the preparation stream has completed
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

// Workspace blocks released by finished runs, reused by later admissions (smallest that fits).
struct Pool {
  std::vector<std::pair<void*, size_t>> free_blocks;
  size_t held = 0;  // bytes of the free blocks
  void* take(size_t need, size_t* got) {
    size_t best = free_blocks.size();
    for (size_t i = 0; i < free_blocks.size(); ++i)
      if (free_blocks[i].second >= need && (best == free_blocks.size() || free_blocks[i].second < free_blocks[best].second))
        best = i;
    if (best == free_blocks.size()) return nullptr;
    void* p = free_blocks[best].first;
    *got = free_blocks[best].second;
    held -= *got;
    free_blocks.erase(free_blocks.begin() + (long)best);
    return p;
  }
  void give(void* p, size_t bytes) {
    free_blocks.push_back({p, bytes});
    held += bytes;
  }
  // release blocks (largest first) until `want` more bytes could be allocated within `budget`
  void shrink(size_t in_use, size_t want, size_t budget) {
    std::sort(free_blocks.begin(), free_blocks.end(), [](auto& x, auto& y) { return x.second < y.second; });
    while (!free_blocks.empty() && in_use + held + want > budget) {
      (void)hipFree(free_blocks.back().first);
      held -= free_blocks.back().second;
      free_blocks.pop_back();
    }
  }
  void clear() {
    for (auto& b : free_blocks) (void)hipFree(b.first);
    free_blocks.clear();
    held = 0;
  }
};

// Creates and initialises the run of request r on the preparation stream `prep` (its handle keeps
// that stream until it joins the batch).  The workspace comes from the pool or a new allocation.
int prepare(const at_serve_config* sc, const at_request* r, int idx, hipStream_t prep, Pool& pool, Active* out) {
  const at_config c = request_config(sc, r);
  const size_t ws_bytes = at_workspace_bytes(&c);
  if (!ws_bytes) return AT_E_INVAL;
  size_t got = 0;
  void* ws = pool.take(ws_bytes, &got);
  if (!ws) {
    HIP_TRY(hipMalloc(&ws, ws_bytes));
    got = ws_bytes;
  }
  at_sim* s = nullptr;
  hipEvent_t ev = nullptr;
  int rc = at_create(&c, ws, got, prep, &s);
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
  if (!rc && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) rc = fail(AT_E_HIP, "event");
  if (!rc && hipEventRecord(ev, prep) != hipSuccess) rc = fail(AT_E_HIP, "event record");
  if (rc) {
    if (ev) (void)hipEventDestroy(ev);
    if (s) at_destroy(s);
    pool.give(ws, got);
    return rc;
  }
  out->req = idx;
  out->sim = s;
  out->ws = ws;
  out->ws_bytes = got;
  out->bytes = footprint(c, r->steps);
  out->end_step = s->step + r->steps;
  out->ready = ev;
  return AT_OK;
}

// A prepared run joins the batch: the batch stream waits for its set-up, and the run moves to it.
int join(Active& a, at_batch* batch, hipStream_t stream) {
  HIP_TRY(hipStreamWaitEvent(stream, a.ready, 0));
  a.sim->stream = stream;
  return at_batch_add(batch, a.sim);
}

int retire(const at_request* r, Active& a, at_batch* batch, at_result* res, Pool& pool) {
  int rc = at_stats(a.sim, &res->stats);  // synchronises the stream
  if (!rc && r->q_final) rc = at_get_field(a.sim, r->q_final);
  const int rc2 = at_batch_remove(batch, a.sim);
  at_destroy(a.sim);
  if (a.ready) (void)hipEventDestroy(a.ready);
  pool.give(a.ws, a.ws_bytes);
  if (!rc) rc = rc2;
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
  hipStream_t prep = nullptr;
  if (hipStreamCreateWithFlags(&prep, hipStreamNonBlocking) != hipSuccess) {
    at_batch_destroy(batch);
    return fail(AT_E_HIP, "preparation stream");
  }
  for (int i = 0; i < nreq; ++i) {
    results[i] = at_result{};
    results[i].status = 1;  // pending
  }
  std::deque<int> queue;
  std::vector<Active> active, ready;
  Pool pool;
  size_t used = 0;  // footprint of admitted runs (active and prepared)
  int next = 0, done = 0;
  bool chunk_running = false;
  const Clock::time_point t0 = Clock::now();
  auto now = [&] { return std::chrono::duration<double>(Clock::now() - t0).count(); };
  // the budget, capped by what the device has free (less 1 GiB) with the server empty
  size_t dev_free = 0, dev_total = 0;
  if (hipMemGetInfo(&dev_free, &dev_total) != hipSuccess) dev_free = 0;
  const size_t margin = (size_t)1 << 30;
  const size_t budget = std::min((size_t)sc->hbm_budget_bytes, dev_free > margin ? dev_free - margin : 0);
  auto admit_queued = [&]() {
    while (!queue.empty() && (int)(active.size() + ready.size()) < sc->max_active) {
      const int i = queue.front();
      const at_config c = request_config(sc, &reqs[i]);
      const size_t need = footprint(c, reqs[i].steps);
      if (need > budget) {  // can never be admitted
        results[i].status = fail(AT_E_WORKSPACE, "request does not fit the HBM budget or the device");
        queue.pop_front();
        ++done;
        continue;
      }
      if (used + need > budget) break;  // waits for runs to leave
      if (used + pool.held + need > budget) pool.shrink(used, need, budget);
      Active a{};
      const int arc = prepare(sc, &reqs[i], i, prep, pool, &a);
      queue.pop_front();
      if (arc) {
        results[i].status = arc;
        ++done;
        continue;
      }
      results[i].admit_s = now();
      used += a.bytes;
      ready.push_back(a);
    }
  };
  while (done < nreq && !rc) {
    while (next < nreq && reqs[next].arrival_s <= now()) queue.push_back(next++);
    if (chunk_running) {
      // prepare queued requests while the chunk runs, then wait for it
      admit_queued();
      if (hipStreamSynchronize(stream) != hipSuccess) {
        rc = fail(AT_E_HIP, "batch chunk");
        break;
      }
      chunk_running = false;
      // the device is idle: read back and release the runs that have finished
      for (size_t k = 0; k < active.size();) {
        Active& a = active[k];
        if (a.sim->step < a.end_step) {
          ++k;
          continue;
        }
        const int i = a.req;
        const int rrc = retire(&reqs[i], a, batch, &results[i], pool);
        results[i].done_s = now();
        results[i].status = rrc;
        used -= a.bytes;
        ++done;
        active.erase(active.begin() + (long)k);
        if (rrc) rc = rrc;
      }
      if (rc) break;
    } else if (active.empty() && ready.empty()) {
      admit_queued();  // nothing on the GPU: prepare now
    }
    // runs prepared during the last chunk join at this boundary
    for (Active& a : ready) {
      const int jrc = join(a, batch, stream);
      if (jrc) {
        rc = jrc;
        break;
      }
      active.push_back(a);
    }
    ready.clear();
    if (rc) break;
    if (active.empty()) {
      if (next < nreq && queue.empty()) {
        const double wait = reqs[next].arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait < 1e-3 ? wait : 1e-3));
      }
      continue;
    }
    int64_t chunk = kMaxChunk;
    for (const Active& a : active) chunk = std::min(chunk, a.end_step - a.sim->step);
    rc = at_batch_step(batch, (int32_t)std::max<int64_t>(chunk, 1));
    if (rc) break;
    chunk_running = true;
  }
  (void)hipStreamSynchronize(stream);
  (void)hipStreamSynchronize(prep);
  if (makespan_s) *makespan_s = now();
  for (std::vector<Active>* v : {&active, &ready})  // only after an error
    for (Active& a : *v) {
      if (a.sim->batch) at_batch_remove(batch, a.sim);
      at_destroy(a.sim);
      if (a.ready) (void)hipEventDestroy(a.ready);
      (void)hipFree(a.ws);
    }
  at_batch_destroy(batch);
  pool.clear();
  (void)hipStreamDestroy(prep);
  return rc;
}
