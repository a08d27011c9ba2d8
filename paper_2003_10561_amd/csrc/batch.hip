// Batched runs: many independent AT runs advanced together with ONE launch per kernel per RK
// stage over all their workgroups (a device run table plus a (run, workgroup) work list), the
// launches of a chunk of steps captured in a HIP graph and replayed while the batch's membership
// and launch shape stay the same, and the autotuner of the launch shape.
//
// Every run keeps its own workspace, schedule, forcing table, step counter and state buffers; a
// batched step does to each run exactly what its own single-run step does (same arguments, same
// workgroup decomposition), so results are bitwise those of the run stepped alone with the same
// launch shape.  The launch shape changes no field value: each point is computed by the same
// expressions in the same order whatever tile or z chunk covers it; only the summation order of
// the FP64 RK totals (one partial per workgroup) follows the shape.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "sim_internal.h"

using namespace atns;

struct at_batch {
  int precision = AT_FP32;
  hipStream_t stream = nullptr;  // caller's stream: table uploads and graph launches
  hipStream_t cap = nullptr;     // private stream, used only to capture graphs
  // private stream of the AT branch of a stage (the AT sums and the AT launch), forked from and
  // joined back into the launch stream at every stage, so that the plain and the AT launches of a
  // stage (disjoint sets of runs) overlap; default priority
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int device = 0;
  std::vector<at_sim*> runs;
  int tile = 1, zchunk = 64;      // launch shape of the stages that read no delayed level
  int tile_d = 1, zchunk_d = 64;  // and of those that do
  int use_graph = 1;
  // device buffer of one chunk: [stage work][view work][forcing rows][run tables]
  uint8_t* d_buf = nullptr;
  size_t d_cap = 0;
  // pinned host staging, double-buffered; an event marks when a copy out of it has finished
  uint8_t* h_buf[2] = {nullptr, nullptr};
  size_t h_cap[2] = {0, 0};
  hipEvent_t h_done[2] = {nullptr, nullptr};
  bool h_recorded[2] = {false, false};
  int h_next = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> sig;
  int64_t captures = 0, replays = 0;
  double* d_trial_tot = nullptr;  // FP64 totals of autotuning trials (discarded)
  size_t trial_tot_n = 0;
};

namespace {

constexpr int kMaxBatchRuns = 4096;
constexpr size_t kFhatRow = (size_t)kNForce * 6;  // doubles of one step's forcing table

size_t word_of(int precision) { return precision == AT_FP32 ? 4 : 8; }

// Launch shape of kind k (0: stages that read no delayed level, 1: those that do).
int kind_tile(const at_batch* b, int k) { return k ? b->tile_d : b->tile; }
int run_zchunk(const at_batch* b, const at_sim* s, int k) { return std::min(k ? b->zchunk_d : b->zchunk, s->cfg.n[2]); }

bool any_forced(const at_batch* b) {
  for (const at_sim* s : b->runs)
    if (s->cfg.forcing) return true;
  return false;
}

// Does the run read delayed levels at any step of its schedule.
bool ever_delayed(const at_sim* s) {
  for (uint8_t d : s->step_delayed)
    if (d) return true;
  return false;
}

void drop_graph(at_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->sig.clear();
}

// Placement of one chunk's tables in the device buffer.
struct ChunkPlan {
  int K = 0;
  int64_t nsw[2] = {0, 0}, nvw = 0;  // stage work-list entries of either launch shape; view entries
  bool views = false;                 // launch the batched AT sums and AT stages at every stage
  int at_kinds = 0;                   // AT instantiations its delayed runs need (kAtMasked, kAtGhost)
  std::vector<int> forced;   // indices of forced runs

  size_t off_sw[2] = {0, 0}, off_vw = 0, off_fh = 0, off_args[2] = {0, 0}, total = 0, argb = 0;
};

ChunkPlan plan_chunk(const at_batch* b, int K) {
  ChunkPlan p;
  p.K = K;
  p.argb = b->precision == AT_FP32 ? batch_arg_bytes<float>() : batch_arg_bytes<double>();
  for (size_t m = 0; m < b->runs.size(); ++m) {
    const at_sim* s = b->runs[m];
    p.nsw[0] += fused_blocks(s->g, b->tile, run_zchunk(b, s, 0));
    p.nsw[1] += fused_blocks(s->g, b->tile_d, run_zchunk(b, s, 1));
    if (ever_delayed(s)) {
      p.views = true;
      p.nvw += view_blocks(s->g);
      p.at_kinds |= tile_aligned(s->g, b->tile_d) ? kAtGhost : kAtMasked;
    }
    if (s->cfg.forcing) p.forced.push_back((int)m);
  }

  if (!p.views) p.nsw[1] = 0;
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    p.off_sw[k] = off;
    off = align_up(off + (size_t)p.nsw[k] * sizeof(uint2));
  }
  p.off_vw = off;
  off = align_up(off + (size_t)p.nvw * sizeof(uint2));
  p.off_fh = off;
  off = align_up(off + p.forced.size() * (size_t)K * kFhatRow * sizeof(double));
  for (int k = 0; k < 2; ++k) {
    p.off_args[k] = off;
    if (k == 0 || p.views) off = align_up(off + (size_t)K * 3 * b->runs.size() * p.argb);
  }
  p.total = off;
  return p;
}

// Wait until the last copy out of a staging half has completed.
hipError_t wait_staging(at_batch* b, int slot) {
  return b->h_recorded[slot] ? hipEventSynchronize(b->h_done[slot]) : hipSuccess;
}

hipError_t upload(at_batch* b, int slot, size_t bytes) {
  hipError_t e = hipMemcpyAsync(b->d_buf, b->h_buf[slot], bytes, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->h_done[slot], b->stream);
  if (e == hipSuccess) b->h_recorded[slot] = true;
  b->h_next ^= 1;
  return e;
}

int ensure_buffers(at_batch* b, size_t bytes, int slot) {
  if (bytes > b->d_cap) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    drop_graph(b);  // captured launches point into the old buffer
    if (b->d_buf) HIP_TRY(hipFree(b->d_buf));
    b->d_buf = nullptr;
    b->d_cap = 0;
    HIP_TRY(hipMalloc(&b->d_buf, bytes));
    b->d_cap = bytes;
  }
  if (bytes > b->h_cap[slot]) {
    if (b->h_buf[slot]) {
      HIP_TRY(wait_staging(b, slot));
      HIP_TRY(hipHostFree(b->h_buf[slot]));
    }
    b->h_buf[slot] = nullptr;
    b->h_cap[slot] = 0;
    HIP_TRY(hipHostMalloc(&b->h_buf[slot], bytes, hipHostMallocDefault));
    b->h_cap[slot] = bytes;
  }
  return AT_OK;
}

// Stage arguments of run s at step (s->step + bstep), stage st.
template <typename T>
StageArgs<T> chunk_args(at_sim* s, int bstep, int st, double* tot_override) {
  StageArgs<T> a = base_args<T>(s);
  const int64_t n = s->step + bstep;
  const int cur = s->qcur ^ ((3 * bstep + st) & 1);
  a.q = (T*)(s->ws + s->L.q[cur]);
  a.q_out = (T*)(s->ws + s->L.q[1 - cur]);
  a.delays = s->d_sched + (size_t)n * s->g.ntiles * 6;
  a.step = n;
  a.step_mod_r = (int)(n % s->g.R);
  a.gv = a.gv_out + (size_t)st * s->g.ring_slot;
  a.rk_a = (T)kRkA[st];
  a.rk_b = (T)kRkB[st];
  a.publish = st == 0;
  a.store_dq = st < 2;
  if (s->cfg.forcing) a.force.table = (T*)(s->ws + s->L.force_table);
  if (tot_override) a.tot_part = tot_override;
  return a;
}

// Work lists and run tables of a chunk of K steps into host staging.
template <typename T>
void fill_chunk(at_batch* b, const ChunkPlan& p, uint8_t* h) {
  const int nk = p.views ? 2 : 1;
  uint2* vw = (uint2*)(h + p.off_vw);
  int64_t is[2] = {0, 0}, iv = 0;
  for (size_t m = 0; m < b->runs.size(); ++m) {
    const at_sim* s = b->runs[m];
    for (int kd = 0; kd < nk; ++kd) {
      uint2* sw = (uint2*)(h + p.off_sw[kd]);
      const int64_t nb = fused_blocks(s->g, kind_tile(b, kd), run_zchunk(b, s, kd));
      for (int64_t k = 0; k < nb; ++k) sw[is[kd]++] = make_uint2((unsigned)m, (unsigned)k);
    }
    if (ever_delayed(s)) {
      const int64_t nv = view_blocks(s->g);
      for (int64_t k = 0; k < nv; ++k) vw[iv++] = make_uint2((unsigned)m, (unsigned)k);
    }
  }
  double* fh = (double*)(h + p.off_fh);
  for (size_t f = 0; f < p.forced.size(); ++f) {
    const at_sim* s = b->runs[(size_t)p.forced[f]];
    std::memcpy(fh + f * (size_t)p.K * kFhatRow, s->h_fhat.data() + (size_t)s->step * kFhatRow,
                (size_t)p.K * kFhatRow * sizeof(double));
  }
  const size_t M = b->runs.size();
  for (int bs = 0; bs < p.K; ++bs)
    for (int st = 0; st < 3; ++st)
      for (size_t m = 0; m < M; ++m) {
        at_sim* s = b->runs[m];
        StageArgs<T> a = chunk_args<T>(s, bs, st, nullptr);
        a.at_ghost = tile_aligned(s->g, b->tile_d) ? 1 : 0;  // the batch's delayed-stage shape
        const int views = s->step_delayed[(size_t)(s->step + bs)] ? 1 : 0;
        for (int kd = 0; kd < nk; ++kd)
          pack_batch_arg<T>(a, kind_tile(b, kd), run_zchunk(b, s, kd), views,
                            h + p.off_args[kd] + ((size_t)(bs * 3 + st) * M + m) * p.argb);
      }
}

// The launches of a chunk (recorded into a graph when capturing).
template <typename T>
hipError_t enqueue_chunk(at_batch* b, const ChunkPlan& p, hipStream_t st) {
  const size_t M = b->runs.size();
  const bool forced = !p.forced.empty();
  const uint2* sw = (const uint2*)(b->d_buf + p.off_sw[0]);
  const uint2* swd = (const uint2*)(b->d_buf + p.off_sw[1]);
  const uint2* vw = (const uint2*)(b->d_buf + p.off_vw);
  const double* fh = (const double*)(b->d_buf + p.off_fh);
  for (int bs = 0; bs < p.K; ++bs) {
    for (size_t f = 0; f < p.forced.size(); ++f) {
      at_sim* s = b->runs[(size_t)p.forced[f]];
      hipError_t e = launch_force_table<T>(s->g, fh + (f * (size_t)p.K + bs) * kFhatRow, s->d_wv, s->d_wv + kNForce,
                                           s->npair, (T*)(s->ws + s->L.force_table),
                                           (const T*)(s->ws + s->L.phase_x), st, nullptr);
      if (e != hipSuccess) return e;
    }
    for (int stg = 0; stg < 3; ++stg) {
      const void* tab = b->d_buf + p.off_args[0] + (size_t)(bs * 3 + stg) * M * p.argb;
      const void* tabd = b->d_buf + p.off_args[1] + (size_t)(bs * 3 + stg) * M * p.argb;
      // runs that read delayed levels at this step run the AT instantiation (in its own launch
      // shape), the others the plain one (each leaves the other's launch at once); both are
      // launched at every stage of a batch with any delayed schedule, so that a chunk's graph
      // depends only on membership, launch shapes and length.  The AT branch (with the AT sums of
      // the step at stage 1) runs on the side stream, concurrently with the plain launch: a run's
      // stage touches only its own buffers, and the join orders every run's stages.
      hipError_t e = hipSuccess;
      if (p.views) {
        if ((e = hipEventRecord(b->ev_fork, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(b->side, b->ev_fork, 0)) != hipSuccess) return e;
        if (stg == 0 && p.nvw > 0) {  // the AT sums of all three stages of the step
          e = launch_at_sums_batch<T>(tab, vw, p.nvw, kRkC, b->side);
          if (e != hipSuccess) return e;
        }
        e = launch_fused_batch<T>(tabd, swd, p.nsw[1], b->tile_d, forced, stg == 0, p.at_kinds, kModeStepH, b->side);
        if (e != hipSuccess) return e;
      }
      e = launch_fused_batch<T>(tab, sw, p.nsw[0], b->tile, forced, stg == 0, 0, kModeStepH, st);
      if (e != hipSuccess) return e;
      if (p.views) {
        if ((e = hipEventRecord(b->ev_join, b->side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, b->ev_join, 0)) != hipSuccess) return e;
      }
    }
  }
  return hipSuccess;
}

std::vector<uint64_t> chunk_signature(const at_batch* b, const ChunkPlan& p) {
  std::vector<uint64_t> sg = {(uint64_t)b->tile, (uint64_t)b->zchunk, (uint64_t)b->tile_d, (uint64_t)b->zchunk_d,
                              (uint64_t)p.K, (uint64_t)b->precision, (uint64_t)(uintptr_t)b->d_buf,
                              (uint64_t)p.nsw[0], (uint64_t)p.nsw[1], (uint64_t)p.nvw, (uint64_t)p.views,
                              (uint64_t)p.at_kinds,
                              (uint64_t)p.off_args[0], (uint64_t)p.off_args[1], (uint64_t)p.off_fh,
                              (uint64_t)p.off_vw};
  for (const at_sim* s : b->runs) {
    sg.push_back((uint64_t)(uintptr_t)s);
    sg.push_back((uint64_t)s->cfg.forcing);
  }
  return sg;
}

template <typename T>
int do_batch_steps(at_batch* b, int K) {
  const ChunkPlan p = plan_chunk(b, K);
  const int slot = b->h_next;
  int rc = ensure_buffers(b, p.total, slot);
  if (rc) return rc;
  // the staging half is reused only after its previous copy has completed
  HIP_TRY(wait_staging(b, slot));
  fill_chunk<T>(b, p, b->h_buf[slot]);
  HIP_TRY(upload(b, slot, p.total));
  if (b->use_graph) {
    std::vector<uint64_t> sg = chunk_signature(b, p);
    if (!b->exec || sg != b->sig) {
      drop_graph(b);
      HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_chunk<T>(b, p, b->cap);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(b->cap, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(AT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
      }
      b->graph = g;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->sig = sg;
      b->captures++;
    }
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    b->replays++;
  } else {
    HIP_TRY(enqueue_chunk<T>(b, p, b->stream));
  }
  for (at_sim* s : b->runs) {
    s->tot_used = std::max({s->tot_used, fused_blocks(s->g, b->tile, run_zchunk(b, s, 0)),
                            fused_blocks(s->g, b->tile_d, run_zchunk(b, s, 1))});
    s->step += K;
    s->ab2_prev = 0;  // Runge-Kutta steps: the register no longer holds dt f^{n-1}
    s->qcur ^= (K & 1);
  }
  return AT_OK;
}

// First step at or after the run's current step that reads delayed levels, or -1.
int64_t first_delayed_step(const at_sim* s) {
  for (size_t n = (size_t)s->step; n < s->step_delayed.size(); ++n)
    if (s->step_delayed[n]) return (int64_t)n;
  return -1;
}

// One trial stage (stage 1, no publication, no register store, FP64 totals discarded) of every
// run with the given launch shape: synchronous (every run in the plain instantiation), or delayed
// (every run that ever reads delayed levels takes the delays of its first such step and the AT
// instantiation).  It rewrites only the other state buffer, which holds no live data between
// steps; the RK register is left alone, since after Adams-Bashforth steps it carries dt f^{n-1}.
template <typename T>
int trial_stage(at_batch* b, int tile, int zchunk, int reps, bool delayed, double* ms) {
  // both kinds of stage in the trial shape; the tables of kind 0 serve both launches
  const int t0 = b->tile, z0 = b->zchunk, t1 = b->tile_d, z1 = b->zchunk_d;
  b->tile = b->tile_d = tile;
  b->zchunk = b->zchunk_d = zchunk;
  const ChunkPlan p = plan_chunk(b, 1);
  b->tile = t0;
  b->zchunk = z0;
  b->tile_d = t1;
  b->zchunk_d = z1;
  const int slot = b->h_next;
  int rc = ensure_buffers(b, p.total, slot);
  if (rc) return rc;
  HIP_TRY(wait_staging(b, slot));
  uint8_t* h = b->h_buf[slot];
  uint2* sw = (uint2*)(h + p.off_sw[0]);
  int64_t is = 0;
  size_t tot_off = 0;
  int at_kinds = 0;
  const size_t M = b->runs.size();
  for (size_t m = 0; m < M; ++m) {
    at_sim* s = b->runs[m];
    const int zc = std::min(zchunk, s->cfg.n[2]);
    const int64_t nb = fused_blocks(s->g, tile, zc);
    for (int64_t k = 0; k < nb; ++k) sw[is++] = make_uint2((unsigned)m, (unsigned)k);
    StageArgs<T> a = chunk_args<T>(s, 0, 0, b->d_trial_tot + tot_off);
    a.publish = 0;
    a.store_dq = 0;
    a.at_ghost = tile_aligned(s->g, tile) ? 1 : 0;
    if (s->cfg.forcing) a.force.table = (T*)(s->ws + s->L.force_table);
    tot_off += (size_t)s->L.ntot * kNQ;
    int views = 0;
    const int64_t nd = delayed ? first_delayed_step(s) : -1;
    if (nd >= 0) {
      a.delays = s->d_sched + (size_t)nd * s->g.ntiles * 6;
      a.step_mod_r = (int)(nd % s->g.R);
      views = 1;
      at_kinds |= a.at_ghost ? kAtGhost : kAtMasked;
    }
    pack_batch_arg<T>(a, tile, zc, views, h + p.off_args[0] + m * p.argb);
  }
  HIP_TRY(upload(b, slot, p.total));
  const bool forced = !p.forced.empty();
  const void* tab = b->d_buf + p.off_args[0];
  const uint2* dsw = (const uint2*)(b->d_buf + p.off_sw[0]);
  auto trial = [&]() -> hipError_t {
    hipError_t e = launch_fused_batch<T>(tab, dsw, p.nsw[0], tile, forced, false, 0, kModeStepH, b->stream);
    if (e == hipSuccess && at_kinds)
      e = launch_fused_batch<T>(tab, dsw, p.nsw[0], tile, forced, false, at_kinds, kModeStepH, b->stream);
    return e;
  };
  HIP_TRY(trial());
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  hipError_t err = hipEventRecord(e0, b->stream);
  for (int r = 0; r < reps && err == hipSuccess; ++r)
    err = trial();
  if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float el = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&el, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(err);
  *ms = el / reps;
  return AT_OK;
}

bool tile_fits(const at_batch* b, int tile) {
  return fused_lds_bytes(tile, word_of(b->precision), any_forced(b)) <= kLdsBytes;
}

std::string tune_key(const at_batch* b) {
  hipDeviceProp_t prop{};
  std::ostringstream k;
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess)
    k << prop.gcnArchName << "/" << prop.multiProcessorCount << "cu";
  k << "|" << (b->precision == AT_FP32 ? "fp32" : "fp64") << "|";
  std::vector<std::string> shapes;
  for (const at_sim* s : b->runs) {
    std::ostringstream r;
    r << s->cfg.n[0] << "x" << s->cfg.n[1] << "x" << s->cfg.n[2] << "/" << s->cfg.p[0] << "x" << s->cfg.p[1] << "x"
      << s->cfg.p[2] << (s->cfg.forcing ? "f" : "");
    shapes.push_back(r.str());
  }
  std::sort(shapes.begin(), shapes.end());
  // run multiset as (shape, count)
  for (size_t i = 0; i < shapes.size();) {
    size_t j = i;
    while (j < shapes.size() && shapes[j] == shapes[i]) ++j;
    k << shapes[i] << "*" << (j - i) << ";";
    i = j;
  }
  return k.str();
}

// Cache file: one JSON object per line, {"key": "...", "tile": t, "zchunk": z, "tile_delayed": td,
// "zchunk_delayed": zd, "ms": m} (a line without the delayed shape gives both kinds (t, z)).
bool cache_lookup(const char* path, const std::string& key, int* tile, int* zchunk, int* tile_d, int* zchunk_d,
                  double* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  const std::string want = "\"key\": \"" + key + "\"";
  bool found = false;
  while (std::getline(f, line)) {
    if (line.find(want) == std::string::npos) continue;
    int t = -1, z = -1;
    double m = 0.0;
    const size_t pt = line.find("\"tile\": "), pz = line.find("\"zchunk\": "), pm = line.find("\"ms\": ");
    if (pt == std::string::npos || pz == std::string::npos || pm == std::string::npos) continue;
    if (std::sscanf(line.c_str() + pt + 8, "%d", &t) != 1 || std::sscanf(line.c_str() + pz + 10, "%d", &z) != 1 ||
        std::sscanf(line.c_str() + pm + 6, "%lf", &m) != 1)
      continue;
    if (t < 0 || t >= kTileCount || z < 4) continue;
    int td = t, zd = z;
    const size_t ptd = line.find("\"tile_delayed\": "), pzd = line.find("\"zchunk_delayed\": ");
    if (ptd != std::string::npos && pzd != std::string::npos &&
        (std::sscanf(line.c_str() + ptd + 16, "%d", &td) != 1 || std::sscanf(line.c_str() + pzd + 18, "%d", &zd) != 1 ||
         td < 0 || td >= kTileCount || zd < 4))
      continue;
    *tile = t;
    *zchunk = z;
    *tile_d = td;
    *zchunk_d = zd;
    *ms = m;
    found = true;  // the last matching line wins
  }
  return found;
}

void cache_store(const char* path, const std::string& key, int tile, int zchunk, int tile_d, int zchunk_d,
                 double ms) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  char buf[192];
  std::snprintf(buf, sizeof(buf),
                "\", \"tile\": %d, \"zchunk\": %d, \"tile_delayed\": %d, \"zchunk_delayed\": %d, \"ms\": %.17g}\n",
                tile, zchunk, tile_d, zchunk_d, ms);
  f << "{\"key\": \"" << key << buf;
}

// Fraction of the members' remaining scheduled steps that read delayed levels.
double delayed_fraction(const at_batch* b) {
  double tot = 0.0, del = 0.0;
  for (const at_sim* s : b->runs)
    for (size_t n = (size_t)s->step; n < s->step_delayed.size(); ++n) {
      tot += 1.0;
      del += s->step_delayed[n] ? 1.0 : 0.0;
    }
  return tot > 0.0 ? del / tot : 0.0;
}

// Launch shapes from timed trial stages: for every feasible (tile, z chunk) the synchronous and
// (if any remaining step reads delayed levels) the delayed trial; the fastest shape of each kind.
// The reported time weights the two by the fraction of remaining steps that read delayed levels.
template <typename T>
int do_autotune(at_batch* b, const char* cache, int reps, double* best_ms) {
  const double f = delayed_fraction(b);
  char fbuf[32];
  std::snprintf(fbuf, sizeof(fbuf), "|delayed=%.2f", f);
  const std::string key = tune_key(b) + fbuf;
  int t = -1, z = -1, td = -1, zd = -1;
  double ms = 0.0;
  if (cache_lookup(cache, key, &t, &z, &td, &zd, &ms) && tile_fits(b, t) && tile_fits(b, td)) {
    b->tile = t;
    b->zchunk = z;
    b->tile_d = td;
    b->zchunk_d = zd;
    if (best_ms) *best_ms = ms;
    return AT_OK;
  }
  size_t need = 0;
  for (const at_sim* s : b->runs) need += (size_t)s->L.ntot * kNQ;
  if (need > b->trial_tot_n) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->d_trial_tot) HIP_TRY(hipFree(b->d_trial_tot));
    b->d_trial_tot = nullptr;
    b->trial_tot_n = 0;
    HIP_TRY(hipMalloc(&b->d_trial_tot, need * sizeof(double)));
    b->trial_tot_n = need;
  }
  int maxz = 4;
  for (const at_sim* s : b->runs) maxz = std::max(maxz, s->cfg.n[2]);
  double best_s = 1e300, best_d = 1e300;
  int bt = b->tile, bz = b->zchunk, btd = b->tile_d, bzd = b->zchunk_d;
  static const int kZ[] = {8, 16, 32, 64, 128, 256, 512};
  for (int tile = 0; tile < kTileCount; ++tile) {
    if (!tile_fits(b, tile)) continue;
    for (int zc : kZ) {
      if (zc > maxz && zc != kZ[0]) break;
      double m_sync = 0.0, m_at = 0.0;
      int rc = trial_stage<T>(b, tile, zc, reps, false, &m_sync);
      if (!rc && f > 0.0) rc = trial_stage<T>(b, tile, zc, reps, true, &m_at);
      if (rc) return rc;
      if (m_sync < best_s) {
        best_s = m_sync;
        bt = tile;
        bz = zc;
      }
      if (f > 0.0 && m_at < best_d) {
        best_d = m_at;
        btd = tile;
        bzd = zc;
      }
    }
  }
  if (!(f > 0.0)) {  // no delayed stage ahead: both kinds in the synchronous choice
    btd = bt;
    bzd = bz;
    best_d = 0.0;
  }
  b->tile = bt;
  b->zchunk = bz;
  b->tile_d = btd;
  b->zchunk_d = bzd;
  const double best = (1.0 - f) * best_s + f * best_d;
  if (best_ms) *best_ms = best;
  cache_store(cache, key, bt, bz, btd, bzd, best);
  return AT_OK;
}

}  // namespace

namespace atns {
void batch_forget(at_batch* b, at_sim* s) {
  if (!b) return;
  b->runs.erase(std::remove(b->runs.begin(), b->runs.end(), s), b->runs.end());
  drop_graph(b);
}
}  // namespace atns

extern "C" {

int at_batch_create(int32_t precision, void* stream, at_batch** out) {
  if (!out) return fail(AT_E_INVAL, "out is NULL");
  if (precision != AT_FP32 && precision != AT_FP64) return fail(AT_E_INVAL, "bad precision");
  at_batch* b = new (std::nothrow) at_batch();
  if (!b) return fail(AT_E_INVAL, "out of host memory");
  b->precision = precision;
  b->stream = (hipStream_t)stream;
  b->tile = b->tile_d = fused_lds_bytes(1, word_of(precision), false) <= kLdsBytes ? 1 : 5;
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&b->h_done[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    at_batch_destroy(b);
    return fail(AT_E_HIP, std::string("batch set-up: ") + hipGetErrorString(e));
  }
  *out = b;
  return AT_OK;
}

int at_batch_add(at_batch* b, at_sim* s) {
  if (!b || !s) return fail(AT_E_INVAL, "NULL argument");
  if (s->batch) return fail(AT_E_STATE, "run is already a member of a batch");
  if (!s->initialised) return fail(AT_E_STATE, "at_init_field before adding a run to a batch");
  if (s->cfg.precision != b->precision) return fail(AT_E_INVAL, "run precision differs from the batch's");
  if (s->stream != b->stream) return fail(AT_E_INVAL, "run and batch must use the same stream");
  if (s->device != b->device) return fail(AT_E_INVAL, "run and batch must be on the same device");
  if ((int)b->runs.size() >= kMaxBatchRuns) return fail(AT_E_INVAL, "batch is full");
  if (s->cfg.order != 4) return fail(AT_E_INVAL, "batched runs use the fourth-order scheme");
  if (s->cfg.form != 0) return fail(AT_E_INVAL, "batched runs use the total-energy flux form");
  if (s->cfg.forcing && (fused_lds_bytes(b->tile, word_of(b->precision), true) > kLdsBytes ||
                         fused_lds_bytes(b->tile_d, word_of(b->precision), true) > kLdsBytes))
    return fail(AT_E_INVAL, "the batch's tile shape does not fit a forced run; set a smaller tile first");
  b->runs.push_back(s);
  s->batch = b;
  drop_graph(b);
  return AT_OK;
}

int at_batch_remove(at_batch* b, at_sim* s) {
  if (!b || !s) return fail(AT_E_INVAL, "NULL argument");
  if (s->batch != b) return fail(AT_E_STATE, "run is not a member of this batch");
  batch_forget(b, s);
  s->batch = nullptr;
  return AT_OK;
}

int at_batch_size(at_batch* b, int32_t* n) {
  if (!b || !n) return fail(AT_E_INVAL, "NULL argument");
  *n = (int32_t)b->runs.size();
  return AT_OK;
}

int at_batch_step(at_batch* b, int32_t n_steps) {
  if (!b) return fail(AT_E_INVAL, "NULL handle");
  if (n_steps < 0 || n_steps > 4096) return fail(AT_E_INVAL, "n_steps out of 0 .. 4096");
  if (n_steps == 0 || b->runs.empty()) return AT_OK;
  for (at_sim* s : b->runs) {
    int rc = check_step_tables(s, s->step, n_steps);
    if (rc) return rc;
    if (s->cfg.forcing && (int64_t)s->h_fhat.size() < (s->step + n_steps) * (int64_t)kFhatRow)
      return fail(AT_E_SCHEDULE, "forcing table does not cover the requested steps");
  }
  return b->precision == AT_FP32 ? do_batch_steps<float>(b, n_steps) : do_batch_steps<double>(b, n_steps);
}

int at_batch_set_stage_tuning(at_batch* b, int32_t tile_sync, int32_t zchunk_sync, int32_t tile_delayed,
                              int32_t zchunk_delayed) {
  if (!b) return fail(AT_E_INVAL, "NULL handle");
  for (int k = 0; k < 2; ++k) {
    const int32_t tile = k ? tile_delayed : tile_sync, zchunk = k ? zchunk_delayed : zchunk_sync;
    if (tile < 0 || tile >= kTileCount) return fail(AT_E_INVAL, "unknown tile shape");
    if (zchunk < 4) return fail(AT_E_INVAL, "z chunk must be >= 4");
    if (!tile_fits(b, tile)) return fail(AT_E_INVAL, "tile shape needs more LDS than a compute unit has");
  }
  b->tile = tile_sync;
  b->zchunk = zchunk_sync;
  b->tile_d = tile_delayed;
  b->zchunk_d = zchunk_delayed;
  return AT_OK;
}

int at_batch_get_stage_tuning(at_batch* b, int32_t* tile_sync, int32_t* zchunk_sync, int32_t* tile_delayed,
                              int32_t* zchunk_delayed) {
  if (!b || !tile_sync || !zchunk_sync || !tile_delayed || !zchunk_delayed) return fail(AT_E_INVAL, "NULL argument");
  *tile_sync = b->tile;
  *zchunk_sync = b->zchunk;
  *tile_delayed = b->tile_d;
  *zchunk_delayed = b->zchunk_d;
  return AT_OK;
}

int at_batch_set_tuning(at_batch* b, int32_t tile, int32_t zchunk) {
  return at_batch_set_stage_tuning(b, tile, zchunk, tile, zchunk);
}

int at_batch_get_tuning(at_batch* b, int32_t* tile, int32_t* zchunk) {
  if (!b || !tile || !zchunk) return fail(AT_E_INVAL, "NULL argument");
  *tile = b->tile;
  *zchunk = b->zchunk;
  return AT_OK;
}

int at_batch_autotune(at_batch* b, const char* cache_path, int32_t reps, double* best_ms) {
  if (!b) return fail(AT_E_INVAL, "NULL handle");
  if (reps < 1 || reps > 100) return fail(AT_E_INVAL, "reps out of 1 .. 100");
  if (b->runs.empty()) return fail(AT_E_STATE, "autotuning needs at least one run in the batch");
  for (at_sim* s : b->runs) {
    int rc = check_step_tables(s, s->step, 1);
    if (rc) return rc;
  }
  return b->precision == AT_FP32 ? do_autotune<float>(b, cache_path, reps, best_ms)
                                 : do_autotune<double>(b, cache_path, reps, best_ms);
}

int at_batch_set_graph(at_batch* b, int32_t enable) {
  if (!b) return fail(AT_E_INVAL, "NULL handle");
  b->use_graph = enable ? 1 : 0;
  if (!enable) drop_graph(b);
  return AT_OK;
}

int at_batch_graph_stats(at_batch* b, int64_t* captures, int64_t* replays) {
  if (!b || !captures || !replays) return fail(AT_E_INVAL, "NULL argument");
  *captures = b->captures;
  *replays = b->replays;
  return AT_OK;
}

int at_batch_destroy(at_batch* b) {
  if (!b) return AT_OK;
  (void)hipStreamSynchronize(b->stream);
  for (at_sim* s : b->runs) s->batch = nullptr;
  drop_graph(b);
  if (b->d_buf) (void)hipFree(b->d_buf);
  if (b->d_trial_tot) (void)hipFree(b->d_trial_tot);
  for (int i = 0; i < 2; ++i) {
    (void)wait_staging(b, i);
    if (b->h_buf[i]) (void)hipHostFree(b->h_buf[i]);
    if (b->h_done[i]) (void)hipEventDestroy(b->h_done[i]);
  }
  if (b->side) {
    (void)hipStreamSynchronize(b->side);
    (void)hipStreamDestroy(b->side);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return AT_OK;
}

}  // extern "C"
