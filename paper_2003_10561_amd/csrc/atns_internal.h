// Internal declarations shared by the host side of the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "atns.h"

namespace atns {

constexpr int kNQ = 5;        // conserved variables
constexpr int kNPub = 4;      // published primitives per ghost point: u, v, w, T
constexpr int kNRing = 9;     // ring components per slab point: u, v, w, T, F_d(0..4)
constexpr int kNGrad = 12;    // du_i/dx_j (9, index 3 i + j) and dT/dx_j (3, index 9 + j)
constexpr int kNForce = 40;   // forcing wavevectors
constexpr int kMaxPairs = 16; // distinct (ky, kz) pairs among them (11 in practice)
constexpr int kNStat = 13;    // per-block statistic partials
constexpr int kMaxDelay = 8;
// Statistics output region: 18 doubles (13 statistics, 5 RK totals) in the first kStatOutSlots,
// then the kStatRed level-1 rows of the two-level reduction.
constexpr int kStatOutSlots = 32;
// Slots kStatInit .. kStatInit + 4 of the output region keep the FP64 sums of the conserved
// variables of the state loaded by at_init_field (the start of the RK-accumulated totals).
constexpr int kStatInit = 24;
constexpr int kStatRed = 256;
constexpr size_t kStatOutBytes = sizeof(double) * (kStatOutSlots + (size_t)kStatRed * (kNStat + 5));

// Grid, virtual-PE tiling and ring geometry (shared by every kernel of one run).
struct Geom {
  int form;           // 0: total-energy flux form; 1: the paper's own discretisation (rho e)
  int order;          // spatial order: 4 or 6
  int M;              // layers each PE publishes per face (order / 2); the stencils' reach
  int tl;             // levels of one AT extrapolation (M + 1)
  int n[3];           // points per direction
  int p[3];           // virtual PEs per direction
  int e[3];           // PE edge n[d] / p[d]
  int64_t npts;
  int64_t slab[3];    // points of one direction's slab set: 2 M p_d n_a n_b
  int64_t ring_dir_off[3];  // element offset of direction d inside one ring slot
  int64_t ring_slot;  // elements per ring slot = 9 * sum_d slab[d] (form 1: 5 * sum_d slab[d])
  int R;              // ring slots = max_delay + tl
  int ntiles;
};

// Physical constants in the working precision.
template <typename T>
struct Coef {
  T inv12h[3];      // 1 / (12 h_d)
  T inv60h[3];      // 1 / (60 h_d)
  T gas_r, inv_cv, cp_over_pr, mu_ref, inv_tref, mu_exp;
  T suth_s;         // Sutherland's constant (visc = 1)
  int visc;         // 0 power law, 1 Sutherland (form 1 only)
  int form;         // 0 total energy E, 1 internal energy rho e as the fifth variable
};

// Forcing: per-step table A[pair][x][c] = sum_kx fhat(kx, pair, c) e^{i kx x} (complex), and the
// y / z phase tables e^{i ky y} (ky = -2..2) and e^{i kz z} (kz = 0..2).
template <typename T>
struct ForceArgs {
  const T* table;     // [npair][nx][3][2], or null when unforced
  const T* phase_y;   // [5][ny][2]
  const T* phase_z;   // [3][nz][2]
  const int* pair_kyz; // [npair][2]: ky, kz of each pair (device memory)
  int npair;
};

// Work of one RK stage (or one RHS evaluation).
template <typename T>
struct StageArgs {
  Geom g;
  Coef<T> cf;
  T* q;               // conserved state [5][N] read by the stage
  T* q_out;           // conserved state written by the stage (the other buffer)
  T* dq;              // RK register [5][N]
  T* ring;            // ring base
  T* gv_out;          // AT sums of the face-layer readers, three slot-sized regions (one per stage
                      // of the step), written by k_at_sums
  const T* gv;        // the region of this stage, read by the stage kernel
  T* rhs_out;         // RHS-only mode output [5][N] (null in stepping mode)
  const int8_t* delays;  // [ntiles][6] for this step
  int64_t step;       // absolute step index n
  int step_mod_r;     // n mod R: ring slot of level n
  T rk_a, rk_b, dt;
  T c_prev;           // Adams-Bashforth: Q += rk_b dQ + c_prev dQ_prev (dQ = dt RHS); 0 for RK
  int publish;        // stage 1: write level n into the ring
  int store_dq;       // 0 in the last stage (the register is not read again)
  int at_ghost;       // the delayed stages of this step run on tiles aligned with the PEs: the x / y
                      // entries of gv are extrapolated halo values, not per-reader sums
  double* tot_part;   // [nblk][5] FP64 running sums of B_s * sum(dQ) * h^3
  double vol;         // h_x h_y h_z
  ForceArgs<T> force;
};

// Fused-stage launch shapes: BX x BY columns per workgroup and the FP32 occupancy target in
// waves per SIMD (FP64 uses half).  Chosen per run by the autotuner; results never depend on it.
struct TileShape {
  int bx, by, waves;
};
constexpr int kTileCount = 7;
__host__ __device__ constexpr TileShape tile_shape(int t) {
  return t == 0 ? TileShape{64, 8, 4}
       : t == 1 ? TileShape{32, 8, 2}
       : t == 2 ? TileShape{32, 8, 4}
       : t == 3 ? TileShape{32, 4, 2}
       : t == 4 ? TileShape{64, 4, 3}
       : t == 5 ? TileShape{16, 8, 2}
                : TileShape{16, 16, 4};
}
__host__ __device__ inline int tile_bx(int t) { return tile_shape(t).bx; }
__host__ __device__ inline int tile_by(int t) { return tile_shape(t).by; }
// Every workgroup tile of this shape lies inside one PE along x and y (PE edges multiples of the
// tile's): delayed stages then place the extrapolated values in the tile halo.
inline bool tile_aligned(const Geom& g, int t) { return g.e[0] % tile_bx(t) == 0 && g.e[1] % tile_by(t) == 0; }
int64_t fused_blocks(const Geom& g, int tile, int zchunk);
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per compute unit on gfx950
size_t fused_lds_bytes(int tile, size_t word, bool forced);
// `at`: some face of the run is delayed at this stage (selects the instantiation with the AT logic).
template <typename T>
hipError_t launch_fused(const StageArgs<T>& a, int tile, int zchunk, int mode, bool at, hipStream_t stream);
template <typename T>
// cs: c_s of stages 1-3; nst: the stages written (3, or 1 for an Adams-Bashforth step: c_s = cs[0])
hipError_t launch_at_sums(const StageArgs<T>& a, const double* cs, hipStream_t stream, int nst = 3);

// Batched launches (one launch over the workgroups of many runs).  A run table is an array of
// batch_arg_bytes<T>() records written by pack_batch_arg; work lists hold (run, local block).
template <typename T>
size_t batch_arg_bytes();
template <typename T>
void pack_batch_arg(const StageArgs<T>& s, int tile, int zchunk, int views, void* dst);
// at: 0 for the plain instantiation; else which AT instantiations to launch over the work list,
// kAtMasked (runs without at_ghost) and / or kAtGhost (runs with it)
constexpr int kAtMasked = 1, kAtGhost = 2;
template <typename T>
hipError_t launch_fused_batch(const void* runs, const uint2* work, int64_t nblk, int tile, bool forced, bool publish,
                              int at, int mode, hipStream_t stream);
template <typename T>
hipError_t launch_at_sums_batch(const void* runs, const uint2* work, int64_t nblk, const double* cs,
                                hipStream_t stream);
int64_t view_blocks(const Geom& g);  // 256-point blocks of k_at_sums for one run
constexpr int kModeStepH = 0, kModeRhsH = 1, kModePublishH = 2;

// Kernel identities for timing (names in kernel_name()).
enum KernelId {
  kKStage = 0, kKRhs = 1, kKPublish = 2, kKForce = 3, kKStats = 4, kKGhost = 5, kK6Grad = 6, kK6Div = 7,
  kKPPublish = 8, kKPGrad = 9, kKPRhs = 10, kK6Ghost = 11, kKCount = 12
};

// The paper's own discretisation (stagep.hip, form 1): publication of the conserved variables,
// then per stage the AT gradients and the right-hand side with the update, one point per thread.
template <typename T>
struct StagePArgs {
  Geom g;
  Coef<T> cf;
  T* q;
  T* q_out;
  T* dq;
  T* grad;            // [12][N]
  T* ring;            // R slots of 5 * sum_d slab[d]
  T* rhs_out;
  const int8_t* delays;
  double* tot_part;
  int step_mod_r, slot, store_dq, mode;
  T cs, rk_a, rk_b, dt, c_prev;
  double vol;
};
constexpr int kPPublish = 0, kPGrad = 1, kPRhs = 2, kPGradPublish = 3;
int64_t paper_blocks(const Geom& g);
template <typename T>
hipError_t launch_stagep(const StagePArgs<T>& s, int which, hipStream_t stream);

// Sixth-order stage (stage6.hip): gradients and fluxes, then divergence and update; tiles of
// bx x by columns inside one PE, one workgroup per (tile, z-PE).
template <typename T>
struct Stage6Args {
  Geom g;
  Coef<T> cf;
  T i60h[3];
  T* q;
  T* q_out;
  T* dq;
  T* flux;            // [3][5][N]
  T* ring;
  T* gv;              // extrapolated values behind the faces: one ring slot per stage of a step
  T* rhs_out;
  const int8_t* delays;
  double* tot_part;
  int bx, by;
  int step_mod_r, publish, store_dq, mode;
  T cs, rk_a, rk_b, dt, c_prev;
  T cs3[3];           // the ghost pass: c_s of each of its nst stages
  int nst;
  double vol;
};
void tile6_of(const Geom& g, int* bx, int* by);
int64_t blocks6(const Geom& g);
// gradflux: the gradient / flux launch; otherwise the divergence / update launch
template <typename T>
hipError_t launch_stage6(const Stage6Args<T>& s, bool gradflux, hipStream_t stream);
// the extrapolated face values of nst stages (c_s in cs3) into gv, gv + ring_slot, ...
template <typename T>
hipError_t launch_ghosts6(const Stage6Args<T>& s, hipStream_t stream);
const char* kernel_name(int id);

// Optional event bracketing of each launch (host side implements it).
struct LaunchHook {
  virtual void before(int kernel_id, hipStream_t s) = 0;
  virtual void after(int kernel_id, hipStream_t s) = 0;
  virtual ~LaunchHook() = default;
};

// Launchers (kernels.hip).  All enqueue on `stream`; `hook` may be null.
template <typename T>
hipError_t launch_convert(const double* src, T* dst, int64_t n, hipStream_t stream);
template <typename T>
hipError_t launch_to_double(const T* src, double* dst, int64_t n, hipStream_t stream);
// Statistics with the synchronous central derivatives of the run's order (g.order).
template <typename T>
hipError_t launch_stats(const Geom& g, const Coef<T>& cf, const T* q, double* part, double* out,
                        const double* tot_part, int64_t ntot_blocks, double gamma, hipStream_t stream,
                        LaunchHook* hook);
template <typename T>
hipError_t launch_force_table(const Geom& g, const double* fhat_step, const int* wv_kx,
                              const int* wv_pair, int npair, T* table, const T* phase_x,
                              hipStream_t stream, LaunchHook* hook);
// The statistics record of reduced sums `raw` (the output region of launch_stats) into a device
// at_stats_t, with step 0, time 0 and the RK totals equal to the direct sums.
hipError_t launch_stats_record(const double* raw, at_stats_t* dst, double npts, double vol, double gamma,
                               double gas_r, hipStream_t stream);
int64_t update_blocks(const Geom& g);
int64_t stats_blocks(const Geom& g);

}  // namespace atns
