/* atns.h - C ABI of the MI355X Asynchrony-Tolerant (AT) compressible Navier-Stokes library.
 *
 * Method: Kumari & Donzis, "Direct Numerical Simulations of turbulent flows using high-order
 * Asynchrony-Tolerant schemes: accuracy and performance".  The library evaluates the right-hand
 * side of the compressible Navier-Stokes equations (Sec. 2, Eqs. cont, mome, ie, written in
 * total-energy flux form) on the triply periodic box [0, 2 pi)^3 with 4th-order central first
 * derivatives, replacing every stencil point that lies across a face of a processing element
 * (PE) by the AT combination of that face's past published levels (Sec. 2.1, Eq. at; Appendix B,
 * Table atschemes, (1,4) rows), and advances it with a low-storage third-order Runge-Kutta step.
 * The PEs of the paper's domain decomposition (Sec. 3, Eqs. NT, NI, NB) are virtual here: they
 * tile one GPU's grid, each publishes the two layers next to each of its six faces into a
 * device-resident ring of time levels (the send buffers of Sec. 3.1), and a delay schedule
 * (Sec. 3.1.1 Alg. SAA, Sec. 3.1.2 Alg. CAA) says which level each face reads at each step.
 *
 * Conventions for every call:
 *   - Return value: AT_OK (0) or a negative at_status; no exception crosses the ABI.
 *     at_last_error() gives a message for the calling thread's last failure.
 *   - Fields are structure-of-arrays, index order [component][z][y][x], x fastest.  Conserved
 *     components: 0 rho, 1 rho u, 2 rho v, 3 rho w, 4 E = rho (c_v T + |u|^2 / 2).
 *   - Host arrays passed in are read during the call only and never retained.
 *   - The device workspace and the HIP stream belong to the caller, who keeps both alive until
 *     at_destroy; the library never frees them.  The library itself allocates (hipMalloc) only the
 *     delay table, the forcing table and a small staging buffer, and frees them in at_destroy.
 *   - All device work is ordered on the caller's stream; calls returning host data
 *     (at_stats, at_get_field) synchronise that stream.  Batches fork the AT launches of each
 *     stage onto a stream of their own and join it back into the caller's stream within the
 *     call, so that when a call's work on the caller's stream has completed, all of it has.  One
 *     host thread per handle.
 *   - NaN / Inf in the state is reported through at_stats.nonfinite, not as an error.
 */
#ifndef ATNS_H
#define ATNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ATNS_API __attribute__((visibility("default")))

/* Opaque handle of one simulation (state, ring, schedule) bound to one device and stream. */
typedef struct at_sim at_sim;

typedef enum at_status {
  AT_OK = 0,
  AT_E_INVAL = -1,      /* bad argument, shape, divisibility or physical parameter          */
  AT_E_WORKSPACE = -2,  /* workspace pointer NULL / misaligned or smaller than required     */
  AT_E_SCHEDULE = -3,   /* delay > max_delay, a read of a level never published, or a step  */
                        /* beyond the schedule / forcing table                               */
  AT_E_HIP = -4,        /* a HIP runtime call failed (message in at_last_error)             */
  AT_E_STATE = -5       /* call out of order (e.g. stepping before at_init_field)           */
} at_status;

typedef enum at_precision { AT_FP64 = 0, AT_FP32 = 1 } at_precision;

/* Delay modes (Sec. 3.1).  t_l is the number of levels one AT extrapolation combines: 3 for the
 * fourth-order scheme, 4 for the sixth-order one.  SYNC: every face reads the current level.
 * CAA (Alg. CAA): PEs exchange every c_r steps, so from step max(c_r, t_l) on the delay is
 * n mod c_r on every face, with L = c_r - 1.  SAA (Alg. SAA): one exchange per step, delays random
 * and bounded by L; from step L + t_l on each (step, PE, face) delay is an independent uniform draw in {0..L} made with
 * SplitMix64 (Steele, Lea & Flood, 2014): z = output number ((n P + t) 6 + f) + 1 of the
 * generator seeded with `seed`, k = ((z >> 32) (L + 1)) >> 32.  EXPLICIT: a caller table. */
typedef enum at_delay_mode { AT_SYNC = 0, AT_CAA = 1, AT_SAA = 2, AT_EXPLICIT = 3 } at_delay_mode;

typedef struct at_config {
  int32_t n[3];        /* grid points in x, y, z; h_d = 2 pi / n[d]                            */
  int32_t p[3];        /* virtual PEs per direction; n[d] % p[d] == 0 and n[d] / p[d] >= 4      */
  int32_t order;       /* spatial order: 4 (the (1,4) rows of Appendix B: 2 face layers, t_l = 3)  */
                       /* or 6 (the (1,6) rows, Sec. 4.1.2: 3 face layers, t_l = 4; PE edges >= 6, */
                       /* unforced, single runs only)                                            */
  int32_t max_delay;   /* largest delay any face may use (0..8); the ring keeps max_delay + t_l */
                       /* levels (L + t_l levels per PE, Sec. 3.1)                              */
  int32_t precision;   /* AT_FP64 or AT_FP32 (fields, fluxes, ring and stencils); reductions of */
                       /* statistics and of the conserved totals are FP64 in both modes         */
  int32_t forcing;     /* 0: unforced; 1: add rho f to momentum and rho f.u to energy, with f   */
                       /* from at_set_forcing (Sec. 4.2)                                        */
  double gamma;        /* ratio of specific heats (1.4)                                          */
  double prandtl;      /* Prandtl number; conductivity k = mu c_p / Pr (0.7)                    */
  double gas_r;        /* gas constant R; p = rho R T, c_v = R / (gamma - 1) (1.0)              */
  double mu_ref;       /* viscosity mu = mu_ref (T / t_ref)^mu_exp                               */
  double t_ref;        /* reference temperature of the viscosity law (1.0)                      */
  double mu_exp;       /* viscosity exponent (0.76)                                              */
  double dt;           /* fixed time step (Sec. 2.2: no CFL reduction inside the step loop)     */
  int32_t form;        /* 0: total-energy flux form (the fifth variable is E = rho (c_v T +     */
                       /*    |u|^2/2); viscous and heat fluxes differentiated twice by the first- */
                       /*    derivative rows).  1: the paper's own discretisation (Sec. 2, Eqs.   */
                       /*    cont, mome, ie): the fifth variable is rho e = rho c_v T, the viscous */
                       /*    and conduction terms expanded into (2,4) AT second derivatives (App. */
                       /*    B) and mixed derivatives taken in the three steps of Sec. 2.1, the    */
                       /*    published layers hold the conserved variables (Sec. 3.1); order 4,    */
                       /*    PE edges >= 5, unforced, single runs                                  */
  int32_t visc_law;    /* 0: mu = mu_ref (T / t_ref)^mu_exp; 1 (form 1 only): Sutherland's law   */
                       /*    named in Sec. 2, mu = mu_ref (T / t_ref)^(3/2) (t_ref + S) / (T + S)  */
  double sutherland_s; /* Sutherland's constant S (same units as T; > 0 with visc_law 1)         */
} at_config;

typedef struct at_stats_s {
  int64_t step;        /* steps taken since the first supplied level                           */
  double time;         /* step * dt                                                             */
  double mass, mom[3], energy;           /* FP64 sums of the current field times h^3          */
  double mass_rk, mom_rk[3], energy_rk;  /* initial totals plus the FP64 sum over all RK     */
                                         /* stages of B_s * sum(dQ) * h^3                     */
  double K;            /* <rho |u|^2 / 2>                                 (Sec. 4.1)            */
  double eps;          /* <sigma_ij du_i/dx_j>, mean viscous dissipation  (Sec. 4.1)            */
  double enstrophy;    /* <|curl u|^2>                                    (Sec. 4.1)            */
  double Mt;           /* <|u|^2>^{1/2} / (gamma R <T>)^{1/2}             (Sec. 4, set-up)      */
  double umax;         /* max over points of |u|                                                */
  int32_t nonfinite;   /* 1 if any conserved value is NaN or Inf                                */
  int32_t reserved;
} at_stats_t;

/* Library version string. */
ATNS_API const char* at_version(void);

/* Message for the calling thread's last failing call ("" if none). */
ATNS_API const char* at_last_error(void);

/* Bytes of device workspace at_create needs for `cfg` (0 if cfg is invalid).  Holds two conserved
 * state buffers (a stage reads one and writes the other), the RK register, the ring of
 * published face layers: (max_delay + t_l) levels x 9 components (u, v, w, T and the face-normal flux of the five
 * conserved variables) x 2 M (1/ex + 1/ey + 1/ez) N^3 points (M = order / 2 layers per face); for
 * order 4 three level-sized buffers of the AT sums of the face-layer readers (one per RK stage of
 * a step; for the x and y faces, when the delayed-stage tile is aligned with the PEs, the
 * extrapolated values themselves), for order 6 the 15 flux components of every point; plus small
 * reduction scratch. */
ATNS_API size_t at_workspace_bytes(const at_config* cfg);

/* Create a simulation handle.  dev_workspace: device memory of at least at_workspace_bytes(cfg)
 * bytes, 256-byte aligned, owned by the caller.  hip_stream: a hipStream_t (NULL = default
 * stream) on the current device.  Errors: AT_E_INVAL (config), AT_E_WORKSPACE (size/alignment),
 * AT_E_HIP. */
ATNS_API int at_create(const at_config* cfg, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                       at_sim** out);

/* Load the state.  q_host: host float64 [n_levels][5][nz][ny][nx], oldest level first; the last
 * level becomes the current state Q^{n0}, n0 = n_levels - 1, and the older ones are published as
 * levels 0 .. n0 - 1 with synchronous derivatives (the synchronous start-up loop of Algs. SAA and
 * CAA fills L + t_l levels).  1 <= n_levels <= max_delay + t_l.  q_host is copied before the call
 * returns; the device work (conversion, publication, the initial conserved totals) is enqueued on
 * the stream without waiting for it.  Resets the step counter to n0, the
 * RK register and the conserved-total accumulators.  Errors: AT_E_INVAL, AT_E_HIP. */
ATNS_API int at_init_field(at_sim* sim, const double* q_host, int32_t n_levels);

/* Set the delay schedule for absolute steps 0 .. n_steps-1 (see at_delay_mode).  L and c_r are
 * used by CAA (L must equal c_r - 1) and SAA; seed by SAA; table (host int8
 * [n_steps][p_x p_y p_z][6], PE index (tz p_y + ty) p_x + tx, faces -x,+x,-y,+y,-z,+z) by
 * EXPLICIT only (NULL otherwise).  Every entry must satisfy 0 <= k <= max_delay and, if k > 0,
 * n - k - (t_l - 1) >= 0.  Errors: AT_E_INVAL, AT_E_SCHEDULE (entry invalid), AT_E_HIP. */
ATNS_API int at_set_delay_schedule(at_sim* sim, int32_t mode, int32_t L, int32_t c_r,
                                   uint64_t seed, const int8_t* table, int64_t n_steps);

/* Forcing of the stationary runs (Sec. 4.2: a large-scale force f added as rho f to the momentum
 * and rho f.u to the energy equation), amplitudes for absolute steps 0 .. n_steps-1: host float64
 * [n_steps][40][3][2] (re, im), copied before the call returns.  The 40 wavevectors are the half
 * space (kz > 0, or kz = 0 and ky > 0, or kz = ky = 0 and kx > 0) of the integer k with
 * 0 < |k|^2 <= 6, ordered by kz, then ky, then kx ascending; f(x) = sum_k 2 Re(fhat_k exp(i k.x)),
 * held fixed within a step.  Errors: AT_E_INVAL (forcing disabled in the config, bad sizes),
 * AT_E_HIP. */
ATNS_API int at_set_forcing(at_sim* sim, const double* fhat_host, int64_t n_steps);

/* RHS of the compressible Navier-Stokes equations (Sec. 2, Eqs. cont, mome, ie, in total-energy
 * flux form) at the current state and step: gradients and flux divergences by the central rows of
 * cfg->order, replaced across every delayed PE face by the AT stencils (Sec. 2.1, Eq. at; Appendix
 * B, the (1,4) or (1,6) rows) with that step's delays at stage time c = 0, plus the forcing
 * source of at_set_forcing; the state is neither published nor changed.  dev_out: device
 * [5][nz][ny][nx] in the config's precision, owned by the caller.
 * Errors: AT_E_STATE, AT_E_SCHEDULE, AT_E_HIP. */
ATNS_API int at_rhs(at_sim* sim, void* dev_out);

/* Enqueue n_steps full steps of Williamson's low-storage RK3 (A = 0, -5/9, -153/128;
 * B = 1/3, 15/16, 8/15; c = 0, 1/3, 3/4).  Stage 1 of step n publishes level n.  A delayed face
 * (k >= 1) at stage s extrapolates levels n-k, n-k-1, n-k-2 to t_n + c_s dt with weights
 * w_0 = (kappa+1)(kappa+2)/2, w_1 = -kappa(kappa+2), w_2 = kappa(kappa+1)/2, kappa = k + c_s
 * (the Appendix B polynomials at c_s = 0); the sixth-order scheme extrapolates levels n-k .. n-k-3
 * with w_0 = (kappa+1)(kappa+2)(kappa+3)/6, w_1 = -kappa(kappa+2)(kappa+3)/2,
 * w_2 = kappa(kappa+1)(kappa+3)/2, w_3 = -kappa(kappa+1)(kappa+2)/6 (the (1,6) rows at c_s = 0);
 * k = 0 reads the neighbour's current stage.
 * Asynchronous: returns after enqueueing.  Errors: AT_E_STATE, AT_E_SCHEDULE, AT_E_HIP. */
ATNS_API int at_rk_step(at_sim* sim, int32_t n_steps);

/* Enqueue n_steps steps of second-order Adams-Bashforth (Sec. 2.2, Eq. time_ab with T = 2):
 * Q^{n+1} = Q^n + dt (3/2 f^n - 1/2 f^{n-1}), one RHS per step at t_n, which publishes level n;
 * a delayed face extrapolates levels n-k, n-k-1, n-k-2 to t_n (kappa = k, the Appendix B
 * weights).  dt f^n is kept in the RK register for the next step, so a step with no stored
 * f^{n-1} (the first after at_init_field, at_rk_step or a batch step) is forward Euler.  Not
 * available through batches.  Asynchronous.  Errors: AT_E_STATE, AT_E_SCHEDULE, AT_E_HIP. */
ATNS_API int at_ab2_step(at_sim* sim, int32_t n_steps);

/* Statistics of the current state (synchronous derivatives on the whole periodic grid; global
 * reductions are the only all-PE operations, as in Sec. 3.1) into *out.  Synchronises the stream.
 * Errors: AT_E_STATE, AT_E_HIP. */
ATNS_API int at_stats(at_sim* sim, at_stats_t* out);

/* Copy the current conserved state to host float64 [5][nz][ny][nx].  Synchronises the stream. */
ATNS_API int at_get_field(at_sim* sim, double* q_host);

/* Device pointer to the current conserved state (config precision, [5][nz][ny][nx]); valid until
 * the next call on the handle.  Errors: AT_E_STATE. */
ATNS_API int at_field_device(at_sim* sim, void** dev_ptr);

/* Launch shape of the fused stage kernel: `tile` (0 .. AT_N_TILES-1) selects the workgroup column
 * tile and register budget (0: 64x8, 1: 32x8, 2: 32x8 at higher occupancy, 3: 32x4, 4: 64x4,
 * 5: 16x8, 6: 16x16 points in x-y), `zchunk` (>= 4) the number of z planes each workgroup marches through.
 * Results do not depend on either (every point is computed by the same arithmetic); only speed
 * does.  Set by the autotuner.  at_set_tuning sets the shape of every stage, at_get_tuning returns
 * that of the stages that read no delayed level.  Errors: AT_E_INVAL. */
#define AT_N_TILES 7
ATNS_API int at_set_tuning(at_sim* sim, int32_t tile, int32_t zchunk);
ATNS_API int at_get_tuning(at_sim* sim, int32_t* tile, int32_t* zchunk);

/* Separate launch shapes for the stages that read no delayed level (tile_sync, zchunk_sync) and
 * for those that do (tile_delayed, zchunk_delayed): the two are compiled differently (the AT code
 * of Sec. 2.1 is left out of the first), and their fastest shapes can differ.  A delayed-stage tile
 * whose width and height divide the PE edges (aligned) puts the extrapolated values of Sec. 2.1
 * into the tile halo; other tiles replace the crossing half of each stencil by the reader's AT sum.
 * The two round identically, so fields are the same bit for bit.  Same meaning and errors as
 * at_set_tuning. */
ATNS_API int at_set_stage_tuning(at_sim* sim, int32_t tile_sync, int32_t zchunk_sync, int32_t tile_delayed,
                                 int32_t zchunk_delayed);
ATNS_API int at_get_stage_tuning(at_sim* sim, int32_t* tile_sync, int32_t* zchunk_sync, int32_t* tile_delayed,
                                 int32_t* zchunk_delayed);

/* Kernel timing.  While enabled, every kernel the handle launches is bracketed by two HIP events
 * recorded on the handle's stream; at_kernel_timing synchronises the stream and returns, for kernel
 * `kernel` (0 .. AT_N_KERNELS-1, named by at_kernel_name), the summed event time in ms and the
 * number of launches since timing was enabled.  Errors: AT_E_INVAL, AT_E_HIP. */
#define AT_N_KERNELS 12
ATNS_API int at_set_kernel_timing(at_sim* sim, int32_t enable);
ATNS_API int at_kernel_timing(at_sim* sim, int32_t kernel, double* total_ms, int64_t* launches);
ATNS_API const char* at_kernel_name(int32_t kernel);

/* Release the handle and the library's own allocations (not the workspace or stream).  A run that
 * is a member of a batch leaves it. */
ATNS_API int at_destroy(at_sim* sim);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the statistics of at_stats for a field the caller holds,
 * with no handle, no allocation (no hipMalloc, hipFree or allocating library routine) and no
 * synchronisation.
 *   cfg:       the field's configuration; used: n, precision, gamma, gas_r, prandtl, mu_ref, t_ref,
 *              mu_exp (the PE grid, delays, forcing and dt play no part), validated as at_create does.
 *   dev_q:     device conserved state [5][nz][ny][nx] in cfg->precision (read only).
 *   dev_out:   device memory for one at_stats_t (8-byte aligned), written on the stream: mass, mom,
 *              energy, K, eps, enstrophy, Mt, umax and nonfinite as at_stats gives them for this
 *              field (same kernels, same reduction order); step and time are 0 and the _rk fields
 *              repeat the direct sums (there is no step count or RK history without a handle).
 *   hip_stream: the stream (NULL = default) on the current device; the call only enqueues.
 * The per-block partials and the reduction live in a static device array of the library, one per
 * device, sized for AT_STATS_NOALLOC_MAX_BLOCKS blocks of 64 x 4 points of one z plane
 * (ceil(nx / 64) ceil(ny / 4) nz <= 65536, e.g. up to 256^3; about 6.9 MB), held until the process
 * ends.  Every call on a device shares that array and leaves its contents there: calls that overlap
 * on one device (other streams or host threads without ordering between them) race.
 * Errors: AT_E_INVAL (NULL pointers, bad config, a grid beyond the block limit), AT_E_HIP. */
#define AT_STATS_NOALLOC_MAX_BLOCKS 65536
ATNS_API int at_field_stats_noalloc(const at_config* cfg, const void* dev_q, at_stats_t* dev_out, void* hip_stream);

/* ---------------------------------------------------------------------------------------------
 * Turbulence diagnostics of one field (Sec. 4.1): the statistics the paper compares between the
 * synchronous and asynchronous runs, computed on the device in FP64 for a field in either
 * precision.  With u_k the discrete Fourier coefficient of u (the forward sum over the grid of
 * u(x) exp(-i k.x), divided by the number of points N) and the shells kappa = round(|k|) of the
 * integer wavevectors (index j of an axis of n points is wavenumber j for j <= n/2, else j - n):
 *   E(kappa)   = sum over the shell of (|u_k|^2 + |v_k|^2 + |w_k|^2) / 2   (Sec. 4.1.2, Eq. ener;
 *                the shells add up to <u.u> / 2)
 *   E_p(kappa) = sum over the shell of |p_k|^2, p = rho R T                 (Eq. pres; E_p(0) = <p>^2)
 *   S = <g^3> / <g^2>^(3/2), F = <g^4> / <g^2>^2 of g = du/dx               (Sec. 4.1.3; 0 if <g^2> = 0)
 *   counts of x = eps / <eps> and of x = Omega / <Omega> (eps = sigma_ij du_i/dx_j, Omega =
 *   |curl u|^2; Sec. 4.1.3, Fig. enst_pdf) in nbins equal bins of [0, x_max), bin =
 *   floor(x (nbins / x_max)) in FP64, values below 0 in bin 0 and values >= x_max in bin nbins; a
 *   PDF whose mean is not positive and finite has all counts 0.
 * Derivatives are the synchronous central ones of cfg->order on the periodic grid (those of
 * at_stats).  Spectra come from in-place FFTs of the four real fields along x, y and z; the shell
 * sums and all reductions run in a fixed order (results do not change from call to call), the
 * counts are exact integers.
 * ------------------------------------------------------------------------------------------- */
#define AT_DIAG_MAX_SHELLS 4096
#define AT_DIAG_MAX_BINS 4096
#define AT_DIAG_N_SCALARS 8
typedef struct at_diag_params {
  int32_t nshell;      /* shells 0 .. nshell-1 reported (1 .. AT_DIAG_MAX_SHELLS); higher ones are    */
                       /* left out of E and E_p                                                        */
  int32_t nbins;       /* bins of each PDF (1 .. AT_DIAG_MAX_BINS), plus one for x >= x_max           */
  double eps_max;      /* x_max of eps / <eps> (> 0)                                                   */
  double ens_max;      /* x_max of Omega / <Omega> (> 0)                                               */
} at_diag_params;

/* Bytes of device workspace at_field_diagnostics needs (0 if cfg or prm is invalid): the half
 * spectra of u, v, w, p (4 nz ny px complex doubles, px = nx/2 + 1 rounded up to a multiple of 8),
 * eps and Omega of every point (2 N doubles), plus reduction partials: about 50 N bytes at 512^3. */
ATNS_API size_t at_diag_workspace_bytes(const at_config* cfg, const at_diag_params* prm);

/* Diagnostics of the device field dev_q ([5][nz][ny][nx] conserved variables in cfg->precision,
 * read only), enqueued on hip_stream (NULL = default) without synchronising.
 *   cfg:     used: n (each a power of two from 8 to 1024), order, precision, gamma, gas_r, mu_ref,
 *            t_ref, mu_exp; validated as at_create does.
 *   dev_ws:  device workspace of at least at_diag_workspace_bytes bytes, 256-byte aligned, owned by
 *            the caller; overwritten.
 *   dev_out: device doubles, 2 nshell + AT_DIAG_N_SCALARS + 2 (nbins + 1) of them: E[nshell],
 *            E_p[nshell], then S, F, <g^2>, <g^3>, <g^4>, <eps>, <Omega>, <p>, then the counts of
 *            eps / <eps> [nbins + 1] and of Omega / <Omega> [nbins + 1] (exact integers).
 * Errors: AT_E_INVAL (config, grid sizes, parameters, NULL pointers), AT_E_WORKSPACE, AT_E_HIP. */
ATNS_API int at_field_diagnostics(const at_config* cfg, const void* dev_q, void* dev_ws, size_t ws_bytes,
                                  const at_diag_params* prm, double* dev_out, void* hip_stream);

/* ---------------------------------------------------------------------------------------------
 * Batched runs.  Many independent runs (any grid, PE grid, delays, forcing, time step and
 * viscosity; one precision) advanced together: one launch per kernel per RK stage covers the
 * workgroups of every member, reading each member's arguments from a device run table through a
 * (run, workgroup) work list; the launches of a call are captured in a HIP graph and the graph is
 * replayed while membership, launch shape and chunk length stay the same.  Each member's state,
 * step counter and outputs are bitwise those it would have if stepped alone with at_rk_step at the
 * batch's launch shape.  Members keep their own handles (at_stats, at_get_field, at_rhs work as
 * usual between batched steps) and must use the batch's stream and device.
 * ------------------------------------------------------------------------------------------- */
typedef struct at_batch at_batch;

/* New empty batch for runs of `precision` (AT_FP32 / AT_FP64) enqueueing on hip_stream (NULL =
 * default stream).  The library allocates the batch's run tables and pinned staging itself.
 * Errors: AT_E_INVAL, AT_E_HIP. */
ATNS_API int at_batch_create(int32_t precision, void* hip_stream, at_batch** out);

/* Add an initialised run (joins at its current step; members may be at different steps).
 * Errors: AT_E_INVAL (precision, stream or device differ; batch full; a forced run with a tile
 * shape that does not fit; a sixth-order run), AT_E_STATE (not initialised, already in a batch). */
ATNS_API int at_batch_add(at_batch* batch, at_sim* sim);

/* Remove a member (it keeps its state and can be stepped alone).  Errors: AT_E_STATE. */
ATNS_API int at_batch_remove(at_batch* batch, at_sim* sim);
ATNS_API int at_batch_size(at_batch* batch, int32_t* n_runs);

/* Enqueue n_steps (0 .. 4096) RK steps of every member, each at its own step counter and with its
 * own schedule and forcing.  Asynchronous on the batch stream.  Errors: AT_E_SCHEDULE (a member's
 * tables do not cover its steps), AT_E_INVAL, AT_E_HIP. */
ATNS_API int at_batch_step(at_batch* batch, int32_t n_steps);

/* Launch shapes of the batched stage launches (same meaning as at_set_tuning and
 * at_set_stage_tuning; never change a field value).  Errors: AT_E_INVAL. */
ATNS_API int at_batch_set_tuning(at_batch* batch, int32_t tile, int32_t zchunk);
ATNS_API int at_batch_get_tuning(at_batch* batch, int32_t* tile, int32_t* zchunk);
ATNS_API int at_batch_set_stage_tuning(at_batch* batch, int32_t tile_sync, int32_t zchunk_sync,
                                       int32_t tile_delayed, int32_t zchunk_delayed);
ATNS_API int at_batch_get_stage_tuning(at_batch* batch, int32_t* tile_sync, int32_t* zchunk_sync,
                                       int32_t* tile_delayed, int32_t* zchunk_delayed);

/* Choose the launch shapes: looks up the device, the members' shapes and the fraction f of their
 * remaining scheduled steps that read delayed levels in cache_path (JSON lines; NULL = no cache);
 * otherwise times, for every feasible (tile, z chunk) (z chunks 8, 16, ..., 512, up to the members'
 * largest n_z), `reps` synchronous trial stages and (if
 * f > 0) `reps` delayed ones (each member at the delays of its first delayed step), keeps the
 * fastest shape of each kind (as at_batch_set_stage_tuning) and appends them to the cache.  A trial
 * rewrites only the second state buffer (dead between steps), neither stores the RK register (which
 * may hold the dt f^{n-1} of Adams-Bashforth steps) nor publishes, and discards its conserved
 * totals, so the members' states, including a stored Adams-Bashforth register, are unchanged.  *best_ms (may be NULL) receives
 * (1 - f) t_sync + f t_delayed of the chosen shapes.  Synchronises.  Errors: AT_E_STATE (empty batch), AT_E_SCHEDULE,
 * AT_E_INVAL, AT_E_HIP. */
ATNS_API int at_batch_autotune(at_batch* batch, const char* cache_path, int32_t reps, double* best_ms);

/* Graph capture on (default) or off (launches enqueued directly); graph capture and replay counts. */
ATNS_API int at_batch_set_graph(at_batch* batch, int32_t enable);
ATNS_API int at_batch_graph_stats(at_batch* batch, int64_t* captures, int64_t* replays);

/* Release the batch (members stay valid and leave it). */
ATNS_API int at_batch_destroy(at_batch* batch);

/* ---------------------------------------------------------------------------------------------
 * Served runs (continuous batching).  at_serve replays a request trace against the wall clock:
 * a request becomes visible at its arrival time, is admitted first come first served when fewer
 * than max_active runs are admitted and its device footprint (workspace, staging, schedule) fits
 * the HBM budget (capped by the device memory free when serving starts, less 1 GiB), is prepared
 * on a second stream while the batch computes (handle, field upload and conversion, schedule),
 * joins the batch at the next step boundary, and leaves at the boundary where it has done its
 * steps, after its final statistics (and field, if asked) are read back.  The batch advances by the
 * fewest steps any active run has left, at most 8, between boundaries.  The server allocates the
 * workspaces itself, reuses those of finished runs and frees them at the end.  Unforced
 * fourth-order cubes only; each request's delays are AT_SYNC, AT_CAA (c_r = L + 1) or AT_SAA (seed).
 * ------------------------------------------------------------------------------------------- */
typedef struct {
  int32_t precision;        /* AT_FP32 | AT_FP64 */
  int32_t max_active;       /* slots: runs served at once */
  int32_t tile, zchunk;     /* batch launch shape (tile < 0: library default) */
  double hbm_budget_bytes;  /* device bytes the server may hold for admitted runs */
  int32_t tile_delayed, zchunk_delayed; /* shape of the stages that read delayed levels (tile_delayed
                                           < 0: the same as tile, zchunk) */
} at_serve_config;

typedef struct {
  double arrival_s;         /* arrival, seconds after the start of serving; non-decreasing */
  int32_t n, p;             /* n^3 grid, p^3 virtual PEs */
  int32_t steps;            /* RK steps to run */
  int32_t mode, L;          /* AT_SYNC | AT_CAA | AT_SAA, delay bound (max_delay = L) */
  uint64_t seed;            /* AT_SAA seed */
  double dt, mu_ref;
  const double* q0;         /* host float64 [5][n][n][n]: initial state (read at admission) */
  double* q_final;          /* host float64 [5][n][n][n] for the final state, or NULL */
} at_request;

typedef struct {
  double admit_s, done_s;   /* seconds after the start: admission (preparation begins), completion */
                            /* (statistics read back)                                            */
  at_stats_t stats;         /* final statistics */
  int32_t status;           /* AT_OK, or the error that ended this request */
  int32_t reserved;
} at_result;

/* Serve nreq requests on hip_stream; blocks until every request has completed or failed.
 * results[i] belongs to reqs[i]; *makespan_s (may be NULL) receives the serving wall time.
 * Errors: AT_E_INVAL (bad arguments or an invalid request), AT_E_HIP; a request that can never
 * fit gets status AT_E_WORKSPACE without failing the call. */
ATNS_API int at_serve(const at_serve_config* cfg, const at_request* reqs, int32_t nreq, void* hip_stream,
                      at_result* results, double* makespan_s);

#ifdef __cplusplus
}
#endif
#endif /* ATNS_H */
