// gfx950 support kernels of the AT compressible Navier-Stokes library: FP64 statistics with
// synchronous 4th-order central derivatives (the k = 0 rows of the (1,4) schemes, Appendix B) and
// fixed-order reductions, precision conversion, and the separable forcing table.
#include "atns_internal.h"

namespace atns {
namespace {

constexpr int kBX = 64;  // one wavefront along x
constexpr int kBY = 4;

template <typename T>
__device__ __forceinline__ T tpow(T a, T b);
template <>
__device__ __forceinline__ double tpow<double>(double a, double b) { return pow(a, b); }
template <>
__device__ __forceinline__ float tpow<float>(float a, float b) { return powf(a, b); }

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// rho, u, v, w, T from the fifth variable E (form 0) or rho e (form 1, the paper's own form).
template <typename T>
__device__ __forceinline__ void primitives(const T* q, int64_t N, int64_t i, T inv_cv, int form, T pr[5]) {
  const T rho = q[i];
  const T rinv = T(1) / rho;
  const T u = q[N + i] * rinv, v = q[2 * N + i] * rinv, w = q[3 * N + i] * rinv;
  pr[0] = rho;
  pr[1] = u;
  pr[2] = v;
  pr[3] = w;
  pr[4] = form == 1 ? q[4 * N + i] * rinv * inv_cv : (q[4 * N + i] * rinv - T(0.5) * (u * u + v * v + w * w)) * inv_cv;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Statistics partials per block with synchronous periodic derivatives (no PE faces) of the run's
// order: the (1,4) central stencil (M = 2) or the (1,6) one (M = 3).
template <typename T, int M>
__global__ __launch_bounds__(256) void k_stats(Geom g, Coef<T> cf, const T* __restrict__ q,
                                               double* __restrict__ part) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool valid = x < g.n[0] && y < g.n[1];
  double s[kNStat];
#pragma unroll
  for (int c = 0; c < kNStat; ++c) s[c] = 0.0;
  if (valid) {
    const int64_t N = g.npts;
    const int64_t i = ((int64_t)z * g.n[1] + y) * g.n[0] + x;
    const int pt[3] = {x, y, z};
    T G[kNGrad];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T v[2 * M][4];
#pragma unroll
      for (int mi = 0; mi < 2 * M; ++mi) {
        const int m = mi < M ? mi - M : mi - M + 1;
        int r[3] = {x, y, z};
        r[d] = wrap1(pt[d] + m, g.n[d]);
        const int64_t ir = ((int64_t)r[2] * g.n[1] + r[1]) * g.n[0] + r[0];
        T pr[5];
        primitives<T>(q, N, ir, cf.inv_cv, cf.form, pr);
        v[mi][0] = pr[1];
        v[mi][1] = pr[2];
        v[mi][2] = pr[3];
        v[mi][3] = pr[4];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T num = M == 2 ? (v[0][c] - T(8) * v[1][c] + T(8) * v[2][c] - v[3][c])
                             : (T(9) * v[1][c] - v[0][c]) + T(45) * (v[3][c] - v[2][c]) + (v[5][c] - T(9) * v[4][c]);
        G[c < 3 ? 3 * c + d : 9 + d] = num * (M == 2 ? cf.inv12h[d] : cf.inv60h[d]);
      }
    }
    T pr[5];
    primitives<T>(q, N, i, cf.inv_cv, cf.form, pr);
    const double tt = (double)pr[4] * (double)cf.inv_tref;
    const double mu = cf.visc == 1 ? (double)cf.mu_ref * tt * sqrt(tt) * (1.0 / (double)cf.inv_tref + (double)cf.suth_s) /
                                         ((double)pr[4] + (double)cf.suth_s)
                                   : (double)cf.mu_ref * pow(tt, (double)cf.mu_exp);
    const double th = (double)G[0] + (double)G[4] + (double)G[8];
    double eps = 0.0;
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        double sg = mu * ((double)G[3 * ii + jj] + (double)G[3 * jj + ii]);
        if (ii == jj) sg -= (2.0 / 3.0) * mu * th;
        eps += sg * (double)G[3 * ii + jj];
      }
    const double ox = (double)G[7] - (double)G[5];
    const double oy = (double)G[2] - (double)G[6];
    const double oz = (double)G[3] - (double)G[1];
    const double u = pr[1], v = pr[2], w = pr[3];
    const double uu = u * u + v * v + w * w;
    int nonfin = 0;
#pragma unroll
    for (int c = 0; c < kNQ; ++c) {
      const double qv = (double)q[c * N + i];
      s[c] = qv;
      if (!isfinite(qv)) nonfin = 1;
    }
    s[5] = 0.5 * (double)pr[0] * uu;
    s[6] = eps;
    s[7] = ox * ox + oy * oy + oz * oz;
    s[8] = uu;
    s[9] = (double)pr[4];
    s[10] = sqrt(uu);
    s[11] = nonfin;
  }
  __shared__ double red[4][kNStat];
  const int lane = threadIdx.x, wave = threadIdx.y;
#pragma unroll
  for (int c = 0; c < kNStat; ++c) {
    double v = s[c];
    if (c == 10 || c == 11) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    } else {
      v = wave_sum(v);
    }
    if (lane == 0) red[wave][c] = v;
  }
  __syncthreads();
  if (wave == 0 && lane < kNStat) {
    double v;
    if (lane == 10 || lane == 11)
      v = fmax(fmax(red[0][lane], red[1][lane]), fmax(red[2][lane], red[3][lane]));
    else
      v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[blk * kNStat + lane] = v;
  }
}

// Fixed-order final reduction: out[0..12] statistics, out[13..17] RK totals partial sums.
// Fixed-order two-level reduction of the per-block partials (deterministic: the order depends only
// on the partial counts).  Level 1: workgroup j reduces its contiguous share of the statistic
// partials [nblk][13] and of the FP64 RK-total slots [ntot][5] into mid[j][18]; level 2 reduces
// the kStatRed rows of mid into out[18].  Components 10 (max |u|) and 11 (non-finite flag) take
// the maximum, the others the sum.
constexpr int kStatOut = kNStat + kNQ;
static_assert(kStatRed == 256, "level 2 gives one thread per level-1 row");

__device__ __forceinline__ double tree256(double* red, double v, bool is_max) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = is_max ? fmax(red[t], red[t + s]) : red[t] + red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_stats_reduce(const double* __restrict__ part, int64_t nblk,
                                                      const double* __restrict__ tot_part, int64_t ntot,
                                                      double* __restrict__ mid) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int64_t j = blockIdx.x;
  const int64_t lp = (nblk + kStatRed - 1) / kStatRed, lt = (ntot + kStatRed - 1) / kStatRed;
  const int64_t p0 = j * lp, p1 = min(p0 + lp, nblk), t0 = j * lt, t1 = min(t0 + lt, ntot);
  for (int c = 0; c < kStatOut; ++c) {
    const bool is_max = (c == 10 || c == 11);
    double v = 0.0;
    if (c < kNStat) {
      for (int64_t b = p0 + t; b < p1; b += 256) {
        const double pv = part[b * kNStat + c];
        v = is_max ? fmax(v, pv) : v + pv;
      }
    } else if (tot_part) {
      for (int64_t b = t0 + t; b < t1; b += 256) v += tot_part[b * kNQ + (c - kNStat)];
    }
    const double r = tree256(red, v, is_max);
    if (t == 0) mid[j * kStatOut + c] = r;
  }
}

__global__ __launch_bounds__(256) void k_stats_final(const double* __restrict__ mid, double* __restrict__ out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  for (int c = 0; c < kStatOut; ++c) {
    const bool is_max = (c == 10 || c == 11);
    const double r = tree256(red, t < kStatRed ? mid[t * kStatOut + c] : 0.0, is_max);
    if (t == 0) out[c] = r;
  }
}

// The statistics record of a field from the reduced sums (the conversions at_stats makes on the
// host), for a caller without a handle: no step count and no RK history, so step and time are 0
// and the RK-accumulated totals repeat the direct sums.
__global__ void k_stats_record(const double* __restrict__ st, at_stats_t* __restrict__ o, double npts, double vol,
                               double gamma, double gas_r) {
  if (threadIdx.x != 0) return;
  o->step = 0;
  o->time = 0.0;
  o->mass = st[0] * vol;
  for (int a = 0; a < 3; ++a) o->mom[a] = st[1 + a] * vol;
  o->energy = st[4] * vol;
  o->mass_rk = o->mass;
  for (int a = 0; a < 3; ++a) o->mom_rk[a] = o->mom[a];
  o->energy_rk = o->energy;
  o->K = st[5] / npts;
  o->eps = st[6] / npts;
  o->enstrophy = st[7] / npts;
  o->Mt = sqrt(st[8] / npts) / sqrt(gamma * gas_r * (st[9] / npts));
  o->umax = st[10];
  o->nonfinite = st[11] != 0.0 ? 1 : 0;
  o->reserved = 0;
}

template <typename T>
__global__ void k_convert(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

template <typename T>
__global__ void k_to_double(const T* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// A[pair][x][c] = sum over wavevectors of that (ky, kz) pair of fhat(c) e^{i kx x}.
template <typename T>
__global__ void k_force_table(int nx, const double* __restrict__ fhat, const int* __restrict__ wv_kx,
                              const int* __restrict__ wv_pair, int npair, T* __restrict__ table,
                              const T* __restrict__ phase_x) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= npair * nx) return;
  const int pidx = tid / nx, x = tid - pidx * nx;
  double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  for (int w = 0; w < kNForce; ++w) {
    if (wv_pair[w] != pidx) continue;
    const T* ph = phase_x + ((int64_t)(wv_kx[w] + 2) * nx + x) * 2;
    const double ec = (double)ph[0], es = (double)ph[1];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double fr = fhat[(w * 3 + c) * 2], fi = fhat[(w * 3 + c) * 2 + 1];
      acc[c][0] += fr * ec - fi * es;
      acc[c][1] += fr * es + fi * ec;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    table[(int64_t)tid * 6 + 2 * c] = (T)acc[c][0];
    table[(int64_t)tid * 6 + 2 * c + 1] = (T)acc[c][1];
  }
}

dim3 grid_of(const Geom& g) {
  return dim3((g.n[0] + kBX - 1) / kBX, (g.n[1] + kBY - 1) / kBY, g.n[2]);
}

}  // namespace

int64_t update_blocks(const Geom& g) {
  const dim3 gr = grid_of(g);
  return (int64_t)gr.x * gr.y * gr.z;
}
int64_t stats_blocks(const Geom& g) { return update_blocks(g); }

const char* kernel_name(int id) {
  static const char* names[kKCount] = {"k_stage", "k_stage(rhs)", "k_stage(publish)", "k_force_table",
                                       "k_stats", "k_at_sums", "k6_gradflux", "k6_divupdate",
                                       "kp_publish", "kp_grad", "kp_rhs", "k6_ghosts"};
  return (id >= 0 && id < kKCount) ? names[id] : "";
}

#define HOOKED(id, launch)              \
  do {                                  \
    if (hook) hook->before(id, stream); \
    launch;                             \
    if (hook) hook->after(id, stream);  \
  } while (0)

template <typename T>
hipError_t launch_convert(const double* src, T* dst, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_convert<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_to_double(const T* src, double* dst, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_to_double<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stats(const Geom& g, const Coef<T>& cf, const T* q, double* part, double* out,
                        const double* tot_part, int64_t ntot_blocks, double gamma, hipStream_t stream,
                        LaunchHook* hook) {
  (void)gamma;
  const dim3 blk(kBX, kBY, 1);
  const dim3 gr = grid_of(g);
  if (g.order == 6)
    HOOKED(kKStats, hipLaunchKernelGGL((k_stats<T, 3>), gr, blk, 0, stream, g, cf, q, part));
  else
    HOOKED(kKStats, hipLaunchKernelGGL((k_stats<T, 2>), gr, blk, 0, stream, g, cf, q, part));
  double* mid = out + kStatOutSlots;
  hipLaunchKernelGGL(k_stats_reduce, dim3(kStatRed), dim3(256), 0, stream, part, stats_blocks(g), tot_part,
                     ntot_blocks, mid);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, stream, (const double*)mid, out);
  return hipGetLastError();
}

hipError_t launch_stats_record(const double* raw, at_stats_t* dst, double npts, double vol, double gamma,
                               double gas_r, hipStream_t stream) {
  hipLaunchKernelGGL(k_stats_record, dim3(1), dim3(64), 0, stream, raw, dst, npts, vol, gamma, gas_r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force_table(const Geom& g, const double* fhat_step, const int* wv_kx,
                              const int* wv_pair, int npair, T* table, const T* phase_x,
                              hipStream_t stream, LaunchHook* hook) {
  const int n = npair * g.n[0];
  HOOKED(kKForce, hipLaunchKernelGGL(k_force_table<T>, dim3((n + 255) / 256), dim3(256), 0, stream,
                                     g.n[0], fhat_step, wv_kx, wv_pair, npair, table, phase_x));
  return hipGetLastError();
}

#define ATNS_INSTANTIATE(T)                                                                          \
  template hipError_t launch_convert<T>(const double*, T*, int64_t, hipStream_t);                    \
  template hipError_t launch_to_double<T>(const T*, double*, int64_t, hipStream_t);                  \
  template hipError_t launch_stats<T>(const Geom&, const Coef<T>&, const T*, double*, double*,       \
                                      const double*, int64_t, double, hipStream_t, LaunchHook*);     \
  template hipError_t launch_force_table<T>(const Geom&, const double*, const int*, const int*, int, \
                                            T*, const T*, hipStream_t, LaunchHook*);
ATNS_INSTANTIATE(double)
ATNS_INSTANTIATE(float)

}  // namespace atns
