// gfx950 kernels of the AT compressible Navier-Stokes step: primitives and AT gradients,
// total fluxes, AT flux divergence with the low-storage RK3 update, statistics and forcing.
//
// The stencil is the 4th-order central first derivative (the k = 0 rows of the (1,4) schemes,
// Appendix B, Table atschemes).  A stencil point outside the PE that owns the evaluation point is
// a buffer point (Sec. 2, Fig. domain): with delay k = 0 it is the neighbour's current value, with
// k >= 1 it is w_0 v^{n-k} + w_1 v^{n-k-1} + w_2 v^{n-k-2} from the ring (Sec. 2.1, Eq. at).
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

// Layer of local index l inside a PE of edge e: 0, 1 next to the low face, 2, 3 next to the high
// face, -1 for points that publish nothing in this direction.
__device__ __forceinline__ int layer_of(int l, int e) {
  return l < 2 ? l : (l >= e - 2 ? l - e + 4 : -1);
}

// Position of global point (x, y, z) in direction d's slab set, plane jp = 4 tile + layer.
__device__ __forceinline__ int64_t slab_index(const Geom& g, int d, int x, int y, int z, int jp) {
  if (d == 0) return ((int64_t)z * g.n[1] + y) * (4 * g.p[0]) + jp;
  if (d == 1) return ((int64_t)z * (4 * g.p[1]) + jp) * g.n[0] + x;
  return ((int64_t)jp * g.n[1] + y) * g.n[0] + x;
}

template <typename T>
__device__ __forceinline__ void at_weights(T kap, T w[3]) {
  w[0] = (kap + T(1)) * (kap + T(2)) * T(0.5);
  w[1] = -kap * (kap + T(2));
  w[2] = kap * (kap + T(1)) * T(0.5);
}

template <typename T>
__device__ __forceinline__ void primitives(const T* q, int64_t N, int64_t i, T inv_cv, T pr[5]) {
  const T rho = q[i];
  const T rinv = T(1) / rho;
  const T u = q[N + i] * rinv, v = q[2 * N + i] * rinv, w = q[3 * N + i] * rinv;
  pr[0] = rho;
  pr[1] = u;
  pr[2] = v;
  pr[3] = w;
  pr[4] = (q[4 * N + i] * rinv - T(0.5) * (u * u + v * v + w * w)) * inv_cv;
}

// Extrapolated ring value of component `comp` of direction d at slab position sidx.
template <typename T>
__device__ __forceinline__ T ring_extrap(const StageArgs<T>& a, int d, int comp, int64_t sidx, int k) {
  T w[3];
  at_weights<T>(T(k) + a.cstage, w);
  const Geom& g = a.g;
  T v = T(0);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int64_t lev = a.step - k - l;
    const int slot = (int)(lev % g.R);
    v += w[l] * a.ring[slot * g.ring_slot + g.ring_dir_off[d] + (int64_t)comp * g.slab[d] + sidx];
  }
  return v;
}

// Velocity and temperature gradients with AT ghosts; at stage 1 publish u, v, w, T.
template <typename T>
__global__ __launch_bounds__(256) void k_grad(StageArgs<T> a, int sync) {
  const Geom& g = a.g;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.n[0] || y >= g.n[1]) return;
  const int pt[3] = {x, y, z};
  int tl[3], lc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    tl[d] = pt[d] / g.e[d];
    lc[d] = pt[d] - tl[d] * g.e[d];
  }
  const int tile = (tl[2] * g.p[1] + tl[1]) * g.p[0] + tl[0];
  const int8_t* kf = a.delays + tile * 6;
  const int64_t N = g.npts;
  const int64_t i = ((int64_t)z * g.n[1] + y) * g.n[0] + x;
  T gr[kNGrad];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T v[4][4];
    const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
      const int m = ms[mi];
      const int lr = lc[d] + m;
      int r[3] = {x, y, z};
      r[d] = wrap1(pt[d] + m, g.n[d]);
      int k = 0;
      if (!sync) {
        if (lr < 0) k = kf[2 * d];
        else if (lr >= g.e[d]) k = kf[2 * d + 1];
      }
      if (k == 0) {
        const int64_t ir = ((int64_t)r[2] * g.n[1] + r[1]) * g.n[0] + r[0];
        T pr[5];
        primitives<T>(a.q, N, ir, a.cf.inv_cv, pr);
        v[mi][0] = pr[1];
        v[mi][1] = pr[2];
        v[mi][2] = pr[3];
        v[mi][3] = pr[4];
      } else {
        const int tr = r[d] / g.e[d];
        const int jp = 4 * tr + layer_of(r[d] - tr * g.e[d], g.e[d]);
        const int64_t sidx = slab_index(g, d, r[0], r[1], r[2], jp);
#pragma unroll
        for (int c = 0; c < kNPub; ++c) v[mi][c] = ring_extrap<T>(a, d, c, sidx, k);
      }
    }
#pragma unroll
    for (int c = 0; c < kNPub; ++c) {
      const T dd = (v[0][c] - T(8) * v[1][c] + T(8) * v[2][c] - v[3][c]) * a.cf.inv12h[d];
      gr[c < 3 ? 3 * c + d : 9 + d] = dd;
    }
  }
#pragma unroll
  for (int j = 0; j < kNGrad; ++j) a.grad[j * N + i] = gr[j];
  if (a.publish) {
    T pr[5];
    primitives<T>(a.q, N, i, a.cf.inv_cv, pr);
    const int slot = (int)(a.step % g.R);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lay = layer_of(lc[d], g.e[d]);
      if (lay < 0) continue;
      const int64_t sidx = slab_index(g, d, x, y, z, 4 * tl[d] + lay);
      T* base = a.ring + slot * g.ring_slot + g.ring_dir_off[d] + sidx;
#pragma unroll
      for (int c = 0; c < kNPub; ++c) base[(int64_t)c * g.slab[d]] = pr[1 + c];
    }
  }
}

// Total fluxes F_j of (rho, rho u_i, E) at every point (Sec. 2, Eqs. cont, mome, ie in
// total-energy form); at stage 1 publish the face-normal flux F_d on the slab layers.
template <typename T>
__global__ __launch_bounds__(256) void k_flux(StageArgs<T> a) {
  const Geom& g = a.g;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.n[0] || y >= g.n[1]) return;
  const int64_t N = g.npts;
  const int64_t i = ((int64_t)z * g.n[1] + y) * g.n[0] + x;
  T pr[5], G[kNGrad];
  primitives<T>(a.q, N, i, a.cf.inv_cv, pr);
#pragma unroll
  for (int j = 0; j < kNGrad; ++j) G[j] = a.grad[j * N + i];
  const T mu = a.cf.mu_ref * tpow<T>(pr[4] * a.cf.inv_tref, a.cf.mu_exp);
  const T kt = mu * a.cf.cp_over_pr;
  const T theta = G[0] + G[4] + G[8];
  T sig[9];
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      T s = mu * (G[3 * ii + jj] + G[3 * jj + ii]);
      if (ii == jj) s -= T(2.0 / 3.0) * mu * theta;
      sig[3 * ii + jj] = s;
    }
  const T p = pr[0] * a.cf.gas_r * pr[4];
  const T E = a.q[4 * N + i];
  T F[3][kNQ];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    F[j][0] = a.q[(1 + j) * N + i];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
      F[j][1 + ii] = a.q[(1 + ii) * N + i] * pr[1 + j] + (ii == j ? p : T(0)) - sig[3 * ii + j];
    F[j][4] = (E + p) * pr[1 + j] - (pr[1] * sig[j] + pr[2] * sig[3 + j] + pr[3] * sig[6 + j]) -
              kt * G[9 + j];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int c = 0; c < kNQ; ++c) a.flux[(j * kNQ + c) * N + i] = F[j][c];
  if (a.publish) {
    const int pt[3] = {x, y, z};
    const int slot = (int)(a.step % g.R);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int tl = pt[d] / g.e[d];
      const int lay = layer_of(pt[d] - tl * g.e[d], g.e[d]);
      if (lay < 0) continue;
      const int64_t sidx = slab_index(g, d, x, y, z, 4 * tl + lay);
      T* base = a.ring + slot * g.ring_slot + g.ring_dir_off[d] + (int64_t)kNPub * g.slab[d] + sidx;
#pragma unroll
      for (int c = 0; c < kNQ; ++c) base[(int64_t)c * g.slab[d]] = F[d][c];
    }
  }
}

template <typename T>
__device__ __forceinline__ void force_at(const ForceArgs<T>& f, const Geom& g, int x, int y, int z,
                                         T out[3]) {
  out[0] = out[1] = out[2] = T(0);
  for (int pidx = 0; pidx < f.npair; ++pidx) {
    const T* ey = f.phase_y + ((int64_t)(f.pair_ky[pidx] + 2) * g.n[1] + y) * 2;
    const T* ez = f.phase_z + ((int64_t)f.pair_kz[pidx] * g.n[2] + z) * 2;
    const T er = ey[0] * ez[0] - ey[1] * ez[1];
    const T ei = ey[0] * ez[1] + ey[1] * ez[0];
    const T* A = f.table + ((int64_t)pidx * g.n[0] + x) * 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] += T(2) * (A[2 * c] * er - A[2 * c + 1] * ei);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// AT divergence of the fluxes, source, and the LS-RK3 register / state update.
template <typename T>
__global__ __launch_bounds__(256) void k_update(StageArgs<T> a) {
  const Geom& g = a.g;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool valid = x < g.n[0] && y < g.n[1];
  double part[kNQ] = {0, 0, 0, 0, 0};
  if (valid) {
    const int pt[3] = {x, y, z};
    int tl[3], lc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      tl[d] = pt[d] / g.e[d];
      lc[d] = pt[d] - tl[d] * g.e[d];
    }
    const int tile = (tl[2] * g.p[1] + tl[1]) * g.p[0] + tl[0];
    const int8_t* kf = a.delays + tile * 6;
    const int64_t N = g.npts;
    const int64_t i = ((int64_t)z * g.n[1] + y) * g.n[0] + x;
    T div[kNQ] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T v[4][kNQ];
      const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) {
        const int m = ms[mi];
        const int lr = lc[d] + m;
        int r[3] = {x, y, z};
        r[d] = wrap1(pt[d] + m, g.n[d]);
        int k = 0;
        if (lr < 0) k = kf[2 * d];
        else if (lr >= g.e[d]) k = kf[2 * d + 1];
        if (k == 0) {
          const int64_t ir = ((int64_t)r[2] * g.n[1] + r[1]) * g.n[0] + r[0];
#pragma unroll
          for (int c = 0; c < kNQ; ++c) v[mi][c] = a.flux[(d * kNQ + c) * N + ir];
        } else {
          const int tr = r[d] / g.e[d];
          const int jp = 4 * tr + layer_of(r[d] - tr * g.e[d], g.e[d]);
          const int64_t sidx = slab_index(g, d, r[0], r[1], r[2], jp);
#pragma unroll
          for (int c = 0; c < kNQ; ++c) v[mi][c] = ring_extrap<T>(a, d, kNPub + c, sidx, k);
        }
      }
#pragma unroll
      for (int c = 0; c < kNQ; ++c)
        div[c] += (v[0][c] - T(8) * v[1][c] + T(8) * v[2][c] - v[3][c]) * a.cf.inv12h[d];
    }
    T src[kNQ] = {T(0), T(0), T(0), T(0), T(0)};
    if (a.force.table) {
      T f[3];
      force_at<T>(a.force, g, x, y, z, f);
      const T rho = a.q[i];
      src[1] = rho * f[0];
      src[2] = rho * f[1];
      src[3] = rho * f[2];
      src[4] = a.q[N + i] * f[0] + a.q[2 * N + i] * f[1] + a.q[3 * N + i] * f[2];
    }
    if (a.rhs_out) {
#pragma unroll
      for (int c = 0; c < kNQ; ++c) a.rhs_out[c * N + i] = src[c] - div[c];
    } else {
#pragma unroll
      for (int c = 0; c < kNQ; ++c) {
        const T r = src[c] - div[c];
        const T d = (a.rk_a == T(0)) ? a.dt * r : a.rk_a * a.dq[c * N + i] + a.dt * r;
        a.dq[c * N + i] = d;
        a.q[c * N + i] = a.q[c * N + i] + a.rk_b * d;
        part[c] = (double)d;
      }
    }
  }
  if (a.rhs_out) return;  // uniform across the grid
  __shared__ double red[4][kNQ];
  const int lane = threadIdx.x;  // blockDim.x == 64: one wavefront per threadIdx.y
  const int wave = threadIdx.y;
#pragma unroll
  for (int c = 0; c < kNQ; ++c) {
    const double s = wave_sum(part[c]);
    if (lane == 0) red[wave][c] = s;
  }
  __syncthreads();
  if (wave == 0 && lane < kNQ) {
    const double s = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    a.tot_part[blk * kNQ + lane] += (double)a.rk_b * s * a.vol;
  }
}

// Statistics partials per block with synchronous periodic derivatives (no PE faces).
template <typename T>
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
      T v[4][4];
      const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) {
        int r[3] = {x, y, z};
        r[d] = wrap1(pt[d] + ms[mi], g.n[d]);
        const int64_t ir = ((int64_t)r[2] * g.n[1] + r[1]) * g.n[0] + r[0];
        T pr[5];
        primitives<T>(q, N, ir, cf.inv_cv, pr);
        v[mi][0] = pr[1];
        v[mi][1] = pr[2];
        v[mi][2] = pr[3];
        v[mi][3] = pr[4];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
        G[c < 3 ? 3 * c + d : 9 + d] = (v[0][c] - T(8) * v[1][c] + T(8) * v[2][c] - v[3][c]) * cf.inv12h[d];
    }
    T pr[5];
    primitives<T>(q, N, i, cf.inv_cv, pr);
    const double mu = (double)cf.mu_ref * pow((double)pr[4] * (double)cf.inv_tref, (double)cf.mu_exp);
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
__global__ __launch_bounds__(256) void k_stats_final(const double* __restrict__ part, int64_t nblk,
                                                     const double* __restrict__ tot_part,
                                                     int64_t ntot, double* __restrict__ out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  for (int c = 0; c < kNStat + kNQ; ++c) {
    const bool is_max = (c == 10 || c == 11);
    double v = 0.0;
    if (c < kNStat) {
      for (int64_t b = t; b < nblk; b += 256) {
        const double pv = part[b * kNStat + c];
        v = is_max ? fmax(v, pv) : v + pv;
      }
    } else if (tot_part) {
      for (int64_t b = t; b < ntot; b += 256) v += tot_part[b * kNQ + (c - kNStat)];
    }
    red[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] = is_max ? fmax(red[t], red[t + s]) : red[t] + red[t + s];
      __syncthreads();
    }
    if (t == 0) out[c] = red[0];
    __syncthreads();
  }
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
  static const char* names[kKCount] = {"k_grad", "k_flux", "k_update", "k_force_table", "k_stats",
                                       "k_grad(history)"};
  return (id >= 0 && id < kKCount) ? names[id] : "";
}

#define HOOKED(id, launch)              \
  do {                                  \
    if (hook) hook->before(id, stream); \
    launch;                             \
    if (hook) hook->after(id, stream);  \
  } while (0)

template <typename T>
hipError_t launch_stage(const StageArgs<T>& a, hipStream_t stream, LaunchHook* hook) {
  const dim3 blk(kBX, kBY, 1);
  const dim3 gr = grid_of(a.g);
  HOOKED(kKGrad, hipLaunchKernelGGL(k_grad<T>, gr, blk, 0, stream, a, 0));
  HOOKED(kKFlux, hipLaunchKernelGGL(k_flux<T>, gr, blk, 0, stream, a));
  HOOKED(kKUpdate, hipLaunchKernelGGL(k_update<T>, gr, blk, 0, stream, a));
  return hipGetLastError();
}

// Publish one history level: synchronous gradients and fluxes of the state in a.q into slot
// a.step mod R.
template <typename T>
hipError_t launch_publish_history(const StageArgs<T>& a, hipStream_t stream) {
  const dim3 blk(kBX, kBY, 1);
  const dim3 gr = grid_of(a.g);
  hipLaunchKernelGGL(k_grad<T>, gr, blk, 0, stream, a, 1);
  hipLaunchKernelGGL(k_flux<T>, gr, blk, 0, stream, a);
  return hipGetLastError();
}

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
  HOOKED(kKStats, hipLaunchKernelGGL(k_stats<T>, gr, blk, 0, stream, g, cf, q, part));
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, stream, part, stats_blocks(g), tot_part,
                     ntot_blocks, out);
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
  template hipError_t launch_stage<T>(const StageArgs<T>&, hipStream_t, LaunchHook*);                \
  template hipError_t launch_publish_history<T>(const StageArgs<T>&, hipStream_t);                   \
  template hipError_t launch_convert<T>(const double*, T*, int64_t, hipStream_t);                    \
  template hipError_t launch_to_double<T>(const T*, double*, int64_t, hipStream_t);                  \
  template hipError_t launch_stats<T>(const Geom&, const Coef<T>&, const T*, double*, double*,       \
                                      const double*, int64_t, double, hipStream_t, LaunchHook*);     \
  template hipError_t launch_force_table<T>(const Geom&, const double*, const int*, const int*, int, \
                                            T*, const T*, hipStream_t, LaunchHook*);
ATNS_INSTANTIATE(double)
ATNS_INSTANTIATE(float)

}  // namespace atns
