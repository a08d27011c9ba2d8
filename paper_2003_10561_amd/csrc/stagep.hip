// The paper's own discretisation on gfx950 (form 1): Sec. 2, Eqs. cont, mome, ie in the variables
// (rho, rho u_i, rho e), e = c_v T, which each PE stores and publishes (Sec. 3.1), with
//   d sigma_ij/dx_j   = mu (d2 u_i/dx_j dx_j + 1/3 d/dx_i du_k/dx_k)
//                       + mu'(T) dT/dx_j (du_i/dx_j + du_j/dx_i - 2/3 delta_ij du_k/dx_k),
//   d(k dT/dx_j)/dx_j = k d2T/dx_j dx_j + k'(T) (dT/dx_j)^2,  k = mu c_p / Pr,
// first derivatives by the (1,4) AT scheme and pure second derivatives by the (2,4) AT scheme
// (Appendix B); a value across a face with delay k >= 1 is sum_l w_l(k + c_s) f(q^{n-k-l}), f the
// differentiated function of the published conserved variables.  Mixed derivatives take three
// steps (Sec. 2.1): the AT first derivatives along both directions, then a derivative of each
// along the other direction with the PE's own points only (central (1,4) where it fits, the
// standard fourth-order one-sided and biased stencils on the two points next to a face), then the
// average.  Viscosity: the power law or Sutherland's law (Sec. 2).
//
// Launches: per stage kp_grad (the 12 AT gradients of u, v, w, T into a workspace buffer; at stage 1
// of a step the points of every PE's two layers next to each face also publish their conserved
// variables into ring slot n mod R) and kp_rhs (every term above at one point per thread, the
// gradients of the PE-local mixed-derivative lines read back from that buffer, then the Runge-Kutta
// or Adams-Bashforth update and FP64 block totals); kp_publish publishes a history level alone.
#include "atns_internal.h"

namespace atns {
namespace {

constexpr int kBXp = 64, kBYp = 4;
constexpr double kTwoPiP = 6.283185307179586476925286766559;

template <typename T>
struct PA {
  const T* q;
  T* q_out;
  T* dq;
  T* grad;           // [12][N]: du_i/dx_j at 3 i + j, then dT/dx_j at 9 + j
  T* ring;
  T* rhs_out;
  const int8_t* delays;
  double* tot_part;
  uint32_t N;
  int n[3], e[3], p[3];
  uint32_t slab[3], rdir[3], rslot;  // ring element: slot rslot + rdir[d] + c slab[d] + j
  int R, step_mod_r, slot, store_dq, mode;
  T cs, rk_a, rk_b, dt, c_prev;
  T gas_r, inv_cv, cp_over_pr, mu_ref, inv_tref, mu_exp, suth_s;
  int visc;
  T i12h[3], i12h2[3];
  double vol;
};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Index of point r inside the slab set of direction d (r lies in one of its PE's 2 + 2 face
// layers along d, local index l): planes (PE along d) * 4 + layer, then the two other directions,
// the faster one first (y for d = x, x otherwise).
template <typename T>
__device__ __forceinline__ uint32_t slab_of(const PA<T>& a, int d, const int r[3], int l) {
  const int e = a.e[d];
  const int j = l < 2 ? l : l - e + 4;
  const int plane = (r[d] / e) * 4 + j;
  const int ia = d == 0 ? 1 : 0, ib = d == 2 ? 1 : 2;
  return ((uint32_t)plane * (uint32_t)a.n[ib] + (uint32_t)r[ib]) * (uint32_t)a.n[ia] + (uint32_t)r[ia];
}

// u, v, w, T, p, then for direction d: m_d, m_i m_d / rho (i = 0..2), rho e m_d / rho.
template <typename T>
__device__ __forceinline__ void derive(const PA<T>& a, const T q[5], int d, T v[10]) {
  const T rinv = T(1) / q[0];
  v[0] = q[1] * rinv;
  v[1] = q[2] * rinv;
  v[2] = q[3] * rinv;
  v[3] = q[4] * rinv * a.inv_cv;
  v[4] = q[0] * a.gas_r * v[3];
  const T md = d == 0 ? q[1] : (d == 1 ? q[2] : q[3]);
  const T ud = md * rinv;
  v[5] = md;
  v[6] = q[1] * ud;
  v[7] = q[2] * ud;
  v[8] = q[3] * ud;
  v[9] = q[4] * ud;
}

// The derived values at r = p + m e_d as the PE of p (tile `tile`) sees them.
template <typename T>
__device__ __forceinline__ void seen(const PA<T>& a, const int p[3], int tile, int d, int m, T v[10]) {
  int r[3] = {p[0], p[1], p[2]};
  r[d] = wrapi(p[d] + m, a.n[d]);
  const int lr = p[d] % a.e[d] + m;
  int k = 0;
  if (lr < 0 || lr >= a.e[d]) k = a.delays[tile * 6 + 2 * d + (lr < 0 ? 0 : 1)];
  if (k == 0) {
    const uint32_t ir = ((uint32_t)r[2] * a.n[1] + r[1]) * a.n[0] + r[0];
    T q[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) q[c] = a.q[(uint32_t)c * a.N + ir];
    derive(a, q, d, v);
    return;
  }
  const T kap = T(k) + a.cs;
  const T w[3] = {(kap + T(1)) * (kap + T(2)) * T(0.5), -kap * (kap + T(2)), kap * (kap + T(1)) * T(0.5)};
  const uint32_t j = slab_of(a, d, r, r[d] % a.e[d]);
#pragma unroll
  for (int c = 0; c < 10; ++c) v[c] = T(0);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    int slot = a.step_mod_r - k - l;
    while (slot < 0) slot += a.R;
    const T* base = a.ring + (uint32_t)slot * a.rslot + a.rdir[d] + j;
    T q[5], vl[10];
#pragma unroll
    for (int c = 0; c < 5; ++c) q[c] = base[(uint32_t)c * a.slab[d]];
    derive(a, q, d, vl);
#pragma unroll
    for (int c = 0; c < 10; ++c) v[c] += w[l] * vl[c];
  }
}

template <typename T>
__device__ __forceinline__ T viscosity(const PA<T>& a, T temp, T* dmu) {
  if (a.visc == 1) {
    const T t = temp * a.inv_tref;
    const T mu = a.mu_ref * t * sqrt(t) * (T(1) / a.inv_tref + a.suth_s) / (temp + a.suth_s);
    *dmu = mu * (T(1.5) / temp - T(1) / (temp + a.suth_s));
    return mu;
  }
  const T mu = a.mu_ref * pow(temp * a.inv_tref, a.mu_exp);
  *dmu = a.mu_exp * mu / temp;
  return mu;
}

// Derivative along direction d of gradient component gc at point i (local index l inside its
// PE of edge e) from the PE's own points: central (1,4) for 2 <= l <= e - 3, else the standard
// fourth-order one-sided (l = 0, e - 1) and biased (l = 1, e - 2) stencils.
template <typename T>
__device__ __forceinline__ T pe_d1(const PA<T>& a, int gc, int d, uint32_t i, int l) {
  const int e = a.e[d];
  const uint32_t st = d == 0 ? 1u : (d == 1 ? (uint32_t)a.n[0] : (uint32_t)a.n[0] * a.n[1]);
  const T* g = a.grad + (uint32_t)gc * a.N + i;
  auto at = [&](int o) { return g[(int64_t)o * (int64_t)st]; };
  T s;
  if (l >= 2 && l <= e - 3) {
    s = (at(-2) - T(8) * at(-1)) + (T(8) * at(1) - at(2));
  } else if (l == 0) {
    s = ((T(-25) * at(0) + T(48) * at(1)) - T(36) * at(2)) + (T(16) * at(3) - T(3) * at(4));
  } else if (l == 1) {
    s = ((T(-3) * at(-1) - T(10) * at(0)) + T(18) * at(1)) + (T(-6) * at(2) + at(3));
  } else if (l == e - 2) {
    s = ((T(3) * at(1) + T(10) * at(0)) - T(18) * at(-1)) + (T(6) * at(-2) - at(-3));
  } else {
    s = ((T(25) * at(0) - T(48) * at(-1)) + T(36) * at(-2)) + (T(-16) * at(-3) + T(3) * at(-4));
  }
  return s * a.i12h[d];
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Stage 1 publication: every point of the slab sets of the three directions.
template <typename T>
__global__ __launch_bounds__(256) void kp_publish(PA<T> a) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  const uint32_t total = a.slab[0] + a.slab[1] + a.slab[2];
  if (t >= total) return;
  const int d = t < a.slab[0] ? 0 : (t < a.slab[0] + a.slab[1] ? 1 : 2);
  const uint32_t j = t - (d == 0 ? 0u : (d == 1 ? a.slab[0] : a.slab[0] + a.slab[1]));
  const int ia = d == 0 ? 1 : 0, ib = d == 2 ? 1 : 2;
  const uint32_t na = a.n[ia], nb = a.n[ib];
  const int ra = (int)(j % na), rb = (int)((j / na) % nb), plane = (int)(j / (na * nb));
  const int layer = plane % 4, pe = plane / 4;
  const int e = a.e[d];
  int r[3];
  r[d] = pe * e + (layer < 2 ? layer : e - 4 + layer);
  r[ia] = ra;
  r[ib] = rb;
  const uint32_t i = ((uint32_t)r[2] * a.n[1] + r[1]) * a.n[0] + r[0];
  T* dst = a.ring + (uint32_t)a.slot * a.rslot + a.rdir[d] + j;
#pragma unroll
  for (int c = 0; c < 5; ++c) dst[(uint32_t)c * a.slab[d]] = a.q[(uint32_t)c * a.N + i];
}

// Workgroups: 64 x 4 columns marching through kZC planes (the z neighbours of a plane are read
// again from the caches by the same threads), numbered XCD-major: the hardware deals consecutive
// workgroups to the 8 XCDs in turn, so logical workgroup L = xcd_major(w) gives each XCD (one L2)
// a contiguous range of bricks.
constexpr int kZC = 16;
constexpr uint32_t kNumXcd = 8;
__device__ __forceinline__ uint32_t xcd_major(uint32_t w, uint32_t nb) {
  const uint32_t c = w % kNumXcd, i = w / kNumXcd, q = nb / kNumXcd, r = nb % kNumXcd;
  return c * q + min(c, r) + i;
}

struct Brick {
  int x, y, z0, z1;
  uint32_t L;
};
template <typename T>
__device__ __forceinline__ Brick brick(const PA<T>& a) {
  const uint32_t gx = (uint32_t)(a.n[0] + kBXp - 1) / kBXp, gy = (uint32_t)(a.n[1] + kBYp - 1) / kBYp;
  const uint32_t L = xcd_major(blockIdx.x, gridDim.x);
  const uint32_t bz = L / (gx * gy), r = L - bz * gx * gy, by = r / gx, bx = r - by * gx;
  Brick b;
  b.x = (int)bx * kBXp + threadIdx.x;
  b.y = (int)by * kBYp + threadIdx.y;
  b.z0 = (int)bz * kZC;
  b.z1 = min(b.z0 + kZC, a.n[2]);
  b.L = L;
  return b;
}

// The 12 AT gradients of u, v, w, T at every point; with `publish`, the points on the face layers
// also write their conserved variables into ring slot a.slot (stage 1 of a step).
template <typename T>
__global__ __launch_bounds__(256) void kp_grad(PA<T> a, int publish) {
  const Brick b = brick(a);
  if (b.x >= a.n[0] || b.y >= a.n[1]) return;
  for (int z = b.z0; z < b.z1; ++z) {
    const int p[3] = {b.x, b.y, z};
    const int tile = (z / a.e[2] * a.p[1] + b.y / a.e[1]) * a.p[0] + b.x / a.e[0];
    const uint32_t i = ((uint32_t)z * a.n[1] + b.y) * a.n[0] + b.x;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T g[4] = {T(0), T(0), T(0), T(0)};
      const T c1[4] = {T(1), T(-8), T(8), T(-1)};
      const int off[4] = {-2, -1, 1, 2};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        T v[10];
        seen(a, p, tile, d, off[s], v);
#pragma unroll
        for (int c = 0; c < 4; ++c) g[c] += c1[s] * v[c];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) a.grad[(uint32_t)(c < 3 ? 3 * c + d : 9 + d) * a.N + i] = g[c] * a.i12h[d];
    }
    if (publish) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int l = p[d] % a.e[d];
        if (l < 2 || l >= a.e[d] - 2) {
          T* dst = a.ring + (uint32_t)a.slot * a.rslot + a.rdir[d] + slab_of(a, d, p, l);
#pragma unroll
          for (int c = 0; c < 5; ++c) dst[(uint32_t)c * a.slab[d]] = a.q[(uint32_t)c * a.N + i];
        }
      }
    }
  }
}

// Every term of the right-hand side at one point per thread and plane, then the update.
template <typename T>
__global__ __launch_bounds__(256) void kp_rhs(PA<T> a) {
  const Brick b = brick(a);
  const bool valid = b.x < a.n[0] && b.y < a.n[1];
  double tsum[5] = {0, 0, 0, 0, 0};
  for (int z = b.z0; valid && z < b.z1; ++z) {
    const int p[3] = {b.x, b.y, z};
    const int tile = (z / a.e[2] * a.p[1] + b.y / a.e[1]) * a.p[0] + b.x / a.e[0];
    const uint32_t i = ((uint32_t)z * a.n[1] + b.y) * a.n[0] + b.x;
    T qc[5], vc[10];
#pragma unroll
    for (int c = 0; c < 5; ++c) qc[c] = a.q[(uint32_t)c * a.N + i];
    derive(a, qc, 0, vc);
    T cont = T(0), conve = T(0), lapT = T(0), conv[3] = {T(0), T(0), T(0)}, lap[3] = {T(0), T(0), T(0)},
      pg[3], pure[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // the first-derivative rows (1, -8, 8, -1) / 12h and the second-derivative rows
      // (-1, 16, -30, 16, -1) / 12h^2, accumulated one offset at a time
      const T c1[4] = {T(1), T(-8), T(8), T(-1)}, c2[4] = {T(-1), T(16), T(16), T(-1)};
      const int off[4] = {-2, -1, 1, 2};
      T s1[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};  // m_d, uu_0d, uu_1d, uu_2d, eu_d, p
      T s2[4] = {T(0), T(0), T(0), T(0)};              // u, v, w, T
#pragma unroll 1  // one neighbour at a time: 116 VGPRs in FP32 (4 waves per SIMD) against 229 unrolled
      for (int s = 0; s < 4; ++s) {
        T v[10];
        seen(a, p, tile, d, off[s], v);
#pragma unroll
        for (int c = 0; c < 5; ++c) s1[c] += c1[s] * v[5 + c];
        s1[5] += c1[s] * v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) s2[c] += c2[s] * v[c];
      }
      cont += s1[0] * a.i12h[d];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        conv[c] += s1[1 + c] * a.i12h[d];
        const T l2 = (s2[c] - T(30) * vc[c]) * a.i12h2[d];
        lap[c] += l2;
        if (c == d) pure[d] = l2;
      }
      conve += s1[4] * a.i12h[d];
      pg[d] = s1[5] * a.i12h[d];
      lapT += (s2[3] - T(30) * vc[3]) * a.i12h2[d];
    }
    T G[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) G[c] = a.grad[(uint32_t)c * a.N + i];
    const T temp = vc[3], pres = vc[4];
    T dmu;
    const T mu = viscosity(a, temp, &dmu);
    const T kt = mu * a.cp_over_pr, dkt = dmu * a.cp_over_pr;
    const T th = G[0] + G[4] + G[8];
    const int loc[3] = {b.x % a.e[0], b.y % a.e[1], z % a.e[2]};
    T rhs[5];
    rhs[0] = -cont;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // d/dx_c (du_k/dx_k): the pure second derivative, and the mixed ones in three steps
      T gd = pure[c];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != c) gd += T(0.5) * (pe_d1(a, 3 * k + k, c, i, loc[c]) + pe_d1(a, 3 * k + c, k, i, loc[k]));
      T visc = mu * (lap[c] + gd / T(3));
#pragma unroll
      for (int j = 0; j < 3; ++j)
        visc += dmu * G[9 + j] * (G[3 * c + j] + G[3 * j + c] - (c == j ? T(2) / T(3) * th : T(0)));
      rhs[1 + c] = (-conv[c] - pg[c]) + visc;
    }
    T diss = T(0), grT = T(0);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      grT += G[9 + ii] * G[9 + ii];
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        T sg = mu * (G[3 * ii + jj] + G[3 * jj + ii]);
        if (ii == jj) sg -= T(2) / T(3) * mu * th;
        diss += sg * G[3 * ii + jj];
      }
    }
    rhs[4] = ((-conve - pres * th) + (kt * lapT + dkt * grT)) + diss;
    if (a.mode == kModeRhsH) {
#pragma unroll
      for (int c = 0; c < 5; ++c) a.rhs_out[(uint32_t)c * a.N + i] = rhs[c];
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const T prev = (a.rk_a != T(0) || a.c_prev != T(0)) ? a.dq[(uint32_t)c * a.N + i] : T(0);
        const T dqv = a.rk_a * prev + a.dt * rhs[c];
        const T inc = a.rk_b * dqv + a.c_prev * prev;
        if (a.store_dq) a.dq[(uint32_t)c * a.N + i] = dqv;
        a.q_out[(uint32_t)c * a.N + i] = qc[c] + inc;
        tsum[c] += a.c_prev != T(0) ? (double)inc : (double)dqv;
      }
    }
  }
  if (a.mode != kModeStepH) return;  // uniform across the grid
  __shared__ double red[kBYp][5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double v = wsum(tsum[c]);
    if (threadIdx.x == 0) red[threadIdx.y][c] = v;
  }
  __syncthreads();
  const int tid = threadIdx.y * kBXp + threadIdx.x;
  if (tid < 5) {
    const double scale = a.c_prev != T(0) ? 1.0 : (double)a.rk_b;
    a.tot_part[b.L * kNQ + tid] += scale * ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) * a.vol;
  }
}

template <typename T>
PA<T> pack(const StagePArgs<T>& s) {
  PA<T> a{};
  const Geom& g = s.g;
  a.q = s.q;
  a.q_out = s.q_out;
  a.dq = s.dq;
  a.grad = s.grad;
  a.ring = s.ring;
  a.rhs_out = s.rhs_out;
  a.delays = s.delays;
  a.tot_part = s.tot_part;
  a.N = (uint32_t)g.npts;
  uint32_t off = 0;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = g.n[d];
    a.e[d] = g.e[d];
    a.p[d] = g.p[d];
    a.slab[d] = (uint32_t)g.slab[d];
    a.rdir[d] = off;
    off += kNQ * a.slab[d];
    const double h = kTwoPiP / g.n[d];
    a.i12h[d] = (T)(1.0 / (12.0 * h));
    a.i12h2[d] = (T)(1.0 / (12.0 * h * h));
  }
  a.rslot = off;
  a.R = g.R;
  a.step_mod_r = s.step_mod_r;
  a.slot = s.slot;
  a.store_dq = s.store_dq;
  a.mode = s.mode;
  a.cs = s.cs;
  a.rk_a = s.rk_a;
  a.rk_b = s.rk_b;
  a.dt = s.dt;
  a.c_prev = s.c_prev;
  a.gas_r = s.cf.gas_r;
  a.inv_cv = s.cf.inv_cv;
  a.cp_over_pr = s.cf.cp_over_pr;
  a.mu_ref = s.cf.mu_ref;
  a.inv_tref = s.cf.inv_tref;
  a.mu_exp = s.cf.mu_exp;
  a.suth_s = s.cf.suth_s;
  a.visc = s.cf.visc;
  a.vol = s.vol;
  return a;
}

}  // namespace

int64_t paper_blocks(const Geom& g) {
  return (int64_t)((g.n[0] + kBXp - 1) / kBXp) * ((g.n[1] + kBYp - 1) / kBYp) * ((g.n[2] + kZC - 1) / kZC);
}

template <typename T>
hipError_t launch_stagep(const StagePArgs<T>& s, int which, hipStream_t stream) {
  const PA<T> a = pack(s);
  if (which == kPPublish) {
    const uint64_t total = (uint64_t)a.slab[0] + a.slab[1] + a.slab[2];
    hipLaunchKernelGGL((kp_publish<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)paper_blocks(s.g));
  if (which == kPGrad || which == kPGradPublish)
    hipLaunchKernelGGL((kp_grad<T>), grid, dim3(kBXp, kBYp), 0, stream, a, which == kPGradPublish ? 1 : 0);
  else hipLaunchKernelGGL((kp_rhs<T>), grid, dim3(kBXp, kBYp), 0, stream, a);
  return hipGetLastError();
}

template hipError_t launch_stagep<float>(const StagePArgs<float>&, int, hipStream_t);
template hipError_t launch_stagep<double>(const StagePArgs<double>&, int, hipStream_t);

}  // namespace atns
