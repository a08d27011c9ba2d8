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

// A value select (a conditional of two array elements would select their addresses, which puts
// the array in scratch when the condition is not known at compile time).
template <typename T>
__device__ __forceinline__ T sel(bool c, T x, T y) {
  return c ? x : y;
}

// 1 / x: the hardware reciprocal in FP32 (1 ulp, as the fourth-order stage kernel uses), a
// correctly rounded division in FP64.
template <typename T>
__device__ __forceinline__ T prcp(T x) {
  return T(1) / x;
}
template <>
__device__ __forceinline__ float prcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// u, v, w, T, p, then for direction d: m_d, m_i m_d / rho (i = 0..2), rho e m_d / rho.
template <typename T>
__device__ __forceinline__ void derive(const PA<T>& a, const T q[5], int d, T v[10]) {
  const T rinv = prcp<T>(q[0]);
  v[0] = q[1] * rinv;
  v[1] = q[2] * rinv;
  v[2] = q[3] * rinv;
  v[3] = q[4] * rinv * a.inv_cv;
  v[4] = q[0] * a.gas_r * v[3];
  const T md = sel<T>(d == 0, q[1], sel<T>(d == 1, q[2], q[3]));
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
    const T rts = prcp<T>(temp + a.suth_s);
    const T mu = a.mu_ref * t * sqrt(t) * (T(1) / a.inv_tref + a.suth_s) * rts;
    *dmu = mu * (T(1.5) * prcp<T>(temp) - rts);
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

// The right-hand side at one point from its derivative sums (Sec. 2, Eqs. cont, mome, ie): vc the
// point's own u, v, w, T, p; G its 12 AT gradients; cont, conv, conve, pg the first derivatives of
// m_j, m_i u_j, rho e u_j (summed over j) and of p; lap, lapT the (2,4) Laplacians of u_i and T;
// pure the pure second derivatives d2 u_c / dx_c^2; mixed the averaged mixed terms of
// d/dx_c du_k/dx_k.
template <typename T>
__device__ __forceinline__ void assemble(const PA<T>& a, const T vc[10], const T G[12], T cont, const T conv[3],
                                         T conve, const T pg[3], const T lap[3], T lapT, const T pure[3],
                                         const T mixed[3], T rhs[5]) {
  const T temp = vc[3], pres = vc[4];
  T dmu;
  const T mu = viscosity(a, temp, &dmu);
  const T kt = mu * a.cp_over_pr, dkt = dmu * a.cp_over_pr;
  const T th = G[0] + G[4] + G[8];
  rhs[0] = -cont;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T gd = pure[c] + mixed[c];  // d/dx_c (du_k/dx_k)
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
}

// The Runge-Kutta or Adams-Bashforth update of point i (or the RHS alone), with this thread's
// running FP64 sums of the increments.
template <typename T>
__device__ __forceinline__ void update_point(const PA<T>& a, uint32_t i, const T qc[5], const T rhs[5],
                                             double tsum[5]) {
  if (a.mode == kModeRhsH) {
#pragma unroll
    for (int c = 0; c < 5; ++c) a.rhs_out[(uint32_t)c * a.N + i] = rhs[c];
    return;
  }
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

// FP64 totals of a workgroup of 256 threads (4 waves) into its slot L of the partial sums.
template <typename T>
__device__ __forceinline__ void block_totals(const PA<T>& a, const double tsum[5], uint32_t L, int tid) {
  __shared__ double red[4][5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double v = wsum(tsum[c]);
    if ((tid & 63) == 0) red[tid >> 6][c] = v;
  }
  __syncthreads();
  if (tid < 5) {
    const double scale = a.c_prev != T(0) ? 1.0 : (double)a.rk_b;
    a.tot_part[L * kNQ + tid] += scale * ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) * a.vol;
  }
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
    const int loc[3] = {b.x % a.e[0], b.y % a.e[1], z % a.e[2]};
    T mixed[3];  // sum over k != c of the averaged mixed derivatives d/dx_c du_k/dx_k
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mixed[c] = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != c) mixed[c] += T(0.5) * (pe_d1(a, 3 * k + k, c, i, loc[c]) + pe_d1(a, 3 * k + c, k, i, loc[k]));
    }
    T rhs[5];
    assemble(a, vc, G, cont, conv, conve, pg, lap, lapT, pure, mixed, rhs);
    update_point(a, i, qc, rhs, tsum);
  }
  if (a.mode != kModeStepH) return;  // uniform across the grid
  block_totals(a, tsum, b.L, threadIdx.y * kBXp + threadIdx.x);
}

// Tiled kernels, for PEs whose x and y edges are multiples of kTB: a workgroup owns a kTB x kTB
// column tile inside one PE and marches it through kTZ planes.  Per plane, the tile's points and
// their 2-wide x and y halos are written once to LDS as the differentiated functions that the
// tile's PE sees (a halo point behind a delayed face of that PE is the extrapolation of its ring
// levels, as `seen` forms it), so every x and y stencil reads LDS; each column keeps a five-plane
// register window of its own planes for the z stencils.  kp_rhs_tile also stages the PE-local
// lines of the gradients that the mixed derivatives differentiate: along x and y in 4-wide halos
// (the one-sided stencils reach 4 points), along z in a nine-plane LDS ring.
//
// The march is software-pipelined: what plane z + 1 needs from memory (the column's plane z + 3
// or z + 4, the halo points, the gradients and the register dQ) is fetched while plane z is
// computed, after the last use of the registers it refills, and consumed after the plane's second
// barrier.  Loads complete in order, so the compute phase issues no loads of its own (only the
// planes next to a delayed z face fetch their ring levels there).
constexpr int kTB = 16, kTZ = 64, kTH = 2, kTG = 4, kTRing = 2 * kTG + 1;
constexpr int kMaxZPe = kTZ / 5 + 2;  // z-PEs a chunk can touch (PE edges are at least 5)

struct TBrick {
  int x0, y0, z0, z1;
  uint32_t L;
};
template <typename T>
__device__ __forceinline__ TBrick tbrick(const PA<T>& a) {
  const uint32_t gx = (uint32_t)a.n[0] / kTB, gy = (uint32_t)a.n[1] / kTB;
  const uint32_t L = xcd_major(blockIdx.x, gridDim.x);
  const uint32_t bz = L / (gx * gy), r = L - bz * gx * gy, by = r / gx, bx = r - by * gx;
  TBrick b;
  b.x0 = (int)bx * kTB;
  b.y0 = (int)by * kTB;
  b.z0 = (int)bz * kTZ;
  b.z1 = min(b.z0 + kTZ, a.n[2]);
  b.L = L;
  return b;
}

template <typename T>
__device__ __forceinline__ int pe_of(const PA<T>& a, int x, int y, int z) {
  return (z / a.e[2] * a.p[1] + y / a.e[1]) * a.p[0] + x / a.e[0];
}

// The six face delays of the tile's PE for each z-PE of the chunk: s_kd[zpe - z0 / e_z][face].
template <typename T>
__device__ __forceinline__ void load_delays(const PA<T>& a, const TBrick& b, int (*s_kd)[6], int tid) {
  const int zp0 = b.z0 / a.e[2], nzp = (b.z1 - 1) / a.e[2] - zp0 + 1;
  if (tid < 6 * nzp) {
    const int zl = tid / 6, f = tid % 6;
    s_kd[zl][f] = a.delays[pe_of(a, b.x0, b.y0, (zp0 + zl) * a.e[2]) * 6 + f];
  }
}

// A halo point of the tile's 2-wide x (d = 0) or y (d = 1) halo, h in [0, 4 kTB): the row (or
// column) h / 4 of the tile and the offset m in {-2, -1, +1, +2} from the tile's edge point of it;
// `pt` the halo point itself (x, y; wrapped), `lds` its index along d in the LDS plane, `face` the
// face of the tile's PE it lies behind (2 d or 2 d + 1) and `out` whether it does (outside the PE).
struct Halo {
  int pt[2], m, lds, face, along;
  bool out;
};
template <typename T>
__device__ __forceinline__ Halo halo_of(const PA<T>& a, int d, int h, int x0, int y0) {
  Halo o;
  o.along = h / 4;
  const int j = h % 4;
  o.m = j < 2 ? j - 2 : j - 1;
  o.lds = j < 2 ? j : kTB + j;
  // (selects in place of indexing by d, which would put the arrays in scratch)
  const int e = d == 0 ? a.e[0] : a.e[1], n = d == 0 ? a.n[0] : a.n[1];
  const int edge = (d == 0 ? x0 : y0) + (j < 2 ? 0 : kTB - 1);
  const int le = edge % e + o.m;
  o.out = le < 0 || le >= e;
  o.face = 2 * d + (o.m < 0 ? 0 : 1);
  const int c = wrapi(edge + o.m, n);
  o.pt[0] = d == 0 ? c : x0 + o.along;
  o.pt[1] = d == 0 ? y0 + o.along : c;
  return o;
}

// The raw values behind one point as a reader's PE sees it: its five conserved variables, or,
// behind a face with delay k >= 1, those of the three ring levels n - k - l (l = 0, 1, 2).
template <typename T>
struct Raw {
  T q[3][5];
};

template <typename T>
__device__ __forceinline__ void fetch_raw(const PA<T>& a, int x, int y, int z, int d, int k, Raw<T>& w) {
  // slab_of for a point of the x (d = 0) or y (d = 1) face layers, with selects in place of
  // indexing by d; level 0 comes from the state (k = 0) or from ring slot n - k, through one load
  // loop (separate loops for the two sources would keep their registers in scratch)
  const int e = d == 0 ? a.e[0] : a.e[1], rd = d == 0 ? x : y, ra = d == 0 ? y : x;
  const uint32_t na = d == 0 ? (uint32_t)a.n[1] : (uint32_t)a.n[0], nb = (uint32_t)a.n[2];
  const int l = rd % e, jl = l < 2 ? l : l - e + 4;
  const uint32_t j = (((uint32_t)((rd / e) * 4 + jl)) * nb + (uint32_t)z) * na + (uint32_t)ra;
  const uint32_t sl = d == 0 ? a.slab[0] : a.slab[1], rdir = d == 0 ? a.rdir[0] : a.rdir[1];
  auto level = [&](int lv) {
    int slot = a.step_mod_r - k - lv;
    while (slot < 0) slot += a.R;
    return a.ring + (uint32_t)slot * a.rslot + rdir + j;
  };
  const T* src = k == 0 ? a.q + (((uint32_t)z * a.n[1] + y) * a.n[0] + x) : level(0);
  const uint32_t cs = k == 0 ? a.N : sl;
#pragma unroll
  for (int c = 0; c < 5; ++c) w.q[0][c] = src[(uint32_t)c * cs];
  if (k > 0) {
#pragma unroll
    for (int lv = 1; lv < 3; ++lv) {
      const T* base = level(lv);
#pragma unroll
      for (int c = 0; c < 5; ++c) w.q[lv][c] = base[(uint32_t)c * sl];
    }
  }
}

// The ten functions of `derive` from fetched raw values (the same sums as `seen`).
template <typename T>
__device__ __forceinline__ void finish_raw(const PA<T>& a, int d, int k, const Raw<T>& w, T v[10]) {
  if (k == 0) {
    derive(a, w.q[0], d, v);
    return;
  }
  const T kap = T(k) + a.cs;
  const T wt[3] = {(kap + T(1)) * (kap + T(2)) * T(0.5), -kap * (kap + T(2)), kap * (kap + T(1)) * T(0.5)};
#pragma unroll
  for (int c = 0; c < 10; ++c) v[c] = T(0);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    T vl[10];
    derive(a, w.q[l], d, vl);
#pragma unroll
    for (int c = 0; c < 10; ++c) v[c] += wt[l] * vl[c];
  }
}

template <typename T>
__device__ __forceinline__ void load_q(const PA<T>& a, int x, int y, int z, T q[5]) {
  const uint32_t i = ((uint32_t)z * a.n[1] + y) * a.n[0] + x;
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = a.q[(uint32_t)c * a.N + i];
}

template <typename T>
__device__ __forceinline__ void publish_point(const PA<T>& a, const int p[3], const T q[5]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int l = p[d] % a.e[d];
    if (l < 2 || l >= a.e[d] - 2) {
      T* dst = a.ring + (uint32_t)a.slot * a.rslot + a.rdir[d] + slab_of(a, d, p, l);
#pragma unroll
      for (int c = 0; c < 5; ++c) dst[(uint32_t)c * a.slab[d]] = q[c];
    }
  }
}

// Halo role of a thread: threads [0, 4 kTB) the x halo, [4 kTB, 8 kTB) the y halo.
struct HaloRole {
  bool on;
  int d;
};
__device__ __forceinline__ HaloRole halo_role(int tid) {
  HaloRole r;
  r.on = tid < 8 * kTB;
  r.d = tid < 4 * kTB ? 0 : 1;
  return r;
}

// Delay with which the tile's PE at plane z sees a halo point (0 inside the PE).
__device__ __forceinline__ int halo_k(const int (*s_kd)[6], int zl, const Halo& h) {
  return h.out ? s_kd[zl][h.face] : 0;
}

template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) void kp_grad_tile(PA<T> a, int publish) {
  constexpr int LW = kTB + 2 * kTH;
  __shared__ T s_u[4][LW][LW];  // u, v, w, T of the plane, tile and x / y halos (corners unused)
  __shared__ int s_kd[kMaxZPe][6];
  const TBrick b = tbrick(a);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTB + tx;
  const int x = b.x0 + tx, y = b.y0 + ty;
  const int nz = a.n[2], ez = a.e[2];
  const HaloRole hr = halo_role(tid);
  const Halo h = halo_of(a, hr.d, hr.on ? tid - 4 * kTB * hr.d : 0, b.x0, b.y0);
  load_delays(a, b, s_kd, tid);
  __syncthreads();

  // prologue: the window (planes z0 - 2 .. z0 + 2), the published planes among them, plane z0 in
  // LDS, then the fetches for plane z0 + 1
  T win[4][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const int zz = b.z0 - 2 + j;
    T q[5], v[10];
    load_q(a, x, y, wrapi(zz, nz), q);
    derive(a, q, 0, v);
#pragma unroll
    for (int c = 0; c < 4; ++c) win[c][j] = v[c];
    if (publish && zz >= b.z0 && zz < b.z1) {
      const int p[3] = {x, y, zz};
      publish_point(a, p, q);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) s_u[c][ty + kTH][tx + kTH] = win[c][2];
  Raw<T> hw;
  int hk = 0;
  if (hr.on) {
    hk = halo_k(s_kd, 0, h);
    fetch_raw(a, h.pt[0], h.pt[1], b.z0, hr.d, hk, hw);
    T v[10];
    finish_raw(a, hr.d, hk, hw, v);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (hr.d == 0) s_u[c][h.along + kTH][h.lds] = v[c];
      else s_u[c][h.lds][h.along + kTH] = v[c];
    }
  }
  T qn[5];
  load_q(a, x, y, wrapi(b.z0 + 3, nz), qn);
  if (hr.on && b.z0 + 1 < b.z1) {
    hk = halo_k(s_kd, (b.z0 % ez) + 1 >= ez ? 1 : 0, h);
    fetch_raw(a, h.pt[0], h.pt[1], b.z0 + 1, hr.d, hk, hw);
  }

  int lz = b.z0 % ez, zl = 0;  // plane z: its index in its z-PE, that z-PE within the chunk
  for (int z = b.z0; z < b.z1; ++z) {
    __syncthreads();
    const uint32_t i = ((uint32_t)z * a.n[1] + y) * a.n[0] + x;
    const T c1[4] = {T(1), T(-8), T(8), T(-1)};
    const int off[4] = {-2, -1, 1, 2};
    T gx[4] = {T(0), T(0), T(0), T(0)}, gy[4] = {T(0), T(0), T(0), T(0)}, gz[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        gx[c] += c1[s] * s_u[c][ty + kTH][tx + kTH + off[s]];
        gy[c] += c1[s] * s_u[c][ty + kTH + off[s]][tx + kTH];
      }
    const bool zface = (lz < 2 && s_kd[zl][4] > 0) || (lz >= ez - 2 && s_kd[zl][5] > 0);  // uniform
    if (!zface) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) gz[c] += c1[s] * win[c][2 + off[s]];
    } else {
      const int p[3] = {x, y, z};
      const int pe = pe_of(a, b.x0, b.y0, z);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        T v[10];
        seen(a, p, pe, 2, off[s], v);
#pragma unroll
        for (int c = 0; c < 4; ++c) gz[c] += c1[s] * v[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {  // streamed out (read by the next launch)
      const uint32_t g0 = (uint32_t)(c < 3 ? 3 * c : 9);
      __builtin_nontemporal_store(gx[c] * a.i12h[0], a.grad + (g0 + 0) * a.N + i);
      __builtin_nontemporal_store(gy[c] * a.i12h[1], a.grad + (g0 + 1) * a.N + i);
      __builtin_nontemporal_store(gz[c] * a.i12h[2], a.grad + (g0 + 2) * a.N + i);
    }
    __syncthreads();
    if (z + 1 < b.z1) {  // uniform
      // consume: the column's plane z + 3 into the window, plane z + 1 into LDS
      {
        T v[10];
        derive(a, qn, 0, v);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int j = 0; j < 4; ++j) win[c][j] = win[c][j + 1];
          win[c][4] = v[c];
        }
        if (publish && z + 3 < b.z1) {
          const int p[3] = {x, y, z + 3};
          publish_point(a, p, qn);
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) s_u[c][ty + kTH][tx + kTH] = win[c][2];
      if (hr.on) {
        T v[10];
        finish_raw(a, hr.d, hk, hw, v);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (hr.d == 0) s_u[c][h.along + kTH][h.lds] = v[c];
          else s_u[c][h.lds][h.along + kTH] = v[c];
        }
      }
      // fetch for plane z + 2: the column's plane z + 4 and the halo points
      load_q(a, x, y, wrapi(z + 4, nz), qn);
      if (hr.on && z + 2 < b.z1) {
        hk = halo_k(s_kd, zl + (lz + 2 >= ez ? 1 : 0), h);
        fetch_raw(a, h.pt[0], h.pt[1], z + 2, hr.d, hk, hw);
      }
    }
    if (++lz == ez) {
      lz = 0;
      ++zl;
    }
  }
}

// Derivative of a line at the PE-local index l (PE edge e), at(o) its value at offset o, with the
// stencils of pe_d1.
template <typename T, typename F>
__device__ __forceinline__ T line_d1(F at, int l, int e, T i12h) {
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
  return s * i12h;
}

// The five-point window of the PE-local first derivative at local index l of a PE of edge e (the
// stencils of pe_d1): its case (0 central, 1 l = 0, 2 l = 1, 3 l = e - 2, 4 l = e - 1), whose
// row of kLineCoef holds the numerators, and its first offset.
__device__ __forceinline__ int line_case(int l, int e) {
  return l >= 2 && l <= e - 3 ? 0 : (l == 0 ? 1 : (l == 1 ? 2 : (l == e - 2 ? 3 : 4)));
}
__device__ __forceinline__ int line_first(int cs) {
  return cs == 0 ? -2 : (cs == 1 ? 0 : (cs == 2 ? -1 : (cs == 3 ? -3 : -4)));
}
__device__ __forceinline__ double line_coef(int cs, int j) {
  constexpr double k[5][5] = {{1, -8, 0, 8, -1},
                              {-25, 48, -36, 16, -3},
                              {-3, -10, 18, -6, 1},
                              {-1, 6, -18, 10, 3},
                              {3, -16, 36, -48, 25}};
  return k[cs][j];
}

// Gradient components whose PE-local lines the mixed derivatives take along x (dv/dy, dw/dz,
// du/dy, du/dz), along y (dv/dx, du/dx, dw/dz, dw/dy) and along z (du/dx, dv/dy, dw/dx, dw/dy).
__host__ __device__ constexpr int kGx(int c) { return c == 0 ? 4 : (c == 1 ? 8 : (c == 2 ? 1 : 2)); }
__host__ __device__ constexpr int kGy(int c) { return c == 0 ? 3 : (c == 1 ? 0 : (c == 2 ? 8 : 5)); }
__host__ __device__ constexpr int kGz(int c) { return c == 0 ? 0 : (c == 1 ? 4 : (c == 2 ? 6 : 7)); }
// the tile's own gradients that go to the x / y line planes: 0, 1, 2, 3, 4, 5, 8
__host__ __device__ constexpr int kGo(int c) { return c < 6 ? c : 8; }

template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void kp_rhs_tile(PA<T> a) {
  constexpr int LW = kTB + 2 * kTH, GW = kTB + 2 * kTG, NP = kTB * kTB;
  __shared__ T s_u[5][LW][LW];         // u, v, w, T, p: tile and x / y halos (corners unused)
  __shared__ T s_fx[5][kTB][LW];       // m_x, m_i u, rho e u on the tile rows with the x halo
  __shared__ T s_fy[5][LW][kTB];       // m_y, m_i v, rho e v on the tile columns with the y halo
  __shared__ T s_gx[4][kTB][GW];       // gradients kGx on the tile rows, x halo 4
  __shared__ T s_gy[4][GW][kTB];       // gradients kGy on the tile columns, y halo 4
  __shared__ T s_gz[kTRing][4][NP];    // gradients kGz of planes z - 4 .. z + 4 (slot by plane)
  __shared__ int s_kd[kMaxZPe][6];
  __shared__ T s_lc[5][5];             // line stencil numerators by case
  const TBrick b = tbrick(a);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTB + tx;
  const int x = b.x0 + tx, y = b.y0 + ty;
  // this thread's PE-local x and y line windows (fixed for the march): case and first offset
  const int cxs = line_case(x % a.e[0], a.e[0]), cys = line_case(y % a.e[1], a.e[1]);
  const int ox = line_first(cxs), oy = line_first(cys);
  if (tid < 25) s_lc[tid / 5][tid % 5] = (T)line_coef(tid / 5, tid % 5);
  const int nz = a.n[2], ez = a.e[2];
  const bool need_dq = a.rk_a != T(0) || a.c_prev != T(0);
  const HaloRole hr = halo_role(tid);
  const Halo h = halo_of(a, hr.d, hr.on ? tid - 4 * kTB * hr.d : 0, b.x0, b.y0);
  // this thread's point of the 4-wide gradient halos: x (tid < 8 kTB), then y
  const int gd = tid < 8 * kTB ? 0 : 1, gh = tid - 8 * kTB * gd, galong = gh / 8, gj = gh % 8;
  const int gl = gj < 4 ? gj : kTB + gj;
  const int ghx = gd == 0 ? wrapi(b.x0 + (gj < 4 ? gj - 4 : kTB + gj - 4), a.n[0]) : b.x0 + galong;
  const int ghy = gd == 0 ? b.y0 + galong : wrapi(b.y0 + (gj < 4 ? gj - 4 : kTB + gj - 4), a.n[1]);
  auto gidx = [&](int xx, int yy, int zz) {  // zz may lie a few planes outside the grid
    int zw = zz;
    while (zw < 0) zw += nz;
    while (zw >= nz) zw -= nz;
    return ((uint32_t)zw * a.n[1] + yy) * a.n[0] + xx;
  };
  auto ring_add = [](int sl, int o) {  // ring slot o planes from slot sl, |o| < kTRing
    const int t = sl + o;
    return t < 0 ? t + kTRing : (t >= kTRing ? t - kTRing : t);
  };
  load_delays(a, b, s_kd, tid);

  // plane-z registers and the fetches for the next plane
  T wq[5][5];  // conserved variables of the column's planes z - 2 .. z + 2
  T dqc[5], gT[3];
  T qn[5], gon[7], grn[4], ghn[4], dqn[5], gTn[3];
  Raw<T> hw;
  int hk = 0;

  // prologue
#pragma unroll
  for (int j = 0; j < 5; ++j) load_q(a, x, y, wrapi(b.z0 - 2 + j, nz), wq[j]);
  for (int zz = b.z0 - kTG; zz <= b.z0 + kTG; ++zz) {
    const uint32_t iz = gidx(x, y, zz);
#pragma unroll
    for (int c = 0; c < 4; ++c) s_gz[zz - b.z0 + kTG][c][tid] = a.grad[(uint32_t)kGz(c) * a.N + iz];
  }
  {
    const uint32_t i0 = gidx(x, y, b.z0), ih = gidx(ghx, ghy, b.z0);
#pragma unroll
    for (int c = 0; c < 7; ++c) gon[c] = a.grad[(uint32_t)kGo(c) * a.N + i0];
#pragma unroll
    for (int c = 0; c < 4; ++c) ghn[c] = a.grad[(uint32_t)(gd == 0 ? kGx(c) : kGy(c)) * a.N + ih];
#pragma unroll
    for (int c = 0; c < 3; ++c) gT[c] = a.grad[(uint32_t)(9 + c) * a.N + i0];
#pragma unroll
    for (int c = 0; c < 5; ++c) dqc[c] = need_dq ? a.dq[(uint32_t)c * a.N + i0] : T(0);
  }
  __syncthreads();  // s_kd
  if (hr.on) {
    hk = halo_k(s_kd, 0, h);
    fetch_raw(a, h.pt[0], h.pt[1], b.z0, hr.d, hk, hw);
  }

  // Writes plane zz's own values, halo values and gradient lines to LDS from the registers.
  auto stage_plane = [&]() {
    T vx[10], vy[10];
    derive(a, wq[2], 0, vx);
    derive(a, wq[2], 1, vy);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      s_u[c][ty + kTH][tx + kTH] = vx[c];
      s_fx[c][ty][tx + kTH] = vx[5 + c];
      s_fy[c][ty + kTH][tx] = vy[5 + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // own gradients: kGx = (4, 8, 1, 2), kGy = (3, 0, 8, 5) among kGo = (0, 1, 2, 3, 4, 5, 8)
      const int ox = c == 0 ? 4 : (c == 1 ? 6 : (c == 2 ? 1 : 2));
      const int oy = c == 0 ? 3 : (c == 1 ? 0 : (c == 2 ? 6 : 5));
      s_gx[c][ty][tx + kTG] = gon[ox];
      s_gy[c][ty + kTG][tx] = gon[oy];
      if (gd == 0) s_gx[c][galong][gl] = ghn[c];
      else s_gy[c][gl][galong] = ghn[c];
    }
    if (hr.on) {
      T v[10];
      finish_raw(a, hr.d, hk, hw, v);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        if (hr.d == 0) {
          s_u[c][h.along + kTH][h.lds] = v[c];
          s_fx[c][h.along][h.lds] = v[5 + c];
        } else {
          s_u[c][h.lds][h.along + kTH] = v[c];
          s_fy[c][h.lds][h.along] = v[5 + c];
        }
      }
    }
  };
  // Issues the loads for plane zz (the column's plane zz + 2, the ring plane zz + 4).
  auto fetch_plane = [&](int zz, int zzl) {  // zzl: the z-PE of plane zz within the chunk
    load_q(a, x, y, wrapi(zz + 2, nz), qn);
    const uint32_t io = gidx(x, y, zz), ih = gidx(ghx, ghy, zz), ir = gidx(x, y, zz + kTG);
#pragma unroll
    for (int c = 0; c < 7; ++c) gon[c] = a.grad[(uint32_t)kGo(c) * a.N + io];
#pragma unroll
    for (int c = 0; c < 4; ++c) ghn[c] = a.grad[(uint32_t)(gd == 0 ? kGx(c) : kGy(c)) * a.N + ih];
#pragma unroll
    for (int c = 0; c < 4; ++c) grn[c] = a.grad[(uint32_t)kGz(c) * a.N + ir];
#pragma unroll
    for (int c = 0; c < 3; ++c) gTn[c] = a.grad[(uint32_t)(9 + c) * a.N + io];
#pragma unroll
    for (int c = 0; c < 5; ++c) dqn[c] = need_dq ? __builtin_nontemporal_load(a.dq + (uint32_t)c * a.N + io) : T(0);
    if (hr.on && zz < b.z1) {
      hk = halo_k(s_kd, zzl, h);
      fetch_raw(a, h.pt[0], h.pt[1], zz, hr.d, hk, hw);
    }
  };
  stage_plane();
  const int lz0 = b.z0 % ez;
  fetch_plane(b.z0 + 1, lz0 + 1 >= ez ? 1 : 0);

  double tsum[5] = {0, 0, 0, 0, 0};
  int lz = lz0, zl = 0, s0 = kTG;  // plane z: its index in its z-PE, that z-PE, its ring slot
  for (int z = b.z0; z < b.z1; ++z) {
    __syncthreads();
    const uint32_t i = ((uint32_t)z * a.n[1] + y) * a.n[0] + x;
    T vc[10];
    derive(a, wq[2], 0, vc);
    T cont = T(0), conve = T(0), lapT = T(0), conv[3] = {T(0), T(0), T(0)}, lap[3] = {T(0), T(0), T(0)},
      pg[3], pure[3];
    const T c1[4] = {T(1), T(-8), T(8), T(-1)}, c2[4] = {T(-1), T(16), T(16), T(-1)};
    const int off[4] = {-2, -1, 1, 2};
    const bool zface = (lz < 2 && s_kd[zl][4] > 0) || (lz >= ez - 2 && s_kd[zl][5] > 0);  // uniform
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T s1[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};  // m_d, uu_0d, uu_1d, uu_2d, eu_d, p
      T s2[4] = {T(0), T(0), T(0), T(0)};              // u, v, w, T
      auto acc = [&](int s, const T v[10]) {
#pragma unroll
        for (int c = 0; c < 5; ++c) s1[c] += c1[s] * v[5 + c];
        s1[5] += c1[s] * v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) s2[c] += c2[s] * v[c];
      };
      if (d < 2) {
#pragma unroll 1  // one neighbour at a time from LDS (register pressure)
        for (int s = 0; s < 4; ++s) {
          const int o = s < 2 ? s - 2 : s - 1;
          const int ux = tx + kTH + (d == 0 ? o : 0), uy = ty + kTH + (d == 1 ? o : 0);
          T v[10];
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            v[c] = s_u[c][uy][ux];
            v[5 + c] = d == 0 ? s_fx[c][ty][ux] : s_fy[c][uy][tx];
          }
          acc(s, v);
        }
      } else if (!zface) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          T v[10];
          derive(a, wq[2 + off[s]], 2, v);
          acc(s, v);
        }
      } else {
        const int p[3] = {x, y, z};
        const int pe = pe_of(a, b.x0, b.y0, z);
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
          T v[10];
          seen(a, p, pe, 2, s < 2 ? s - 2 : s - 1, v);
          acc(s, v);
        }
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
    // mixed derivatives: d/dx_c du_k/dx_k as the average of the PE-local derivative along x_c of
    // du_k/dx_k and along x_k of du_k/dx_c (k != c)
    T dx[4], dy[4], dzl[4];
    {
      T kx[5], ky[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        kx[j] = s_lc[cxs][j];
        ky[j] = s_lc[cys][j];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        // x and y: the thread's window, branch-free; z: uniform cases
        T sx = kx[0] * s_gx[c][ty][tx + kTG + ox], sy = ky[0] * s_gy[c][ty + kTG + oy][tx];
#pragma unroll
        for (int j = 1; j < 5; ++j) {
          sx += kx[j] * s_gx[c][ty][tx + kTG + ox + j];
          sy += ky[j] * s_gy[c][ty + kTG + oy + j][tx];
        }
        dx[c] = sx * a.i12h[0];
        dy[c] = sy * a.i12h[1];
        dzl[c] = line_d1<T>([&](int o) { return s_gz[ring_add(s0, o)][c][tid]; }, lz, ez, a.i12h[2]);
      }
    }
    // dx: G4 G8 G1 G2; dy: G3 G0 G8 G5; dzl: G0 G4 G6 G7
    T mixed[3];
    mixed[0] = T(0.5) * (dx[0] + dy[0]) + T(0.5) * (dx[1] + dzl[2]);
    mixed[1] = T(0.5) * (dy[1] + dx[2]) + T(0.5) * (dy[2] + dzl[3]);
    mixed[2] = T(0.5) * (dzl[0] + dx[3]) + T(0.5) * (dzl[1] + dy[3]);
    T G[12];
    G[0] = s_gy[1][ty + kTG][tx];
    G[1] = s_gx[2][ty][tx + kTG];
    G[2] = s_gx[3][ty][tx + kTG];
    G[3] = s_gy[0][ty + kTG][tx];
    G[4] = s_gx[0][ty][tx + kTG];
    G[5] = s_gy[3][ty + kTG][tx];
    G[6] = s_gz[s0][2][tid];
    G[7] = s_gz[s0][3][tid];
    G[8] = s_gx[1][ty][tx + kTG];
#pragma unroll
    for (int c = 0; c < 3; ++c) G[9 + c] = gT[c];
    T rhs[5];
    assemble(a, vc, G, cont, conv, conve, pg, lap, lapT, pure, mixed, rhs);
    // the update (or the RHS alone), with dQ of this plane from registers
    if (a.mode == kModeRhsH) {
#pragma unroll
      for (int c = 0; c < 5; ++c) __builtin_nontemporal_store(rhs[c], a.rhs_out + (uint32_t)c * a.N + i);
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const T prev = dqc[c];
        const T dqv = a.rk_a * prev + a.dt * rhs[c];
        const T inc = a.rk_b * dqv + a.c_prev * prev;
        if (a.store_dq) __builtin_nontemporal_store(dqv, a.dq + (uint32_t)c * a.N + i);
        __builtin_nontemporal_store(wq[2][c] + inc, a.q_out + (uint32_t)c * a.N + i);
        tsum[c] += a.c_prev != T(0) ? (double)inc : (double)dqv;
      }
    }
    __syncthreads();
    if (z + 1 < b.z1) {  // uniform: consume the fetches for plane z + 1, then fetch for z + 2
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < 5; ++c) wq[j][c] = wq[j + 1][c];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        wq[4][c] = qn[c];
        dqc[c] = dqn[c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) gT[c] = gTn[c];
#pragma unroll
      for (int c = 0; c < 4; ++c) s_gz[ring_add(s0, kTG + 1)][c][tid] = grn[c];  // plane z + 5
      stage_plane();
      fetch_plane(z + 2, zl + (lz + 2 >= ez ? 1 : 0));
    }
    s0 = ring_add(s0, 1);
    if (++lz == ez) {
      lz = 0;
      ++zl;
    }
  }
  if (a.mode != kModeStepH) return;  // uniform across the grid
  block_totals(a, tsum, b.L, tid);
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

bool paper_tiled(const Geom& g) { return g.e[0] % kTB == 0 && g.e[1] % kTB == 0; }

int64_t paper_tiled_blocks(const Geom& g) {
  return (int64_t)(g.n[0] / kTB) * (g.n[1] / kTB) * ((g.n[2] + kTZ - 1) / kTZ);
}

// Workgroup slots of the FP64 totals: enough for either kernel.
int64_t paper_blocks(const Geom& g) {
  const int64_t pt = (int64_t)((g.n[0] + kBXp - 1) / kBXp) * ((g.n[1] + kBYp - 1) / kBYp) * ((g.n[2] + kZC - 1) / kZC);
  return paper_tiled(g) ? std::max(pt, paper_tiled_blocks(g)) : pt;
}

template <typename T>
hipError_t launch_stagep(const StagePArgs<T>& s, int which, hipStream_t stream) {
  const PA<T> a = pack(s);
  if (which == kPPublish) {
    const uint64_t total = (uint64_t)a.slab[0] + a.slab[1] + a.slab[2];
    hipLaunchKernelGGL((kp_publish<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
  }
  if (paper_tiled(s.g)) {
    const dim3 grid((unsigned)paper_tiled_blocks(s.g)), block(kTB, kTB);
    if (which == kPGrad || which == kPGradPublish)
      hipLaunchKernelGGL((kp_grad_tile<T>), grid, block, 0, stream, a, which == kPGradPublish ? 1 : 0);
    else hipLaunchKernelGGL((kp_rhs_tile<T>), grid, block, 0, stream, a);
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
