// Turbulence diagnostics of one field on gfx950 (Sec. 4.1): the energy spectrum E(kappa) and the
// pressure spectrum E_p(kappa) over the shells kappa = round(|k|) (Eqs. ener, pres), the skewness
// and flatness of du/dx (Sec. 4.1.3), and the PDFs of eps / <eps> and Omega / <Omega> (Fig.
// enst_pdf) as integer counts.  Everything in FP64 whatever the field precision.
//
// Passes (one stream, no host synchronisation):
//   1. k_diag_pts: synchronous central gradients of the run's order; per-workgroup FP64 sums of
//      g^2, g^3, g^4 (g = du/dx), eps = sigma_ij du_i/dx_j, Omega = |curl u|^2 and p, reduced in a
//      fixed order (k_mom_reduce, k_mom_final) into the means and S, F; eps and Omega of every
//      point kept in the workspace.
//   2. k_diag_hist: eps and Omega binned against the means; LDS histograms, flushed with 64-bit
//      integer atomics (exact and order-free).
//   3. k_fft_x: rows of the conservative field -> u, v, w, p in FP64 -> (u + i v) and (w + i p)
//      transformed along x in LDS -> separated into the half spectra (kx = 0 .. nx/2) of the four
//      real fields.
//   4. k_fft_y: in-place transform along y of every (field, z, kx) column block.
//   5. k_fft_z_shell: transform along z in LDS, then the shell sums of the workgroup's columns,
//      each shell summed by one thread over contiguous runs of kz (no atomics), into per-workgroup
//      partials that k_shell_reduce1/2 add in a fixed order.
// The line transforms are in-place decimation-in-frequency radix-8 (plus one radix-4 or radix-2
// stage) FFTs, so their outputs sit in the mixed-radix digit-reversed order of the stages; no
// reordering pass is made - pos_of / freq_of map between positions and frequencies wherever one is
// needed (the x separation and the shell sums).
#include <algorithm>
#include <cmath>

#include "sim_internal.h"

using namespace atns;

namespace {

constexpr int kThreads = 256;
constexpr int kMaxN = 1024;       // points per direction (the line transforms live in LDS)
constexpr int kMinN = 8;
constexpr int kMaxStages = 4;     // 1024 = 8 * 8 * 8 * 2
constexpr int kMom = 6;           // g^2, g^3, g^4, eps, Omega, p
constexpr int kRed = 256;         // level-1 rows of the fixed-order reductions
constexpr int kLdsFft = 64 * 1024;
constexpr int kPtsBX = 64, kPtsBY = 4, kPtsZC = 32;  // point-pass workgroup: 64 x 4 columns, 32 planes
constexpr int kMaxShells = AT_DIAG_MAX_SHELLS;
constexpr int kMaxBins = AT_DIAG_MAX_BINS;

// Radix plan of one axis of n = 2^m points: m / 3 radix-8 stages, then one radix-2 or radix-4 stage
// for the rest.
struct Axis {
  int n;
  int lg;              // log2 n
  int nst;
  int lr[kMaxStages];  // log2 of each stage's radix, in the order the stages run
  int tws;             // twiddle table stride: table length / n
};

Axis make_axis(int n, int ntw) {
  Axis a{};
  a.n = n;
  int m = 0;
  while ((1 << m) < n) ++m;
  a.lg = m;
  for (int i = 0; i < m / 3; ++i) a.lr[a.nst++] = 3;
  if (m % 3) a.lr[a.nst++] = m % 3;
  a.tws = ntw / n;
  return a;
}

// Position, after the in-place transform, of frequency index f (0 .. n-1), and its inverse.
// Stage i splits the current span L into R_i blocks; frequency f = t_1 + R_1 (t_2 + R_2 (...)) sits
// at position sum_i t_i n / (R_1 ... R_i).
__device__ __forceinline__ int pos_of(const Axis& a, int f) {
  int p = 0, L = a.n;
  for (int i = 0; i < a.nst; ++i) {
    L >>= a.lr[i];
    p += (f & ((1 << a.lr[i]) - 1)) * L;
    f >>= a.lr[i];
  }
  return p;
}
__device__ __forceinline__ int freq_of(const Axis& a, int p) {
  int k = 0, sh = 0, lgL = a.lg;
  for (int i = 0; i < a.nst; ++i) {
    lgL -= a.lr[i];
    k += (p >> lgL) << sh;
    p &= (1 << lgL) - 1;
    sh += a.lr[i];
  }
  return k;
}
__device__ __forceinline__ int signed_k(int f, int n) { return f <= n / 2 ? f : f - n; }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }  // a * (-i)

// R-point forward DFTs in registers: y_t = sum_s x_s exp(-2 pi i s t / R).
__device__ __forceinline__ void dft2(double2& a, double2& b) {
  const double2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3) {
  const double2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mul_mi(csub(x1, x3));
  x0 = cadd(a, c);
  x1 = cadd(b, d);
  x2 = csub(a, c);
  x3 = csub(b, d);
}
__device__ __forceinline__ void dft8(double2* x) {
  constexpr double r = 0.70710678118654752440084436210485;  // 1 / sqrt 2
  double2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  double2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  o1 = make_double2(r * (o1.x + o1.y), r * (o1.y - o1.x));     // * exp(-i pi / 4)
  o2 = mul_mi(o2);                                             // * exp(-i pi / 2)
  o3 = make_double2(r * (o3.y - o3.x), -r * (o3.x + o3.y));    // * exp(-3 i pi / 4)
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

// LDS position of element e of an x line: one pad element after every 8, so that the strided
// butterflies of the later stages (inputs 8 or 1 elements apart, 128 bytes and more) spread over
// the banks instead of falling on the same half of them (the lines of the y and z passes are
// interleaved by column, where those strides already fall on different banks).
__device__ __forceinline__ int pe(int e) { return e + (e >> 3); }
__host__ __device__ constexpr int padded(int n) { return n + n / 8; }

// One in-place decimation-in-frequency stage of radix R = 2^LR on every line: span L, butterfly
// inputs Ls = L / R apart; output t of butterfly j is multiplied by exp(-2 pi i j t / L).  Element
// e of line l lives at buf[l * ls + e' * es], e' = pe(e) with PAD, else e.  line_fast: consecutive threads take consecutive lines
// (strided axes, where the lines are interleaved), else consecutive butterflies of one line.
template <int LR, int NT, bool PAD>
__device__ __forceinline__ void dif_stage(double2* buf, const Axis& a, int L, int nlines, int ls, int es,
                                          const double2* __restrict__ tw, bool line_fast) {
  constexpr int R = 1 << LR;
  const int Ls = L >> LR, nb = a.n >> LR, total = nlines * nb;
  const int twstep = (a.n / L) * a.tws;
  for (int t = threadIdx.x; t < total; t += NT) {
    int line, b;
    if (line_fast) {
      line = t % nlines;
      b = t / nlines;
    } else {
      b = t % nb;
      line = t / nb;
    }
    const int blk = b / Ls, j = b - blk * Ls;
    double2* base = buf + line * ls;
    const int e0 = blk * L + j;
    double2 x[R];
#pragma unroll
    for (int s = 0; s < R; ++s) x[s] = base[(PAD ? pe(e0 + s * Ls) : e0 + s * Ls) * es];
    if constexpr (R == 8) dft8(x);
    else if constexpr (R == 4) dft4(x[0], x[1], x[2], x[3]);
    else dft2(x[0], x[1]);
#pragma unroll
    for (int s = 1; s < R; ++s) x[s] = cmul(x[s], tw[j * s * twstep]);
#pragma unroll
    for (int s = 0; s < R; ++s) base[(PAD ? pe(e0 + s * Ls) : e0 + s * Ls) * es] = x[s];
  }
}

template <int NT, bool PAD>
__device__ void fft_lines(double2* buf, const Axis& a, int nlines, int ls, int es, const double2* __restrict__ tw,
                          bool line_fast) {
  int L = a.n;
  for (int i = 0; i < a.nst; ++i) {
    if (a.lr[i] == 3) dif_stage<3, NT, PAD>(buf, a, L, nlines, ls, es, tw, line_fast);
    else if (a.lr[i] == 2) dif_stage<2, NT, PAD>(buf, a, L, nlines, ls, es, tw, line_fast);
    else dif_stage<1, NT, PAD>(buf, a, L, nlines, ls, es, tw, line_fast);
    L >>= a.lr[i];
    __syncthreads();
  }
}

// Twiddle table exp(-2 pi i e / ntw), e = 0 .. ntw-1 (sincospi of an exact argument).
// Streamed accesses of the pass buffers (each written once by one pass and read once by the
// next, far beyond the caches at the sizes these passes serve).
typedef double dvec2 __attribute__((ext_vector_type(2)));  // 16 bytes, the layout of double2
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  const dvec2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<dvec2*>(p));
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const dvec2 w = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
  return make_double2(w.x, w.y);
}

__global__ void k_twiddle(double2* tw, int ntw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntw) return;
  double s, c;
  sincospi(-2.0 * (double)e / (double)ntw, &s, &c);
  tw[e] = make_double2(c, s);
}

struct Phys {
  double inv_cv, gas_r, mu_ref, inv_tref, mu_exp, suth_s;
  int form, visc;   // fifth variable E (0) or rho e (1); power law (0) or Sutherland (1)
  double inv_h[3];  // 1 / (12 h) for order 4, 1 / (60 h) for order 6
};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ void prims(const T* __restrict__ q, int64_t N, int64_t i, const Phys& ph, double pr[5]) {
  const double rho = (double)q[i];
  const double rinv = 1.0 / rho;
  const double u = (double)q[N + i] * rinv, v = (double)q[2 * N + i] * rinv, w = (double)q[3 * N + i] * rinv;
  pr[0] = rho;
  pr[1] = u;
  pr[2] = v;
  pr[3] = w;
  pr[4] = ph.form == 1 ? (double)q[4 * N + i] * rinv * ph.inv_cv
                       : ((double)q[4 * N + i] * rinv - 0.5 * (u * u + v * v + w * w)) * ph.inv_cv;
}

// Per-point values of one point: g = du/dx, eps, Omega, p (synchronous periodic derivatives).
template <typename T, int M>
__device__ __forceinline__ void point_values(const T* __restrict__ q, int nx, int ny, int nz, int64_t N, int x, int y,
                                             int z, const Phys& ph, double& g, double& eps, double& om, double& p) {
  const int pt[3] = {x, y, z};
  const int nn[3] = {nx, ny, nz};
  double G[9];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double v[2 * M][3];
#pragma unroll
    for (int mi = 0; mi < 2 * M; ++mi) {
      const int m = mi < M ? mi - M : mi - M + 1;
      int r[3] = {x, y, z};
      r[d] = wrapi(pt[d] + m, nn[d]);
      const int64_t ir = ((int64_t)r[2] * ny + r[1]) * nx + r[0];
      double pr[5];
      prims<T>(q, N, ir, ph, pr);
      v[mi][0] = pr[1];
      v[mi][1] = pr[2];
      v[mi][2] = pr[3];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double num = M == 2 ? (v[0][c] - 8.0 * v[1][c] + 8.0 * v[2][c] - v[3][c])
                                : (9.0 * v[1][c] - v[0][c]) + 45.0 * (v[3][c] - v[2][c]) + (v[5][c] - 9.0 * v[4][c]);
      G[3 * c + d] = num * ph.inv_h[d];
    }
  }
  const int64_t i = ((int64_t)z * ny + y) * nx + x;
  double pr[5];
  prims<T>(q, N, i, ph, pr);
  const double tt = pr[4] * ph.inv_tref;
  const double mu = ph.visc == 1 ? ph.mu_ref * tt * sqrt(tt) * (1.0 / ph.inv_tref + ph.suth_s) / (pr[4] + ph.suth_s)
                                 : ph.mu_ref * pow(tt, ph.mu_exp);
  const double th = G[0] + G[4] + G[8];
  double e = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double sg = mu * (G[3 * a + b] + G[3 * b + a]);
      if (a == b) sg -= (2.0 / 3.0) * mu * th;
      e += sg * G[3 * a + b];
    }
  const double ox = G[7] - G[5], oy = G[2] - G[6], oz = G[3] - G[1];
  g = G[0];
  eps = e;
  om = ox * ox + oy * oy + oz * oz;
  p = pr[0] * ph.gas_r * pr[4];
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int pdf_bin(double x, double scale, int nbins) {
  double b = floor(x * scale);
  if (!(b >= 0.0)) b = 0.0;
  if (b > (double)nbins) b = (double)nbins;
  return (int)b;
}

// Point pass over 64 x 4 columns and kPtsZC planes per workgroup: partial sums [blk][kMom] of
// g^2, g^3, g^4, eps, Omega and p, and (eps, Omega) of every point for the histogram pass.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_diag_pts(const T* __restrict__ q, int nx, int ny, int nz, Phys ph,
                                                  double* __restrict__ part, double2* __restrict__ eo) {
  const int x = blockIdx.x * kPtsBX + threadIdx.x;
  const int y = blockIdx.y * kPtsBY + threadIdx.y;
  const int z0 = blockIdx.z * kPtsZC, z1 = min(z0 + kPtsZC, nz);
  const int tid = threadIdx.y * kPtsBX + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  double s[kMom] = {0, 0, 0, 0, 0, 0};
  if (x < nx && y < ny) {
    for (int z = z0; z < z1; ++z) {
      double g, e, o, p;
      point_values<T, M>(q, nx, ny, nz, N, x, y, z, ph, g, e, o, p);
      st_stream(&eo[((int64_t)z * ny + y) * nx + x], make_double2(e, o));
      const double g2 = g * g;
      s[0] += g2;
      s[1] += g2 * g;
      s[2] += g2 * g2;
      s[3] += e;
      s[4] += o;
      s[5] += p;
    }
  }
  __shared__ double red[kPtsBY][kMom];
#pragma unroll
  for (int c = 0; c < kMom; ++c) {
    const double v = wsum(s[c]);
    if (threadIdx.x == 0) red[threadIdx.y][c] = v;
  }
  __syncthreads();
  if (tid < kMom) {
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[blk * kMom + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
  }
}

constexpr int kHistPts = 16;  // points per thread of the histogram pass

// Counts of eps / <eps> and Omega / <Omega> (means from the reduced sums) in LDS, flushed with
// 64-bit integer atomics.
__global__ __launch_bounds__(256) void k_diag_hist(const double2* __restrict__ eo, int64_t N,
                                                   const double* __restrict__ sums,
                                                   unsigned long long* __restrict__ hist, int nbins, double scale_e,
                                                   double scale_o) {
  extern __shared__ unsigned int hs[];  // [2][nbins + 1]
  const double inv_n = 1.0 / (double)N;
  const double me = sums[3] * inv_n, mo = sums[4] * inv_n;
  const bool do_e = me > 0.0 && isfinite(me), do_o = mo > 0.0 && isfinite(mo);
  for (int b = threadIdx.x; b < 2 * (nbins + 1); b += kThreads) hs[b] = 0u;
  __syncthreads();
  if (do_e || do_o) {
    const int64_t i0 = (int64_t)blockIdx.x * kThreads * kHistPts;
#pragma unroll 4
    for (int c = 0; c < kHistPts; ++c) {
      const int64_t i = i0 + c * kThreads + threadIdx.x;
      if (i < N) {
        const double2 v = ld_stream(&eo[i]);
        if (do_e) atomicAdd(&hs[pdf_bin(v.x / me, scale_e, nbins)], 1u);
        if (do_o) atomicAdd(&hs[nbins + 1 + pdf_bin(v.y / mo, scale_o, nbins)], 1u);
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 2 * (nbins + 1); b += kThreads)
    if (hs[b]) atomicAdd(&hist[b], (unsigned long long)hs[b]);
}

__device__ __forceinline__ double tree(double* red, double v) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Fixed-order reduction of the moment partials: workgroup j sums its contiguous share into mid[j].
__global__ __launch_bounds__(256) void k_mom_reduce(const double* __restrict__ part, int64_t nblk,
                                                    double* __restrict__ mid) {
  __shared__ double red[kThreads];
  const int64_t per = (nblk + kRed - 1) / kRed, b0 = blockIdx.x * per, b1 = min(b0 + per, nblk);
  for (int c = 0; c < kMom; ++c) {
    double v = 0.0;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += kThreads) v += part[b * kMom + c];
    const double r = tree(red, v);
    if (threadIdx.x == 0) mid[blockIdx.x * kMom + c] = r;
  }
}

// Level 2: sums[kMom], and the scalars S, F, <g^2>, <g^3>, <g^4>, <eps>, <Omega>, <p> at out.
__global__ __launch_bounds__(256) void k_mom_final(const double* __restrict__ mid, double npts,
                                                   double* __restrict__ sums, double* __restrict__ out) {
  __shared__ double red[kThreads];
  __shared__ double sm[kMom];
  for (int c = 0; c < kMom; ++c) {
    const double r = tree(red, threadIdx.x < kRed ? mid[threadIdx.x * kMom + c] : 0.0);
    if (threadIdx.x == 0) sm[c] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double inv = 1.0 / npts;
    const double g2 = sm[0] * inv, g3 = sm[1] * inv, g4 = sm[2] * inv;
    for (int c = 0; c < kMom; ++c) sums[c] = sm[c];
    out[0] = g2 > 0.0 ? g3 / (g2 * sqrt(g2)) : 0.0;
    out[1] = g2 > 0.0 ? g4 / (g2 * g2) : 0.0;
    out[2] = g2;
    out[3] = g3;
    out[4] = g4;
    out[5] = sm[3] * inv;
    out[6] = sm[4] * inv;
    out[7] = sm[5] * inv;
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_counts_out(const unsigned long long* __restrict__ hist, int n, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)hist[i];
}

// Transform along x of `rows` rows (z, y) per workgroup: u, v, w, p from the conservative state,
// (u + i v) and (w + i p) transformed together, then the half spectra of the four real fields,
// A(k) = (Z(k) + conj Z(-k)) / 2 and B(k) = (Z(k) - conj Z(-k)) / (2 i), for kx = 0 .. nx/2 into
// S[f][z][y][kx] (row pitch px).
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x(const T* __restrict__ q, int nx, int64_t N, int rows, Axis ax,
                                               const double2* __restrict__ tw, Phys ph, double2* __restrict__ S,
                                               int px, int64_t fstride) {
  extern __shared__ double2 lds[];  // [rows][2][padded(nx)]
  const int64_t row0 = (int64_t)blockIdx.x * rows;
  const int lx = padded(nx);
  for (int t = threadIdx.x; t < rows * nx; t += kThreads) {
    const int r = t / nx, x = t - r * nx;
    double pr[5];
    prims<T>(q, N, (row0 + r) * nx + x, ph, pr);
    lds[(2 * r) * lx + pe(x)] = make_double2(pr[1], pr[2]);
    lds[(2 * r + 1) * lx + pe(x)] = make_double2(pr[3], pr[0] * ph.gas_r * pr[4]);
  }
  __syncthreads();
  fft_lines<kThreads, true>(lds, ax, 2 * rows, lx, 1, tw, false);
  const int nh = nx / 2 + 1;
  for (int t = threadIdx.x; t < 2 * rows * nh; t += kThreads) {
    const int kx = t % nh, rl = t / nh;
    const double2* line = lds + rl * lx;
    const double2 zk = line[pe(pos_of(ax, kx))], zm = line[pe(pos_of(ax, (nx - kx) & (nx - 1)))];
    const double2 A = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
    const double2 B = make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x));
    const int f = 2 * (rl & 1);
    const int64_t o = (row0 + (rl >> 1)) * px + kx;
    st_stream(&S[f * fstride + o], A);
    st_stream(&S[(f + 1) * fstride + o], B);
  }
}

// In-place transform along y of the columns kx0 .. kx0 + bx - 1 of one (field, z) plane.
constexpr int kThreadsYZ = 512;  // 8 waves: twice the loads in flight of a 256-thread workgroup
__global__ __launch_bounds__(kThreadsYZ) void k_fft_y(double2* __restrict__ S, int nx, int ny, int px, int bx, Axis ay,
                                                      const double2* __restrict__ tw, int64_t fstride) {
  extern __shared__ double2 lds[];  // [ny][bx]
  const int kx0 = blockIdx.x * bx, z = blockIdx.y, f = blockIdx.z;
  const int nv = min(bx, nx / 2 + 1 - kx0);
  double2* base = S + f * fstride + (int64_t)z * ny * px + kx0;
  for (int t = threadIdx.x; t < ny * bx; t += kThreadsYZ) {
    const int y = t / bx, l = t - y * bx;
    lds[t] = l < nv ? ld_stream(&base[(int64_t)y * px + l]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_lines<kThreadsYZ, false>(lds, ay, bx, 1, bx, tw, true);
  for (int t = threadIdx.x; t < ny * bx; t += kThreadsYZ) {
    const int y = t / bx, l = t - y * bx;
    if (l < nv) st_stream(&base[(int64_t)y * px + l], lds[t]);
  }
}

// floor(sqrt(v)) of an integer 0 <= v < 2^24 (exact in FP32; corrected in integers).
__device__ __forceinline__ int isqrt_floor(int v) {
  int s = (int)sqrtf((float)v);
  while (s * s > v) --s;
  while ((s + 1) * (s + 1) <= v) ++s;
  return s;
}
// round(sqrt(k2)) of an integer k2 >= 0: no integer lies on a tie.
__device__ __forceinline__ int shell_of(int k2) {
  const int s = isqrt_floor(k2);
  return k2 > s * s + s ? s + 1 : s;
}

constexpr int kMaxPerThread = kLdsFft / (int)sizeof(double2) / kThreadsYZ;  // points per thread in the z pass

// Transform along z of the columns kx0 .. kx0 + bx - 1 of one (field, y-position) row, then the
// workgroup's shell sums.  |S|^2 of every point (times 2 on the columns 0 < kx < nx/2, whose mirror
// images -k carry the same |F|^2) is first laid out per column in natural frequency order over the
// transform's buffer.  Shell s >= 1 holds the k with s^2 - s < |k|^2 <= s^2 + s (shell 0 is k = 0):
// on every column a contiguous run of |kz|, so one thread sums shell s over the columns (kx
// ascending) and both halves of kz (kz >= 0, then kz < 0, |kz| ascending) with no atomics.
// part[wg][j] is shell lo + j, hdr[wg] = (lo, count); velocity fields carry the factor 1/2 of the
// energy.  |k|^2 <= 3 (n/2)^2 < 2^24 for n <= 1024.
__global__ __launch_bounds__(kThreadsYZ) void k_fft_z_shell(const double2* __restrict__ S, int nx, int ny, int nz, int px,
                                                     int bx, Axis ay, Axis az, const double2* __restrict__ tw,
                                                     int64_t fstride, int nshell, int spanmax,
                                                     double* __restrict__ part, int* __restrict__ hdr,
                                                     double inv_n2) {
  extern __shared__ double2 lds[];  // [nz][bx]; then [bx][nz + 1] doubles
  const int kx0 = blockIdx.x * bx, py = blockIdx.y, f = blockIdx.z;
  const int nv = min(bx, nx / 2 + 1 - kx0);
  const double2* base = S + f * fstride + (int64_t)py * px + kx0;
  const int64_t zs = (int64_t)ny * px;
  for (int t = threadIdx.x; t < nz * bx; t += kThreadsYZ) {
    const int z = t / bx, l = t - z * bx;
    lds[t] = l < nv ? ld_stream(&base[z * zs + l]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_lines<kThreadsYZ, false>(lds, az, bx, 1, bx, tw, true);
  const int nzp = nz + 1;
  double ev[kMaxPerThread];
  int ei[kMaxPerThread];
#pragma unroll
  for (int c = 0; c < kMaxPerThread; ++c) {
    const int t = threadIdx.x + c * kThreadsYZ;
    ei[c] = -1;
    if (t < nz * bx) {
      const int p = t / bx, l = t - p * bx;
      const double2 v = lds[t];
      const int kx = kx0 + l;
      ev[c] = (kx == 0 || kx == nx / 2 ? 1.0 : 2.0) * (v.x * v.x + v.y * v.y);
      ei[c] = l * nzp + freq_of(az, p);
    }
  }
  __syncthreads();
  double* en = (double*)lds;
#pragma unroll
  for (int c = 0; c < kMaxPerThread; ++c)
    if (ei[c] >= 0) en[ei[c]] = ev[c];
  __syncthreads();
  const int ky = signed_k(freq_of(ay, py), ny);
  const int kxa = kx0, kxb = kx0 + nv - 1, kzh = nz / 2;
  const int s_lo = shell_of(kxa * kxa + ky * ky);
  const int s_hi = min(shell_of(kxb * kxb + ky * ky + kzh * kzh), nshell - 1);
  const int span = max(0, s_hi - s_lo + 1);
  const int64_t wg = ((int64_t)f * gridDim.y + py) * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    hdr[2 * wg] = s_lo;
    hdr[2 * wg + 1] = span;
  }
  const double scale = (f < 3 ? 0.5 : 1.0) * inv_n2;
  for (int j = threadIdx.x; j < span; j += kThreadsYZ) {
    const int s = s_lo + j;
    const int lo2 = s == 0 ? 0 : s * s - s + 1, hi2 = s * s + s;
    double tot = 0.0;
    for (int l = 0; l < nv; ++l) {
      const int kx = kx0 + l, r = kx * kx + ky * ky;
      if (hi2 < r) continue;
      const int a = lo2 <= r ? 0 : isqrt_floor(lo2 - r - 1) + 1;  // ceil(sqrt(lo2 - r))
      const int b = min(isqrt_floor(hi2 - r), kzh);
      const double* row = en + l * nzp;
      double acc = 0.0;
      for (int kz = a; kz <= b; ++kz) acc += row[kz];
      for (int kz = max(a, 1); kz <= min(b, kzh - 1); ++kz) acc += row[nz - kz];
      tot += acc;
    }
    part[wg * spanmax + j] = tot * scale;
  }
}

// Shell partials of workgroups [j per, (j + 1) per) added in workgroup order: mid[j][0][s] the
// velocity fields (E), mid[j][1][s] the pressure (E_p).
__global__ __launch_bounds__(256) void k_shell_reduce1(const double* __restrict__ part, const int* __restrict__ hdr,
                                                       int64_t nwg, int64_t nwg_vel, int spanmax, int nshell,
                                                       double* __restrict__ mid) {
  const int64_t per = (nwg + kRed - 1) / kRed, w0 = blockIdx.x * per, w1 = min(w0 + per, nwg);
  for (int s = threadIdx.x; s < nshell; s += kThreads) {
    double e = 0.0, ep = 0.0;
    for (int64_t w = w0; w < w1; ++w) {
      const int lo = hdr[2 * w], cnt = hdr[2 * w + 1];
      if (s >= lo && s < lo + cnt) {
        const double v = part[w * spanmax + (s - lo)];
        if (w < nwg_vel) e += v;
        else ep += v;
      }
    }
    mid[((int64_t)blockIdx.x * 2) * nshell + s] = e;
    mid[((int64_t)blockIdx.x * 2 + 1) * nshell + s] = ep;
  }
}

__global__ __launch_bounds__(256) void k_shell_reduce2(const double* __restrict__ mid, int nshell,
                                                       double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshell) return;
  double e = 0.0, ep = 0.0;
  for (int j = 0; j < kRed; ++j) {
    e += mid[((int64_t)j * 2) * nshell + s];
    ep += mid[((int64_t)j * 2 + 1) * nshell + s];
  }
  out[s] = e;
  out[nshell + s] = ep;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Workspace plan of one call.
struct Plan {
  int nx, ny, nz, px, bxy, bxz, rows, ntw, nbxy, nbxz;
  int64_t nblk_pts, nwgz, spanmax;
  size_t off_S, off_eo, off_tw, off_part, off_mid, off_sums, off_hist, off_spart, off_hdr, off_smid, total;
  dim3 pts_grid;
};

int plan_of(const at_config* cfg, const at_diag_params* prm, Plan* pl) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!prm) return fail(AT_E_INVAL, "NULL diagnostics parameters");
  for (int d = 0; d < 3; ++d)
    if (!pow2(cfg->n[d]) || cfg->n[d] < kMinN || cfg->n[d] > kMaxN)
      return fail(AT_E_INVAL, "diagnostics need powers of two from 8 to 1024 points per direction");
  if (prm->nshell < 1 || prm->nshell > kMaxShells) return fail(AT_E_INVAL, "nshell outside 1 .. AT_DIAG_MAX_SHELLS");
  if (prm->nbins < 1 || prm->nbins > kMaxBins) return fail(AT_E_INVAL, "nbins outside 1 .. AT_DIAG_MAX_BINS");
  if (!(prm->eps_max > 0.0) || !(prm->ens_max > 0.0) || !std::isfinite(prm->eps_max) || !std::isfinite(prm->ens_max))
    return fail(AT_E_INVAL, "PDF ranges must be positive and finite");
  Plan& p = *pl;
  p.nx = cfg->n[0];
  p.ny = cfg->n[1];
  p.nz = cfg->n[2];
  const int nh = p.nx / 2 + 1;
  p.px = (nh + 7) & ~7;
  p.ntw = std::max(p.nx, std::max(p.ny, p.nz));
  p.rows = std::min(kLdsFft / (int)(2 * sizeof(double2)) / p.nx, p.ny * p.nz);
  p.bxy = std::min(8, kLdsFft / (int)sizeof(double2) / p.ny);
  p.bxz = std::min(8, kLdsFft / (int)sizeof(double2) / p.nz);
  p.nbxy = (nh + p.bxy - 1) / p.bxy;
  p.nbxz = (nh + p.bxz - 1) / p.bxz;
  p.pts_grid = dim3((p.nx + kPtsBX - 1) / kPtsBX, (p.ny + kPtsBY - 1) / kPtsBY, (p.nz + kPtsZC - 1) / kPtsZC);
  p.nblk_pts = (int64_t)p.pts_grid.x * p.pts_grid.y * p.pts_grid.z;
  p.nwgz = (int64_t)4 * p.ny * p.nbxz;
  p.spanmax = p.nz / 2 + p.bxz + 2;  // |k| grows by at most bx - 1 + nz/2 across one workgroup
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  p.off_S = take((size_t)4 * p.nz * p.ny * p.px * sizeof(double2));
  p.off_eo = take((size_t)p.nx * p.ny * p.nz * sizeof(double2));
  p.off_tw = take((size_t)p.ntw * sizeof(double2));
  p.off_part = take((size_t)p.nblk_pts * kMom * sizeof(double));
  p.off_mid = take((size_t)kRed * kMom * sizeof(double));
  p.off_sums = take(8 * sizeof(double));
  p.off_hist = take((size_t)2 * (prm->nbins + 1) * sizeof(unsigned long long));
  p.off_spart = take((size_t)p.nwgz * p.spanmax * sizeof(double));
  p.off_hdr = take((size_t)p.nwgz * 2 * sizeof(int));
  p.off_smid = take((size_t)kRed * 2 * prm->nshell * sizeof(double));
  p.total = o;
  return AT_OK;
}

template <typename T, int M>
int run_diag(const at_config* cfg, const Plan& pl, const at_diag_params* prm, const T* q, uint8_t* ws, double* out,
             hipStream_t st) {
  Phys ph;
  ph.inv_cv = (cfg->gamma - 1.0) / cfg->gas_r;
  ph.gas_r = cfg->gas_r;
  ph.mu_ref = cfg->mu_ref;
  ph.inv_tref = 1.0 / cfg->t_ref;
  ph.mu_exp = cfg->mu_exp;
  ph.suth_s = cfg->sutherland_s;
  ph.form = cfg->form;
  ph.visc = cfg->visc_law;
  for (int d = 0; d < 3; ++d) ph.inv_h[d] = 1.0 / ((M == 2 ? 12.0 : 60.0) * (kTwoPi / cfg->n[d]));
  double2* S = (double2*)(ws + pl.off_S);
  double2* tw = (double2*)(ws + pl.off_tw);
  double* part = (double*)(ws + pl.off_part);
  double* mid = (double*)(ws + pl.off_mid);
  double* sums = (double*)(ws + pl.off_sums);
  auto* hist = (unsigned long long*)(ws + pl.off_hist);
  double* spart = (double*)(ws + pl.off_spart);
  int* hdr = (int*)(ws + pl.off_hdr);
  double* smid = (double*)(ws + pl.off_smid);
  double2* eo = (double2*)(ws + pl.off_eo);
  const int nshell = prm->nshell, nb = prm->nbins;
  const int64_t N = (int64_t)pl.nx * pl.ny * pl.nz;
  double* o_scal = out + 2 * nshell;
  double* o_cnt = o_scal + AT_DIAG_N_SCALARS;

  hipLaunchKernelGGL(k_twiddle, dim3((pl.ntw + 255) / 256), dim3(256), 0, st, tw, pl.ntw);
  const dim3 pblk(kPtsBX, kPtsBY);
  hipLaunchKernelGGL((k_diag_pts<T, M>), pl.pts_grid, pblk, 0, st, q, pl.nx, pl.ny, pl.nz, ph, part, eo);
  hipLaunchKernelGGL(k_mom_reduce, dim3(kRed), dim3(kThreads), 0, st, (const double*)part, pl.nblk_pts, mid);
  hipLaunchKernelGGL(k_mom_final, dim3(1), dim3(kThreads), 0, st, (const double*)mid, (double)N, sums, o_scal);
  const int nh2 = 2 * (nb + 1);
  hipLaunchKernelGGL(k_zero_u64, dim3((nh2 + 255) / 256), dim3(256), 0, st, hist, nh2);
  hipLaunchKernelGGL(k_diag_hist, dim3((unsigned)((N + kThreads * kHistPts - 1) / (kThreads * kHistPts))), dim3(kThreads),
                     (size_t)nh2 * sizeof(unsigned int), st, (const double2*)eo, N, (const double*)sums, hist, nb,
                     (double)nb / prm->eps_max, (double)nb / prm->ens_max);
  hipLaunchKernelGGL(k_counts_out, dim3((nh2 + 255) / 256), dim3(256), 0, st, (const unsigned long long*)hist, nh2,
                     o_cnt);

  const int64_t fstride = (int64_t)pl.nz * pl.ny * pl.px;
  const Axis ax = make_axis(pl.nx, pl.ntw), ay = make_axis(pl.ny, pl.ntw), az = make_axis(pl.nz, pl.ntw);
  const int64_t nrows = (int64_t)pl.ny * pl.nz;
  hipLaunchKernelGGL((k_fft_x<T>), dim3((unsigned)(nrows / pl.rows)), dim3(kThreads),
                     (size_t)pl.rows * 2 * padded(pl.nx) * sizeof(double2), st, q, pl.nx, N, pl.rows, ax,
                     (const double2*)tw, ph, S, pl.px, fstride);
  hipLaunchKernelGGL(k_fft_y, dim3(pl.nbxy, pl.nz, 4), dim3(kThreadsYZ), (size_t)pl.ny * pl.bxy * sizeof(double2), st,
                     S, pl.nx, pl.ny, pl.px, pl.bxy, ay, (const double2*)tw, fstride);
  const double inv_n2 = 1.0 / ((double)N * (double)N);
  hipLaunchKernelGGL(k_fft_z_shell, dim3(pl.nbxz, pl.ny, 4), dim3(kThreadsYZ), (size_t)pl.nz * pl.bxz * sizeof(double2),
                     st, (const double2*)S, pl.nx, pl.ny, pl.nz, pl.px, pl.bxz, ay, az, (const double2*)tw, fstride,
                     nshell, (int)pl.spanmax, spart, hdr, inv_n2);
  hipLaunchKernelGGL(k_shell_reduce1, dim3(kRed), dim3(kThreads), 0, st, (const double*)spart, (const int*)hdr,
                     pl.nwgz, (int64_t)3 * pl.ny * pl.nbxz, (int)pl.spanmax, nshell, smid);
  hipLaunchKernelGGL(k_shell_reduce2, dim3((nshell + 255) / 256), dim3(256), 0, st, (const double*)smid, nshell, out);
  HIP_TRY(hipGetLastError());
  return AT_OK;
}

}  // namespace

extern "C" {

size_t at_diag_workspace_bytes(const at_config* cfg, const at_diag_params* prm) {
  Plan pl;
  if (plan_of(cfg, prm, &pl)) return 0;
  return pl.total;
}

int at_field_diagnostics(const at_config* cfg, const void* dev_q, void* dev_ws, size_t ws_bytes,
                         const at_diag_params* prm, double* dev_out, void* hip_stream) {
  Plan pl;
  int rc = plan_of(cfg, prm, &pl);
  if (rc) return rc;
  if (!dev_q || !dev_ws || !dev_out) return fail(AT_E_INVAL, "NULL field, workspace or output pointer");
  if (ws_bytes < pl.total || ((uintptr_t)dev_ws & 255))
    return fail(AT_E_WORKSPACE, "diagnostics workspace smaller than at_diag_workspace_bytes or not 256-byte aligned");
  const hipStream_t st = (hipStream_t)hip_stream;
  uint8_t* ws = (uint8_t*)dev_ws;
  if (cfg->precision == AT_FP32)
    return cfg->order == 6 ? run_diag<float, 3>(cfg, pl, prm, (const float*)dev_q, ws, dev_out, st)
                           : run_diag<float, 2>(cfg, pl, prm, (const float*)dev_q, ws, dev_out, st);
  return cfg->order == 6 ? run_diag<double, 3>(cfg, pl, prm, (const double*)dev_q, ws, dev_out, st)
                         : run_diag<double, 2>(cfg, pl, prm, (const double*)dev_q, ws, dev_out, st);
}

}  // extern "C"
