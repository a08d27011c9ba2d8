// Sixth-order AT step (gfx950): the (1,6) first derivative of Appendix B (Table atschemes, (1,6)
// rows) in the flux form of the fourth-order path, with three ghost layers per face and ghost
// values extrapolated from four published levels (cubic in time; the Appendix B weights at c_s = 0).
//
// Work decomposition.  A workgroup owns a BX x BY column tile that lies inside one PE along x and y
// (the PE edges are multiples of the tile's, chosen by the host) and marches through the whole z
// extent of one PE.  Every point outside the workgroup's box that a stencil reaches is therefore
// across exactly one face of the workgroup's own PE, or inside that PE: a point across a face whose
// delay k is >= 1 takes the extrapolated value w_0 v^{n-k} + w_1 v^{n-k-1} + w_2 v^{n-k-2} +
// w_3 v^{n-k-3} (kappa = k + c_s), any other point its current value.  Each stage is two launches:
//
//  k6_gradflux: primitives, the 12 velocity and temperature gradients at the tile's points (x, y
//    from an LDS plane with a 3-point halo, z from a 7-plane register window of the column), the
//    total fluxes F_x, F_y, F_z (written to the flux buffer), and at stage 1 the publication of the
//    three layers next to each PE face (u, v, w, T and the face-normal flux) into ring slot n mod R;
//  k6_divupdate: the flux divergence (F_x, F_y through LDS planes with a 3-point halo, F_z through a
//    7-plane register window) with ghost fluxes from the ring across delayed faces, then the
//    low-storage RK3 (or Adams-Bashforth) update and the FP64 block totals, or the RHS output.
//
// The fluxes make one round trip through HBM (15 words written, then read), which the fused
// fourth-order kernel avoids; in exchange every point's flux is computed once.
#include "atns_internal.h"

namespace atns {
namespace {

constexpr int kM6 = 3;  // layers per face

template <typename T>
struct A6 {
  const T* q;
  T* q_out;
  T* dq;
  T* flux;           // [3][5][N]: F_d of conserved component c at [(d 5 + c) N + i]
  T* ring;
  T* gv;             // extrapolated values behind the faces, ring-slot layout: this stage's (stage
                     // kernels), or the first of nst consecutive ones (k6_ghosts)
  T* rhs_out;
  const int8_t* delays;  // [ntiles][6] for this step
  double* tot_part;
  uint32_t N, plane;
  uint32_t slab0, slab1, slab2, rdir1, rdir2, rslot;
  int nx, ny, nz, px, py, pz, ex, ey, ez;
  int bx, by;        // tile (columns in x and y), dividing ex and ey
  int gbx, gby;      // workgroups along x and y
  int R, step_mod_r, publish, store_dq, mode;
  T cs;              // c_s of this stage
  T cs3[3];          // k6_ghosts: c_s of each stage it forms
  int nst;
  T i60x, i60y, i60z, gas_r, inv_cv, cp_over_pr, mu_ref, inv_tref, mu_exp;
  T rk_a, rk_b, dt, c_prev;
  double vol;
};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ T rcp6(T x) { return T(1) / x; }
template <>
__device__ __forceinline__ float rcp6<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ T visc6(const A6<T>& a, T t) { return a.mu_ref * pow(t * a.inv_tref, a.mu_exp); }
template <>
__device__ __forceinline__ float visc6<float>(const A6<float>& a, float t) {
  return a.mu_ref * __builtin_amdgcn_exp2f(a.mu_exp * __builtin_amdgcn_logf(t * a.inv_tref));
}

// u, v, w, T of conserved values q (rho, m, E).
template <typename T>
__device__ __forceinline__ void prims(const T q[5], T inv_cv, T& u, T& v, T& w, T& t) {
  const T ri = rcp6<T>(q[0]);
  u = q[1] * ri;
  v = q[2] * ri;
  w = q[3] * ri;
  t = (q[4] * ri - T(0.5) * (u * u + v * v + w * w)) * inv_cv;
}

template <typename T>
__device__ __forceinline__ void load_prims(const A6<T>& a, uint32_t i, T& u, T& v, T& w, T& t) {
  T q[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = a.q[c * a.N + i];
  prims<T>(q, a.inv_cv, u, v, w, t);
}

// The (1,6) central numerator: -v(-3) + 9 v(-2) - 45 v(-1) + 45 v(+1) - 9 v(+2) + v(+3).
template <typename T>
__device__ __forceinline__ T c6(T m3, T m2, T m1, T p1, T p2, T p3) {
  return (T(9) * m2 - m3) + T(45) * (p1 - m1) + (p3 - T(9) * p2);
}

// Cubic extrapolation weights to kappa = k + c_s from levels n-k .. n-k-3.
template <typename T>
__device__ __forceinline__ void weights6(T kap, T w[4]) {
  w[0] = (kap + T(1)) * (kap + T(2)) * (kap + T(3)) * T(1.0 / 6.0);
  w[1] = -kap * (kap + T(2)) * (kap + T(3)) * T(0.5);
  w[2] = kap * (kap + T(1)) * (kap + T(3)) * T(0.5);
  w[3] = -kap * (kap + T(1)) * (kap + T(2)) * T(1.0 / 6.0);
}

// Ring element offset (slot 0, component 0) of direction d at global point (x, y, z) on one of the
// six published layers of its PE along d: layer jp = 6 t + (l < 3 ? l : l - e + 6).
template <typename T>
__device__ __forceinline__ uint32_t ring_off6(const A6<T>& a, int d, int x, int y, int z) {
  if (d == 0) {
    const int t = x / a.ex, l = x - t * a.ex;
    const int jp = 6 * t + (l < kM6 ? l : l - a.ex + 2 * kM6);
    return ((uint32_t)z * a.ny + y) * (uint32_t)(6 * a.px) + jp;
  }
  if (d == 1) {
    const int t = y / a.ey, l = y - t * a.ey;
    const int jp = 6 * t + (l < kM6 ? l : l - a.ey + 2 * kM6);
    return a.rdir1 + ((uint32_t)z * (6 * a.py) + jp) * (uint32_t)a.nx + x;
  }
  const int t = z / a.ez, l = z - t * a.ez;
  const int jp = 6 * t + (l < kM6 ? l : l - a.ez + 2 * kM6);
  return a.rdir2 + ((uint32_t)jp * a.ny + y) * (uint32_t)a.nx + x;
}

template <typename T>
__device__ __forceinline__ uint32_t slab6(const A6<T>& a, int d) {
  return d == 0 ? a.slab0 : (d == 1 ? a.slab1 : a.slab2);
}

// Extrapolated value of ring component `comp` (0..3 u, v, w, T; 4..8 face-normal flux) at ring
// offset `off` of direction d, as the PE reading it across its delayed face sees it at this stage
// (formed by k6_ghosts for that reader's delay).
template <typename T>
__device__ __forceinline__ T ghost6(const A6<T>& a, int d, int comp, uint32_t off) {
  return a.gv[off + (uint32_t)comp * slab6(a, d)];
}

// Extrapolated values behind the PE faces for the stages of one step (Sec. 2.1, Eq. at; Appendix
// B, (1,6) rows), one thread per element e of a ring slot.  Element e (direction d, component c,
// layer jp = 6 t + j of PE t along d) is read across a face by one PE only, its neighbour on the
// layer's side: PE t - 1 across its upper face for the lower layers (j < 3), PE t + 1 across its
// lower face for the upper ones.  With that reader's delay k >= 1, stage s gets the cubic
// extrapolation to kappa = k + c_s of levels n - k .. n - k - 3, written at e of its slot-sized
// buffer; elements whose reader is not delayed are left alone (no stage reads them).  The four
// levels are read once for all the stages, coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k6_ghosts(A6<T> a) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= a.rslot) return;
  const int d = e < a.rdir1 ? 0 : (e < a.rdir2 ? 1 : 2);
  const uint32_t pos = (e - (d == 0 ? 0u : (d == 1 ? a.rdir1 : a.rdir2))) % slab6(a, d);
  int jp, tx, ty, tz;
  if (d == 0) {  // pos = (z ny + y) 6 px + jp
    const uint32_t w6 = 6u * (uint32_t)a.px, zy = pos / w6;
    jp = (int)(pos - zy * w6);
    ty = (int)(zy % (uint32_t)a.ny) / a.ey;
    tz = (int)(zy / (uint32_t)a.ny) / a.ez;
    tx = jp / 6;
  } else if (d == 1) {  // pos = (z 6 py + jp) nx + x
    const uint32_t r = pos / (uint32_t)a.nx, h6 = 6u * (uint32_t)a.py;
    tx = (int)(pos - r * (uint32_t)a.nx) / a.ex;
    jp = (int)(r % h6);
    tz = (int)(r / h6) / a.ez;
    ty = jp / 6;
  } else {  // pos = (jp ny + y) nx + x
    const uint32_t r = pos / (uint32_t)a.nx;
    tx = (int)(pos - r * (uint32_t)a.nx) / a.ex;
    ty = (int)(r % (uint32_t)a.ny) / a.ey;
    jp = (int)(r / (uint32_t)a.ny);
    tz = jp / 6;
  }
  const bool low = jp - 6 * (jp / 6) < kM6;
  const int np = d == 0 ? a.px : (d == 1 ? a.py : a.pz);
  int t = jp / 6;
  t = low ? (t == 0 ? np - 1 : t - 1) : (t == np - 1 ? 0 : t + 1);
  tx = d == 0 ? t : tx;
  ty = d == 1 ? t : ty;
  tz = d == 2 ? t : tz;
  const int k = a.delays[((tz * a.py + ty) * a.px + tx) * 6 + 2 * d + (low ? 1 : 0)];
  if (k <= 0) return;
  T lev[4];
  int s = a.step_mod_r - k;
  s += s < 0 ? a.R : 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    lev[l] = a.ring[(uint32_t)s * a.rslot + e];
    s = s == 0 ? a.R - 1 : s - 1;
  }
  for (int st = 0; st < a.nst; ++st) {
    T w[4];
    weights6<T>(T(k) + a.cs3[st], w);
    T v = T(0);
#pragma unroll
    for (int l = 0; l < 4; ++l) v += w[l] * lev[l];
    __builtin_nontemporal_store(v, a.gv + (uint32_t)st * a.rslot + e);
  }
}

// Workgroups are dealt to the 8 XCDs in turn (dispatch index w to XCD w mod 8), each with its own
// L2.  Logical workgroup xcd_major(w, nb) gives each XCD a contiguous range of tiles, so the tiles
// whose 3-point halos overlap run on the same L2 (a bijection of [0, nb)).
constexpr uint32_t kNumXcd = 8;
__device__ __forceinline__ uint32_t xcd_major(uint32_t w, uint32_t nb) {
  const uint32_t c = w % kNumXcd, i = w / kNumXcd, q = nb / kNumXcd, r = nb % kNumXcd;
  return c * q + min(c, r) + i;
}

// Workgroup decode: tile (bkx, bky), z-PE bkz of the logical workgroup, which is returned.
template <typename T>
__device__ __forceinline__ uint32_t decode6(const A6<T>& a, int& bkx, int& bky, int& bkz) {
  const uint32_t L = xcd_major(blockIdx.x, gridDim.x);
  const int b = (int)L;
  const int gxy = a.gbx * a.gby;
  bkz = b / gxy;
  const int r = b - bkz * gxy;
  bky = r / a.gbx;
  bkx = r - bky * a.gbx;
  return L;
}

// Primitives u, v, w, T at global (x, y, z) as the workgroup's PE sees them: across its face f
// (crossed = the face index 0..5, or -1 inside the PE) with delay k >= 1 the extrapolation of the
// published values, else the current state.
template <typename T>
__device__ __forceinline__ void seen_prims(const A6<T>& a, int x, int y, int z, int crossed, const int kf[6],
                                           T& u, T& v, T& w, T& t) {
  x = wrapi(x, a.nx);
  y = wrapi(y, a.ny);
  z = wrapi(z, a.nz);
  if (crossed >= 0 && kf[crossed] > 0) {
    const int d = crossed >> 1;
    const uint32_t o = ring_off6(a, d, x, y, z);
    u = ghost6(a, d, 0, o);
    v = ghost6(a, d, 1, o);
    w = ghost6(a, d, 2, o);
    t = ghost6(a, d, 3, o);
  } else {
    load_prims(a, ((uint32_t)z * a.ny + y) * (uint32_t)a.nx + x, u, v, w, t);
  }
}

// Face-normal flux F_d, component c, at global (x, y, z) as the workgroup's PE sees it.
template <typename T>
__device__ __forceinline__ T seen_flux(const A6<T>& a, int d, int c, int x, int y, int z, int crossed,
                                       const int kf[6]) {
  x = wrapi(x, a.nx);
  y = wrapi(y, a.ny);
  z = wrapi(z, a.nz);
  if (crossed >= 0 && kf[crossed] > 0) return ghost6(a, d, 4 + c, ring_off6(a, d, x, y, z));
  return a.flux[(uint32_t)(d * 5 + c) * a.N + ((uint32_t)z * a.ny + y) * (uint32_t)a.nx + x];
}

template <typename T>
__global__ __launch_bounds__(256) void k6_gradflux(A6<T> a) {
  extern __shared__ unsigned char s_raw[];
  const int BX = a.bx, BY = a.by, LW = BX + 2 * kM6, LH = BY + 2 * kM6;
  T* s_p = reinterpret_cast<T*>(s_raw);  // [4][LH][LW]
  const int plane_lds = LW * LH;
  int bkx, bky, bkz;
  decode6(a, bkx, bky, bkz);
  const int tid = threadIdx.x, lx = tid % BX, ly = tid / BX;
  const int x0 = bkx * BX, y0 = bky * BY, z0 = bkz * a.ez, z1 = z0 + a.ez;
  const int tx = x0 / a.ex, ty = y0 / a.ey, tz = bkz;
  const int X = x0 + lx, Y = y0 + ly;
  int kf[6];
  {
    const int8_t* k = a.delays + ((tz * a.py + ty) * a.px + tx) * 6;
#pragma unroll
    for (int f = 0; f < 6; ++f) kf[f] = k[f];
  }
  const int pxl = tx * a.ex, pxh = pxl + a.ex, pyl = ty * a.ey, pyh = pyl + a.ey;
  // z window: u, v, w, T at planes zc-3 .. zc+3 (slot j = 0 .. 6)
  T win[4][7];
  auto zcross = [&](int z) { return z < z0 ? 4 : (z >= z1 ? 5 : -1); };
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int z = z0 - 3 + j;
    seen_prims(a, X, Y, z, zcross(z), kf, win[0][j], win[1][j], win[2][j], win[3][j]);
  }
  const int nhalo = 2 * kM6 * (BX + BY);
  T* rb = a.ring + (uint32_t)a.step_mod_r * a.rslot;
  for (int zc = z0; zc < z1; ++zc) {
    // density and energy of this plane, issued first so that they arrive in the round trip of the
    // window and halo fetches (a wave's loads complete in order)
    const uint32_t i = ((uint32_t)zc * a.ny + Y) * (uint32_t)a.nx + X;
    const T rho = a.q[i], E = a.q[4 * a.N + i];
    {
      const int z = zc + 3;
      seen_prims(a, X, Y, z, zcross(z), kf, win[0][6], win[1][6], win[2][6], win[3][6]);
    }
    // LDS plane zc: own points and the x / y halos (3 points beyond each side of the tile)
#pragma unroll
    for (int c = 0; c < 4; ++c) s_p[c * plane_lds + (ly + kM6) * LW + lx + kM6] = win[c][3];
    for (int h = tid; h < nhalo; h += BX * BY) {
      int hx, hy;
      if (h < 2 * kM6 * BY) {  // x halo
        const int side = h / (kM6 * BY), r = h % (kM6 * BY);
        hy = y0 + r / kM6;
        hx = side == 0 ? x0 - kM6 + r % kM6 : x0 + BX + r % kM6;
      } else {
        const int h2 = h - 2 * kM6 * BY, side = h2 / (kM6 * BX), r = h2 % (kM6 * BX);
        hx = x0 + r % BX;
        hy = side == 0 ? y0 - kM6 + r / BX : y0 + BY + r / BX;
      }
      const int crossed = hx < pxl ? 0 : hx >= pxh ? 1 : hy < pyl ? 2 : hy >= pyh ? 3 : -1;
      T u, v, w, t;
      seen_prims(a, hx, hy, zc, crossed, kf, u, v, w, t);
      const int li = (hy - y0 + kM6) * LW + (hx - x0 + kM6);
      s_p[0 * plane_lds + li] = u;
      s_p[1 * plane_lds + li] = v;
      s_p[2 * plane_lds + li] = w;
      s_p[3 * plane_lds + li] = t;
    }
    __syncthreads();
    T G[kNGrad];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T* p = s_p + c * plane_lds + (ly + kM6) * LW + lx + kM6;
      const T gx = c6(p[-3], p[-2], p[-1], p[1], p[2], p[3]) * a.i60x;
      const T gy = c6(p[-3 * LW], p[-2 * LW], p[-LW], p[LW], p[2 * LW], p[3 * LW]) * a.i60y;
      const T gz = c6(win[c][0], win[c][1], win[c][2], win[c][4], win[c][5], win[c][6]) * a.i60z;
      const int base = c < 3 ? 3 * c : 9;
      G[base + 0] = gx;
      G[base + 1] = gy;
      G[base + 2] = gz;
    }
    const T u = win[0][3], v = win[1][3], w = win[2][3], t = win[3][3];
    const T mu = visc6<T>(a, t);
    const T kt = mu * a.cp_over_pr;
    const T th = G[0] + G[4] + G[8];
    const T s00 = mu * (G[0] + G[0]) - T(2.0 / 3.0) * mu * th;
    const T s11 = mu * (G[4] + G[4]) - T(2.0 / 3.0) * mu * th;
    const T s22 = mu * (G[8] + G[8]) - T(2.0 / 3.0) * mu * th;
    const T s01 = mu * (G[1] + G[3]);
    const T s02 = mu * (G[2] + G[6]);
    const T s12 = mu * (G[5] + G[7]);
    const T p = rho * a.gas_r * t;
    const T mx = rho * u, my = rho * v, mz = rho * w, Ep = E + p;
    T F[3][5];
    F[0][0] = mx;
    F[0][1] = mx * u + p - s00;
    F[0][2] = my * u - s01;
    F[0][3] = mz * u - s02;
    F[0][4] = Ep * u - (u * s00 + v * s01 + w * s02) - kt * G[9];
    F[1][0] = my;
    F[1][1] = mx * v - s01;
    F[1][2] = my * v + p - s11;
    F[1][3] = mz * v - s12;
    F[1][4] = Ep * v - (u * s01 + v * s11 + w * s12) - kt * G[10];
    F[2][0] = mz;
    F[2][1] = mx * w - s02;
    F[2][2] = my * w - s12;
    F[2][3] = mz * w + p - s22;
    F[2][4] = Ep * w - (u * s02 + v * s12 + w * s22) - kt * G[11];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int c = 0; c < 5; ++c)  // streamed out: read by the next launch, far beyond the caches
        __builtin_nontemporal_store(F[d][c], a.flux + (uint32_t)(d * 5 + c) * a.N + i);
    if (a.publish) {
      const int lxe = X - pxl, lye = Y - pyl, lze = zc - z0;
      const bool on[3] = {lxe < kM6 || lxe >= a.ex - kM6, lye < kM6 || lye >= a.ey - kM6,
                          lze < kM6 || lze >= a.ez - kM6};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (!on[d]) continue;
        const uint32_t o = ring_off6(a, d, X, Y, zc), sl = slab6(a, d);
        T* b = rb + o;
        b[0] = u;
        b[sl] = v;
        b[2 * sl] = w;
        b[3 * sl] = t;
#pragma unroll
        for (int c = 0; c < 5; ++c) b[(4 + c) * sl] = F[d][c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 6; ++j) win[c][j] = win[c][j + 1];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k6_divupdate(A6<T> a) {
  extern __shared__ unsigned char s_raw[];
  const int BX = a.bx, BY = a.by, LWX = BX + 2 * kM6, LHY = BY + 2 * kM6;
  T* s_fx = reinterpret_cast<T*>(s_raw);  // [5][BY][LWX]
  T* s_fy = s_fx + 5 * BY * LWX;          // [5][LHY][BX]
  double* s_red = reinterpret_cast<double*>(s_fy + 5 * LHY * BX + ((5 * LHY * BX + 5 * BY * LWX) & 1));
  int bkx, bky, bkz;
  const uint32_t blk = decode6(a, bkx, bky, bkz);  // slot of the FP64 block totals
  const int tid = threadIdx.x, lx = tid % BX, ly = tid / BX, NT = BX * BY;
  const int x0 = bkx * BX, y0 = bky * BY, z0 = bkz * a.ez, z1 = z0 + a.ez;
  const int tx = x0 / a.ex, ty = y0 / a.ey, tz = bkz;
  const int X = x0 + lx, Y = y0 + ly;
  int kf[6];
  {
    const int8_t* k = a.delays + ((tz * a.py + ty) * a.px + tx) * 6;
#pragma unroll
    for (int f = 0; f < 6; ++f) kf[f] = k[f];
  }
  const int pxl = tx * a.ex, pxh = pxl + a.ex, pyl = ty * a.ey, pyh = pyl + a.ey;
  auto zcross = [&](int z) { return z < z0 ? 4 : (z >= z1 ? 5 : -1); };
  T fz[5][7];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int z = z0 - 3 + j;
#pragma unroll
    for (int c = 0; c < 5; ++c) fz[c][j] = seen_flux(a, 2, c, X, Y, z, zcross(z), kf);
  }
  double tsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int nhx = 2 * kM6 * BY, nhy = 2 * kM6 * BX;
  const bool upd = a.mode != kModeRhsH, keep = a.rk_a != T(0) || a.c_prev != T(0);
  for (int zc = z0; zc < z1; ++zc) {
    const uint32_t i = ((uint32_t)zc * a.ny + Y) * (uint32_t)a.nx + X;
    // this plane's state and RK register, issued before the fluxes so that they arrive in the
    // same round trip (a wave's loads complete in order)
    T qv[5], prev[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      qv[c] = upd ? a.q[(uint32_t)c * a.N + i] : T(0);
      prev[c] = upd && keep ? __builtin_nontemporal_load(a.dq + (uint32_t)c * a.N + i) : T(0);
    }
    {
      const int z = zc + 3;
#pragma unroll
      for (int c = 0; c < 5; ++c) fz[c][6] = seen_flux(a, 2, c, X, Y, z, zcross(z), kf);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      s_fx[(c * BY + ly) * LWX + lx + kM6] = a.flux[(uint32_t)c * a.N + i];
      s_fy[(c * LHY + ly + kM6) * BX + lx] = a.flux[(uint32_t)(5 + c) * a.N + i];
    }
    for (int h = tid; h < nhx + nhy; h += NT) {
      if (h < nhx) {  // F_x beyond the tile's x sides
        const int side = h / (kM6 * BY), r = h % (kM6 * BY);
        const int hy = y0 + r / kM6, hx = side == 0 ? x0 - kM6 + r % kM6 : x0 + BX + r % kM6;
        const int crossed = hx < pxl ? 0 : hx >= pxh ? 1 : -1;
#pragma unroll
        for (int c = 0; c < 5; ++c)
          s_fx[(c * BY + (hy - y0)) * LWX + hx - x0 + kM6] = seen_flux(a, 0, c, hx, hy, zc, crossed, kf);
      } else {  // F_y beyond the tile's y sides
        const int h2 = h - nhx, side = h2 / (kM6 * BX), r = h2 % (kM6 * BX);
        const int hx = x0 + r % BX, hy = side == 0 ? y0 - kM6 + r / BX : y0 + BY + r / BX;
        const int crossed = hy < pyl ? 2 : hy >= pyh ? 3 : -1;
#pragma unroll
        for (int c = 0; c < 5; ++c)
          s_fy[(c * LHY + hy - y0 + kM6) * BX + hx - x0] = seen_flux(a, 1, c, hx, hy, zc, crossed, kf);
      }
    }
    __syncthreads();
    T rhs[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const T* px_ = s_fx + (c * BY + ly) * LWX + lx + kM6;
      const T* py_ = s_fy + (c * LHY + ly + kM6) * BX + lx;
      const T dfx = c6(px_[-3], px_[-2], px_[-1], px_[1], px_[2], px_[3]) * a.i60x;
      const T dfy = c6(py_[-3 * BX], py_[-2 * BX], py_[-BX], py_[BX], py_[2 * BX], py_[3 * BX]) * a.i60y;
      const T dfz = c6(fz[c][0], fz[c][1], fz[c][2], fz[c][4], fz[c][5], fz[c][6]) * a.i60z;
      rhs[c] = -((dfx + dfy) + dfz);
    }
    if (a.mode == kModeRhsH) {
#pragma unroll
      for (int c = 0; c < 5; ++c) __builtin_nontemporal_store(rhs[c], a.rhs_out + (uint32_t)c * a.N + i);
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const T d = a.rk_a * prev[c] + a.dt * rhs[c];
        const T inc = a.rk_b * d + a.c_prev * prev[c];
        if (a.store_dq) __builtin_nontemporal_store(d, a.dq + (uint32_t)c * a.N + i);
        __builtin_nontemporal_store(qv[c] + inc, a.q_out + (uint32_t)c * a.N + i);
        tsum[c] += a.c_prev != T(0) ? (double)inc : (double)d;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
      for (int j = 0; j < 6; ++j) fz[c][j] = fz[c][j + 1];
  }
  if (a.mode != kModeStepH) return;  // uniform across the grid
  // FP64 block sums in a fixed order: B_s * sum(dQ) * h^3 (or the Adams-Bashforth increment)
  for (int c = 0; c < 5; ++c) {
    s_red[tid] = tsum[c];
    __syncthreads();
    for (int len = 128; len > 0; len >>= 1) {
      if (tid < len && tid + len < NT) s_red[tid] += s_red[tid + len];
      __syncthreads();
    }
    if (tid == 0) {
      const double scale = a.c_prev != T(0) ? 1.0 : (double)a.rk_b;
      a.tot_part[blk * kNQ + c] += scale * s_red[0] * a.vol;
    }
    __syncthreads();
  }
}

template <typename T>
A6<T> pack6(const Stage6Args<T>& s) {
  A6<T> a{};
  const Geom& g = s.g;
  a.q = s.q;
  a.q_out = s.q_out;
  a.dq = s.dq;
  a.flux = s.flux;
  a.ring = s.ring;
  a.gv = s.gv;
  a.rhs_out = s.rhs_out;
  a.delays = s.delays;
  a.tot_part = s.tot_part;
  a.N = (uint32_t)g.npts;
  a.plane = (uint32_t)g.n[0] * (uint32_t)g.n[1];
  a.slab0 = (uint32_t)g.slab[0];
  a.slab1 = (uint32_t)g.slab[1];
  a.slab2 = (uint32_t)g.slab[2];
  a.rdir1 = (uint32_t)g.ring_dir_off[1];
  a.rdir2 = (uint32_t)g.ring_dir_off[2];
  a.rslot = (uint32_t)g.ring_slot;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.px = g.p[0];
  a.py = g.p[1];
  a.pz = g.p[2];
  a.ex = g.e[0];
  a.ey = g.e[1];
  a.ez = g.e[2];
  a.bx = s.bx;
  a.by = s.by;
  a.gbx = g.n[0] / s.bx;
  a.gby = g.n[1] / s.by;
  a.R = g.R;
  a.step_mod_r = s.step_mod_r;
  a.publish = s.publish;
  a.store_dq = s.store_dq;
  a.mode = s.mode;
  a.cs = s.cs;
  for (int st = 0; st < 3; ++st) a.cs3[st] = s.cs3[st];
  a.nst = s.nst;
  for (int d = 0; d < 3; ++d) (d == 0 ? a.i60x : d == 1 ? a.i60y : a.i60z) = s.i60h[d];
  a.gas_r = s.cf.gas_r;
  a.inv_cv = s.cf.inv_cv;
  a.cp_over_pr = s.cf.cp_over_pr;
  a.mu_ref = s.cf.mu_ref;
  a.inv_tref = s.cf.inv_tref;
  a.mu_exp = s.cf.mu_exp;
  a.rk_a = s.rk_a;
  a.rk_b = s.rk_b;
  a.dt = s.dt;
  a.c_prev = s.c_prev;
  a.vol = s.vol;
  return a;
}

}  // namespace

void tile6_of(const Geom& g, int* bx, int* by) {
  int b = 32;
  while (b > 1 && g.e[0] % b) b >>= 1;
  int c = 8;
  while (c > 1 && g.e[1] % c) c >>= 1;
  *bx = b;
  *by = c;
}

int64_t blocks6(const Geom& g) {
  int bx, by;
  tile6_of(g, &bx, &by);
  return (int64_t)(g.n[0] / bx) * (g.n[1] / by) * g.p[2];
}

template <typename T>
hipError_t launch_stage6(const Stage6Args<T>& s, bool gradflux, hipStream_t stream) {
  const A6<T> a = pack6<T>(s);
  const Geom& g = s.g;
  const dim3 grid((unsigned)blocks6(g)), block((unsigned)(s.bx * s.by));
  if (gradflux) {
    const size_t lds = sizeof(T) * 4 * (s.bx + 2 * kM6) * (s.by + 2 * kM6);
    hipLaunchKernelGGL(k6_gradflux<T>, grid, block, lds, stream, a);
  } else {
    const size_t nel = (size_t)5 * s.by * (s.bx + 2 * kM6) + (size_t)5 * (s.by + 2 * kM6) * s.bx;
    const size_t lds = sizeof(T) * (nel + (nel & 1)) + sizeof(double) * 256;
    hipLaunchKernelGGL(k6_divupdate<T>, grid, block, lds, stream, a);
  }
  return hipGetLastError();
}

template hipError_t launch_stage6<float>(const Stage6Args<float>&, bool, hipStream_t);
template hipError_t launch_stage6<double>(const Stage6Args<double>&, bool, hipStream_t);

template <typename T>
hipError_t launch_ghosts6(const Stage6Args<T>& s, hipStream_t stream) {
  if (s.nst < 1 || s.nst > 3 || !s.gv) return hipErrorInvalidValue;
  const A6<T> a = pack6<T>(s);
  const dim3 grid((unsigned)((a.rslot + 255u) / 256u)), block(256);
  hipLaunchKernelGGL(k6_ghosts<T>, grid, block, 0, stream, a);
  return hipGetLastError();
}

template hipError_t launch_ghosts6<float>(const Stage6Args<float>&, hipStream_t);
template hipError_t launch_ghosts6<double>(const Stage6Args<double>&, hipStream_t);

}  // namespace atns
