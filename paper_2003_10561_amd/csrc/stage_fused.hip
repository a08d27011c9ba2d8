// Fused RK-stage kernel of the AT compressible Navier-Stokes step (gfx950).
//
// One launch per Runge-Kutta stage does, for every grid point: primitives, the 12 velocity and
// temperature gradients, the total fluxes, the flux divergence, the forcing source and the
// low-storage RK3 update, plus (stage 1) the publication of the PE face layers into the ring.
// Stencil points across a PE face are replaced by the AT combination of published levels
// (Sec. 2.1, Eq. at; Appendix B, (1,4) rows) using the delay of the PE that owns the point being
// evaluated (every point - own or halo - is computed with its own PE's rules).
//
// Work decomposition.  A workgroup owns a BX x BY column tile and marches through a z chunk.
// One thread per column of the tile and of its 2-wide x and y halos (wave-uniform roles, see
// Tile), each keeping a five-plane register window of its column's primitives for the z
// derivatives and writing the current plane to LDS for the x and y derivatives; the remaining
// halo points the x / y derivatives need are loaded one plane ahead by the first threads.  The
// tile computes all three fluxes, the halo rows F_y and the halo columns F_x; F_x and F_y reach
// the tile through LDS, F_z stays in the owning thread and is scattered into a five-plane register
// accumulator, so the z divergence needs no LDS.  The state is read from one buffer and written
// to the other, so halo reads never see updated values.
//
// Indexing is 32-bit (element offsets below 2^32, checked by the host) and every per-column
// quantity is computed once; per-plane quantities are uniform across the workgroup.
#include <cstring>

#include "atns_internal.h"

namespace atns {
namespace {

constexpr int kModeStep = kModeStepH, kModeRhs = kModeRhsH, kModePublish = kModePublishH;

// Compact kernel arguments: what the stage needs, 32-bit where possible.
template <typename T>
struct FArgs {
  const T* q;
  T* q_out;
  T* dq;
  T* ring;
  const T* gv;         // AT views of the face layers for this stage (one ring slot's layout)
  T* rhs_out;
  const int8_t* delays;
  const T* ftab;
  const T* phase_y;
  const T* phase_z;
  const int* pair_kyz;
  double* tot_part;
  uint32_t N, plane;
  uint32_t slab0, slab1, slab2;
  uint32_t rdir1, rdir2, rslot;  // ring offsets of directions 1, 2 in a slot; slot size
  int nx, ny, nz, px, py, ex, ey, ez;
  int R, step_mod_r, npair, zchunk, publish, store_dq;
  int gbx, gby;  // workgroups along x and y (a batched launch decodes its local block with them)
  int views;     // batched ghost views: does this run read delayed levels at this stage
  T i12x, i12y, i12z, gas_r, inv_cv, cp_over_pr, mu_ref, inv_tref, mu_exp;
  T cstage, rk_a, rk_b, dt;
  double vol;
};

template <typename T>
__device__ __forceinline__ T frcp(T x) { return T(1) / x; }
template <>
__device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// mu = mu_ref (T / T_ref)^n
template <typename T>
__device__ __forceinline__ T visc(const FArgs<T>& a, T t) { return a.mu_ref * pow(t * a.inv_tref, a.mu_exp); }
template <>
__device__ __forceinline__ float visc<float>(const FArgs<float>& a, float t) {
  return a.mu_ref * __builtin_amdgcn_exp2f(a.mu_exp * __builtin_amdgcn_logf(t * a.inv_tref));
}

__device__ __forceinline__ int pmod(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int layer_of(int l, int e) { return l < 2 ? l : l - e + 4; }

// Ring element offset (slot 0, component 0) of direction d at a global point on a published layer.
template <typename T>
__device__ __forceinline__ uint32_t slab_off(const FArgs<T>& a, int d, int x, int y, int z) {
  if (d == 0) {
    const int t = x / a.ex;
    const int jp = 4 * t + layer_of(x - t * a.ex, a.ex);
    return ((uint32_t)z * a.ny + y) * (uint32_t)(4 * a.px) + jp;
  }
  if (d == 1) {
    const int t = y / a.ey;
    const int jp = 4 * t + layer_of(y - t * a.ey, a.ey);
    return a.rdir1 + ((uint32_t)z * (4 * a.py) + jp) * (uint32_t)a.nx + x;
  }
  const int t = z / a.ez;
  const int jp = 4 * t + layer_of(z - t * a.ez, a.ez);
  return a.rdir2 + ((uint32_t)jp * a.ny + y) * (uint32_t)a.nx + x;
}

template <typename T>
__device__ __forceinline__ uint32_t slab_size(const FArgs<T>& a, int d) {
  return d == 0 ? a.slab0 : (d == 1 ? a.slab1 : a.slab2);
}

// AT value of ring component `comp` (0..3 primitives u, v, w, T; 4..8 face-normal flux) of a face
// layer point at ring offset `off`, as seen from across its face at this stage: precomputed by
// k_ghost_views (the extrapolation sum_l w_l(k + c) v^{n-k-l} with the reading PE's delay k).
template <typename T>
__device__ __forceinline__ T ghost(const FArgs<T>& a, int d, int comp, uint32_t off, int k) {
  (void)k;
  return a.gv[off + (uint32_t)comp * slab_size(a, d)];
}

// Primitives from conserved values: rho, u, v, w, T.
template <typename T>
__device__ __forceinline__ void prim_of(const T q[5], T inv_cv, T& r, T& u, T& v, T& w, T& t) {
  r = q[0];
  const T ri = frcp<T>(q[0]);
  u = q[1] * ri;
  v = q[2] * ri;
  w = q[3] * ri;
  t = (q[4] * ri - T(0.5) * (u * u + v * v + w * w)) * inv_cv;
}

// Thread roles of a workgroup (one column of the z march each, wave-uniform):
//   [0, NOWN)            the BX x BY tile columns (fluxes F_x, F_y, F_z, divergence, update)
//   [NOWN, NOWN + NY2)   the 2 + 2 rows of y-halo columns (flux F_y only)
//   [.., NCOL)           the 2 + 2 columns of x-halo columns (flux F_x only)
// and, per plane, NXTRA plane-only points (x halo 3-4, y halo 3-4, the 16 corners) that feed the
// x / y derivatives of the halo columns, loaded one plane ahead by the first NXTRA threads.
template <int BX, int BY>
struct Tile {
  static constexpr int NOWN = BX * BY;
  static constexpr int NY2 = 4 * BX;
  static constexpr int NX2 = 4 * BY;
  static constexpr int NCOL = NOWN + NY2 + NX2;
  static constexpr int NT = ((NCOL + 63) / 64) * 64;
  static constexpr int NXTRA = 4 * BY + 4 * BX + 16;
  static constexpr int LW = BX + 8, LH = BY + 8;  // LDS plane: x halo 4, y halo 4
  static_assert(NXTRA <= NT, "every thread loads at most one plane-only point");
};

template <typename T>
__device__ __forceinline__ void set_grad(T G[kNGrad], int c, int d, T val) {
  switch (c) {
    case 0: G[0 + d] = val; break;
    case 1: G[3 + d] = val; break;
    case 2: G[6 + d] = val; break;
    default: G[9 + d] = val; break;
  }
}
template <typename T>
__device__ __forceinline__ void add5(T acc[kNQ], int c, T val) {
  switch (c) {
    case 0: acc[0] += val; break;
    case 1: acc[1] += val; break;
    case 2: acc[2] += val; break;
    case 3: acc[3] += val; break;
    default: acc[4] += val; break;
  }
}

// window element of component c (0 u, 1 v, 2 w, 3 T) at plane index j (plane zc - 2 + j)
#define WIN(c, j) s_win[5 * (c) + sl5[j]][wc]

// One workgroup of a stage: the BX x BY column tile (bkx, bky) and z chunk bkz of run `a`; `blk`
// is its slot among the run's workgroups for the FP64 totals.
template <typename T, int BX, int BY>
__device__ __forceinline__ void stage_body(const FArgs<T>& a, const int mode, const int bkx, const int bky,
                                           const int bkz, const uint32_t blk) {
  using TL = Tile<BX, BY>;
  constexpr int LW = TL::LW, LH = TL::LH;
  __shared__ T s_pr[2][4][LH][LW];       // u, v, w, T of a plane (two buffers: planes alternate)
  __shared__ T s_fx[2][5][BY][BX + 4];   // F_x on the tile rows, x halo 2
  __shared__ T s_fy[2][5][BY + 4][BX];   // F_y on the tile columns, y halo 2
  __shared__ double s_tsum[kNQ][TL::NOWN];  // FP64 running sums of dQ per tile column
  // per-column window of the z march (thread-private): u, v, w, T of 5 planes (ring slot
  // z mod 5, index 5 c + slot) and rho, E of 3 planes (index 20 + 3 (c - 4) + z mod 3)
  __shared__ T s_win[26][TL::NCOL];
  extern __shared__ unsigned char s_dyn[];  // forcing coefficients when forced
  T* s_force = reinterpret_cast<T*>(s_dyn);

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const uint32_t N = a.N, plane = a.plane;
  const int tid = threadIdx.x;
  const int x0 = bkx * BX, y0 = bky * BY, z0 = bkz * a.zchunk;
  const int xe = min(x0 + BX, nx), ye = min(y0 + BY, ny), z1 = min(z0 + a.zchunk, nz);

  // role and column of this thread
  const int role = tid < TL::NOWN ? 0 : (tid < TL::NOWN + TL::NY2 ? 1 : (tid < TL::NCOL ? 2 : 3));
  int X = x0, Y = y0;
  if (role == 0) {
    X = x0 + tid % BX;
    Y = y0 + tid / BX;
  } else if (role == 1) {
    const int j = tid - TL::NOWN, r = j / BX;
    X = x0 + j % BX;
    Y = r < 2 ? y0 - 2 + r : y0 + BY + r - 2;
  } else if (role == 2) {
    const int j = tid - TL::NOWN - TL::NY2, c = j / BY;
    X = c < 2 ? x0 - 2 + c : x0 + BX + c - 2;
    Y = y0 + j % BY;
  }
  const bool column = role < 3;
  const bool valid = role == 0 && X < xe && Y < ye;  // a point this workgroup updates
  const int px = X - x0 + 4, py = Y - y0 + 4;        // LDS plane coordinates
  const int gx = pmod(X, nx), gy = pmod(Y, ny);
  // plane-only point of this thread
  int ex_ = -1, exX = x0, exY = y0;
  if (tid < TL::NXTRA) {
    const int e = tid;
    if (e < 4 * BY) {
      const int c = e / BY;
      exX = c < 2 ? x0 - 4 + c : x0 + BX + c;
      exY = y0 + e % BY;
    } else if (e < 4 * BY + 4 * BX) {
      const int f = e - 4 * BY, r = f / BX;
      exX = x0 + f % BX;
      exY = r < 2 ? y0 - 4 + r : y0 + BY + r;
    } else {
      const int g = e - 4 * BY - 4 * BX, cx = g % 4, cy = g / 4;
      exX = cx < 2 ? x0 - 2 + cx : x0 + BX + cx - 2;
      exY = cy < 2 ? y0 - 2 + cy : y0 + BY + cy - 2;
    }
    ex_ = e;
  }
  const int epx = exX - x0 + 4, epy = exY - y0 + 4;
  const uint32_t xcol = (uint32_t)pmod(exY, ny) * nx + pmod(exX, nx);

  const int tx = gx / a.ex, ty = gy / a.ey;
  const int lxe = gx - tx * a.ex, lye = gy - ty * a.ey;
  const bool near_x = lxe < 2 || lxe >= a.ex - 2;
  const bool near_y = lye < 2 || lye >= a.ey - 2;
  const uint32_t col = (uint32_t)gy * nx + gx;
  const T* __restrict__ qin = a.q;
  const T inv_cv = a.inv_cv;

  // forcing coefficients B_kz,c(x, y) = sum over pairs with that kz of A[pair][x][c] e^{i ky y},
  // stored as [c][kz][re, im][BY][BX] (kz = 0 imaginary part unused)
  const bool forced = a.ftab != nullptr;
  if (forced && role == 0) {
    T b[3][3][2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int kz = 0; kz < 3; ++kz) b[c][kz][0] = b[c][kz][1] = T(0);
    for (int pi = 0; pi < a.npair; ++pi) {
      const int ky = a.pair_kyz[2 * pi], kz = a.pair_kyz[2 * pi + 1];
      const T* ey = a.phase_y + ((uint32_t)(ky + 2) * ny + gy) * 2;
      const T* A = a.ftab + ((uint32_t)pi * nx + gx) * 6;
      const T er = ey[0], ei = ey[1];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T pr_ = A[2 * c] * er - A[2 * c + 1] * ei;
        const T pim = A[2 * c] * ei + A[2 * c + 1] * er;
        if (kz == 0) {
          b[c][0][0] += pr_;
        } else if (kz == 1) {
          b[c][1][0] += pr_;
          b[c][1][1] += pim;
        } else {
          b[c][2][0] += pr_;
          b[c][2][1] += pim;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int kz = 0; kz < 3; ++kz) {
        s_force[(c * 6 + 2 * kz) * (BX * BY) + tid] = b[c][kz][0];
        s_force[(c * 6 + 2 * kz + 1) * (BX * BY) + tid] = b[c][kz][1];
      }
  }

  T raw[5], xraw[5];
  T acc[5][kNQ];
  if (role == 0) {
#pragma unroll
    for (int c = 0; c < kNQ; ++c) s_tsum[c][tid] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int c = 0; c < kNQ; ++c) acc[j][c] = T(0);
  const int wc = column ? tid : 0;
  if (column) {
    // planes z0-4 .. z0-1 into the window; z0 arrives through `raw`
#pragma unroll
    for (int j = 1; j < 5; ++j) {
      const int z = z0 - 5 + j;
      const uint32_t i = (uint32_t)pmod(z, nz) * plane + col;
      T q[5], r_, u_, v_, w_, t_;
#pragma unroll
      for (int c = 0; c < 5; ++c) q[c] = qin[c * N + i];
      prim_of<T>(q, inv_cv, r_, u_, v_, w_, t_);
      const int s5 = pmod(z, 5), s3 = pmod(z, 3);
      s_win[0 + s5][wc] = u_;
      s_win[5 + s5][wc] = v_;
      s_win[10 + s5][wc] = w_;
      s_win[15 + s5][wc] = t_;
      s_win[20 + s3][wc] = r_;
      s_win[23 + s3][wc] = q[4];
    }
    const uint32_t i0 = (uint32_t)pmod(z0, nz) * plane + col;
#pragma unroll
    for (int c = 0; c < 5; ++c) raw[c] = qin[c * N + i0];
  }
  if (ex_ >= 0) {
    const uint32_t i1 = (uint32_t)pmod(z0 - 2, nz) * plane + xcol;
#pragma unroll
    for (int c = 0; c < 5; ++c) xraw[c] = qin[c * N + i1];
  }
  // window plane z0, then the LDS plane z0 - 2 (buffer parity (z + 2) & 1)
  if (column) {
    T r_, u_, v_, w_, t_;
    prim_of<T>(raw, inv_cv, r_, u_, v_, w_, t_);
    const int s5 = pmod(z0, 5), s3 = pmod(z0, 3);
    s_win[0 + s5][wc] = u_;
    s_win[5 + s5][wc] = v_;
    s_win[10 + s5][wc] = w_;
    s_win[15 + s5][wc] = t_;
    s_win[20 + s3][wc] = r_;
    s_win[23 + s3][wc] = raw[4];
    if (z0 + 1 <= z1 + 3) {
      const uint32_t i = (uint32_t)pmod(z0 + 1, nz) * plane + col;
#pragma unroll
      for (int c = 0; c < 5; ++c) raw[c] = qin[c * N + i];
    }
    const int sp = pmod(z0 - 2, 5);
    const int b0 = z0 & 1;
    s_pr[b0][0][py][px] = s_win[0 + sp][wc];
    s_pr[b0][1][py][px] = s_win[5 + sp][wc];
    s_pr[b0][2][py][px] = s_win[10 + sp][wc];
    s_pr[b0][3][py][px] = s_win[15 + sp][wc];
  }
  if (ex_ >= 0) {
    T xr, xu, xv, xw, xt;
    prim_of<T>(xraw, inv_cv, xr, xu, xv, xw, xt);
    const uint32_t i = (uint32_t)pmod(z0 - 1, nz) * plane + xcol;
#pragma unroll
    for (int c = 0; c < 5; ++c) xraw[c] = qin[c * N + i];
    const int b0 = z0 & 1;
    s_pr[b0][0][epy][epx] = xu;
    s_pr[b0][1][epy][epx] = xv;
    s_pr[b0][2][epy][epx] = xw;
    s_pr[b0][3][epy][epx] = xt;
  }
  __syncthreads();

  // delays of this column's PE, cached per z-PE: the x / y face delays this column's stencils can
  // cross (0 away from those faces), and both z-face delays; the previous plane's x / y delays are
  // kept for its divergence, which runs one plane behind
  int tz_c = -1, kcx = 0, kcy = 0, kzl = 0, kzh = 0;

  // Iteration zc: fluxes of plane zc (LDS buffers of parity zc), x-y divergence of plane zc - 1,
  // update of plane zc - 2, then the window and LDS plane for zc + 1; one barrier per plane.
  for (int zc = z0 - 2; zc <= z1 + 1; ++zc) {
    const int bc = (zc + 2) & 1, bd = bc ^ 1;
    const int gz = pmod(zc, nz);
    const int tz = gz / a.ez;
    const int lze = gz - tz * a.ez;
    const int kcx_d = kcx, kcy_d = kcy;
    if (column && tz != tz_c) {
      tz_c = tz;
      const int8_t* kf = a.delays + ((tz * a.py + ty) * a.px + tx) * 6;
      kcx = near_x ? (lxe < 2 ? kf[0] : kf[1]) : 0;
      kcy = near_y ? (lye < 2 ? kf[2] : kf[3]) : 0;
      kzl = kf[4];
      kzh = kf[5];
    }
    const int kcz = lze < 2 ? kzl : (lze >= a.ez - 2 ? kzh : 0);
    const bool zin = zc >= z0 && zc < z1;
    const bool zin_d = zc - 1 >= z0 && zc - 1 < z1;
    const int gzd = pmod(zc - 1, nz);
    // plane zc - 2 is finalized in this iteration: fetch its state and register now
    const int zf = zc - 2;
    const bool fin = valid && zf >= z0 && zf < z1 && mode != kModePublish;
    const uint32_t fi = (uint32_t)pmod(zf, nz) * plane + col;
    T fq[5], fd[5];
    if (fin) {
#pragma unroll
      for (int c = 0; c < 5; ++c) fq[c] = qin[c * N + fi];
      if (mode == kModeStep && a.rk_a != T(0)) {
#pragma unroll
        for (int c = 0; c < 5; ++c) fd[c] = a.dq[c * N + fi];
      }
    }
    // ring slots of planes zc-2 .. zc+2 (u, v, w, T) and zc (rho, E)
    const int sb = pmod(zc - 2, 5);
    int sl5[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) sl5[j] = sb + j >= 5 ? sb + j - 5 : sb + j;
    const int sr = pmod(zc, 3);

    // fluxes of this column at plane zc: the tile computes all three (F_z also just outside the
    // chunk, for the z divergence), the halo rows F_y and the halo columns F_x
    const bool pub = valid && zin && a.publish;
    const bool need_fx = (role == 0 || role == 2) && zin && mode != kModePublish;
    const bool need_fy = (role == 0 || role == 1) && zin && mode != kModePublish;
    const bool need_fz = valid && mode != kModePublish;
    if (need_fx || need_fy || need_fz || pub) {
      T G[kNGrad];
      // central derivatives of u, v, w, T: x and y from the LDS plane, z from the window
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        set_grad(G, c, 0, (s_pr[bc][c][py][px - 2] - T(8) * s_pr[bc][c][py][px - 1] +
                           T(8) * s_pr[bc][c][py][px + 1] - s_pr[bc][c][py][px + 2]) * a.i12x);
        set_grad(G, c, 1, (s_pr[bc][c][py - 2][px] - T(8) * s_pr[bc][c][py - 1][px] +
                           T(8) * s_pr[bc][c][py + 1][px] - s_pr[bc][c][py + 2][px]) * a.i12y);
        set_grad(G, c, 2, (WIN(c, 0) - T(8) * WIN(c, 1) + T(8) * WIN(c, 3) - WIN(c, 4)) * a.i12z);
      }
      // a stencil that crosses a face with delay k >= 1 is recomputed with the AT values there
      if (kcx > 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T v[4];
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) {
            const int m = mi < 2 ? mi - 2 : mi - 1;
            const int l = lxe + m;
            v[mi] = (l < 0 || l >= a.ex) ? ghost<T>(a, 0, c, slab_off(a, 0, pmod(gx + m, nx), gy, gz), kcx)
                                          : s_pr[bc][c][py][px + m];
          }
          set_grad(G, c, 0, (v[0] - T(8) * v[1] + T(8) * v[2] - v[3]) * a.i12x);
        }
      }
      if (kcy > 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T v[4];
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) {
            const int m = mi < 2 ? mi - 2 : mi - 1;
            const int l = lye + m;
            v[mi] = (l < 0 || l >= a.ey) ? ghost<T>(a, 1, c, slab_off(a, 1, gx, pmod(gy + m, ny), gz), kcy)
                                          : s_pr[bc][c][py + m][px];
          }
          set_grad(G, c, 1, (v[0] - T(8) * v[1] + T(8) * v[2] - v[3]) * a.i12y);
        }
      }
      if (kcz > 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T v[4];
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) {
            const int m = mi < 2 ? mi - 2 : mi - 1;
            const int l = lze + m;
            v[mi] = (l < 0 || l >= a.ez) ? ghost<T>(a, 2, c, slab_off(a, 2, gx, gy, pmod(gz + m, nz)), kcz)
                                          : WIN(c, 2 + m);
          }
          set_grad(G, c, 2, (v[0] - T(8) * v[1] + T(8) * v[2] - v[3]) * a.i12z);
        }
      }
      // stress, pressure and the total fluxes (Eqs. cont, mome, ie in total-energy form), one
      // direction at a time
      const T rho = s_win[20 + sr][wc], u = WIN(0, 2), v = WIN(1, 2), w = WIN(2, 2), t = WIN(3, 2),
              E = s_win[23 + sr][wc];
      const T mu = visc<T>(a, t);
      const T kt = mu * a.cp_over_pr;
      const T th = G[0] + G[4] + G[8];
      const T s00 = mu * (G[0] + G[0]) - T(2.0 / 3.0) * mu * th;
      const T s11 = mu * (G[4] + G[4]) - T(2.0 / 3.0) * mu * th;
      const T s22 = mu * (G[8] + G[8]) - T(2.0 / 3.0) * mu * th;
      const T s01 = mu * (G[1] + G[3]);
      const T s02 = mu * (G[2] + G[6]);
      const T s12 = mu * (G[5] + G[7]);
      const T p = rho * a.gas_r * t;
      const T mx = rho * u, my = rho * v, mz = rho * w;
      const T Ep = E + p;
      T* rb = a.ring + (uint32_t)a.step_mod_r * a.rslot;
      const bool pubx = pub && near_x;
      const bool puby = pub && near_y;
      const bool pubz = pub && (lze < 2 || lze >= a.ez - 2);
      if (need_fx || pubx) {
        T F[kNQ];
        F[0] = mx;
        F[1] = mx * u + p - s00;
        F[2] = my * u - s01;
        F[3] = mz * u - s02;
        F[4] = Ep * u - (u * s00 + v * s01 + w * s02) - kt * G[9];
        if (need_fx) {
#pragma unroll
          for (int c = 0; c < kNQ; ++c) s_fx[bc][c][py - 4][px - 2] = F[c];
        }
        if (pubx) {
          const uint32_t sl = a.slab0;
          T* b = rb + slab_off(a, 0, gx, gy, gz);
          b[0] = u;
          b[sl] = v;
          b[2 * sl] = w;
          b[3 * sl] = t;
#pragma unroll
          for (int c = 0; c < kNQ; ++c) b[(4 + c) * sl] = F[c];
        }
      }
      if (need_fy || puby) {
        T F[kNQ];
        F[0] = my;
        F[1] = mx * v - s01;
        F[2] = my * v + p - s11;
        F[3] = mz * v - s12;
        F[4] = Ep * v - (u * s01 + v * s11 + w * s12) - kt * G[10];
        if (need_fy) {
#pragma unroll
          for (int c = 0; c < kNQ; ++c) s_fy[bc][c][py - 2][px - 4] = F[c];
        }
        if (puby) {
          const uint32_t sl = a.slab1;
          T* b = rb + slab_off(a, 1, gx, gy, gz);
          b[0] = u;
          b[sl] = v;
          b[2 * sl] = w;
          b[3 * sl] = t;
#pragma unroll
          for (int c = 0; c < kNQ; ++c) b[(4 + c) * sl] = F[c];
        }
      }
      if (need_fz || pubz) {
        T F[kNQ];
        F[0] = mz;
        F[1] = mx * w - s02;
        F[2] = my * w - s12;
        F[3] = mz * w + p - s22;
        F[4] = Ep * w - (u * s02 + v * s12 + w * s22) - kt * G[11];
        if (pubz) {
          const uint32_t sl = a.slab2;
          T* b = rb + slab_off(a, 2, gx, gy, gz);
          b[0] = u;
          b[sl] = v;
          b[2 * sl] = w;
          b[3 * sl] = t;
#pragma unroll
          for (int c = 0; c < kNQ; ++c) b[(4 + c) * sl] = F[c];
        }
        if (need_fz) {
          // scatter F_z(zc) into the receivers zc + r (RHS -= D_z F_z).  The source sits at
          // offset m = -r from receiver zc + r; a receiver in another z-PE whose face is delayed
          // reads the extrapolated flux instead (the receiver's PE owns that decision).
#pragma unroll
          for (int ri = 0; ri < 4; ++ri) {
            const int r = ri < 2 ? ri - 2 : ri - 1;
            const int zp = zc + r;
            if (zp < z0 || zp >= z1) continue;
            const int m = -r;
            const T cm = ((m == -2) ? T(1) : (m == -1) ? T(-8) : (m == 1) ? T(8) : T(-1)) * a.i12z;
            const int gzp = pmod(zp, nz);
            const int tzp = gzp / a.ez;
            const int l = gzp - tzp * a.ez + m;
            int k = 0;
            if (l < 0 || l >= a.ez) k = a.delays[((tzp * a.py + ty) * a.px + tx) * 6 + (l < 0 ? 4 : 5)];
            if (k == 0) {
#pragma unroll
              for (int c = 0; c < kNQ; ++c) acc[2 + r][c] -= cm * F[c];
            } else {
              const uint32_t so = slab_off(a, 2, gx, gy, gz);
#pragma unroll
              for (int c = 0; c < kNQ; ++c) add5(acc[2 + r], c, -cm * ghost<T>(a, 2, 4 + c, so, k));
            }
          }
        }
      }
    }

    if (valid && zin_d && mode != kModePublish) {
      const int fxx = px - 2, fyy = py - 2;  // this point in s_fx (column) and s_fy (row)
#pragma unroll
      for (int c = 0; c < kNQ; ++c) {
        const T dfx = (s_fx[bd][c][py - 4][fxx - 2] - T(8) * s_fx[bd][c][py - 4][fxx - 1] + T(8) * s_fx[bd][c][py - 4][fxx + 1] -
                       s_fx[bd][c][py - 4][fxx + 2]) * a.i12x;
        const T dfy = (s_fy[bd][c][fyy - 2][px - 4] - T(8) * s_fy[bd][c][fyy - 1][px - 4] + T(8) * s_fy[bd][c][fyy + 1][px - 4] -
                       s_fy[bd][c][fyy + 2][px - 4]) * a.i12y;
        acc[1][c] -= dfx + dfy;
      }
      // stencils crossing a delayed face: replace the central value by the AT one
      if (kcx_d > 0) {
#pragma unroll
        for (int c = 0; c < kNQ; ++c) {
          T v[4];
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) {
            const int m = mi < 2 ? mi - 2 : mi - 1;
            const int l = lxe + m;
            v[mi] = (l < 0 || l >= a.ex) ? ghost<T>(a, 0, 4 + c, slab_off(a, 0, pmod(gx + m, nx), gy, gzd), kcx_d)
                                          : s_fx[bd][c][py - 4][fxx + m];
          }
          const T cen = (s_fx[bd][c][py - 4][fxx - 2] - T(8) * s_fx[bd][c][py - 4][fxx - 1] + T(8) * s_fx[bd][c][py - 4][fxx + 1] -
                         s_fx[bd][c][py - 4][fxx + 2]) * a.i12x;
          const T at = (v[0] - T(8) * v[1] + T(8) * v[2] - v[3]) * a.i12x;
          add5(acc[1], c, cen - at);
        }
      }
      if (kcy_d > 0) {
#pragma unroll
        for (int c = 0; c < kNQ; ++c) {
          T v[4];
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) {
            const int m = mi < 2 ? mi - 2 : mi - 1;
            const int l = lye + m;
            v[mi] = (l < 0 || l >= a.ey) ? ghost<T>(a, 1, 4 + c, slab_off(a, 1, gx, pmod(gy + m, ny), gzd), kcy_d)
                                          : s_fy[bd][c][fyy + m][px - 4];
          }
          const T cen = (s_fy[bd][c][fyy - 2][px - 4] - T(8) * s_fy[bd][c][fyy - 1][px - 4] + T(8) * s_fy[bd][c][fyy + 1][px - 4] -
                         s_fy[bd][c][fyy + 2][px - 4]) * a.i12y;
          const T at = (v[0] - T(8) * v[1] + T(8) * v[2] - v[3]) * a.i12y;
          add5(acc[1], c, cen - at);
        }
      }
    }

    // finalize plane zc - 2: source and RK update (or RHS output)
    if (fin) {
      T r[kNQ];
#pragma unroll
      for (int c = 0; c < kNQ; ++c) r[c] = acc[0][c];
      if (forced) {
        // f_c = 2 Re(sum_kz B_kz,c e^{i kz z}), B from LDS, e^{i kz z} for kz = 1, 2 from the table
        const int gzf = pmod(zf, nz);
        const T* ez1 = a.phase_z + ((uint32_t)nz + gzf) * 2;
        const T* ez2 = a.phase_z + ((uint32_t)(2 * nz) + gzf) * 2;
        const T e1r = ez1[0], e1i = ez1[1], e2r = ez2[0], e2i = ez2[1];
        T f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T* b = s_force + (c * 6) * (BX * BY) + tid;
          constexpr int st = BX * BY;
          f[c] = T(2) * (b[0] + (b[2 * st] * e1r - b[3 * st] * e1i) + (b[4 * st] * e2r - b[5 * st] * e2i));
        }
        r[1] += fq[0] * f[0];
        r[2] += fq[0] * f[1];
        r[3] += fq[0] * f[2];
        r[4] += fq[1] * f[0] + fq[2] * f[1] + fq[3] * f[2];
      }
      if (mode == kModeRhs) {
#pragma unroll
        for (int c = 0; c < kNQ; ++c) a.rhs_out[c * N + fi] = r[c];
      } else {
#pragma unroll
        for (int c = 0; c < kNQ; ++c) {
          const T d = (a.rk_a == T(0)) ? a.dt * r[c] : a.rk_a * fd[c] + a.dt * r[c];
          if (a.store_dq) a.dq[c * N + fi] = d;
          a.q_out[c * N + fi] = fq[c] + a.rk_b * d;
          s_tsum[c][tid] += (double)d;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < kNQ; ++c) acc[j][c] = acc[j + 1][c];
#pragma unroll
    for (int c = 0; c < kNQ; ++c) acc[4][c] = T(0);

    // prepare plane zc + 1: window gets plane zc + 3 (replacing zc - 2), LDS plane zc + 1
    if (zc <= z1) {
      const int bn = bd;  // parity of zc + 1
      if (column) {
        T r_, u_, v_, w_, t_;
        prim_of<T>(raw, inv_cv, r_, u_, v_, w_, t_);
        const int s3 = pmod(zc + 3, 3);
        s_win[0 + sl5[0]][wc] = u_;
        s_win[5 + sl5[0]][wc] = v_;
        s_win[10 + sl5[0]][wc] = w_;
        s_win[15 + sl5[0]][wc] = t_;
        s_win[20 + s3][wc] = r_;
        s_win[23 + s3][wc] = raw[4];
        if (zc + 4 <= z1 + 3) {
          const uint32_t i = (uint32_t)pmod(zc + 4, nz) * plane + col;
#pragma unroll
          for (int c = 0; c < 5; ++c) raw[c] = qin[c * N + i];
        }
        s_pr[bn][0][py][px] = s_win[0 + sl5[3]][wc];
        s_pr[bn][1][py][px] = s_win[5 + sl5[3]][wc];
        s_pr[bn][2][py][px] = s_win[10 + sl5[3]][wc];
        s_pr[bn][3][py][px] = s_win[15 + sl5[3]][wc];
      }
      if (ex_ >= 0) {
        T xr, xu, xv, xw, xt;
        prim_of<T>(xraw, inv_cv, xr, xu, xv, xw, xt);
        if (zc + 2 <= z1 + 1) {
          const uint32_t i = (uint32_t)pmod(zc + 2, nz) * plane + xcol;
#pragma unroll
          for (int c = 0; c < 5; ++c) xraw[c] = qin[c * N + i];
        }
        s_pr[bn][0][epy][epx] = xu;
        s_pr[bn][1][epy][epx] = xv;
        s_pr[bn][2][epy][epx] = xw;
        s_pr[bn][3][epy][epx] = xt;
      }
    }
    __syncthreads();
  }


  if (mode != kModeStep) return;  // uniform across the grid
  // FP64 block sums of B_s * sum(dQ) * h^3 into this workgroup's slot (fixed order)
  __syncthreads();
  for (int len = TL::NOWN / 2; len > 0; len >>= 1) {
    if (tid < len) {
#pragma unroll
      for (int c = 0; c < kNQ; ++c) s_tsum[c][tid] += s_tsum[c][tid + len];
    }
    __syncthreads();
  }
  if (tid < kNQ) a.tot_part[blk * kNQ + tid] += (double)a.rk_b * s_tsum[tid][0] * a.vol;
}

// Workgroups are dispatched to the 8 XCDs round-robin (dispatch index w goes to XCD w mod 8), and
// each XCD has its own L2.  Logical workgroup L = xcd_major(w, nb) gives XCD c the contiguous range
// of logical workgroups [c q + min(c, r), ...) (q = nb / 8, r = nb mod 8, XCDs below r take one
// more), so workgroups that share halo planes run on the same L2.  A bijection of [0, nb).
constexpr uint32_t kNumXcd = 8;
__device__ __forceinline__ uint32_t xcd_major(uint32_t w, uint32_t nb) {
  const uint32_t c = w % kNumXcd, i = w / kNumXcd, q = nb / kNumXcd, r = nb % kNumXcd;
  return c * q + min(c, r) + i;
}

// MINW: waves per SIMD the register allocation must allow (occupancy target).
template <typename T, int BX, int BY, int MINW>
__global__ __launch_bounds__((Tile<BX, BY>::NT), MINW) void k_stage(FArgs<T> a, int mode) {
  const uint32_t gx = (uint32_t)a.gbx, gxy = gx * (uint32_t)a.gby;
  const uint32_t L = xcd_major(blockIdx.x, gridDim.x);
  const uint32_t bz = L / gxy, r = L - bz * gxy, by = r / gx, bx = r - by * gx;
  stage_body<T, BX, BY>(a, mode, (int)bx, (int)by, (int)bz, L);
}

// Batched stage: one launch over the workgroups of many runs.  work[b] = (run, local workgroup);
// the run's arguments come from the device run table, so each run sees exactly the workgroup
// decomposition (and therefore the arithmetic) of its own single-run launch.
template <typename T, int BX, int BY, int MINW>
__global__ __launch_bounds__((Tile<BX, BY>::NT), MINW) void k_stage_batch(const FArgs<T>* __restrict__ runs,
                                                                          const uint2* __restrict__ work,
                                                                          int mode) {
  const uint2 w = work[xcd_major(blockIdx.x, gridDim.x)];
  const FArgs<T> a = runs[w.x];
  const uint32_t per = (uint32_t)a.gbx * (uint32_t)a.gby;
  const uint32_t bz = w.y / per, r = w.y - bz * per, by = r / (uint32_t)a.gbx, bx = r - by * (uint32_t)a.gbx;
  stage_body<T, BX, BY>(a, mode, (int)bx, (int)by, (int)bz, w.y);
}

template <typename T>
FArgs<T> pack(const StageArgs<T>& s, int zchunk) {
  FArgs<T> a{};
  const Geom& g = s.g;
  a.q = s.q;
  a.q_out = s.q_out;
  a.dq = s.dq;
  a.ring = s.ring;
  a.gv = s.gv;
  a.rhs_out = s.rhs_out;
  a.delays = s.delays;
  a.ftab = s.force.table;
  a.phase_y = s.force.phase_y;
  a.phase_z = s.force.phase_z;
  a.pair_kyz = s.force.pair_kyz;
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
  a.ex = g.e[0];
  a.ey = g.e[1];
  a.ez = g.e[2];
  a.R = g.R;
  a.step_mod_r = s.step_mod_r;
  a.npair = s.force.npair;
  a.zchunk = zchunk;
  a.gbx = (g.n[0] + 15) / 16;  // set to the launch tile's workgroup counts by the launchers
  a.gby = (g.n[1] + 3) / 4;
  a.views = 0;
  a.publish = s.publish;
  a.store_dq = s.store_dq;
  a.i12x = s.cf.inv12h[0];
  a.i12y = s.cf.inv12h[1];
  a.i12z = s.cf.inv12h[2];
  a.gas_r = s.cf.gas_r;
  a.inv_cv = s.cf.inv_cv;
  a.cp_over_pr = s.cf.cp_over_pr;
  a.mu_ref = s.cf.mu_ref;
  a.inv_tref = s.cf.inv_tref;
  a.mu_exp = s.cf.mu_exp;
  a.cstage = s.cstage;
  a.rk_a = s.rk_a;
  a.rk_b = s.rk_b;
  a.dt = s.dt;
  a.vol = s.vol;
  return a;
}

// Static LDS of the stage kernel (must fit a compute unit: 160 KiB on gfx950).
template <typename T, int BX, int BY>
constexpr size_t stage_static_lds() {
  using TL = Tile<BX, BY>;
  return sizeof(T) * (2 * (4 * TL::LH * TL::LW + 5 * BY * (BX + 4) + 5 * (BY + 4) * BX) + 26 * TL::NCOL) +
         8 * kNQ * TL::NOWN;
}

template <typename T, int BX, int BY, int MINW>
hipError_t launch_cfg(const StageArgs<T>& s, int zchunk, int mode, hipStream_t stream) {
  if constexpr (stage_static_lds<T, BX, BY>() > kLdsBytes) {
    return hipErrorInvalidConfiguration;
  } else {
    const Geom& g = s.g;
    // a 1-D grid (the kernel decodes its logical x / y / z workgroup), with gridDim.y and gridDim.z
    // carried as 1 so that the decode below sees (gx, gy, gz) = (grid x, grid y, grid z)
    const unsigned gx = (unsigned)((g.n[0] + BX - 1) / BX), gy = (unsigned)((g.n[1] + BY - 1) / BY),
                   gz = (unsigned)((g.n[2] + zchunk - 1) / zchunk);
    FArgs<T> a = pack<T>(s, zchunk);
    a.gbx = (int)gx;
    a.gby = (int)gy;
    const size_t dyn = s.force.table ? sizeof(T) * 18 * BX * BY : 0;
    hipLaunchKernelGGL((k_stage<T, BX, BY, MINW>), dim3(gx * gy * gz), dim3(Tile<BX, BY>::NT), dyn, stream, a, mode);
    return hipGetLastError();
  }
}

// AT views of all published face-layer points for one stage: for a point on layer 0/1 (2/3) of
// PE t along d, the reader is the neighbouring PE t-1 (t+1) across that face; with its delay k > 0
// the view is w_0 v^{n-k} + w_1 v^{n-k-1} + w_2 v^{n-k-2}, w from kappa = k + c_s (Sec. 2.1,
// Eq. at; Appendix B weights at c_s = 0).  Points whose reader has k = 0 are not written.
template <typename T>
__device__ __forceinline__ void ghost_body(const FArgs<T>& a, T* __restrict__ gv, const uint32_t tid) {
  const uint32_t total = a.slab0 + a.slab1 + a.slab2;
  if (tid >= total) return;
  int d, x, y, z, jp;
  uint32_t sidx;
  if (tid < a.slab0) {
    d = 0;
    sidx = tid;
    const int q = 4 * a.px;
    jp = (int)(sidx % q);
    const uint32_t r = sidx / q;
    y = (int)(r % a.ny);
    z = (int)(r / a.ny);
    x = 0;
  } else if (tid < a.slab0 + a.slab1) {
    d = 1;
    sidx = tid - a.slab0;
    x = (int)(sidx % a.nx);
    const uint32_t r = sidx / a.nx;
    jp = (int)(r % (4 * a.py));
    z = (int)(r / (4 * a.py));
    y = 0;
  } else {
    d = 2;
    sidx = tid - a.slab0 - a.slab1;
    x = (int)(sidx % a.nx);
    const uint32_t r = sidx / a.nx;
    y = (int)(r % a.ny);
    jp = (int)(r / a.ny);
    z = 0;
  }
  const int t = jp / 4, layer = jp % 4;
  // PE coordinates of the reader: the owner's neighbour across the nearest face along d
  const int pz = a.nz / a.ez;
  int rx = d == 0 ? 0 : x / a.ex, ry = d == 1 ? 0 : y / a.ey, rz = d == 2 ? 0 : z / a.ez;
  const int pd = d == 0 ? a.px : (d == 1 ? a.py : pz);
  const int rt = layer < 2 ? (t == 0 ? pd - 1 : t - 1) : (t == pd - 1 ? 0 : t + 1);
  if (d == 0) rx = rt;
  else if (d == 1) ry = rt;
  else rz = rt;
  const int face = 2 * d + (layer < 2 ? 1 : 0);
  const int k = a.delays[((rz * a.py + ry) * a.px + rx) * 6 + face];
  if (k <= 0) return;
  const T kap = T(k) + a.cstage;
  const T w0 = (kap + T(1)) * (kap + T(2)) * T(0.5);
  const T w1 = -kap * (kap + T(2));
  const T w2 = kap * (kap + T(1)) * T(0.5);
  int s0 = a.step_mod_r - k;
  s0 += s0 < 0 ? a.R : 0;
  const int s1 = s0 == 0 ? a.R - 1 : s0 - 1;
  const int s2 = s1 == 0 ? a.R - 1 : s1 - 1;
  const uint32_t base = (d == 0 ? 0u : (d == 1 ? a.rdir1 : a.rdir2)) + sidx;
  const uint32_t ss = d == 0 ? a.slab0 : (d == 1 ? a.slab1 : a.slab2);
#pragma unroll
  for (int c = 0; c < kNRing; ++c) {
    const uint32_t o = base + (uint32_t)c * ss;
    gv[o] = w0 * a.ring[(uint32_t)s0 * a.rslot + o] + w1 * a.ring[(uint32_t)s1 * a.rslot + o] +
            w2 * a.ring[(uint32_t)s2 * a.rslot + o];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ghost_views(FArgs<T> a, T* __restrict__ gv) {
  ghost_body<T>(a, gv, blockIdx.x * 256u + threadIdx.x);
}

// Batched views: work[b] = (run, local block of 256 face-layer points); runs that read no
// delayed level at this stage leave at once.
template <typename T>
__global__ __launch_bounds__(256) void k_ghost_views_batch(const FArgs<T>* __restrict__ runs,
                                                           const uint2* __restrict__ work) {
  const uint2 w = work[blockIdx.x];
  const FArgs<T> a = runs[w.x];
  if (!a.views) return;
  ghost_body<T>(a, const_cast<T*>(a.gv), w.y * 256u + threadIdx.x);
}

}  // namespace

template <typename T>
hipError_t launch_ghost_views(const StageArgs<T>& a, hipStream_t stream) {
  const Geom& g = a.g;
  const int64_t total = g.slab[0] + g.slab[1] + g.slab[2];
  hipLaunchKernelGGL(k_ghost_views<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                     pack<T>(a, 4), a.gv_out);
  return hipGetLastError();
}
template hipError_t launch_ghost_views<double>(const StageArgs<double>&, hipStream_t);
template hipError_t launch_ghost_views<float>(const StageArgs<float>&, hipStream_t);

int64_t fused_blocks(const Geom& g, int tile, int zchunk) {
  const int bx = tile_bx(tile), by = tile_by(tile);
  return (int64_t)((g.n[0] + bx - 1) / bx) * ((g.n[1] + by - 1) / by) * ((g.n[2] + zchunk - 1) / zchunk);
}

// LDS bytes of a stage launch (static arrays plus the forcing coefficients when forced).
template <int BX, int BY>
size_t stage_lds_bytes(size_t w, bool forced) {
  const size_t stat = w == 4 ? stage_static_lds<float, BX, BY>() : stage_static_lds<double, BX, BY>();
  return stat + (forced ? w * 18 * BX * BY : 0);
}

size_t fused_lds_bytes(int tile, size_t word, bool forced) {
  switch (tile) {
    case 0: return stage_lds_bytes<64, 8>(word, forced);
    case 1: case 2: return stage_lds_bytes<32, 8>(word, forced);
    case 3: return stage_lds_bytes<32, 4>(word, forced);
    case 4: return stage_lds_bytes<64, 4>(word, forced);
    case 5: return stage_lds_bytes<16, 8>(word, forced);
    default: return ~size_t(0);
  }
}

template <typename T>
hipError_t launch_fused(const StageArgs<T>& a, int tile, int zchunk, int mode, hipStream_t stream) {
  if (fused_lds_bytes(tile, sizeof(T), a.force.table != nullptr) > kLdsBytes) return hipErrorInvalidConfiguration;
  constexpr bool f32 = sizeof(T) == 4;
  switch (tile) {
    case 0: return launch_cfg<T, 64, 8, f32 ? 4 : 2>(a, zchunk, mode, stream);
    case 1: return launch_cfg<T, 32, 8, f32 ? 2 : 1>(a, zchunk, mode, stream);
    case 2: return launch_cfg<T, 32, 8, f32 ? 4 : 2>(a, zchunk, mode, stream);
    case 3: return launch_cfg<T, 32, 4, f32 ? 2 : 1>(a, zchunk, mode, stream);
    case 4: return launch_cfg<T, 64, 4, f32 ? 3 : 2>(a, zchunk, mode, stream);
    case 5: return launch_cfg<T, 16, 8, f32 ? 2 : 1>(a, zchunk, mode, stream);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fused<double>(const StageArgs<double>&, int, int, int, hipStream_t);
template hipError_t launch_fused<float>(const StageArgs<float>&, int, int, int, hipStream_t);

template <typename T>
size_t batch_arg_bytes() {
  return sizeof(FArgs<T>);
}

template <typename T>
void pack_batch_arg(const StageArgs<T>& s, int tile, int zchunk, int views, void* dst) {
  FArgs<T> a = pack<T>(s, zchunk);
  a.gbx = (s.g.n[0] + tile_bx(tile) - 1) / tile_bx(tile);
  a.gby = (s.g.n[1] + tile_by(tile) - 1) / tile_by(tile);
  a.views = views;
  std::memcpy(dst, &a, sizeof(a));
}

int64_t view_blocks(const Geom& g) { return (g.slab[0] + g.slab[1] + g.slab[2] + 255) / 256; }

namespace {
template <typename T, int BX, int BY, int MINW>
hipError_t launch_batch_cfg(const void* runs, const uint2* work, int64_t nblk, bool forced, int mode,
                            hipStream_t stream) {
  if constexpr (stage_static_lds<T, BX, BY>() > kLdsBytes) {
    return hipErrorInvalidConfiguration;
  } else {
    const size_t dyn = forced ? sizeof(T) * 18 * BX * BY : 0;
    hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MINW>), dim3((unsigned)nblk), dim3(Tile<BX, BY>::NT), dyn,
                       stream, (const FArgs<T>*)runs, work, mode);
    return hipGetLastError();
  }
}
}  // namespace

template <typename T>
hipError_t launch_fused_batch(const void* runs, const uint2* work, int64_t nblk, int tile, bool forced, int mode,
                              hipStream_t stream) {
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidValue;
  if (fused_lds_bytes(tile, sizeof(T), forced) > kLdsBytes) return hipErrorInvalidConfiguration;
  constexpr bool f32 = sizeof(T) == 4;
  switch (tile) {
    case 0: return launch_batch_cfg<T, 64, 8, f32 ? 4 : 2>(runs, work, nblk, forced, mode, stream);
    case 1: return launch_batch_cfg<T, 32, 8, f32 ? 2 : 1>(runs, work, nblk, forced, mode, stream);
    case 2: return launch_batch_cfg<T, 32, 8, f32 ? 4 : 2>(runs, work, nblk, forced, mode, stream);
    case 3: return launch_batch_cfg<T, 32, 4, f32 ? 2 : 1>(runs, work, nblk, forced, mode, stream);
    case 4: return launch_batch_cfg<T, 64, 4, f32 ? 3 : 2>(runs, work, nblk, forced, mode, stream);
    case 5: return launch_batch_cfg<T, 16, 8, f32 ? 2 : 1>(runs, work, nblk, forced, mode, stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_views_batch(const void* runs, const uint2* work, int64_t nblk, hipStream_t stream) {
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ghost_views_batch<T>, dim3((unsigned)nblk), dim3(256), 0, stream, (const FArgs<T>*)runs,
                     work);
  return hipGetLastError();
}

template size_t batch_arg_bytes<float>();
template size_t batch_arg_bytes<double>();
template void pack_batch_arg<float>(const StageArgs<float>&, int, int, int, void*);
template void pack_batch_arg<double>(const StageArgs<double>&, int, int, int, void*);
template hipError_t launch_fused_batch<float>(const void*, const uint2*, int64_t, int, bool, int, hipStream_t);
template hipError_t launch_fused_batch<double>(const void*, const uint2*, int64_t, int, bool, int, hipStream_t);
template hipError_t launch_views_batch<float>(const void*, const uint2*, int64_t, hipStream_t);
template hipError_t launch_views_batch<double>(const void*, const uint2*, int64_t, hipStream_t);

}  // namespace atns
