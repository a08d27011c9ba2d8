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
// halo points the x / y derivatives need are loaded one plane ahead by the first waves.  The
// tile computes all three fluxes, the halo rows F_y and the halo columns F_x; F_x and F_y reach
// the tile through LDS, F_z stays in the owning thread and is scattered into a five-plane register
// accumulator, so the z divergence needs no LDS.  The state is read from one buffer and written
// to the other, so halo reads never see updated values.
//
// Fetches for a later plane (the state of plane z + 4, the plane-only halo points of z + 2, the AT
// sums of z + 1) are issued after the last use of the registers they refill and on every lane of
// the waves that use them: loads complete in order, and a refill copied into place, or one whose
// use the wait analysis cannot pair with it, would make the wave wait for it before the barrier.
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
  const T* gv;         // AT sums of the face-layer readers for this stage (one ring slot's layout)
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
  int views;     // batched AT sums: does this run read delayed levels at this stage
  int at_ghost;  // x / y AT entries are extrapolated halo values (delayed stages on aligned tiles)
  T i12x, i12y, i12z, gas_r, inv_cv, cp_over_pr, mu_ref, inv_tref, mu_exp;
  T rk_a, rk_b, dt;
  double vol;
  T c_prev;  // coefficient of the stored register in the update (Adams-Bashforth; 0 for RK)
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

// AT sum of component `comp` (0..3 primitives u, v, w, T; 4..8 face-normal flux) for the reader
// at face-layer ring offset `off`: the sum over the reader's stencil offsets m that cross its
// delayed face of a_m view(X + m), precomputed for this stage by k_at_sums.
template <typename T>
__device__ __forceinline__ T at_sum(const FArgs<T>& a, int d, int comp, uint32_t off) {
  return a.gv[off + (uint32_t)comp * slab_size(a, d)];
}

// Numerators a_m of the (1,4) first-derivative stencil at offsets m = -2, -1, +1, +2 (index mi);
// the derivative is (sum_m a_m v(X + m)) / 12h.
template <typename T>
__device__ __forceinline__ constexpr T stencil_a(int mi) {
  return mi == 0 ? T(1) : mi == 1 ? T(-8) : mi == 2 ? T(8) : T(-1);
}

// Bit mi set: offset m(mi) of a point at local index l in a PE of edge e >= 4 crosses a PE face.
__device__ __forceinline__ int crossing_mask(int l, int e) {
  return (l == 0 ? 0x3 : l == 1 ? 0x1 : 0) | (l == e - 1 ? 0xC : l == e - 2 ? 0x8 : 0);
}

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) { return fma(a, b, c); }
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The (1,4) stencil numerator in one fixed association, (v(-2) - 8 v(-1)) + (8 v(+1) - v(+2)), in
// every instantiation.  An AT derivative is this expression with the points across a delayed face
// replaced by their extrapolated values (Sec. 2.1, Eq. at); the two ways of evaluating it round
// identically:
//  * ghost points in the operands (aligned tiles: the halo holds the extrapolated values), or
//  * the reader's AT sum V in place of the half it covers (masked_num): V is that half with the
//    ghost operands, formed by the AT-sum kernel (or ghost_sum) with the same operations.
template <typename T>
__device__ __forceinline__ T central_num(T m2, T m1, T p1, T p2) {
  return fmaT(T(-8), m1, m2) + fmaT(T(8), p1, -p2);
}

// cm = crossing_mask of the reader (nonzero only on one side for e >= 4): layer 0 takes L = V,
// layer 1 L = V - 8 v(-1) (V = v(-1)), layer e-2 R = 8 v(+1) + V (V = -v(+2)), layer e-1 R = V.
template <typename T>
__device__ __forceinline__ T masked_num(T m2, T m1, T p1, T p2, int cm, T V) {
  const T L = (cm & 2) ? V : fmaT(T(-8), m1, (cm & 1) ? V : m2);
  const T R = (cm & 4) ? V : fmaT(T(8), p1, (cm & 8) ? V : -p2);
  return L + R;
}

// AT sum of a reader from the two extrapolated values g0, g1 stored at the slots of its face's
// readers (lower face: g0 at layer -2, g1 at -1; upper: g0 at e, g1 at e+1).
template <typename T>
__device__ __forceinline__ T at_sum_of(bool lower, bool outer, T g0, T g1) {
  // lower: layer 0 (outer) g0 - 8 g1, layer 1 g1; upper: layer e-2 -g0, layer e-1 (outer) 8 g0 - g1
  return lower ? (outer ? fmaT(T(-8), g1, g0) : g1) : (outer ? fmaT(T(8), g0, -g1) : -g0);
}

// Zero, produced by an instruction that reads v.  Added to the address of a fetch that refills the
// registers whose old contents v was computed from, it keeps the fetch behind that computation:
// issued earlier, the fetch would need other registers, and the copy back at the end of the
// iteration would make the wave wait for it there.
template <typename T>
__device__ __forceinline__ uint32_t zero_after(T v) {
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z) : "v"(v));
  return z;
}

// v in a register of its own (FP32): the window keeps rho and E of a plane, and as copies of the
// state registers they would hold those until the end of the iteration, past the refill.
template <typename T>
__device__ __forceinline__ T own_copy(T v) {
  static_assert(sizeof(T) == 4, "a copy into one 32-bit register");
  T r;
  asm volatile("v_mov_b32 %0, %1" : "=&v"(r) : "v"(v));
  return r;
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
// x / y derivatives of the halo columns, held by the first NXTRA threads (fetched one plane ahead).
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

// Per-column window of the z march: u, v, w, T of planes zc-2 .. zc+2 (index j = 0 .. 4) and rho,
// E of plane zc, for the current plane zc; push() brings in plane zc + 3 and advances zc.  It lives
// in registers (shifted one plane per push) in every instantiation: the FP64 AT ones of 4-wave
// workgroups run one wave per SIMD, whose budget (VGPRs plus AGPRs) holds it without scratch; those
// of larger workgroups spill part of their state to scratch, but keep the arithmetic, and so the
// rounding, of the others.
template <typename T>
struct ZWin {
  T w[4][5], re[2][3];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 5; ++j) w[c][j] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) re[0][j] = re[1][j] = T(0);
  }
  __device__ __forceinline__ void fill(int j, T u, T v, T ww, T t) {
    w[0][j] = u;
    w[1][j] = v;
    w[2][j] = ww;
    w[3][j] = t;
  }
  __device__ __forceinline__ void fill_re(int j, T r, T e) {
    re[0][j] = r;
    re[1][j] = e;
  }
  __device__ __forceinline__ T get(int c, int j) const { return w[c][j]; }
  __device__ __forceinline__ T rho() const { return re[0][0]; }
  __device__ __forceinline__ T E() const { return re[1][0]; }
  __device__ __forceinline__ void push(T u, T v, T ww, T t, T r, T e) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) w[c][j] = w[c][j + 1];
    fill(4, u, v, ww, t);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[0][j] = re[0][j + 1];
      re[1][j] = re[1][j + 1];
    }
    fill_re(2, r, e);
  }
};

// window element of component c (0 u, 1 v, 2 w, 3 T) at plane index j (plane zc - 2 + j)
#define WIN(c, j) zw.get(c, j)

// One workgroup of a stage: the BX x BY column tile (bkx, bky) and z chunk bkz of run `a`; `blk`
// is its slot among the run's workgroups for the FP64 totals.  PUB: this stage publishes the face
// layers (stage 1 of a step, or a history level); AT: some face of the run is delayed at this
// stage.  Each is compiled out of the stages that do not need it.  SUB (with AT, tiles aligned with
// the PEs along x and y): the halo columns within 2 of a delayed face of the tile's PE hold the
// extrapolated values (primitives in the LDS plane, the face-normal flux in the flux plane), so the
// tile's columns evaluate the central form; halo columns that compute (their own PE's face delayed,
// the tile's not) form their AT sums from the extrapolated values when they need them.  Without SUB
// every column whose face is delayed uses masked operands and AT sums fetched a plane ahead.
// AB2: the Adams-Bashforth update Q + rk_b dQ + c_prev dQ_prev in place of the Runge-Kutta one.
template <typename T, int BX, int BY, bool PUB, bool AT, bool SUB, bool AB2 = false>
__device__ __forceinline__ void stage_body(const FArgs<T>& a, const int mode, const int bkx, const int bky,
                                           const int bkz, const uint32_t blk) {
  constexpr bool kMask = AT && !SUB, kSub = AT && SUB;
  using TL = Tile<BX, BY>;
  constexpr int LW = TL::LW, LH = TL::LH;
  __shared__ T s_pr[2][4][LH][LW];       // u, v, w, T of a plane (two buffers: planes alternate)
  __shared__ T s_fx[2][5][BY][BX + 4];   // F_x on the tile rows, x halo 2
  __shared__ T s_fy[2][5][BY + 4][BX];   // F_y on the tile columns, y halo 2
  __shared__ double s_tsum[kNQ][TL::NOWN];  // FP64 running sums of dQ per tile column
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
  const bool xwave = (tid >> 6) < (TL::NXTRA + 63) / 64;  // uniform across the wave
  const uint32_t xcol = (uint32_t)pmod(exY, ny) * nx + pmod(exX, nx);

  const int tx = gx / a.ex, ty = gy / a.ey;
  const int lxe = gx - tx * a.ex, lye = gy - ty * a.ey;
  const bool near_x = lxe < 2 || lxe >= a.ex - 2;
  const bool near_y = lye < 2 || lye >= a.ey - 2;
  const uint32_t col = (uint32_t)gy * nx + gx;
  // this column's face-layer ring offsets (less the z term), where it publishes and where its AT
  // sums are: layer index jp = 4 t + (l < 2 ? l : l - e + 4)
  const int jx = 4 * tx + (lxe < 2 ? lxe : lxe - a.ex + 4), jy = 4 * ty + (lye < 2 ? lye : lye - a.ey + 4);
  const uint32_t zsx = (uint32_t)ny * (uint32_t)(4 * a.px), zsy = (uint32_t)(4 * a.py) * (uint32_t)nx;
  const uint32_t opx = (uint32_t)gy * (uint32_t)(4 * a.px) + (uint32_t)jx;    // + z zsx
  const uint32_t opy = a.rdir1 + (uint32_t)jy * (uint32_t)nx + (uint32_t)gx;  // + z zsy
  // AT by masked operands: where this column's PE face is delayed (k >= 1) the reader's AT sum
  // replaces the half of the stencil that crosses it (masked_num)
  const int cxm = crossing_mask(lxe, a.ex), cym = crossing_mask(lye, a.ey);
  // SUB: the tile's PE (ttx, tty); a halo column on the first two layers across one of its faces
  // is that face's ghost (gside 0..3 = lower x, upper x, lower y, upper y; -1 none) and finds the
  // extrapolated values at gofs (+ z term gzs, component stride gss): the slots of that face's
  // tile-PE readers, layer -2, -1 (or e, e+1) at readers 0, 1 (or 2, 3)
  const int ttx = x0 / a.ex, tty = y0 / a.ey;
  int gside = -1;
  uint32_t gofs = 0;
  if (kSub && role == 2) {
    const int c = (tid - TL::NOWN - TL::NY2) / BY;
    if (c < 2 ? x0 == ttx * a.ex : x0 + BX == (ttx + 1) * a.ex) {
      gside = c < 2 ? 0 : 1;
      gofs = (uint32_t)gy * (uint32_t)(4 * a.px) + (uint32_t)(4 * ttx + c);
    }
  } else if (kSub && role == 1) {
    const int r = (tid - TL::NOWN) / BX;
    if (r < 2 ? y0 == tty * a.ey : y0 + BY == (tty + 1) * a.ey) {
      gside = r < 2 ? 2 : 3;
      gofs = a.rdir1 + (uint32_t)(4 * tty + r) * (uint32_t)nx + (uint32_t)gx;
    }
  }
  const uint32_t gzs = role == 2 ? zsx : zsy, gss = role == 2 ? a.slab0 : a.slab1;
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

  // (zero where a lane never fetches them: every path then reads defined values, see below)
  T raw[5], xraw[5] = {}, fq[5] = {}, fd[5] = {};
  T acc[5][kNQ];
  if (role == 0) {
#pragma unroll
    for (int c = 0; c < kNQ; ++c) s_tsum[c][tid] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int c = 0; c < kNQ; ++c) acc[j][c] = T(0);
  ZWin<T> zw;
  zw.init();
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
      zw.fill(j - 1, u_, v_, w_, t_);
      if (j >= 3) zw.fill_re(j - 3, r_, q[4]);
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
  // Delays of this column's PE, cached per z-PE: the x / y face delays its stencils can cross (0
  // away from those faces, and for the tile's columns under SUB), for plane zc (gradients) and,
  // one plane behind, zc - 1 (divergence); the z-face delays in one word kz (bytes: its lower and
  // upper face, the upper face of the z-PE below and the lower face of the one above); under SUB
  // also gk, the delay of the tile-PE face this column is a ghost of (0: none, or not delayed).
  // Without SUB the gradient AT sums are fetched one iteration ahead (vx, vy: plane zc), the
  // divergence ones (vfx, vfy: plane zc - 1) right after the gradients, so that the fluxes hide them.
  int tz_c = -1, kcx = 0, kcy = 0, kz = 0, kcx_d = 0, kcy_d = 0, gk = 0;
  T vx[4], vy[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) vx[c] = vy[c] = T(0);
  auto plane_delays = [&](int zpl) {
    if (!AT) return;
    const int gzp = pmod(zpl, nz), tzp = gzp / a.ez;
    if (tzp != tz_c) {  // uniform: a new z-PE
      tz_c = tzp;
      if (column) {
        const int8_t* kf = a.delays + ((tzp * a.py + ty) * a.px + tx) * 6;
        const bool own = !kSub || role != 0;
        kcx = own && near_x ? (lxe < 2 ? kf[0] : kf[1]) : 0;
        kcy = own && near_y ? (lye < 2 ? kf[2] : kf[3]) : 0;
        const int pz = nz / a.ez;
        const int tzb = tzp == 0 ? pz - 1 : tzp - 1, tza = tzp == pz - 1 ? 0 : tzp + 1;
        const int kb = a.delays[((tzb * a.py + ty) * a.px + tx) * 6 + 5];
        const int ka = a.delays[((tza * a.py + ty) * a.px + tx) * 6 + 4];
        kz = (kf[4] & 0xff) | ((kf[5] & 0xff) << 8) | ((kb & 0xff) << 16) | ((ka & 0xff) << 24);
        if (kSub) gk = gside >= 0 ? a.delays[((tzp * a.py + tty) * a.px + ttx) * 6 + gside] : 0;
      }
    }
    if (kMask && __builtin_expect(kcx > 0, 0)) {
#pragma unroll
      for (int c = 0; c < 4; ++c) vx[c] = at_sum<T>(a, 0, c, (uint32_t)gzp * zsx + opx);
    }
    if (kMask && __builtin_expect(kcy > 0, 0)) {
#pragma unroll
      for (int c = 0; c < 4; ++c) vy[c] = at_sum<T>(a, 1, c, (uint32_t)gzp * zsy + opy);
    }
  };
  // SUB: the extrapolated u, v, w, T of plane zpl at this ghost column into an LDS plane buffer
  auto put_ghost_prims = [&](T (*dst)[LH][LW], int zpl) {
    const uint32_t o = gofs + (uint32_t)pmod(zpl, nz) * gzs;
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[c][py][px] = a.gv[o + (uint32_t)c * gss];
  };
  if (kSub) plane_delays(z0 - 2);
  // SUB: a halo column next to an x face forms the AT sums of its x derivatives (used while its own
  // PE's face is delayed and the tile's is not) a plane ahead: the operands of plane zc + 1 are
  // fetched at the top of iteration zc into the registers the tile's columns use for the finalize
  // fetch (free in halo columns), and the sums go to this thread's LDS slot when that fetch is
  // retired, for the next iteration's gradients; so the halo waves do not wait in their gradients.
  // (The publishing instantiation fetches them when it needs them: measured faster there.)
  constexpr bool kHv = kSub && !PUB;
  __shared__ T s_hv[kHv ? 4 : 1][kHv ? TL::NY2 + TL::NX2 : 1];
  const bool hx = kHv && (role == 1 || role == 2) && near_x;
  const int hslot = kHv ? max(tid - TL::NOWN, 0) : 0;
  auto hx_fetch = [&](int zpl) {
    const uint32_t o = (uint32_t)pmod(zpl, nz) * zsx + opx - (uint32_t)(lxe < 2 ? lxe : lxe - a.ex + 2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      fq[c] = a.gv[o + (uint32_t)c * a.slab0];
      fd[c] = a.gv[o + 1 + (uint32_t)c * a.slab0];
    }
  };
  auto hx_store = [&]() {
    const bool lo = lxe < 2, outer = lxe == 0 || lxe == a.ex - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) s_hv[c][hslot] = at_sum_of<T>(lo, outer, fq[c], fd[c]);
  };

  // window plane z0, then the LDS plane z0 - 2 (buffer parity (z + 2) & 1)
  if (column) {
    T r_, u_, v_, w_, t_;
    prim_of<T>(raw, inv_cv, r_, u_, v_, w_, t_);
    zw.fill(4, u_, v_, w_, t_);
    zw.fill_re(2, r_, raw[4]);
    if (z0 + 1 <= z1 + 3) {
      const uint32_t i = (uint32_t)pmod(z0 + 1, nz) * plane + col;
#pragma unroll
      for (int c = 0; c < 5; ++c) raw[c] = qin[c * N + i];
    }
    const int b0 = z0 & 1;
    if (kSub && gk > 0) {
      put_ghost_prims(s_pr[b0], z0 - 2);
    } else {
      s_pr[b0][0][py][px] = zw.get(0, 2);
      s_pr[b0][1][py][px] = zw.get(1, 2);
      s_pr[b0][2][py][px] = zw.get(2, 2);
      s_pr[b0][3][py][px] = zw.get(3, 2);
    }
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

  if (!kSub) plane_delays(z0 - 2);
  if (hx) {
    hx_fetch(z0 - 2);
    hx_store();
  }

  // Iteration zc: fluxes of plane zc (LDS buffers of parity zc), x-y divergence of plane zc - 1,
  // update of plane zc - 2, then the window and LDS plane for zc + 1; one barrier per plane.
  for (int zc = z0 - 2; zc <= z1 + 1; ++zc) {
    const int bc = (zc + 2) & 1, bd = bc ^ 1;
    const int gz = pmod(zc, nz);
    const int tz = gz / a.ez;
    const int lze = gz - tz * a.ez;
    const int kcz = !AT ? 0 : lze < 2 ? (kz & 0xff) : (lze >= a.ez - 2 ? (kz >> 8) & 0xff : 0);
    T vfx[kNQ], vfy[kNQ];
#pragma unroll
    for (int c = 0; c < kNQ; ++c) vfx[c] = vfy[c] = T(0);
    const bool zin = zc >= z0 && zc < z1;
    const bool zin_d = zc - 1 >= z0 && zc - 1 < z1;
    // plane zc - 2 is finalized in this iteration
    const int zf = zc - 2;
    const bool fin = valid && zf >= z0 && zf < z1 && mode != kModePublish;
    const uint32_t fi = (uint32_t)pmod(zf, nz) * plane + col;

    // fluxes of this column at plane zc: the tile computes all three (F_z also just outside the
    // chunk, for the z divergence), the halo rows F_y and the halo columns F_x
    const bool pub = PUB && valid && zin;
    const bool need_fx = (role == 0 || role == 2) && zin && mode != kModePublish;
    const bool need_fy = (role == 0 || role == 1) && zin && mode != kModePublish;
    const bool need_fz = valid && mode != kModePublish;
    if (kSub && gside >= 0) {
      // a ghost column: while its tile-PE face is delayed, its flux-plane entry of this plane is
      // the extrapolated face-normal flux and its LDS entry of the next plane (a buffer nobody
      // reads in this iteration) the extrapolated primitives; both fetched in one round trip.
      // The next plane's delay: this z-PE's, or the next z-PE's at its first plane (uniform).
      const int zn = pmod(zc + 1, nz), tzn = zn / a.ez;
      const int gkn = tzn == tz_c ? gk : (int)a.delays[((tzn * a.py + tty) * a.px + ttx) * 6 + gside];
      if (gk > 0 || gkn > 0) {
        const uint32_t o = gofs + (uint32_t)gz * gzs, on = gofs + (uint32_t)zn * gzs;
        T F[kNQ], P[4];
#pragma unroll
        for (int c = 0; c < kNQ; ++c) F[c] = a.gv[o + (uint32_t)(4 + c) * gss];
#pragma unroll
        for (int c = 0; c < 4; ++c) P[c] = a.gv[on + (uint32_t)c * gss];
        if (gk > 0 && zin && mode != kModePublish) {
          if (role == 2) {
#pragma unroll
            for (int c = 0; c < kNQ; ++c) s_fx[bc][c][py - 4][px - 2] = F[c];
          } else {
#pragma unroll
            for (int c = 0; c < kNQ; ++c) s_fy[bc][c][py - 2][px - 4] = F[c];
          }
        }
        if (gkn > 0 && zc <= z1) {
#pragma unroll
          for (int c = 0; c < 4; ++c) s_pr[bd][c][py][px] = P[c];
        }
      }
    }
    if (hx && zc <= z1) hx_fetch(zc + 1);  // after the ghost fetches, which are waited for at once
    if (kSub && gk > 0) {
      // computes nothing
    } else if (need_fx || need_fy || need_fz || pub) {
      T G[kNGrad];
      // derivatives of u, v, w, T: x and y from the LDS plane, z from the window.  Where a stencil
      // crosses a delayed face the points across carry coefficient 0 and the reader's AT sum
      // replaces them; elsewhere the central form is the same expression in every instantiation
      // (so a run's result does not depend on whether another run of its batch is delayed)
      // the masked forms only in waves that hold a reader of a delayed face (wave-uniform test)
      const bool wx = AT && __builtin_amdgcn_ballot_w64(kcx > 0) != 0;
      const bool wy = AT && __builtin_amdgcn_ballot_w64(kcy > 0) != 0;
      T sx[4], sy[4];  // the AT sums of this plane's readers: fetched ahead, or (SUB) formed here
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sx[c] = kMask ? vx[c] : T(0);
        sy[c] = kMask ? vy[c] : T(0);
      }
      if (kSub && wx && kcx > 0) {
        // a halo column next to its own delayed x face: its AT sums, formed a plane ahead, or from
        // the two extrapolated values at its face's reader slots
        if (kHv) {
#pragma unroll
          for (int c = 0; c < 4; ++c) sx[c] = s_hv[c][hslot];
        } else {
          const uint32_t o = (uint32_t)gz * zsx + opx - (uint32_t)(lxe < 2 ? lxe : lxe - a.ex + 2);
          const bool lo = lxe < 2, outer = lxe == 0 || lxe == a.ex - 1;
#pragma unroll
          for (int c = 0; c < 4; ++c) sx[c] = at_sum_of<T>(lo, outer, a.gv[o + (uint32_t)c * a.slab0],
                                                            a.gv[o + 1 + (uint32_t)c * a.slab0]);
        }
      }
      if (kSub && wy && kcy > 0) {
        const uint32_t o = (uint32_t)gz * zsy + opy - (uint32_t)(lye < 2 ? lye : lye - a.ey + 2) * (uint32_t)nx;
        const bool lo = lye < 2, outer = lye == 0 || lye == a.ey - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) sy[c] = at_sum_of<T>(lo, outer, a.gv[o + (uint32_t)c * a.slab1],
                                                          a.gv[o + (uint32_t)nx + (uint32_t)c * a.slab1]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T xm2 = s_pr[bc][c][py][px - 2], xm1 = s_pr[bc][c][py][px - 1], xp1 = s_pr[bc][c][py][px + 1],
                xp2 = s_pr[bc][c][py][px + 2];
        const T ym2 = s_pr[bc][c][py - 2][px], ym1 = s_pr[bc][c][py - 1][px], yp1 = s_pr[bc][c][py + 1][px],
                yp2 = s_pr[bc][c][py + 2][px];
        T dx = central_num(xm2, xm1, xp1, xp2);
        T dy = central_num(ym2, ym1, yp1, yp2);
        if (wx && kcx > 0) dx = masked_num(xm2, xm1, xp1, xp2, cxm, sx[c]);
        if (wy && kcy > 0) dy = masked_num(ym2, ym1, yp1, yp2, cym, sy[c]);
        set_grad(G, c, 0, dx * a.i12x);
        set_grad(G, c, 1, dy * a.i12y);
        set_grad(G, c, 2, (WIN(c, 0) - T(8) * WIN(c, 1) + T(8) * WIN(c, 3) - WIN(c, 4)) * a.i12z);
      }
      if (__builtin_expect(kcz > 0, 0)) {
        // near a delayed z face (the same for the whole plane unless the column's PEs differ): the
        // AT sums of all nine components in one round trip, the primitives' for the z derivatives
        // and the face-normal flux's for this plane's z divergence, which takes them in place of
        // the F_z values across the face (left out of the scatter)
        const uint32_t oz = slab_off(a, 2, gx, gy, gz);
        T sz[kNRing];
#pragma unroll
        for (int c = 0; c < kNRing; ++c) sz[c] = at_sum<T>(a, 2, c, oz);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T dz = sz[c];
#pragma unroll
          for (int mi = 0; mi < 4; ++mi) {
            const int m = mi < 2 ? mi - 2 : mi - 1;
            const int l = lze + m;
            if (l >= 0 && l < a.ez) dz += stencil_a<T>(mi) * WIN(c, 2 + m);
          }
          set_grad(G, c, 2, dz * a.i12z);
        }
#pragma unroll
        for (int c = 0; c < kNQ; ++c) acc[2][c] -= sz[4 + c] * a.i12z;
      }
      // fetched now, after the gradients, so that the gradients' wait for their AT sums (fetched in
      // the last iteration) covers no newer fetch; the fluxes hide these: the state and register of
      // the plane finalized in this iteration and the divergence AT sums of plane zc - 1 (the lanes
      // that use them all compute fluxes)
      if (fin) {
  #pragma unroll
        for (int c = 0; c < 5; ++c) fq[c] = qin[c * N + fi];
        if (mode == kModeStep && (AB2 || a.rk_a != T(0))) {
  #pragma unroll
          for (int c = 0; c < 5; ++c) fd[c] = __builtin_nontemporal_load(a.dq + c * N + fi);
        }
      }
      if (kMask && __builtin_expect(valid && kcx_d > 0, 0)) {
        const uint32_t o = (uint32_t)pmod(zc - 1, nz) * zsx + opx;
  #pragma unroll
        for (int c = 0; c < kNQ; ++c) vfx[c] = at_sum<T>(a, 0, 4 + c, o);
      }
      if (kMask && __builtin_expect(valid && kcy_d > 0, 0)) {
        const uint32_t o = (uint32_t)pmod(zc - 1, nz) * zsy + opy;
  #pragma unroll
        for (int c = 0; c < kNQ; ++c) vfy[c] = at_sum<T>(a, 1, 4 + c, o);
      }

      // stress, pressure and the total fluxes (Eqs. cont, mome, ie in total-energy form), one
      // direction at a time
      const T rho = zw.rho(), u = WIN(0, 2), v = WIN(1, 2), w = WIN(2, 2), t = WIN(3, 2), E = zw.E();
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
          T* b = rb + ((uint32_t)gz * zsx + opx);
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
          T* b = rb + ((uint32_t)gz * zsy + opy);
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
          // takes no contribution from it and has added its AT sum instead (the receiver's PE owns
          // that decision).
          // only a source within 2 planes of its z-PE's faces (uniform) has receivers across
          const bool zface = AT && (lze < 2 || lze >= a.ez - 2);
#pragma unroll
          for (int ri = 0; ri < 4; ++ri) {
            const int r = ri < 2 ? ri - 2 : ri - 1;
            const int zp = zc + r;
            if (zp < z0 || zp >= z1) continue;
            const int m = -r;
            const T cm = ((m == -2) ? T(1) : (m == -1) ? T(-8) : (m == 1) ? T(8) : T(-1)) * a.i12z;
            bool keep = true;
            if (zface) {
              const int l = lze - m;  // the receiver in this z-PE's local coordinates
              if (l < 0) keep = ((kz >> 16) & 0xff) == 0;  // in the z-PE below
              if (l >= a.ez) keep = ((kz >> 24) & 0xff) == 0;  // in the one above
            }
            if (keep) {
#pragma unroll
              for (int c = 0; c < kNQ; ++c) acc[2 + r][c] -= cm * F[c];
            }
          }
        }
      }
    }

    if (valid && zin_d && mode != kModePublish) {
      const int fxx = px - 2, fyy = py - 2;  // this point in s_fx (column) and s_fy (row)
      const bool wx = kMask && __builtin_amdgcn_ballot_w64(kcx_d > 0) != 0;
      const bool wy = kMask && __builtin_amdgcn_ballot_w64(kcy_d > 0) != 0;
#pragma unroll
      for (int c = 0; c < kNQ; ++c) {
        const T xm2 = s_fx[bd][c][py - 4][fxx - 2], xm1 = s_fx[bd][c][py - 4][fxx - 1],
                xp1 = s_fx[bd][c][py - 4][fxx + 1], xp2 = s_fx[bd][c][py - 4][fxx + 2];
        const T ym2 = s_fy[bd][c][fyy - 2][px - 4], ym1 = s_fy[bd][c][fyy - 1][px - 4],
                yp1 = s_fy[bd][c][fyy + 1][px - 4], yp2 = s_fy[bd][c][fyy + 2][px - 4];
        T dfx = central_num(xm2, xm1, xp1, xp2);
        T dfy = central_num(ym2, ym1, yp1, yp2);
        if (wx && kcx_d > 0) dfx = masked_num(xm2, xm1, xp1, xp2, cxm, vfx[c]);
        if (wy && kcy_d > 0) dfy = masked_num(ym2, ym1, yp1, yp2, cym, vfy[c]);
        acc[1][c] -= dfx * a.i12x + dfy * a.i12y;
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
        for (int c = 0; c < kNQ; ++c) __builtin_nontemporal_store(r[c], a.rhs_out + c * N + fi);
      } else {
#pragma unroll
        for (int c = 0; c < kNQ; ++c) {
          const T d = (a.rk_a == T(0)) ? a.dt * r[c] : a.rk_a * fd[c] + a.dt * r[c];
          // the register and the new state are not read again in this stage: streaming stores
          // keep the L2 for the halo planes
          if (a.store_dq) __builtin_nontemporal_store(d, a.dq + c * N + fi);
          if constexpr (AB2) {
            // Adams-Bashforth (Sec. 2.2, Eq. time_ab): d = dt f^n, the register dt f^{n-1}
            const T inc = a.rk_b * d + a.c_prev * fd[c];
            __builtin_nontemporal_store(fq[c] + inc, a.q_out + c * N + fi);
            s_tsum[c][tid] += (double)inc;
          } else {
            __builtin_nontemporal_store(fq[c] + a.rk_b * d, a.q_out + c * N + fi);
            s_tsum[c][tid] += (double)d;
          }
        }
      }
    }
    // the fetched state and register are consumed here on every path (no instruction: the wait
    // for them happens now, not at the next write of their registers, after later fetches)
#pragma unroll
    for (int c = 0; c < 5; ++c) asm volatile("" ::"v"(fq[c]), "v"(fd[c]));
    if (hx && zc <= z1) hx_store();  // the sums of plane zc + 1
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < kNQ; ++c) acc[j][c] = acc[j + 1][c];
#pragma unroll
    for (int c = 0; c < kNQ; ++c) acc[4][c] = T(0);

    // prepare plane zc + 1: window gets plane zc + 3 (replacing zc - 2), LDS plane zc + 1
    if (zc <= z1) {
      const int bn = bd;  // parity of zc + 1
      // the divergence of plane zc (next iteration) with this plane's delays; AT sums ahead
      kcx_d = kcx;
      kcy_d = kcy;
      // consume what the last iteration fetched (the plane-only points of zc + 1, the column's
      // plane zc + 3), then fetch ahead: every lane fetches, at a valid address, the plane after
      // (zc + 2, zc + 4, wrapped), so that the wait counts on the fetches are exact
      plane_delays(zc + 1);
      T xt = T(0), t_ = T(0);
      if (ex_ >= 0) {
        T xr, xu, xv, xw;
        prim_of<T>(xraw, inv_cv, xr, xu, xv, xw, xt);
        s_pr[bn][0][epy][epx] = xu;
        s_pr[bn][1][epy][epx] = xv;
        s_pr[bn][2][epy][epx] = xw;
        s_pr[bn][3][epy][epx] = xt;
      }
#pragma unroll
      for (int c = 0; c < 5; ++c) asm volatile("" ::"v"(xraw[c]));  // consumed on every path
      if (column) {
        T r_, u_, v_, w_, e_ = raw[4];
        prim_of<T>(raw, inv_cv, r_, u_, v_, w_, t_);
        if constexpr (sizeof(T) == 4) {
          r_ = own_copy(r_);
          e_ = own_copy(e_);
        }
        zw.push(u_, v_, w_, t_, r_, e_);
        if (!(kSub && gk > 0)) {  // (a ghost's entry is in place; its window keeps its own values)
          s_pr[bn][0][py][px] = zw.get(0, 2);
          s_pr[bn][1][py][px] = zw.get(1, 2);
          s_pr[bn][2][py][px] = zw.get(2, 2);
          s_pr[bn][3][py][px] = zw.get(3, 2);
        }
      }
      {
        const uint32_t i = (uint32_t)pmod(zc + 4, nz) * plane + col + zero_after(t_);
#pragma unroll
        for (int c = 0; c < 5; ++c) raw[c] = qin[c * N + i];
      }
      if (xwave || AT) {  // only the waves that hold plane-only points
        const uint32_t i = (uint32_t)pmod(zc + 2, nz) * plane + xcol + zero_after(xt);
#pragma unroll
        for (int c = 0; c < 5; ++c) xraw[c] = qin[c * N + i];
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
  if (tid < kNQ) a.tot_part[blk * kNQ + tid] += (double)(AB2 ? T(1) : a.rk_b) * s_tsum[tid][0] * a.vol;
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
template <typename T, int BX, int BY, int MINW, bool PUB, bool AT, bool SUB, bool AB2 = false>
__global__ __launch_bounds__((Tile<BX, BY>::NT), MINW) void k_stage(FArgs<T> a, int mode) {
  const uint32_t gx = (uint32_t)a.gbx, gxy = gx * (uint32_t)a.gby;
  const uint32_t L = xcd_major(blockIdx.x, gridDim.x);
  const uint32_t bz = L / gxy, r = L - bz * gxy, by = r / gx, bx = r - by * gx;
  stage_body<T, BX, BY, PUB, AT, SUB, AB2>(a, mode, (int)bx, (int)by, (int)bz, L);
}

// Batched stage: one launch over the workgroups of many runs.  work[b] = (run, local workgroup);
// the run's arguments come from the device run table, so each run sees exactly the workgroup
// decomposition (and therefore the arithmetic) of its own single-run launch.  A run executes in
// the instantiation its own single-run step would use: the AT one where it reads delayed levels
// at this stage (its `views` flag), the other one elsewhere, and of the two AT ones the one for its
// tiles (at_ghost: aligned with its PEs); its workgroups leave the other instantiations' launches
// at once.
template <typename T, int BX, int BY, int MINW, bool PUB, bool AT, bool SUB>
__global__ __launch_bounds__((Tile<BX, BY>::NT), MINW) void k_stage_batch(const FArgs<T>* __restrict__ runs,
                                                                          const uint2* __restrict__ work,
                                                                          int mode) {
  const uint2 w = work[xcd_major(blockIdx.x, gridDim.x)];
  const FArgs<T> a = runs[w.x];
  if ((a.views != 0) != AT || (AT && (a.at_ghost != 0) != SUB)) return;  // uniform across the workgroup
  const uint32_t per = (uint32_t)a.gbx * (uint32_t)a.gby;
  const uint32_t bz = w.y / per, r = w.y - bz * per, by = r / (uint32_t)a.gbx, bx = r - by * (uint32_t)a.gbx;
  stage_body<T, BX, BY, PUB, AT, SUB>(a, mode, (int)bx, (int)by, (int)bz, w.y);
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
  a.at_ghost = s.at_ghost;
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
  a.rk_a = s.rk_a;
  a.rk_b = s.rk_b;
  a.c_prev = s.c_prev;
  a.dt = s.dt;
  a.vol = s.vol;
  return a;
}

// Occupancy target of the AT instantiations: their extra state does not fit the registers of 4
// waves per SIMD without spilling, so workgroups of at most 8 waves (which run at 2 waves per
// SIMD) target 2; larger workgroups keep the target they need to be resident at all.
template <int BX, int BY>
constexpr int at_waves(int minw) {
  return Tile<BX, BY>::NT <= 512 ? (minw < 2 ? minw : 2) : minw;
}

// The publishing AT instantiation of 4-wave FP32 workgroups needs a few registers more than 3
// waves per SIMD allow (172 of 168) and so would run at 2; held to 3 it spills 4 registers to
// scratch and its stages take 18% less time.  (Larger workgroups gain no resident workgroup from
// a third wave, and the other instantiations are slower under the tighter target.)
template <typename T, int BX, int BY>
constexpr int pub_at_waves(int ma) {
  return sizeof(T) == 4 && Tile<BX, BY>::NT <= 256 ? 3 : ma;
}

// Occupancy target of the instantiations for aligned tiles (SUB): in FP32 they fit the registers of
// 4 waves per SIMD (the publishing one with 2 or 3 spilled), whatever the tile's own target; a
// workgroup shape that keeps as many workgroups per CU (16 wave slots) at 3 waves per SIMD as at 4
// (6- and 9-wave workgroups) targets 3.
template <typename T, int BX, int BY>
constexpr int sub_waves(int minw) {
  constexpr int nw = Tile<BX, BY>::NT / 64;
  return sizeof(T) != 4 ? minw : (12 / nw == 16 / nw ? 3 : 4);
}

// Static LDS of the stage kernel (must fit a compute unit: 160 KiB on gfx950); the halo AT-sum
// slots of the aligned-tile instantiations are counted for all.
template <typename T, int BX, int BY>
constexpr size_t stage_static_lds() {
  using TL = Tile<BX, BY>;
  return sizeof(T) * (2 * (4 * TL::LH * TL::LW + 5 * BY * (BX + 4) + 5 * (BY + 4) * BX) +
                      4 * (TL::NY2 + TL::NX2)) +
         8 * kNQ * TL::NOWN;
}

// Occupancy target of the FP64 AT instantiations.  A workgroup of at most 4 waves targets one wave
// per SIMD, so that the z window, the AT state and the gradients fit VGPRs and AGPRs without
// scratch.  Larger workgroups take no more waves per SIMD than their static LDS leaves room for, so
// that they keep the registers of that occupancy.
template <typename T, int BX, int BY>
constexpr int fp64_at_cap(int m) {
  constexpr int nw = Tile<BX, BY>::NT / 64;
  constexpr int wgs = (int)(kLdsBytes / stage_static_lds<T, BX, BY>());
  constexpr int cap = (wgs * nw + 3) / 4 < 1 ? 1 : (wgs * nw + 3) / 4;
  return sizeof(T) == 4 ? m : nw <= 4 ? 1 : m <= cap ? m : cap;
}

template <typename T, int BX, int BY, int MINW>
hipError_t launch_cfg(const StageArgs<T>& s, int zchunk, int mode, bool at, hipStream_t stream) {
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
    const dim3 grid(gx * gy * gz), block(Tile<BX, BY>::NT);
    constexpr int MA = fp64_at_cap<T, BX, BY>(at_waves<BX, BY>(MINW));
    constexpr int MP = fp64_at_cap<T, BX, BY>(pub_at_waves<T, BX, BY>(MA));
    constexpr int MS = fp64_at_cap<T, BX, BY>(sub_waves<T, BX, BY>(MINW));
    const bool sub = at && s.at_ghost;
    if (s.c_prev != T(0)) {  // an Adams-Bashforth step with a stored register (always publishes)
      if (!s.publish || mode != kModeStep) return hipErrorInvalidValue;
      if (sub)
        hipLaunchKernelGGL((k_stage<T, BX, BY, MS, true, true, true, true>), grid, block, dyn, stream, a, mode);
      else if (at)
        hipLaunchKernelGGL((k_stage<T, BX, BY, MP, true, true, false, true>), grid, block, dyn, stream, a, mode);
      else
        hipLaunchKernelGGL((k_stage<T, BX, BY, MINW, true, false, false, true>), grid, block, dyn, stream, a, mode);
    } else if (s.publish && sub)
      hipLaunchKernelGGL((k_stage<T, BX, BY, MS, true, true, true>), grid, block, dyn, stream, a, mode);
    else if (s.publish && at)
      hipLaunchKernelGGL((k_stage<T, BX, BY, MP, true, true, false>), grid, block, dyn, stream, a, mode);
    else if (s.publish)
      hipLaunchKernelGGL((k_stage<T, BX, BY, MINW, true, false, false>), grid, block, dyn, stream, a, mode);
    else if (sub)
      hipLaunchKernelGGL((k_stage<T, BX, BY, MS, false, true, true>), grid, block, dyn, stream, a, mode);
    else if (at)
      hipLaunchKernelGGL((k_stage<T, BX, BY, MA, false, true, false>), grid, block, dyn, stream, a, mode);
    else
      hipLaunchKernelGGL((k_stage<T, BX, BY, MINW, false, false, false>), grid, block, dyn, stream, a, mode);
    return hipGetLastError();
  }
}

// AT sums of the three stages of a step, per reader (Sec. 2.1, Eq. at; Appendix B, (1,4) rows).  A point on face
// layer l of PE t along d reads, across the face on its side (layers 0, 1: the lower face, read
// from PE t-1; layers 2, 3: the upper face, from PE t+1), the stencil offsets m that leave its PE:
// m = -2, -1 (l = 0), -2 (l = 1), +2 (l = 2), +1, +2 (l = 3).  With the reader PE's delay k >= 1 on
// that face the value there is the extrapolation w_0 v^{n-k} + w_1 v^{n-k-1} + w_2 v^{n-k-2},
// w from kappa = k + c_s (the Appendix B weights at c_s = 0); the kernel stores, for each of the 9
// ring components, sum_m a_m (extrapolated value at X + m) at the reader's own ring offset, with
// a = (1, -8, 8, -1) the stencil numerators.  The delays and levels are those of the step, the
// same for its three stages, which differ only in c_s: one launch per step reads the levels once
// and writes the sums of stage s into the s-th of three consecutive slot-sized regions of gv (an
// Adams-Bashforth step writes only the first, c_s = 0).
// One thread serves the two readers of a face (layers 0, 1 or 2, 3), which share their delay and
// the source points across it (each extrapolated once).  Readers whose face has k = 0 are not
// written.  For a run whose stages run on tiles aligned with its PEs (at_ghost), the x and y
// entries hold the two extrapolated values instead (layers -2, -1 at the slots of readers 0, 1;
// layers e, e+1 at those of readers 2, 3), which the stage kernel places in its halo; the sums are
// formed from them as at_sum_of does.
// NST: the stages whose sums are written (3 for Runge-Kutta; 1, c_s = 0, for Adams-Bashforth).
template <typename T, int NST = 3>
__device__ __forceinline__ void at_sums_body(const FArgs<T>& a, T* __restrict__ gv, const uint32_t tid,
                                             const T c0, const T c1, const T c2) {
  const uint32_t h0 = a.slab0 / 2, h1 = a.slab1 / 2, h2 = a.slab2 / 2;
  if (tid >= h0 + h1 + h2) return;
  int d, x, y, z, jp;
  uint32_t sidx, jstride;  // slab index of the pair's first reader, stride of the layer index jp
  if (tid < h0) {
    d = 0;
    const int q = 2 * a.px;  // reader pairs per (y, z) row
    const int jpp = (int)(tid % q);
    const uint32_t r = tid / q;
    y = (int)(r % a.ny);
    z = (int)(r / a.ny);
    x = 0;
    jp = 2 * jpp;
    jstride = 1;
    sidx = r * (uint32_t)(4 * a.px) + (uint32_t)jp;
  } else if (tid < h0 + h1) {
    d = 1;
    const uint32_t u = tid - h0;
    x = (int)(u % a.nx);
    const uint32_t r = u / a.nx;
    const int jpp = (int)(r % (2 * a.py));
    z = (int)(r / (2 * a.py));
    y = 0;
    jp = 2 * jpp;
    jstride = (uint32_t)a.nx;
    sidx = ((uint32_t)z * (uint32_t)(4 * a.py) + (uint32_t)jp) * (uint32_t)a.nx + (uint32_t)x;
  } else {
    d = 2;
    const uint32_t u = tid - h0 - h1;
    x = (int)(u % a.nx);
    const uint32_t r = u / a.nx;
    y = (int)(r % a.ny);
    const int jpp = (int)(r / a.ny);
    z = 0;
    jp = 2 * jpp;
    jstride = (uint32_t)a.nx * (uint32_t)a.ny;
    sidx = ((uint32_t)jp * (uint32_t)a.ny + (uint32_t)y) * (uint32_t)a.nx + (uint32_t)x;
  }
  const int t = jp / 4, lower = (jp % 4) == 0;  // readers on layers 0, 1 (lower face) or 2, 3
  // the readers' PE: t along d, from the point's coordinates across
  const int rx = d == 0 ? t : x / a.ex, ry = d == 1 ? t : y / a.ey, rz = d == 2 ? t : z / a.ez;
  const int k = a.delays[((rz * a.py + ry) * a.px + rx) * 6 + 2 * d + (lower ? 0 : 1)];
  if (k <= 0) return;
  const int pd = d == 0 ? a.px : (d == 1 ? a.py : a.nz / a.ez);
  const int tn = lower ? (t == 0 ? pd - 1 : t - 1) : (t == pd - 1 ? 0 : t + 1);
  // sources: lower face: layers 2, 3 of PE tn; upper face: layers 0, 1 of PE tn
  const int sl = lower ? 2 : 0;
  const bool ghost = a.at_ghost != 0 && d < 2;
  T w[3][3];
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    const T kap = T(k) + (st == 0 ? c0 : st == 1 ? c1 : c2);
    w[st][0] = (kap + T(1)) * (kap + T(2)) * T(0.5);
    w[st][1] = -kap * (kap + T(2));
    w[st][2] = kap * (kap + T(1)) * T(0.5);
  }
  int s0 = a.step_mod_r - k;
  s0 += s0 < 0 ? a.R : 0;
  const int s1 = s0 == 0 ? a.R - 1 : s0 - 1;
  const int s2 = s1 == 0 ? a.R - 1 : s1 - 1;
  const uint32_t base = d == 0 ? 0u : (d == 1 ? a.rdir1 : a.rdir2);
  const uint32_t ss = d == 0 ? a.slab0 : (d == 1 ? a.slab1 : a.slab2);
  const uint32_t srcA = base + sidx + (uint32_t)(4 * tn + sl - jp) * jstride;  // layer sl
  const uint32_t srcB = srcA + jstride;                                        // layer sl + 1
  const uint32_t dst = base + sidx;
  const T* r0 = a.ring + (uint32_t)s0 * a.rslot;
  const T* r1 = a.ring + (uint32_t)s1 * a.rslot;
  const T* r2 = a.ring + (uint32_t)s2 * a.rslot;
#pragma unroll
  for (int c = 0; c < kNRing; ++c) {
    const uint32_t oa = srcA + (uint32_t)c * ss, ob = srcB + (uint32_t)c * ss;
    const T a0 = r0[oa], a1 = r1[oa], a2 = r2[oa], b0 = r0[ob], b1 = r1[ob], b2 = r2[ob];
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const T va = w[st][0] * a0 + w[st][1] * a1 + w[st][2] * a2;
      const T vb = w[st][0] * b0 + w[st][1] * b1 + w[st][2] * b2;
      // lower face: reader 0 = 1 va - 8 vb (offsets -2, -1), reader 1 = 1 vb (offset -2);
      // upper face: reader 2 = -1 va (offset +2), reader 3 = 8 va - 1 vb (offsets +1, +2); or,
      // for the x / y faces of a run on aligned tiles, the extrapolated values va, vb themselves
      const T v0 = ghost ? va : at_sum_of<T>(lower, lower, va, vb);
      const T v1 = ghost ? vb : at_sum_of<T>(lower, !lower, va, vb);
      T* g = gv + (uint32_t)st * a.rslot;
      g[dst + (uint32_t)c * ss] = v0;
      g[dst + jstride + (uint32_t)c * ss] = v1;
    }
  }
}

template <typename T, int NST>
__global__ __launch_bounds__(256) void k_at_sums(FArgs<T> a, T* __restrict__ gv, T c0, T c1, T c2) {
  at_sums_body<T, NST>(a, gv, blockIdx.x * 256u + threadIdx.x, c0, c1, c2);
}

// Batched sums: work[b] = (run, local block of 256 reader pairs); runs that read no delayed level
// at this step leave at once.  The run table is that of the step's first stage, whose gv is the
// base of the three regions.
template <typename T>
__global__ __launch_bounds__(256) void k_at_sums_batch(const FArgs<T>* __restrict__ runs,
                                                           const uint2* __restrict__ work, T c0, T c1, T c2) {
  const uint2 w = work[blockIdx.x];
  const FArgs<T> a = runs[w.x];
  if (!a.views) return;
  at_sums_body<T>(a, const_cast<T*>(a.gv), w.y * 256u + threadIdx.x, c0, c1, c2);
}

}  // namespace

template <typename T>
hipError_t launch_at_sums(const StageArgs<T>& a, const double* cs, hipStream_t stream, int nst) {
  const Geom& g = a.g;
  const int64_t total = (g.slab[0] + g.slab[1] + g.slab[2]) / 2;  // reader pairs
  if (nst != 1 && nst != 3) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (nst == 3)
    hipLaunchKernelGGL((k_at_sums<T, 3>), grid, block, 0, stream, pack<T>(a, 4), a.gv_out, (T)cs[0], (T)cs[1], (T)cs[2]);
  else
    hipLaunchKernelGGL((k_at_sums<T, 1>), grid, block, 0, stream, pack<T>(a, 4), a.gv_out, (T)cs[0], (T)cs[1], (T)cs[2]);
  return hipGetLastError();
}
template hipError_t launch_at_sums<double>(const StageArgs<double>&, const double*, hipStream_t, int);
template hipError_t launch_at_sums<float>(const StageArgs<float>&, const double*, hipStream_t, int);

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
    case 6: return stage_lds_bytes<16, 16>(word, forced);
    default: return ~size_t(0);
  }
}

template <typename T>
hipError_t launch_fused(const StageArgs<T>& a, int tile, int zchunk, int mode, bool at, hipStream_t stream) {
  if (fused_lds_bytes(tile, sizeof(T), a.force.table != nullptr) > kLdsBytes) return hipErrorInvalidConfiguration;
  if (at && a.at_ghost && !tile_aligned(a.g, tile)) return hipErrorInvalidValue;  // halo values need aligned tiles
  constexpr bool f32 = sizeof(T) == 4;
  switch (tile) {
    case 0: return launch_cfg<T, 64, 8, f32 ? 4 : 2>(a, zchunk, mode, at, stream);
    case 1: return launch_cfg<T, 32, 8, f32 ? 2 : 1>(a, zchunk, mode, at, stream);
    case 2: return launch_cfg<T, 32, 8, f32 ? 4 : 2>(a, zchunk, mode, at, stream);
    case 3: return launch_cfg<T, 32, 4, f32 ? 2 : 1>(a, zchunk, mode, at, stream);
    case 4: return launch_cfg<T, 64, 4, f32 ? 3 : 2>(a, zchunk, mode, at, stream);
    case 5: return launch_cfg<T, 16, 8, 2>(a, zchunk, mode, at, stream);
    case 6: return launch_cfg<T, 16, 16, f32 ? 4 : 2>(a, zchunk, mode, at, stream);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fused<double>(const StageArgs<double>&, int, int, int, bool, hipStream_t);
template hipError_t launch_fused<float>(const StageArgs<float>&, int, int, int, bool, hipStream_t);

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

int64_t view_blocks(const Geom& g) { return (g.slab[0] + g.slab[1] + g.slab[2]) / 2 / 256 + 1; }

namespace {
template <typename T, int BX, int BY, int MINW>
hipError_t launch_batch_cfg(const void* runs, const uint2* work, int64_t nblk, bool forced, bool publish, int at,
                            int mode, hipStream_t stream) {
  if constexpr (stage_static_lds<T, BX, BY>() > kLdsBytes) {
    return hipErrorInvalidConfiguration;
  } else {
    const size_t dyn = forced ? sizeof(T) * 18 * BX * BY : 0;
    const dim3 grid((unsigned)nblk), block(Tile<BX, BY>::NT);
    const FArgs<T>* r = (const FArgs<T>*)runs;
    constexpr int MA = fp64_at_cap<T, BX, BY>(at_waves<BX, BY>(MINW));
    constexpr int MP = fp64_at_cap<T, BX, BY>(pub_at_waves<T, BX, BY>(MA));
    constexpr int MS = fp64_at_cap<T, BX, BY>(sub_waves<T, BX, BY>(MINW));
    if (at == 0) {
      if (publish)
        hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MINW, true, false, false>), grid, block, dyn, stream, r, work, mode);
      else
        hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MINW, false, false, false>), grid, block, dyn, stream, r, work, mode);
    }
    if (at & kAtMasked) {
      if (publish)
        hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MP, true, true, false>), grid, block, dyn, stream, r, work, mode);
      else
        hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MA, false, true, false>), grid, block, dyn, stream, r, work, mode);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (at & kAtGhost) {
      if (publish)
        hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MS, true, true, true>), grid, block, dyn, stream, r, work, mode);
      else
        hipLaunchKernelGGL((k_stage_batch<T, BX, BY, MS, false, true, true>), grid, block, dyn, stream, r, work, mode);
    }
    return hipGetLastError();
  }
}
}  // namespace

template <typename T>
hipError_t launch_fused_batch(const void* runs, const uint2* work, int64_t nblk, int tile, bool forced, bool publish,
                              int at, int mode, hipStream_t stream) {
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidValue;
  if (fused_lds_bytes(tile, sizeof(T), forced) > kLdsBytes) return hipErrorInvalidConfiguration;
  constexpr bool f32 = sizeof(T) == 4;
  switch (tile) {
    case 0: return launch_batch_cfg<T, 64, 8, f32 ? 4 : 2>(runs, work, nblk, forced, publish, at, mode, stream);
    case 1: return launch_batch_cfg<T, 32, 8, f32 ? 2 : 1>(runs, work, nblk, forced, publish, at, mode, stream);
    case 2: return launch_batch_cfg<T, 32, 8, f32 ? 4 : 2>(runs, work, nblk, forced, publish, at, mode, stream);
    case 3: return launch_batch_cfg<T, 32, 4, f32 ? 2 : 1>(runs, work, nblk, forced, publish, at, mode, stream);
    case 4: return launch_batch_cfg<T, 64, 4, f32 ? 3 : 2>(runs, work, nblk, forced, publish, at, mode, stream);
    case 5: return launch_batch_cfg<T, 16, 8, 2>(runs, work, nblk, forced, publish, at, mode, stream);
    case 6: return launch_batch_cfg<T, 16, 16, f32 ? 4 : 2>(runs, work, nblk, forced, publish, at, mode, stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_at_sums_batch(const void* runs, const uint2* work, int64_t nblk, const double* cs,
                                hipStream_t stream) {
  if (nblk <= 0 || nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_at_sums_batch<T>, dim3((unsigned)nblk), dim3(256), 0, stream, (const FArgs<T>*)runs,
                     work, (T)cs[0], (T)cs[1], (T)cs[2]);
  return hipGetLastError();
}

template size_t batch_arg_bytes<float>();
template size_t batch_arg_bytes<double>();
template void pack_batch_arg<float>(const StageArgs<float>&, int, int, int, void*);
template void pack_batch_arg<double>(const StageArgs<double>&, int, int, int, void*);
template hipError_t launch_fused_batch<float>(const void*, const uint2*, int64_t, int, bool, bool, int, int, hipStream_t);
template hipError_t launch_fused_batch<double>(const void*, const uint2*, int64_t, int, bool, bool, int, int, hipStream_t);
template hipError_t launch_at_sums_batch<float>(const void*, const uint2*, int64_t, const double*, hipStream_t);
template hipError_t launch_at_sums_batch<double>(const void*, const uint2*, int64_t, const double*, hipStream_t);

}  // namespace atns
