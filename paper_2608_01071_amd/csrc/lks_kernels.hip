// lks_kernels.hip -- gfx950 kernels of the LKS + Brinkman forward march, its
// exact discrete adjoint and the paper's ALKS reverse sweep, and the
// optimiser-side design prelude (Tanabe, Yaji, Ushijima, Secs. 2.2-2.6, 3.1).
//
// Data layout: analysis fields are SoA planes [d+1][N] (x fastest); the
// pressure plane holds p - 1/3, which keeps the 1/3 offset out of every
// rounding in FP32.  Body fields live on the step's support box (fixed
// strides).  Sums that span the whole run (objective, shape and motion
// sensitivities) are FP64 in fixed order; nothing on the hot path uses
// floating-point atomics, so results are reproducible bit for bit.
//
// Kernel map:
//   k_fwd2d / k_fwd3d   one LKS step: velocity gradient, Inamuro equilibrium,
//                       neighbour gather, Brinkman correction, wall rule,
//                       J1 partials.  LDS tile with a 2-node halo; the 3D
//                       kernel marches z through a 3-plane ring.
//   k_adj2d / k_adj3d   exact transpose of one step (objective seed, wall
//                       rule, Brinkman correction, gather, equilibrium,
//                       velocity gradient), emitting dJ/dkappa and dJ/du_s
//                       on the body box.  The ALK instantiations run the
//                       ALKS of Sec. 2.5 instead: the same adjoint
//                       equilibrium, with the seed and Brinkman sources on
//                       the raw first moment only.
//   k_map2d / k_map3d   per-step rigid transform and cosine-kernel transfer
//                       design grid -> analysis box (deterministic gather).
//   k_mapadj            transpose of the transfer per design point:
//                       dJ/dkappa_ref accumulation and per-step motion
//                       partials (block-reduced, fixed order).
//   prelude / epilogue  temporal filter, bounds, time differences, box and
//                       domain check, kappa_ref, objective finalisation and
//                       the sensitivity chain rule.
//   k_design_* k_con_*  once per design iteration: density filter and
//                       Heaviside projection with their chain rule, and the
//                       constraint functionals G1-G3 (Sec. 3.1, Sec. 2.6).
#include <math.h>
#include <string.h>

#include <mutex>
#include <type_traits>

#include "lks_internal.h"

namespace lks {

// ------------------------------------------------------------ helpers
__device__ __forceinline__ bool wrap_axis(const Geo& g, int a, int& v) {
  if (v >= 0 && v < g.n[a]) return true;
  if (g.bc[a] == 0) {
    v %= g.n[a];
    if (v < 0) v += g.n[a];
    return true;
  }
  return false;
}
__device__ __forceinline__ bool on_wall(const Geo& g, int a, int v) {
  return g.bc[a] == 1 && (v == 0 || v == g.n[a] - 1);
}
__device__ __forceinline__ bool is_wall(const Geo& g, int x, int y, int z) {
  bool w = on_wall(g, 0, x) || on_wall(g, 1, y);
  if (g.d == 3) w = w || on_wall(g, 2, z);
  return w;
}
__device__ __forceinline__ long long nidx(const Geo& g, int x, int y, int z) {
  return x + (long long)g.n[0] * (y + (long long)g.n[1] * z);
}
__device__ __forceinline__ int inward(const Geo& g, int a, int v) {
  if (g.bc[a] != 1) return v;
  if (v == 0) return 1;
  if (v == g.n[a] - 1) return g.n[a] - 2;
  return v;
}
__device__ __forceinline__ long long wall_src(const Geo& g, int x, int y, int z) {
  return nidx(g, inward(g, 0, x), inward(g, 1, y), g.d == 3 ? inward(g, 2, z) : z);
}
// Imposed velocity at a wall node (the highest wall axis wins).
__device__ __forceinline__ void wall_vel(const Geo& g, int x, int y, int z, double u[3]) {
  u[0] = u[1] = u[2] = 0.0;
  const int c[3] = {x, y, z};
  _Pragma("unroll") for (int a = 0; a < 3; ++a) if (a < g.d) {
    if (g.bc[a] != 1) continue;
    int side = -1;
    if (c[a] == 0) side = 0;
    if (c[a] == g.n[a] - 1) side = 1;
    if (side < 0) continue;
    for (int k = 0; k < 3; ++k) u[k] = g.uw[a][side][k];
  }
}
__device__ __forceinline__ bool in_target(const Geo& g, int x, int y, int z) {
  if (x < g.tlo[0] || x >= g.thi[0] || y < g.tlo[1] || y >= g.thi[1]) return false;
  if (g.d == 3 && (z < g.tlo[2] || z >= g.thi[2])) return false;
  return true;
}
// Body-box local index of a (wrapped) node, -1 outside this step's box.
__device__ __forceinline__ long long box_index(const Geo& g, const Box& b, int x, int y, int z) {
  const int c[3] = {x, y, z};
  int r[3] = {0, 0, 0};
  _Pragma("unroll") for (int a = 0; a < 3; ++a) if (a < g.d) {
    int v = c[a] - b.lo[a];
    if (g.bc[a] == 0) {
      v %= g.n[a];
      if (v < 0) v += g.n[a];
    }
    if (v < 0 || v >= b.ext[a]) return -1;
    r[a] = v;
  }
  return r[0] + (long long)b.sx * (r[1] + (long long)b.sy * r[2]);
}

// Whether (wrapped) coordinate v of axis ax lies in [lo, lo + ext) of a
// step's body box (periodic axes measure the offset modulo n).
__device__ __forceinline__ bool in_step_box(const Geo& g, const StepInfo* si, int ax, int v) {
  int r = v - si->lo[ax];
  if (g.bc[ax] == 0) {
    r %= g.n[ax];
    if (r < 0) r += g.n[ax];
  }
  return r >= 0 && r < si->ext[ax];
}

// Step box from the device table (when given).
__device__ __forceinline__ void apply_step(Box& b, const StepInfo* si) {
  if (!si) return;
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = si->lo[k];
    b.ext[k] = si->ext[k];
  }
}

// Cosine kernel w(r) = (1 + cos(pi r / 2)) / 4 and its derivative (Sec. 2.3),
// for |r| <= 2, as w = cos^2(y) / 2 and w' = -(pi / 4) sin(y) cos(y) with
// y = pi r / 4 in [-pi/2, pi/2].  Single precision takes the Taylor series of
// cos through y^12 and of sin through y^13 (below 7e-9 from the functions),
// double precision those through y^20 and y^21 (below 2e-17); the
// coefficients absorb the powers of pi / 4 so the polynomials run in r^2.
namespace wpoly {
constexpr double Q = 0.78539816339744830962;  // pi / 4
constexpr double Q2 = Q * Q;
constexpr float c1 = (float)(-Q2 / 2), c2 = (float)(Q2 * Q2 / 24),
                c3 = (float)(-Q2 * Q2 * Q2 / 720), c4 = (float)(Q2 * Q2 * Q2 * Q2 / 40320),
                c5 = (float)(-Q2 * Q2 * Q2 * Q2 * Q2 / 3628800.0),
                c6 = (float)(Q2 * Q2 * Q2 * Q2 * Q2 * Q2 / 479001600.0);
constexpr float s0 = (float)Q, s1 = (float)(-Q * Q2 / 6), s2 = (float)(Q * Q2 * Q2 / 120),
                s3 = (float)(-Q * Q2 * Q2 * Q2 / 5040), s4 = (float)(Q * Q2 * Q2 * Q2 * Q2 / 362880),
                s5 = (float)(-Q * Q2 * Q2 * Q2 * Q2 * Q2 / 39916800.0),
                s6 = (float)(Q * Q2 * Q2 * Q2 * Q2 * Q2 * Q2 / 6227020800.0);
__device__ __forceinline__ float cosq(float z) {  // cos(pi r / 4), z = r^2
  return fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(c6, z, c5), z, c4), z, c3), z, c2), z, c1), z, 1.0f);
}
__device__ __forceinline__ float sinq(float r, float z) {  // sin(pi r / 4)
  return r * fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(s6, z, s5), z, s4), z, s3), z, s2), z, s1), z, s0);
}
// double precision: coefficient k of cos(pi r / 4) and of sin(pi r / 4) / r
// as series in z = r^2
constexpr double ccos(int k) {
  double v = 1.0;
  for (int i = 1; i <= k; ++i) v *= -Q2 / ((2.0 * i - 1.0) * (2.0 * i));
  return v;
}
constexpr double csin(int k) {
  double v = Q;
  for (int i = 1; i <= k; ++i) v *= -Q2 / ((2.0 * i) * (2.0 * i + 1.0));
  return v;
}
__device__ __forceinline__ double cosq(double z) {
  constexpr double a0 = ccos(0), a1 = ccos(1), a2 = ccos(2), a3 = ccos(3), a4 = ccos(4),
                   a5 = ccos(5), a6 = ccos(6), a7 = ccos(7), a8 = ccos(8), a9 = ccos(9),
                   a10 = ccos(10);
  double p = fma(fma(fma(fma(fma(a10, z, a9), z, a8), z, a7), z, a6), z, a5);
  return fma(fma(fma(fma(fma(p, z, a4), z, a3), z, a2), z, a1), z, a0);
}
__device__ __forceinline__ double sinq(double r, double z) {
  constexpr double b0 = csin(0), b1 = csin(1), b2 = csin(2), b3 = csin(3), b4 = csin(4),
                   b5 = csin(5), b6 = csin(6), b7 = csin(7), b8 = csin(8), b9 = csin(9),
                   b10 = csin(10);
  double p = fma(fma(fma(fma(fma(b10, z, b9), z, b8), z, b7), z, b6), z, b5);
  return r * fma(fma(fma(fma(fma(p, z, b4), z, b3), z, b2), z, b1), z, b0);
}
}  // namespace wpoly
__device__ __forceinline__ float wk(float r) {
  const float c = wpoly::cosq(r * r);
  return 0.5f * c * c;
}
__device__ __forceinline__ double wk(double r) {
  const double c = wpoly::cosq(r * r);
  return 0.5 * c * c;
}
__device__ __forceinline__ float wkd(float r) {
  const float z = r * r;
  return -0.78539816f * wpoly::sinq(r, z) * wpoly::cosq(z);
}
__device__ __forceinline__ double wkd(double r) {
  const double z = r * r;
  return -0.78539816339744830962 * wpoly::sinq(r, z) * wpoly::cosq(z);
}

// Derivative along one axis from an LDS row (stride st): central, or
// second-order one-sided on a wall node.  The one-sided forms name their
// fused multiply-add (a sum of two products may otherwise be fused either
// way), so every kernel that inlines this rounds alike.
template <class R>
__device__ __forceinline__ R dnum(const Geo& g, int a, int v, const R* s, int c, int st) {
  if (g.bc[a] == 1) {
    if (v == 0) return fma(R(-1.5), s[c], R(2) * s[c + st]) - R(0.5) * s[c + 2 * st];
    if (v == g.n[a] - 1) return fma(R(1.5), s[c], R(-2) * s[c - st]) + R(0.5) * s[c - 2 * st];
  }
  return R(0.5) * (s[c + st] - s[c - st]);
}
// Transpose of dnum at node coordinate v: sum_x D[x][v] gv(x), reading the
// LDS row around index c.
template <class R>
__device__ __forceinline__ R dnumT(const Geo& g, int a, int v, const R* s, int c, int st) {
  if (g.bc[a] != 1) return R(0.5) * (s[c - st] - s[c + st]);
  const int n = g.n[a];
  R r = R(0);
  if (v == 0) r += R(-1.5) * s[c];
  if (v == n - 1) r += R(1.5) * s[c];
  if (v - 1 >= 0) r += (v - 1 == 0 ? R(2) : R(0.5)) * s[c - st];
  if (v + 1 <= n - 1) r += (v + 1 == n - 1 ? R(-2) : R(-0.5)) * s[c + st];
  if (v - 2 == 0) r += R(-0.5) * s[c - 2 * st];
  if (v + 2 == n - 1) r += R(0.5) * s[c + 2 * st];
  return r;
}

// dnumT at node coordinate v as weights of the row entries at offsets
// -2 .. +2 (k[2 + o]): the same terms, so a wall node's transpose is one
// straight-line 5-tap sum.
template <class R>
__device__ __forceinline__ void dnumT_taps(const Geo& g, int a, int v, R k[5]) {
  const int n = g.n[a];
  for (int q = 0; q < 5; ++q) k[q] = R(0);
  if (g.bc[a] != 1) {
    k[1] = R(0.5);
    k[3] = R(-0.5);
    return;
  }
  if (v == 0) k[2] += R(-1.5);
  if (v == n - 1) k[2] += R(1.5);
  if (v - 1 >= 0) k[1] = v - 1 == 0 ? R(2) : R(0.5);
  if (v + 1 <= n - 1) k[3] = v + 1 == n - 1 ? R(-2) : R(-0.5);
  if (v - 2 == 0) k[0] = R(-0.5);
  if (v + 2 == n - 1) k[4] = R(0.5);
}

// XCD-aware tile order.  Workgroups are dealt to the device's XCDs (nx, 8
// on MI355X, queried at plan time) round robin by their linear id, and each
// XCD has its own L2; this remap gives every XCD a contiguous run of tiles
// (x fastest, then y, then z segment), so tiles that share halo nodes run on
// the same XCD and hit the same L2.
__device__ __forceinline__ int xcd_tile_of(int b, int nx, int nbx, int nby, int nbz, int& bx,
                                           int& by, int& bz) {
  const int total = nbx * nby * nbz;
  const int xcd = b % nx, slot = b / nx;
  const int q = total / nx, r = total % nx;
  const int t = (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
  bx = t % nbx;
  by = (t / nbx) % nby;
  bz = t / (nbx * nby);
  return t;
}
__device__ __forceinline__ int xcd_tile(int nx, int nbx, int nby, int nbz, int& bx, int& by,
                                        int& bz) {
  return xcd_tile_of(blockIdx.x, nx, nbx, nby, nbz, bx, by, bz);
}
__device__ __forceinline__ int tiles_x(const Geo& g) { return (g.n[0] - g.org[0] + TILE_X - 1) / TILE_X; }
__device__ __forceinline__ int tiles_y(const Geo& g) { return (g.n[1] - g.org[1] + g.ty3 - 1) / g.ty3; }
__host__ __device__ inline int adj2d_tiles_y(const Geo& g) {
  return (g.n[1] - g.org[1] + ADJ2D_TY - 1) / ADJ2D_TY;
}
__device__ __forceinline__ int tiles_z(const Geo& g) { return g.d == 3 ? (g.n[2] + g.zseg - 1) / g.zseg : 1; }

// Lattice constants of the equilibria in the state type.  In FP32 the
// nearest floats of the weights sum to 1 + 7e-9 and the velocity
// coefficients 3 w_i (summed over c_ia^2) to 1 + 3e-8: a per-step gain on the
// pressure and velocity that compounds over thousands of steps (a 4e-5
// relative drift of J1 over 5000 steps).  The FP32 set moves one weight and
// one velocity coefficient by one ulp so both sums are exactly 1
// (sum_i w_i = 1, sum_i 3 w_i c_ix^2 = 1); the isotropy error this leaves is
// 1e-7.  FP64 uses the nearest doubles.
template <class R>
struct EqC {
  static constexpr R w0_9 = R(4.0 / 9.0), wa = R(1.0 / 9.0), wd_9 = R(1.0 / 36.0);
  static constexpr R w0_15 = R(2.0 / 9.0), wd_15 = R(1.0 / 72.0);
  static constexpr R ca = R(1.0 / 3.0), cd_9 = R(1.0 / 12.0), cd_15 = R(1.0 / 24.0);
  static constexpr R third_hi = R(1.0 / 3.0), third_lo = R(0);
};
template <>
struct EqC<float> {
  static constexpr float w0_9 = 0x1.c71c72p-2f, wa = 0x1.c71c72p-4f, wd_9 = 0x1.c71c70p-6f;
  static constexpr float w0_15 = 0x1.c71c72p-3f, wd_15 = 0x1.c71c70p-7f;
  static constexpr float ca = 0x1.555556p-2f, cd_9 = 0x1.555554p-4f, cd_15 = 0x1.555554p-5f;
  // 1/3 = third_hi + third_lo to about 1e-16
  static constexpr float third_hi = 0x1.555556p-2f, third_lo = -0x1.555556p-27f;
};
// x / 3 without the bias of the rounded constant 1/3.
template <class R>
__device__ __forceinline__ R third_of(R x) {
  if constexpr (sizeof(R) == 4)
    return fmaf(x, EqC<float>::third_lo, x * EqC<float>::third_hi);
  else
    return x * R(1.0 / 3.0);
}

// Brinkman factor 1 / (1 + kappa).  FP32: the hardware reciprocal refined by
// one Newton step (within an ulp of the quotient, 3 instructions instead of
// the IEEE division sequence); FP64: the division.
template <class R>
__device__ __forceinline__ R brinkman_inv(R k) {
  if constexpr (sizeof(R) == 4) {
    const float d = 1.0f + k;
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(r, fmaf(-d, r, 1.0f), r);
  } else {
    return 1.0 / (1.0 + k);
  }
}

// Buffer-resource access with a per-thread byte offset (VGPR) and a uniform
// byte offset (SGPR): the 3D step kernels keep the per-thread part of every
// address fixed over their z march.  Offsets past the resource's size read 0
// and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
template <class R>
__device__ __forceinline__ R bld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(R) == 4)
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// N consecutive values from a buffer resource at byte offset `off` (4-byte
// aligned), in 16-byte loads and one 8- or 4-byte remainder.
template <class R, int N>
__device__ __forceinline__ void bld_run(__amdgpu_buffer_rsrc_t r, unsigned off, R* out) {
  constexpr int W = 16 / (int)sizeof(R);  // values per 16-byte load
#pragma unroll
  for (int k = 0; k + W <= N; k += W) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(off + k * sizeof(R)), 0, 0);
    const R* pv = reinterpret_cast<const R*>(&v);
#pragma unroll
    for (int q = 0; q < W; ++q) out[k + q] = pv[q];
  }
  constexpr int D = N / W * W;
  if constexpr (N - D >= 2 && sizeof(R) == 4) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(off + D * sizeof(R)), 0, 0);
    const R* pv = reinterpret_cast<const R*>(&v);
    out[D] = pv[0];
    out[D + 1] = pv[1];
    if constexpr (N - D == 3) out[D + 2] = bld<R>(r, off + (D + 2) * sizeof(R), 0);
  } else if constexpr (N - D == 1) {
    out[D] = bld<R>(r, off + D * sizeof(R), 0);
  }
}
template <class R>
__device__ __forceinline__ void bst(R v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(R) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
  } else {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, 0);
  }
}

// Doubled one-sided wall derivative (second order) of an LDS row: at the low
// wall o = +stride, at the high wall o = -stride and the result is negated.
template <class R>
__device__ __forceinline__ R dwall2(const R* s, int c, int o) {
  return R(-3) * s[c] + R(4) * s[c + o] - s[c + 2 * o];
}

// Inamuro equilibria for one node (pairs of opposite directions share
// their even part).  S holds D_a u_b + D_b u_a.  Sums of two products name
// their fused multiply-add, so the 2D kernels that inline this (one step,
// step with map, batched) round alike.
template <class R>
__device__ __forceinline__ void feq9(R p, R ux, R uy, R Sxx, R Syy, R Sxy, R A, R* f) {
  using C = EqC<R>;
  const R base = fma(R(-1.5), fma(uy, uy, ux * ux), R(3) * p);
  f[0] = C::w0_9 * base;
  auto pair = [&](int i, R w, R c3w, R cu, R cSc) {
    R com = w * (base + R(4.5) * cu * cu + A * cSc);
    f[i] = fma(c3w, cu, com);
    f[i + 1] = fma(-c3w, cu, com);
  };
  pair(1, C::wa, C::ca, ux, Sxx);
  pair(3, C::wa, C::ca, uy, Syy);
  pair(5, C::wd_9, C::cd_9, ux + uy, Sxx + Syy + R(2) * Sxy);
  pair(7, C::wd_9, C::cd_9, uy - ux, Sxx + Syy - R(2) * Sxy);
}
// D3Q15: the diagonal arguments are S_aa = 2 D_a u_a as above, the
// off-diagonal ones twice S_ab (the sums of raw central differences, which
// need no scaling).
template <class R>
__device__ __forceinline__ void feq15(R p, R ux, R uy, R uz, R Sxx, R Syy, R Szz, R Txy, R Txz,
                                      R Tyz, R A, R* f) {
  using C = EqC<R>;
  const R base = R(3) * p - R(1.5) * (ux * ux + uy * uy + uz * uz);
  f[0] = C::w0_15 * base;
  // w (base + 4.5 (c.u)^2 + A cSc) +- 3 w c.u, with w base and w A formed
  // once per weight class (4.5 w is 1/2 on the axes, 1/16 on the diagonals)
  const R wab = C::wa * base, wdb = C::wd_15 * base;
  const R waA = C::wa * A, wdA = C::wd_15 * A;
  auto pair = [&](int i, R wb, R w45, R wA, R c3w, R cu, R cSc) {
    const R com = fma(wA, cSc, fma(w45 * cu, cu, wb));
    f[i] = fma(c3w, cu, com);
    f[i + 1] = fma(-c3w, cu, com);
  };
  pair(1, wab, R(0.5), waA, C::ca, ux, Sxx);
  pair(3, wab, R(0.5), waA, C::ca, uy, Syy);
  pair(5, wab, R(0.5), waA, C::ca, uz, Szz);
  // the four diagonal pairs share partial sums of c.u and c S c
  const R tr = Sxx + Syy + Szz;
  const R a = uy + uz, b = uy - uz;
  const R s1 = tr + Tyz, s2 = tr - Tyz, d1 = Txy + Txz, d2 = Txy - Txz;
  pair(7, wdb, R(0.0625), wdA, C::cd_15, ux + a, s1 + d1);    // (1,1,1)
  pair(9, wdb, R(0.0625), wdA, C::cd_15, a - ux, s1 - d1);    // (-1,1,1)
  pair(11, wdb, R(0.0625), wdA, C::cd_15, ux - b, s2 - d2);   // (1,-1,1)
  pair(13, wdb, R(0.0625), wdA, C::cd_15, ux + b, s2 + d2);   // (1,1,-1)
}

// Block-wide fixed-order sum of K doubles per thread into out[0..K) (thread 0).
template <int K, int NT>
__device__ __forceinline__ void block_sum(double (&v)[K], double* out) {
  __shared__ double red[NT / 64][K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) red[wv][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[w][k];
      out[k] = s;
    }
  }
}

// Brinkman correction, wall rule, objective partials and store of one
// output node.  acc = (sum_i feq_i, sum_i c_i feq_i) gathered at x; the body
// fields (bin: node in the box) are loaded by the caller ahead of time.
template <class R>
__device__ __forceinline__ void finish_node(const Geo& g, const FwdArgs& a, int x, int y, int z,
                                            R sp, R sux, R suy, R suz, double& s1, double& s2,
                                            bool bin, R bkv, const R (&buv)[3]) {
  R* out = (R*)a.out;
  const long long N = g.N;
  const long long i = nidx(g, x, y, z);
  R u[3];
  R p;
  if (is_wall(g, x, y, z)) {
    double uw[3];
    wall_vel(g, x, y, z, uw);
    u[0] = (R)uw[0];
    u[1] = (R)uw[1];
    u[2] = (R)uw[2];
    p = R(0);  // wall pressure follows the wall rule when read
  } else {
    p = third_of(sp);
    u[0] = sux;
    u[1] = suy;
    u[2] = suz;
    if (bin) {
      const R inv = brinkman_inv(bkv);
      _Pragma("unroll") for (int c = 0; c < 3; ++c) if (c < g.d) u[c] = (u[c] + bkv * buv[c]) * inv;
    }
    R uu = u[0] * u[0] + u[1] * u[1] + (g.d == 3 ? u[2] * u[2] : R(0));
    if (a.flags && !(uu < R(0.25))) a.flags[0] = 1;  // non-finite or |u| >= 0.5
  }
  out[i] = p;
  out[N + i] = u[0];
  out[2 * N + i] = u[1];
  if (g.d == 3) out[3 * N + i] = u[2];
  if (a.opart && in_target(g, x, y, z)) {
    double un = g.ndir[0] * (double)u[0] + g.ndir[1] * (double)u[1];
    if (g.d == 3) un += g.ndir[2] * (double)u[2];
    s1 += un;
    s2 += un * un;
  }
}

// ------------------------------------------------------ forward, D2Q9
template <class R>
__device__ __forceinline__ void fwd2d_tile(const Geo& g, FwdArgs a, int bid) {
  apply_step(a.box, a.si);
  constexpr int TX = TILE_X, TY = TILE_Y;
  constexpr int LX = TX + 4, LY = TY + 4, FX = TX + 2, FY = TY + 2;
  __shared__ R sp[LY * LX], sx[LY * LX], sy[LY * LX];
  __shared__ R sf[9][FY * FX];
  const R* in = (const R*)a.in;
  const long long N = g.N;
  int tbx, tby, tbz;
  const int tlin = xcd_tile_of(bid, g.nxcd, tiles_x(g), tiles_y(g), 1, tbx, tby, tbz);
  const int x0 = tbx * TX + g.org[0], y0 = tby * TY + g.org[1];
  // the body fields of this thread's output node are loaded first, so their
  // latency overlaps the state loads and the equilibria
  static_assert(STEP_THREADS == TX * TY, "one output node per thread");
  const int otx = threadIdx.x % TX, oty = threadIdx.x / TX;
  const int ogx = x0 + otx, ogy = y0 + oty;
  const bool oown = ogx >= 0 && ogx < g.n[0] && ogy >= 0 && ogy < g.n[1];
  bool bin = false;
  R bkv = R(0), buv[3] = {R(0), R(0), R(0)};
  if (oown && a.bk && !is_wall(g, ogx, ogy, 0)) {
    const long long bi = box_index(g, a.box, ogx, ogy, 0);
    if (bi >= 0) {
      const R* bk = (const R*)a.bk;
      const R* bu = (const R*)a.bu;
      bin = true;
      bkv = bk[bi];
      buv[0] = bu[bi];
      buv[1] = bu[a.box.vol + bi];
    }
  }
  for (int k = threadIdx.x; k < LX * LY; k += STEP_THREADS) {
    int gx = x0 - 2 + k % LX, gy = y0 - 2 + k / LX;
    R p = R(0), ux = R(0), uy = R(0);
    if (wrap_axis(g, 0, gx) && wrap_axis(g, 1, gy)) {
      long long i = nidx(g, gx, gy, 0);
      ux = in[N + i];
      uy = in[2 * N + i];
      long long ip = (a.lazy_wall && is_wall(g, gx, gy, 0)) ? wall_src(g, gx, gy, 0) : i;
      p = in[ip];
    }
    sp[k] = p;
    sx[k] = ux;
    sy[k] = uy;
  }
  __syncthreads();
  const R A = (R)g.A;
  for (int k = threadIdx.x; k < FX * FY; k += STEP_THREADS) {
    int fx = k % FX, fy = k / FX;
    int gx = x0 - 1 + fx, gy = y0 - 1 + fy;
    R f[9];
    if (wrap_axis(g, 0, gx) && wrap_axis(g, 1, gy)) {
      const int c = (fy + 1) * LX + (fx + 1);
      R dxux = dnum(g, 0, gx, sx, c, 1), dxuy = dnum(g, 0, gx, sy, c, 1);
      R dyux = dnum(g, 1, gy, sx, c, LX), dyuy = dnum(g, 1, gy, sy, c, LX);
      feq9(sp[c], sx[c], sy[c], R(2) * dxux, R(2) * dyuy, dxuy + dyux, A, f);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = R(0);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) sf[i][k] = f[i];
  }
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
  {
    const int tx = otx, ty = oty;
    const int gx = ogx, gy = ogy;
    if (oown) {
      const int c = (ty + 1) * FX + (tx + 1);
      R P = R(0), Ux = R(0), Uy = R(0);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int cx = Lat<9>::c[i][0], cy = Lat<9>::c[i][1];
        R v = sf[i][c - cx - cy * FX];
        P += v;
        if (cx == 1) Ux += v;
        if (cx == -1) Ux -= v;
        if (cy == 1) Uy += v;
        if (cy == -1) Uy -= v;
      }
      finish_node<R>(g, a, gx, gy, 0, P, Ux, Uy, R(0), s1, s2, bin, bkv, buv);
    }
  }
  if (a.opart) {
    double v[2] = {s1, s2};
    double tot[2];
    block_sum<2, STEP_THREADS>(v, tot);
    if (threadIdx.x == 0) {
      a.opart[2 * tlin] += tot[0];
      a.opart[2 * tlin + 1] += tot[1];
    }
  }
}

template <class R>
__global__ __launch_bounds__(STEP_THREADS) void k_fwd2d(Geo g, FwdArgs a) {
  fwd2d_tile<R>(g, a, blockIdx.x);
}

// One node's (u_x, u_y, u_z, p) in LDS: the 3D step kernels read a
// neighbour's values with one 16-byte (or, for u alone, 12-byte) access.
template <class R>
struct alignas(4 * sizeof(R)) Q4 {
  R x, y, z, p;
};

// ------------------------------------------------------ forward, D3Q15
// Block = one 32 x Tile3<R>::TY column tile marching z over a z segment
// (the launcher passes the forward's segment length in g.zseg).  Per plane:
// (1) the (p, u) plane with a 2-node halo enters a 3-plane LDS ring from
// registers filled two planes ahead (the global loads overlap the
// arithmetic of the planes in between); (2) the 15 equilibria of the plane
// are formed on the 1-node halo region, the 12 that move within the plane go
// through LDS; (3) each output column adds them into the accumulators of the
// three output planes they feed; the plane below is then complete and is
// finished (Brinkman, walls, J1).  In FP32 (32 x 16 tiles, 768 threads,
// 66 KB of LDS, at most 80 VGPRs) two blocks are resident per CU.
// Node offsets within a plane set are 32-bit (plan validation bounds N).
template <class R>
__global__ __launch_bounds__(Tile3<R>::NT, sizeof(R) == 4 ? 6 : 3) void k_fwd3d(Geo g, FwdArgs a) {
  apply_step(a.box, a.si);
  constexpr int TX = TILE_X, TY = Tile3<R>::TY, NT = Tile3<R>::NT;
  constexpr int LX = TX + 4, LY = TY + 4, FX = TX + 2, FY = TY + 2;
  constexpr int LP = LX * LY, FP = FX * FY;
  static_assert(NT >= LP && NT >= FP, "one load and one equilibrium slot per thread");
  // planes (mod 3): p, ux, uy, uz; entries LP.. take the commits of idle slots
  __shared__ R ring[3][4][NT];
  __shared__ R sf[12][FP];  // the 12 equilibria that move within the plane
  const int N = (int)g.N;
  constexpr unsigned es = sizeof(R);
  const unsigned fb = (unsigned)N * es;  // bytes of one field (4 fields fit 32 bits)
  const __amdgpu_buffer_rsrc_t rin = brsrc(a.in, 4u * fb);
  const int nz = g.n[2];
  const int NP = g.n[0] * g.n[1];
  int tbx, tby, tbz;
  const int tlin = xcd_tile(g.nxcd, tiles_x(g), tiles_y(g), tiles_z(g), tbx, tby, tbz);
  const int x0 = tbx * TX + g.org[0], y0 = tby * TY + g.org[1];
  const int z0 = tbz * g.zseg, z1 = min(z0 + g.zseg, nz);

  const int tid = threadIdx.x;
  const bool outer = tid < TX * TY;
  const int tx = tid % TX, ty = tid / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = outer && gx >= 0 && gx < g.n[0] && gy >= 0 && gy < g.n[1];
  const int oc = (ty + 1) * FX + (tx + 1);
  // column-constant data of the output node
  const bool cwall = own && (on_wall(g, 0, gx) || on_wall(g, 1, gy));
  const bool ctgt = own && a.opart && gx >= g.tlo[0] && gx < g.thi[0] && gy >= g.tlo[1] &&
                    gy < g.thi[1];
  int cbxy = -1;
  if (own && !cwall && a.bk) {
    int r0 = gx - a.box.lo[0], r1 = gy - a.box.lo[1];
    if (g.bc[0] == 0) { r0 %= g.n[0]; if (r0 < 0) r0 += g.n[0]; }
    if (g.bc[1] == 0) { r1 %= g.n[1]; if (r1 < 0) r1 += g.n[1]; }
    if (r0 >= 0 && r0 < a.box.ext[0] && r1 >= 0 && r1 < a.box.ext[1]) cbxy = r0 + a.box.sx * r1;
  }
  R cw[3] = {R(0), R(0), R(0)};
  if (cwall) {
    double uw[3];
    wall_vel(g, gx, gy, 0, uw);
    cw[0] = (R)uw[0];
    cw[1] = (R)uw[1];
    cw[2] = (R)uw[2];
  }
  const int bvol = (int)a.box.vol, bplane = a.box.sx * a.box.sy;
  const bool body = a.bk && bvol > 0;
  const bool wbody = __ballot(cbxy >= 0) != 0;  // some lane of the wave owns a box column
  const unsigned bb = (unsigned)bvol * es;  // bytes of one body field
  const __amdgpu_buffer_rsrc_t rbk = brsrc(a.bk, bb);
  const __amdgpu_buffer_rsrc_t rbu = brsrc(a.bu, 3u * bb);
  const unsigned cvo = cbxy >= 0 ? (unsigned)cbxy * es : 0u;
  const __amdgpu_buffer_rsrc_t rout = brsrc(a.out, 4u * fb);
  const unsigned ovo = own ? (unsigned)(gx + g.n[0] * gy) * es : 0u;

  // load slot of the halo plane (fixed over the march); slots outside the
  // grid or the halo read node 0 of the plane
  unsigned lvo, lpvo;  // byte offsets within a plane of (u) and (p)
  bool lok;
  {
    int hx2 = x0 - 2 + tid % LX, hy2 = y0 - 2 + tid / LX;
    lok = tid < LP && wrap_axis(g, 0, hx2) && wrap_axis(g, 1, hy2);
    const int lofs = lok ? hx2 + g.n[0] * hy2 : 0;
    const int lpofs = (lok && a.lazy_wall && is_wall(g, hx2, hy2, 0))
                          ? inward(g, 0, hx2) + g.n[0] * inward(g, 1, hy2)
                          : lofs;
    lvo = (unsigned)lofs * es;
    lpvo = (unsigned)lpofs * es;
  }
  // Register buffers of two planes in flight.  Every load and every commit
  // is unconditional (clamped plane and node), so the wait before a commit
  // counts only the loads issued after it, never the output stores.
  struct Buf {
    R v[4];
    R bk, bu[3];  // body fields of output plane zp - 2
    bool bin;
  };
  // fetches come in plane order, so the wrapped plane index zp mod nz and
  // the body-box plane (zp - 2 - lo_z) mod nz advance by one per call
  int fzw = (z0 - 2) % nz, fr2 = (z0 - 4 - a.box.lo[2]) % nz;
  if (fzw < 0) fzw += nz;
  if (fr2 < 0) fr2 += nz;
  auto fetch = [&](int zp, Buf& B) {
    const int zw = fzw, r2 = fr2;
    fzw = fzw + 1 == nz ? 0 : fzw + 1;
    fr2 = fr2 + 1 == nz ? 0 : fr2 + 1;
    B.bin = false;
    // wave-uniform skip: waves without an output column in the box (the halo
    // waves among them) and planes outside the box load no body fields
    if (body && wbody && r2 < a.box.ext[2]) {
      B.bin = cbxy >= 0 && zp - 2 >= z0 && zp - 2 < z1;
      const unsigned so = (unsigned)(bplane * r2) * es;
      B.bk = bld<R>(rbk, cvo, so);
      B.bu[0] = bld<R>(rbu, cvo, so);
      B.bu[1] = bld<R>(rbu, cvo, so + bb);
      B.bu[2] = bld<R>(rbu, cvo, so + 2u * bb);
    }
    const unsigned so = (unsigned)(NP * zw) * es;
    B.v[0] = bld<R>(rin, lpvo, so);
    B.v[1] = bld<R>(rin, lvo, so + fb);
    B.v[2] = bld<R>(rin, lvo, so + 2u * fb);
    B.v[3] = bld<R>(rin, lvo, so + 3u * fb);
  };
  // Slots outside the grid (beyond a wall) hold node 0's values, which no
  // equilibrium that is used reads: a wall node takes one-sided derivatives
  // into the grid, and the equilibria of slots outside the grid are zeroed.
  auto commit = [&](int sl, const Buf& B) {
#pragma unroll
    for (int q = 0; q < 4; ++q) ring[sl][q][tid] = B.v[q];
  };

  // equilibrium slot: threads 0..255 take their own output position (the
  // three equilibria that stay in the column, 0 and +-z, never leave
  // registers), threads 256..339 the positions of the 1-node halo ring
  const bool fok = tid < FP;
  int fx, fy;
  if (outer) {
    fx = tx + 1;
    fy = ty + 1;
  } else {
    const int r = tid - TX * TY;
    if (r < FX) {
      fx = r;
      fy = 0;
    } else if (r < 2 * FX) {
      fx = r - FX;
      fy = FY - 1;
    } else {
      const int q = r - 2 * FX;  // 0 .. 2 (FY - 2) - 1
      fx = (q & 1) ? FX - 1 : 0;
      fy = 1 + (q >> 1);
    }
  }
  const int fpos = fx + FX * fy;
  int hx = x0 - 1 + fx, hy = y0 - 1 + fy;
  const bool fin = fok && wrap_axis(g, 0, hx) && wrap_axis(g, 1, hy);
  const int fc = (fy + 1) * LX + (fx + 1);
  // wall positions take one-sided derivatives (rare: handled after the central
  // ones): direction into the grid and sign of the doubled derivative
  const bool fwx = fin && on_wall(g, 0, hx), fwy = fin && on_wall(g, 1, hy);
  const int wox = hx == 0 ? 1 : -1, woy = hy == 0 ? LX : -LX;
  const R wsx = hx == 0 ? R(1) : R(-1), wsy = hy == 0 ? R(1) : R(-1);

  R am[4] = {R(0), R(0), R(0), R(0)}, a0[4] = {R(0), R(0), R(0), R(0)},
    ap[4] = {R(0), R(0), R(0), R(0)};
  double s1 = 0.0, s2 = 0.0;
  bool bad = false;  // instability seen by this thread (reported once at the end)
  const R A = (R)g.A;

  // Iteration zf: commit plane zf+1 (buffer X) | barrier | fetch plane zf+3
  // into X | equilibria of plane zf | barrier | gather of plane zf, finish
  // of plane zf-1.
  // rs = zf mod 3: ring slots of planes zf, zf + 1, zf - 1
  auto iter = [&](int zf, int rs, Buf& X) {
    const int sc = rs, sp1 = rs == 2 ? 0 : rs + 1, sm = rs == 0 ? 2 : rs - 1;
    // the commit and the next plane's loads go out at raised wave priority,
    // so the loads enter the memory system ahead of the other block's
    // arithmetic (a scheduling hint only)
    __builtin_amdgcn_s_setprio(2);
    commit(sp1, X);
    const bool binb = X.bin;
    const R bkv = X.bk, bu0 = X.bu[0], bu1 = X.bu[1], bu2 = X.bu[2];
    __syncthreads();
    fetch(zf + 3, X);
    __builtin_amdgcn_s_setprio(0);
    R f0 = R(0), fzp = R(0), fzm = R(0);
    if (fok) {
      const R* ux = ring[sc][1];
      const R* uy = ring[sc][2];
      const R* uz = ring[sc][3];
      const int c = fc;
      // raw central differences, twice the derivatives (one-sided at walls)
      R xx = ux[c + 1] - ux[c - 1], xy = uy[c + 1] - uy[c - 1], xz = uz[c + 1] - uz[c - 1];
      R yx = ux[c + LX] - ux[c - LX], yy = uy[c + LX] - uy[c - LX], yz = uz[c + LX] - uz[c - LX];
      if (fwx) {
        xx = wsx * dwall2(ux, c, wox);
        xy = wsx * dwall2(uy, c, wox);
        xz = wsx * dwall2(uz, c, wox);
      }
      if (fwy) {
        yx = wsy * dwall2(ux, c, woy);
        yy = wsy * dwall2(uy, c, woy);
        yz = wsy * dwall2(uz, c, woy);
      }
      const R zx = ring[sp1][1][c] - ring[sm][1][c];
      const R zy = ring[sp1][2][c] - ring[sm][2][c];
      const R zz = ring[sp1][3][c] - ring[sm][3][c];
      R f[15];
      feq15(ring[sc][0][c], ux[c], uy[c], uz[c], xx, yy, zz, xy + yx, xz + zx, yz + zy, A, f);
      if (!fin) {
#pragma unroll
        for (int i = 0; i < 15; ++i) f[i] = R(0);
      }
      f0 = f[0];
      fzp = f[5];
      fzm = f[6];
#pragma unroll
      for (int i = 1; i < 15; ++i)
        if (i != 5 && i != 6) sf[i < 5 ? i - 1 : i - 3][fpos] = f[i];
    }
    __syncthreads();
    if (outer) {
      // gather plane zf into the three output planes it feeds; each group of
      // four equilibria enters through sums and differences of its pairs
      auto rd = [&](int i) {
        return sf[i < 5 ? i - 1 : i - 3][oc - Lat<15>::c[i][0] - Lat<15>::c[i][1] * FX];
      };
      const R v1 = rd(1), v2 = rd(2), v3 = rd(3), v4 = rd(4);       // c_z = 0
      const R v7 = rd(7), v9 = rd(9), v11 = rd(11), v14 = rd(14);  // c_z = +1
      const R v8 = rd(8), v10 = rd(10), v12 = rd(12), v13 = rd(13);  // c_z = -1
      a0[0] += (f0 + (v1 + v2)) + (v3 + v4);
      a0[1] += v1 - v2;
      a0[2] += v3 - v4;
      {
        // c_z = +1, the first contributions to plane zf + 1:
        // (1,1,1) (-1,1,1) (1,-1,1) (-1,-1,1)
        const R s1 = v7 + v9, s2 = v11 + v14, d1 = v7 - v9, d2 = v11 - v14;
        const R P = (s1 + s2) + fzp;
        ap[0] = P;
        ap[1] = d1 + d2;
        ap[2] = s1 - s2;
        ap[3] = P;
      }
      {
        // c_z = -1, the last contributions to plane zf - 1:
        // (1,1,-1) (-1,1,-1) (1,-1,-1) (-1,-1,-1)
        const R s1 = v13 + v12, s2 = v10 + v8, d1 = v13 - v12, d2 = v10 - v8;
        const R P = (s1 + s2) + fzm;
        am[0] += P;
        am[1] += d1 + d2;
        am[2] += s1 - s2;
        am[3] -= P;
      }
      const int zo = zf - 1;
      if (zo >= z0 && own) {
        R u0, u1, u2, p;
        if (cwall) {
          u0 = cw[0];
          u1 = cw[1];
          u2 = cw[2];
          p = R(0);  // wall pressure follows the wall rule when read
        } else {
          p = third_of(am[0]);
          u0 = am[1];
          u1 = am[2];
          u2 = am[3];
          if (binb) {
            // named fused multiply-adds: both unrolled copies round alike
            const R inv = brinkman_inv(bkv);
            u0 = fma(bkv, bu0, u0) * inv;
            u1 = fma(bkv, bu1, u1) * inv;
            u2 = fma(bkv, bu2, u2) * inv;
          }
          const R uu = u0 * u0 + u1 * u1 + u2 * u2;
          bad = bad || !(uu < R(0.25));  // non-finite or |u| >= 0.5
        }
        const unsigned so = (unsigned)(NP * zo) * es;
        bst<R>(p, rout, ovo, so);
        bst<R>(u0, rout, ovo, so + fb);
        bst<R>(u1, rout, ovo, so + 2u * fb);
        bst<R>(u2, rout, ovo, so + 3u * fb);
        if (ctgt && zo >= g.tlo[2] && zo < g.thi[2]) {
          const double un = g.ndir[0] * (double)u0 + g.ndir[1] * (double)u1 + g.ndir[2] * (double)u2;
          s1 += un;
          s2 += un * un;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        am[k] = a0[k];
        a0[k] = ap[k];
      }
    }
  };

  Buf bA, bB;
  // z0 - 1 >= -1, so z0 + 2 keeps the residues nonnegative
  const int r0 = (z0 + 2) % 3;  // slot of plane z0 - 1
  {
    // the four planes of the prologue are requested together (one memory
    // round trip before the march, not three); the body fields of t0 and t1
    // feed no output and their loads are dropped
    Buf t0, t1;
    fetch(z0 - 2, t0);
    fetch(z0 - 1, t1);
    fetch(z0, bA);
    fetch(z0 + 1, bB);
    commit(r0 == 0 ? 2 : r0 - 1, t0);
    commit(r0, t1);
  }
  // iterations z0-1 .. z1, two per trip so each buffer stays in fixed
  // registers (and every trip ends with the loads of the other buffer)
  int zf = z0 - 1, rs = r0;
  for (; zf + 1 <= z1; zf += 2) {
    iter(zf, rs, bA);
    rs = rs == 2 ? 0 : rs + 1;
    iter(zf + 1, rs, bB);
    rs = rs == 2 ? 0 : rs + 1;
  }
  if (zf <= z1) iter(zf, rs, bA);
  if (bad && a.flags) a.flags[0] = 1;
  if (a.opart) {
    double v[2] = {s1, s2};
    double tot[2];
    block_sum<2, NT>(v, tot);
    if (threadIdx.x == 0) {
      a.opart[2 * tlin] += tot[0];
      a.opart[2 * tlin + 1] += tot[1];
    }
  }
}

// ---------------------------------------------------------- adjoint helpers
// Adjoint-state value of node (x,y,z) after the objective seed, the
// transposed wall rule and the transposed Brinkman correction:
// returns (pbar*, ubar*).  Wall nodes and nodes outside the grid give 0.
// Owned nodes of the body box also emit dJ/dkappa and dJ/du_s.  ALK: the
// ALKS sources of Sec. 2.5 instead (Eq. au): seed and Brinkman act on the
// raw first-moment part X = 3 u~ alone, the coupling part passes through.
template <class R, bool ALK>
__device__ __forceinline__ void adj_star(const Geo& g, const AdjArgs& a, int x, int y, int z,
                                         bool inside, bool owned, R out[4]) {
  out[0] = out[1] = out[2] = out[3] = R(0);
  if (!inside || is_wall(g, x, y, z)) return;
  const R* lam = (const R*)a.lam;
  const R* uc = (const R*)a.u_cur;
  const long long N = g.N;
  const long long i = nidx(g, x, y, z);
  // pressure adjoint plus the wall nodes that copy this node's pressure
  R pb = lam[i];
  // wall node next to this one along each wall axis (-1: none)
  const int c[3] = {x, y, z};
  int ex[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    ex[ax] = -1;
    if (ax < g.d && g.bc[ax] == 1) {
      if (c[ax] == 1) ex[ax] = 0;
      else if (c[ax] == g.n[ax] - 2) ex[ax] = g.n[ax] - 1;
    }
  }
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    const int kx = m & 1, ky = (m >> 1) & 1, kz = m >> 2;
    if ((kx && ex[0] < 0) || (ky && ex[1] < 0) || (kz && ex[2] < 0)) continue;
    pb += lam[nidx(g, kx ? ex[0] : x, ky ? ex[1] : y, kz ? ex[2] : z)];
  }
  R ub[3];
  ub[0] = lam[N + i];
  ub[1] = lam[2 * N + i];
  ub[2] = g.d == 3 ? lam[3 * N + i] : R(0);
  R un3[3] = {R(0), R(0), R(0)};
  R sd[3] = {R(0), R(0), R(0)};  // objective seed
  bool have_u = false;
  if (a.seed && in_target(g, x, y, z)) {
    _Pragma("unroll") for (int k = 0; k < 3; ++k) if (k < g.d) un3[k] = uc[(k + 1) * N + i];
    have_u = true;
    double un = 0.0;
    _Pragma("unroll") for (int k = 0; k < 3; ++k) if (k < g.d) un += g.ndir[k] * (double)un3[k];
    double gs = a.seed[0] * g.NTinv * (1.0 - 2.0 * g.phi * (un - a.E[0]));
    _Pragma("unroll") for (int k = 0; k < 3; ++k) if (k < g.d) sd[k] = (R)(gs * g.ndir[k]);
  }
  R T[3] = {ub[0], ub[1], ub[2]};  // state as loaded
  _Pragma("unroll") for (int k = 0; k < 3; ++k) ub[k] += sd[k];
  out[0] = pb;
  if (a.bk) {
    long long bi = box_index(g, a.box, x, y, z);
    if (bi >= 0) {
      const R* bk = (const R*)a.bk;
      const R* bu = (const R*)a.bu;
      const R k = bk[bi];
      const R inv = brinkman_inv(k);
      if (a.j2s) {
        const R* js = (const R*)a.j2s;
        _Pragma("unroll") for (int q = 0; q < 2; ++q) {
          sd[q] += js[q * a.box.vol + bi];
          ub[q] += js[q * a.box.vol + bi];
        }
      }
      // the part the Brinkman correction acts on
      R xs[3] = {ub[0], ub[1], ub[2]}, X[3] = {R(0), R(0), R(0)};
      if constexpr (ALK) {
        const R* xi = (const R*)a.xin;
        _Pragma("unroll") for (int q = 0; q < 3; ++q) if (q < g.d) {
          X[q] = xi[q * N + i];
          xs[q] = X[q] + sd[q];
        }
      }
      if (owned) {
        if (!have_u)
          _Pragma("unroll") for (int q = 0; q < 3; ++q) if (q < g.d) un3[q] = uc[(q + 1) * N + i];
        R kb = R(0);
        R* bkbar = (R*)a.bkbar;
        R* bubar = (R*)a.bubar;
        _Pragma("unroll") for (int q = 0; q < 3; ++q) if (q < g.d) {
          kb += xs[q] * (bu[q * a.box.vol + bi] - un3[q]);
          bubar[q * a.box.vol + bi] = k * xs[q] * inv;
        }
        bkbar[bi] = kb * inv;
      }
      if constexpr (ALK) {
        _Pragma("unroll") for (int q = 0; q < 3; ++q) if (q < g.d) ub[q] = xs[q] * inv + (T[q] - X[q]);
      } else {
        _Pragma("unroll") for (int q = 0; q < 3; ++q) if (q < g.d) ub[q] *= inv;
      }
    }
  }
  out[1] = ub[0];
  out[2] = ub[1];
  out[3] = ub[2];
}

// ------------------------------------------------------ adjoint, D2Q9
template <class R, bool ALK>
__device__ __forceinline__ void adj2d_tile(const Geo& g, AdjArgs a, int bid) {
  apply_step(a.box, a.si);
  constexpr int TX = TILE_X, TY = ADJ2D_TY;
  constexpr int LX = TX + 4, LY = TY + 4, FX = TX + 2, FY = TY + 2;
  __shared__ R sl[3][LY * LX];     // pbar*, ubar*_x, ubar*_y
  __shared__ R sm[6][FY * FX];     // M0, M1x, M1y, M2xx, M2yy, M2xy
  const long long N = g.N;
  int tbx, tby, tbz;
  xcd_tile_of(bid, g.nxcd, tiles_x(g), adj2d_tiles_y(g), 1, tbx, tby, tbz);
  const int x0 = tbx * TX + g.org[0], y0 = tby * TY + g.org[1];
  // this thread's output node and its velocity of the previous step, loaded
  // first so the latency overlaps the gather
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool oown = ty < TY && gx >= 0 && gx < g.n[0] && gy >= 0 && gy < g.n[1];
  const long long i = oown ? nidx(g, gx, gy, 0) : 0;
  R ux = R(0), uy = R(0);
  if (oown) {
    const R* up = (const R*)a.u_prev;
    ux = up[N + i];
    uy = up[2 * N + i];
  }
  for (int k = threadIdx.x; k < LX * LY; k += ADJ2D_THREADS) {
    int lx = k % LX, ly = k / LX;
    int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
    bool inside = wrap_axis(g, 0, gx) && wrap_axis(g, 1, gy);
    bool owned = lx >= 2 && lx < TX + 2 && ly >= 2 && ly < TY + 2 && (x0 - 2 + lx) == gx &&
                 (y0 - 2 + ly) == gy;
    R v[4];
    adj_star<R, ALK>(g, a, gx, gy, 0, inside, owned, v);
    sl[0][k] = v[0];
    sl[1][k] = v[1];
    sl[2][k] = v[2];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < FX * FY; k += ADJ2D_THREADS) {
    int fx = k % FX, fy = k / FX;
    const int c = (fy + 1) * LX + (fx + 1);
    R M0 = R(0), M1x = R(0), M1y = R(0), Mxx = R(0), Myy = R(0), Mxy = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int cx = Lat<9>::c[i][0], cy = Lat<9>::c[i][1];
      const int j = c + cx + cy * LX;
      R F = sl[0][j] * R(1.0 / 3.0);
      if (cx == 1) F += sl[1][j];
      if (cx == -1) F -= sl[1][j];
      if (cy == 1) F += sl[2][j];
      if (cy == -1) F -= sl[2][j];
      const R wF = R(Lat<9>::w[i]) * F;
      M0 += wF;
      if (cx == 1) { M1x += wF; Mxx += wF; }
      if (cx == -1) { M1x -= wF; Mxx += wF; }
      if (cy == 1) { M1y += wF; Myy += wF; }
      if (cy == -1) { M1y -= wF; Myy += wF; }
      if (cx * cy == 1) Mxy += wF;
      if (cx * cy == -1) Mxy -= wF;
    }
    sm[0][k] = M0;
    sm[1][k] = M1x;
    sm[2][k] = M1y;
    sm[3][k] = Mxx;
    sm[4][k] = Myy;
    sm[5][k] = Mxy;
  }
  __syncthreads();
  if (!oown) return;
  const int c = (ty + 1) * FX + (tx + 1);
  const R M0 = sm[0][c];
  const R A2 = R(2) * (R)g.A;
  R px = R(3) * M0;
  R bx = R(3) * sm[1][c] + R(9) * (sm[3][c] * ux + sm[5][c] * uy) - R(3) * ux * M0;
  R by = R(3) * sm[2][c] + R(9) * (sm[5][c] * ux + sm[4][c] * uy) - R(3) * uy * M0;
  // velocity-gradient transpose: ubar_b += sum_a D_a^T (2 A M2_ab)
  bx += A2 * (dnumT(g, 0, gx, sm[3], c, 1) + dnumT(g, 1, gy, sm[5], c, FX));
  by += A2 * (dnumT(g, 0, gx, sm[5], c, 1) + dnumT(g, 1, gy, sm[4], c, FX));
  R* lp = (R*)a.lam_prev;
  lp[i] = px;
  lp[N + i] = bx;
  lp[2 * N + i] = by;
  if constexpr (ALK) {
    // raw first-moment part, read by the next step on its body box only
    if (a.xall ||
        (a.si_next && in_step_box(g, a.si_next, 0, gx) && in_step_box(g, a.si_next, 1, gy))) {
      R* xo = (R*)a.xout;
      xo[i] = R(3) * sm[1][c];
      xo[N + i] = R(3) * sm[2][c];
    }
    // the ALKS state itself (p~, u~, s~ = -M0, -M1, -M2), for the carry
    if (a.mout) {
      R* mo = (R*)a.mout;
      mo[i] = -M0;
      mo[N + i] = -sm[1][c];
      mo[2 * N + i] = -sm[2][c];
      mo[3 * N + i] = -sm[3][c];
      mo[4 * N + i] = -sm[4][c];
      mo[5 * N + i] = -sm[5][c];
    }
  }
}

template <class R, bool ALK>
__global__ __launch_bounds__(ADJ2D_THREADS, 2) void k_adj2d(Geo g, AdjArgs a) {
  adj2d_tile<R, ALK>(g, a, blockIdx.x);
}

// ------------------------------------------------------ adjoint, D3Q15
// Same column-tile march as the forward kernel, run on the adjoint state.
// Per plane: the adjoint state of plane z+1 (after objective seed, the
// transposed wall rule and the transposed Brinkman correction; raw loads
// fetched one iteration ahead) enters a 3-plane ring; the gather transpose
// F_i and its moments M0, M1, M2 are formed for plane z on the 1-node halo;
// plane z-1 is then finished: equilibrium transpose plus the transposed
// velocity gradient (in-plane from the moment plane, along z from the
// neighbouring planes' moments of the own column).
template <class R, bool ALK>
__global__ __launch_bounds__(Tile3<R>::NT, sizeof(R) == 4 ? 3 : 2) void k_adj3d(Geo g, AdjArgs a) {
  apply_step(a.box, a.si);
  constexpr int TX = TILE_X, TY = Tile3<R>::TY, NT = Tile3<R>::NT;
  constexpr int LX = TX + 4, LY = TY + 4, FX = TX + 2, FY = TY + 2;
  constexpr int LP = LX * LY, FP = FX * FY;
  static_assert(NT >= LP && NT >= FP, "one load and one moment slot per thread");
  constexpr int NR = AdjRing<R>::NR;  // 3: two barriers per plane, 4: one
  // adjoint star planes (mod NR); entries LP.. take the commits of idle slots
  __shared__ Q4<R> ring[NR][NT];
  __shared__ R mb[2][5][FP];  // in-plane second moments (mod 2): Mxx, Myy, Mxy, Mxz, Myz
  const int N = (int)g.N;
  // the arrays read or written on every plane go through buffer resources
  // (per-thread byte offsets fixed over the march, plane offsets uniform);
  // the conditional body and target accesses keep flat pointers
  constexpr unsigned es = sizeof(R);
  const unsigned fb = (unsigned)N * es;  // bytes of one field (4 fields fit 32 bits)
  const __amdgpu_buffer_rsrc_t rlam = brsrc(a.lam, 4u * fb);
  const __amdgpu_buffer_rsrc_t rup = brsrc(a.u_prev, 4u * fb);
  const __amdgpu_buffer_rsrc_t rlp = brsrc(a.lam_prev, 4u * fb);
  const R* ucur = (const R*)a.u_cur;
  const int bvol = (int)a.box.vol, bplane = a.box.sx * a.box.sy;
  const bool body = a.bk && bvol > 0;
  const R* bkp = (const R*)a.bk;
  const R* bup = (const R*)a.bu;
  R* bkbar = (R*)a.bkbar;
  R* bubar = (R*)a.bubar;
  const int nz = g.n[2];
  const int NP = g.n[0] * g.n[1];
  int tbx, tby, tbz;
  xcd_tile(g.nxcd, tiles_x(g), tiles_y(g), tiles_z(g), tbx, tby, tbz);
  const int x0 = tbx * TX + g.org[0], y0 = tby * TY + g.org[1];
  const int z0 = tbz * g.zseg, z1 = min(z0 + g.zseg, nz);
  const double seed = a.seed ? a.seed[0] : 0.0;
  const double Ebar = a.seed ? a.E[0] : 0.0;
  const R nd0 = (R)g.ndir[0], nd1 = (R)g.ndir[1], nd2 = (R)g.ndir[2];
  const int tid = threadIdx.x;

  // load slot of the halo plane (fixed over the march)
  int lofs, bxy;
  bool lok, ltg, lown;
  int nwn = 0, wofs[3] = {0, 0, 0};  // wall nodes that copy this node's pressure
  {
    const int lx = tid % LX, ly = tid / LX;
    int hx2 = x0 - 2 + lx, hy2 = y0 - 2 + ly;
    bool ok = tid < LP && wrap_axis(g, 0, hx2) && wrap_axis(g, 1, hy2);
    lown = ok && lx >= 2 && lx < TX + 2 && ly >= 2 && ly < TY + 2 && (x0 - 2 + lx) == hx2 &&
           (y0 - 2 + ly) == hy2;
    ok = ok && !(on_wall(g, 0, hx2) || on_wall(g, 1, hy2));
    lok = ok;
    lofs = ok ? hx2 + g.n[0] * hy2 : 0;
    ltg = ok && a.seed && hx2 >= g.tlo[0] && hx2 < g.thi[0] && hy2 >= g.tlo[1] && hy2 < g.thi[1];
    if (ok) {
      int ox[2] = {hx2, hx2}, oy[2] = {hy2, hy2};
      int cx = 1, cy = 1;
      if (g.bc[0] == 1) {
        if (hx2 == 1) ox[cx++] = 0;
        else if (hx2 == g.n[0] - 2) ox[cx++] = g.n[0] - 1;
      }
      if (g.bc[1] == 1) {
        if (hy2 == 1) oy[cy++] = 0;
        else if (hy2 == g.n[1] - 2) oy[cy++] = g.n[1] - 1;
      }
      for (int ky = 0; ky < cy; ++ky)
        for (int kx = 0; kx < cx; ++kx)
          if (kx || ky) wofs[nwn++] = ox[kx] + g.n[0] * oy[ky];
    }
    int bb = -1;
    if (ok && body) {
      int r0 = hx2 - a.box.lo[0], r1 = hy2 - a.box.lo[1];
      if (g.bc[0] == 0) { r0 %= g.n[0]; if (r0 < 0) r0 += g.n[0]; }
      if (g.bc[1] == 0) { r1 %= g.n[1]; if (r1 < 0) r1 += g.n[1]; }
      if (r0 >= 0 && r0 < a.box.ext[0] && r1 >= 0 && r1 < a.box.ext[1]) bb = r0 + a.box.sx * r1;
    }
    bxy = bb;
  }

  const bool outer = tid < TX * TY;
  const int tx = tid % TX, ty = tid / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = outer && gx >= 0 && gx < g.n[0] && gy >= 0 && gy < g.n[1];
  const int oc = (ty + 1) * FX + (tx + 1);
  const int ocol = own ? gx + g.n[0] * gy : 0;
  const unsigned ovo = (unsigned)ocol * es;
  const unsigned lvo = (unsigned)lofs * es;
  // ALKS: the raw first-moment part is stored on the next step's body box
  const bool xcol = ALK && own &&
                    (a.xall || (a.si_next && in_step_box(g, a.si_next, 0, gx) &&
                                in_step_box(g, a.si_next, 1, gy)));

  // Register buffers of two planes in flight.  The per-lane conditional
  // loads of a plane are issued first and the unconditional ones (clamped
  // node) last, so the wait before a commit counts only the other buffer's
  // loads, never the stores.
  struct Buf {
    R l[4];       // raw adjoint state of the slot node, plane zp
    R w[3];       // wall-node pressure adjoints that copy it (0 if none)
    R un[3];      // u^n of the slot node (target or owned body node)
    R bk, bu[3];  // body fields of the slot node
    R up[3];      // own column u^(n-1), output plane zp - 2
    int xo;       // ALKS: node offset of the slot node (its raw moment is read at commit)
    int bi;       // body-box index of the slot node, -1 outside
    bool tg, bown;
  };
  // fetches come in plane order, so the wrapped plane index zp mod nz and
  // the body-box plane (zp - lo_z) mod nz advance by one per call
  int fzw = (z0 - 2) % nz, fr2 = (z0 - 2 - a.box.lo[2]) % nz;
  if (fzw < 0) fzw += nz;
  if (fr2 < 0) fr2 += nz;
  auto fetch = [&](int zp, Buf& B) {
    const int zw = fzw, r2 = fr2;
    fzw = fzw + 1 == nz ? 0 : fzw + 1;
    fr2 = fr2 + 1 == nz ? 0 : fr2 + 1;
    const unsigned so = (unsigned)(NP * zw) * es;
    const bool zbox = r2 < a.box.ext[2];
    const bool ztg = zw >= g.tlo[2] && zw < g.thi[2];
    const bool own_plane = zp >= z0 && zp < z1;
    B.tg = ltg && ztg;
    B.bi = (bxy >= 0 && zbox) ? bxy + bplane * r2 : -1;
    B.bown = B.bi >= 0 && lown && own_plane;
    B.w[0] = B.w[1] = B.w[2] = R(0);
    if (nwn > 0) B.w[0] = bld<R>(rlam, (unsigned)wofs[0] * es, so);
    if (nwn > 1) B.w[1] = bld<R>(rlam, (unsigned)wofs[1] * es, so);
    if (nwn > 2) B.w[2] = bld<R>(rlam, (unsigned)wofs[2] * es, so);
    B.un[0] = B.un[1] = B.un[2] = R(0);
    if (B.tg || B.bown) {
      const R* uc = ucur + NP * zw + lofs;
      B.un[0] = uc[N];
      B.un[1] = uc[2 * N];
      B.un[2] = uc[3 * N];
    }
    B.bk = R(0);
    B.bu[0] = B.bu[1] = B.bu[2] = R(0);
    if (B.bi >= 0) {
      B.bk = bkp[B.bi];
      B.bu[0] = bup[B.bi];
      B.bu[1] = bup[B.bi + bvol];
      B.bu[2] = bup[B.bi + 2 * bvol];
    }
    if constexpr (ALK) B.xo = NP * zw + lofs;
    int zo = zp - 2;
    const bool zown = zo >= z0 && zo < z1;
    const unsigned uso = (unsigned)(zown ? NP * zo : 0) * es;
    B.up[0] = bld<R>(rup, ovo, uso + fb);
    B.up[1] = bld<R>(rup, ovo, uso + 2u * fb);
    B.up[2] = bld<R>(rup, ovo, uso + 3u * fb);
    B.l[0] = bld<R>(rlam, lvo, so);
    B.l[1] = bld<R>(rlam, lvo, so + fb);
    B.l[2] = bld<R>(rlam, lvo, so + 2u * fb);
    B.l[3] = bld<R>(rlam, lvo, so + 3u * fb);
  };
  auto commit = [&](int zp, const Buf& B) {
    const int sl = (zp + 2 * NR) % NR;
    R pb = B.l[0] + (B.w[0] + B.w[1] + B.w[2]);
    R ub0 = B.l[1], ub1 = B.l[2], ub2 = B.l[3];
    R s0 = R(0), s1 = R(0), s2 = R(0);  // objective seed
    if (B.tg) {
      const double un = g.ndir[0] * (double)B.un[0] + g.ndir[1] * (double)B.un[1] +
                        g.ndir[2] * (double)B.un[2];
      const R gs = (R)(seed * g.NTinv * (1.0 - 2.0 * g.phi * (un - Ebar)));
      s0 = gs * nd0;
      s1 = gs * nd1;
      s2 = gs * nd2;
      if constexpr (!ALK) {
        ub0 += s0;
        ub1 += s1;
        ub2 += s2;
      }
    }
    if (B.bi >= 0) {
      const R kk = B.bk;
      const R inv = brinkman_inv(kk);
      // the part the Brinkman correction acts on: all of it, or (ALKS) the
      // raw first-moment part with the seed
      R x0 = ub0, x1 = ub1, x2 = ub2;
      R X0 = R(0), X1 = R(0), X2 = R(0);
      if constexpr (ALK) {
        const R* xp = (const R*)a.xin + B.xo;
        X0 = xp[0];
        X1 = xp[N];
        X2 = xp[2 * N];
        x0 = X0 + s0;
        x1 = X1 + s1;
        x2 = X2 + s2;
      }
      if (B.bown) {
        const R kb = fma(x2, B.bu[2] - B.un[2],
                         fma(x1, B.bu[1] - B.un[1], x0 * (B.bu[0] - B.un[0])));
        bkbar[B.bi] = kb * inv;
        bubar[B.bi] = kk * x0 * inv;
        bubar[B.bi + bvol] = kk * x1 * inv;
        bubar[B.bi + 2 * bvol] = kk * x2 * inv;
      }
      if constexpr (ALK) {
        ub0 = fma(x0, inv, ub0 - X0);
        ub1 = fma(x1, inv, ub1 - X1);
        ub2 = fma(x2, inv, ub2 - X2);
      } else {
        ub0 *= inv;
        ub1 *= inv;
        ub2 *= inv;
      }
    } else if constexpr (ALK) {
      ub0 += s0;
      ub1 += s1;
      ub2 += s2;
    }
    Q4<R> v;
    v.p = lok ? pb * R(1.0 / 3.0) : R(0);  // the gather transpose takes p-bar / 3
    v.x = lok ? ub0 : R(0);
    v.y = lok ? ub1 : R(0);
    v.z = lok ? ub2 : R(0);
    ring[sl][tid] = v;
  };

  // own nodes within two nodes of a wall take the one-sided stencil transposes
  const bool owx = own && g.bc[0] == 1 && (gx <= 2 || gx >= g.n[0] - 3);
  const bool owy = own && g.bc[1] == 1 && (gy <= 2 || gy >= g.n[1] - 3);
  // their transposed stencils, doubled (the central transposes below are the
  // raw differences: the factor 1/2 of the central difference sits in A)
  R kxw[5], kyw[5];
  dnumT_taps(g, 0, gx, kxw);
  dnumT_taps(g, 1, gy, kyw);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    kxw[q] *= R(2);
    kyw[q] *= R(2);
  }
  const R A = (R)g.A;
  // moment slot: threads 0..255 take their own output position (its moments
  // stay in registers for the output), threads 256..339 the 1-node halo ring
  const bool fok = tid < FP;
  int fx, fy;
  if (outer) {
    fx = tx + 1;
    fy = ty + 1;
  } else {
    const int r = tid - TX * TY;
    if (r < FX) {
      fx = r;
      fy = 0;
    } else if (r < 2 * FX) {
      fx = r - FX;
      fy = FY - 1;
    } else {
      const int q = r - 2 * FX;  // 0 .. 2 (FY - 2) - 1
      fx = (q & 1) ? FX - 1 : 0;
      fy = 1 + (q >> 1);
    }
  }
  const int fpos = fx + FX * fy;
  const int fc = (fy + 1) * LX + (fx + 1);
  R Mp[10];                          // own-position moments of plane zs - 1
  R zprev[3] = {R(0), R(0), R(0)};  // own column M2_{zx}, M2_{zy}, M2_{zz} at zs - 2
#pragma unroll
  for (int q = 0; q < 10; ++q) Mp[q] = R(0);

  // Iteration zs: commit plane zs+1 (buffer X) | barrier | fetch plane zs+3
  // into X | moments of plane zs | output of plane zs-1.  The output reads
  // other threads' moments of plane zs-1 only (written before the barrier);
  // the z transposes use the own column's moments of planes zs-2 and zs from
  // registers.  With a 4-plane ring one barrier per plane suffices; a
  // 3-plane ring (less LDS) needs a second one before the next commit.
  auto iter = [&](int zs, Buf& X) {
    // commit and loads at raised wave priority, as in the forward step
    __builtin_amdgcn_s_setprio(2);
    commit(zs + 1, X);
    const R upx = X.up[0], upy = X.up[1], upz = X.up[2];
    __syncthreads();
    fetch(zs + 3, X);
    __builtin_amdgcn_s_setprio(0);
    R M[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) M[q] = R(0);
    if (fok) {
      const int rs[3] = {(zs + 2 * NR - 1) % NR, (zs + 2 * NR) % NR,
                         (zs + 2 * NR + 1) % NR};  // planes zs-1, zs, zs+1
      // F_i(y) = p-bar(y + c_i) / 3 + c_i . u-bar(y + c_i); each opposite pair
      // enters the even moments through its sum and the first moments through
      // its difference
      M[0] = R(Lat<15>::w[0]) * ring[rs[1]][fc].p;
#pragma unroll
      for (int i = 1; i < 15; i += 2) {
        const int cx = Lat<15>::c[i][0], cy = Lat<15>::c[i][1], cz = Lat<15>::c[i][2];
        const int pp = rs[cz + 1], pm = rs[1 - cz];
        const int jp = fc + cx + cy * LX, jm = fc - cx - cy * LX;
        const Q4<R> vp = ring[pp][jp], vm = ring[pm][jm];
        R cu_p = R(0), cu_m = R(0);
        if (cx == 1) { cu_p += vp.x; cu_m += vm.x; }
        if (cx == -1) { cu_p -= vp.x; cu_m -= vm.x; }
        if (cy == 1) { cu_p += vp.y; cu_m += vm.y; }
        if (cy == -1) { cu_p -= vp.y; cu_m -= vm.y; }
        if (cz == 1) { cu_p += vp.z; cu_m += vm.z; }
        if (cz == -1) { cu_p -= vp.z; cu_m -= vm.z; }
        const R Fp = vp.p + cu_p, Fm = vm.p - cu_m;
        const R w = R(Lat<15>::w[i]), S = Fp + Fm, D = Fp - Fm;
        M[0] = fma(w, S, M[0]);
        if (cx != 0) { M[1] = fma(cx > 0 ? w : -w, D, M[1]); M[4] = fma(w, S, M[4]); }
        if (cy != 0) { M[2] = fma(cy > 0 ? w : -w, D, M[2]); M[5] = fma(w, S, M[5]); }
        if (cz != 0) { M[3] = fma(cz > 0 ? w : -w, D, M[3]); M[6] = fma(w, S, M[6]); }
        if (cx * cy != 0) M[7] = fma(cx * cy > 0 ? w : -w, S, M[7]);
        if (cx * cz != 0) M[8] = fma(cx * cz > 0 ? w : -w, S, M[8]);
        if (cy * cz != 0) M[9] = fma(cy * cz > 0 ? w : -w, S, M[9]);
      }
      R(*mo)[FP] = mb[zs & 1];
      mo[0][fpos] = M[4];
      mo[1][fpos] = M[5];
      mo[2][fpos] = M[7];
      mo[3][fpos] = M[8];
      mo[4][fpos] = M[9];
    }
    const int zo = zs - 1;
    if (zo >= z0 && own) {
      R(*m0)[FP] = mb[zo & 1];  // plane zo, written before this iteration's barrier
      const unsigned so = (unsigned)(NP * zo) * es;
      const R ux = upx, uy = upy, uz = upz;
      const R M0 = Mp[0];
      const R Mxx = Mp[4], Myy = Mp[5], Mzz = Mp[6];
      const R Mxy = Mp[7], Mxz = Mp[8], Myz = Mp[9];
      // the fused multiply-adds are named here and below, so that the two
      // unrolled copies of the plane loop round alike (a plane's result must
      // not depend on the parity of its place in the segment)
      auto eqT = [&](R m1, R mx, R my, R mz, R uc) {
        const R t = fma(mz, uz, fma(my, uy, mx * ux));
        return fma(-R(3) * uc, M0, fma(R(9), t, R(3) * m1));
      };
      R bx = eqT(Mp[1], Mxx, Mxy, Mxz, ux);
      R by = eqT(Mp[2], Mxy, Myy, Myz, uy);
      R bz = eqT(Mp[3], Mxz, Myz, Mzz, uz);
      // velocity-gradient transpose: D_x^T, D_y^T in plane (central, then the
      // one-sided transposes next to walls); D_z^T (periodic) from zo -+ 1
      R tx0 = m0[0][oc - 1] - m0[0][oc + 1];
      R tx1 = m0[2][oc - 1] - m0[2][oc + 1];
      R tx2 = m0[3][oc - 1] - m0[3][oc + 1];
      R ty0 = m0[2][oc - FX] - m0[2][oc + FX];
      R ty1 = m0[1][oc - FX] - m0[1][oc + FX];
      R ty2 = m0[4][oc - FX] - m0[4][oc + FX];
      // taps with a zero weight may fall outside the moment plane: their
      // row or column is clamped into it (nonzero weights never leave it)
      if (owx) {
        tx0 = tx1 = tx2 = R(0);
        const int r0 = oc - (tx + 1);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const int j = r0 + min(max(tx + 1 + q - 2, 0), FX - 1);
          tx0 = fma(kxw[q], m0[0][j], tx0);
          tx1 = fma(kxw[q], m0[2][j], tx1);
          tx2 = fma(kxw[q], m0[3][j], tx2);
        }
      }
      if (owy) {
        ty0 = ty1 = ty2 = R(0);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const int j = (tx + 1) + min(max(ty + 1 + q - 2, 0), FY - 1) * FX;
          ty0 = fma(kyw[q], m0[2][j], ty0);
          ty1 = fma(kyw[q], m0[1][j], ty1);
          ty2 = fma(kyw[q], m0[4][j], ty2);
        }
      }
      bx = fma(A, tx0 + ty0 + (zprev[0] - M[8]), bx);
      by = fma(A, tx1 + ty1 + (zprev[1] - M[9]), by);
      bz = fma(A, tx2 + ty2 + (zprev[2] - M[6]), bz);
      bst<R>(R(3) * M0, rlp, ovo, so);
      bst<R>(bx, rlp, ovo, so + fb);
      bst<R>(by, rlp, ovo, so + 2u * fb);
      bst<R>(bz, rlp, ovo, so + 3u * fb);
      if constexpr (ALK) {
        if (xcol && (a.xall || in_step_box(g, a.si_next, 2, zo))) {
          const __amdgpu_buffer_rsrc_t rxo = brsrc(a.xout, 3u * fb);
          bst<R>(R(3) * Mp[1], rxo, ovo, so);
          bst<R>(R(3) * Mp[2], rxo, ovo, so + fb);
          bst<R>(R(3) * Mp[3], rxo, ovo, so + 2u * fb);
        }
        // the ALKS state itself (p~, u~, s~ = -M0, -M1, -M2), for the carry
        if (a.mout) {
          R* mo = (R*)a.mout + NP * zo + ocol;
          mo[0] = -M0;
          mo[N] = -Mp[1];
          mo[2 * N] = -Mp[2];
          mo[3 * N] = -Mp[3];
          mo[4 * N] = -Mxx;
          mo[5 * N] = -Myy;
          mo[6 * N] = -Mzz;
          mo[7 * N] = -Mxy;
          mo[8 * N] = -Mxz;
          mo[9 * N] = -Myz;
        }
      }
    }
    zprev[0] = Mp[8];
    zprev[1] = Mp[9];
    zprev[2] = Mp[6];
#pragma unroll
    for (int q = 0; q < 10; ++q) Mp[q] = M[q];
    // with three ring slots the next commit overwrites plane zs-1, read above
    if (NR == 3) __syncthreads();
  };

  Buf bA, bB;
  fetch(z0 - 2, bA);
  commit(z0 - 2, bA);
  fetch(z0 - 1, bA);
  commit(z0 - 1, bA);
  fetch(z0, bA);
  fetch(z0 + 1, bB);
  int zs = z0 - 1;
  for (; zs + 1 <= z1; zs += 2) {
    iter(zs, bA);
    iter(zs + 1, bB);
  }
  if (zs <= z1) iter(zs, bA);
}

// --------------------------------------------------------------- map
struct Mot {
  double xg[3], ug[3], c, s, om;
};
__host__ __device__ inline Mot make_mot(const double* m8) {
  Mot m;
  for (int k = 0; k < 3; ++k) {
    m.xg[k] = m8[k];
    m.ug[k] = m8[3 + k];
  }
  m.c = cos(m8[6]);
  m.s = sin(m8[6]);
  m.om = m8[7];
  return m;
}

__device__ __forceinline__ void apply_step(Box& b, Mot& m, const StepInfo* si) {
  if (!si) return;
  apply_step(b, si);
  for (int k = 0; k < 3; ++k) {
    m.xg[k] = si->xg[k];
    m.ug[k] = si->ug[k];
  }
  m.c = si->c;
  m.s = si->s;
  m.om = si->om;
}

// Cosine-kernel sums over the design points whose rotated position lies
// within the kernel support of analysis position (bx, by): the W-weighted
// kappa_ref, and from sum W, sum W r1, sum W r2 the transferred rigid
// velocity, in arithmetic type C (kappa_ref read in the state type R; the
// fused multiply-adds are named so every kernel that inlines this rounds
// alike).  The offset of design point e from the analysis node is R (q - e),
// q being the node in design coordinates, so the candidate loop works on
// q - e relative to the window corner (small numbers, exact in the working
// precision) instead of on absolute positions.
template <class R, class C>
__device__ __forceinline__ void map2d_sums(const Geo& g, const R* kref, const Mot& m, int bx,
                                           int by, C& k, C& usx, C& usy) {
  C m0 = C(0), m1 = C(0), m2 = C(0);
  k = C(0);
  const C c = (C)m.c, s = (C)m.s;
  const double rx = bx - m.xg[0], ry = by - m.xg[1];
  const double q0 = m.c * rx + m.s * ry + g.xiG[0];
  const double q1 = -m.s * rx + m.c * ry + g.xiG[1];
  const double h = 2.0 * (fabs(m.c) + fabs(m.s));
  const int i0 = max(0, (int)ceil(q0 - h)), i1 = min(g.D[0] - 1, (int)floor(q0 + h));
  const int j0 = max(0, (int)ceil(q1 - h)), j1 = min(g.D[1] - 1, (int)floor(q1 + h));
  const C f0 = (C)(q0 - i0), f1 = (C)(q1 - j0);  // q - (window corner)
  const C a0 = (C)((double)i0 - g.xiG[0]), a1 = (C)((double)j0 - g.xiG[1]);
  // a window row has at most 6 points (its width is below 2 h + 1 <= 6.7):
  // the row's loads are issued together, clamped into the row
  const int jn = (i0 <= i1) ? j1 : j0 - 1;
  for (int e1 = j0; e1 <= jn; ++e1) {
    const C t1 = f1 - (C)(e1 - j0);
    const C r1 = a1 + (C)(e1 - j0);
    const R* kr = kref + (long long)g.D[0] * e1;
    R v[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) v[u] = kr[min(i0 + u, i1)];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const C t0 = f0 - (C)u;
      const C d0 = fma(c, t0, -s * t1);
      const C d1 = fma(s, t0, c * t1);
      if (i0 + u <= i1 && fabs(d0) < C(2) && fabs(d1) < C(2)) {
        const C W = wk(d0) * wk(d1);
        m0 += W;
        m1 = fma(W, a0 + (C)u, m1);
        m2 = fma(W, r1, m2);
        k = fma(W, (C)v[u], k);
      }
    }
  }
  const C om = (C)m.om;
  usx = fma(om, fma(-s, m1, -c * m2), (C)m.ug[0] * m0);
  usy = fma(om, fma(c, m1, -s * m2), (C)m.ug[1] * m0);
}

// The transfer of one box node; a block is a MAP2_TX x MAP2_TY patch of the
// box.  J2F (kernels launched for single-precision plans with the objective
// J2 only): the sums are taken in FP64 and the outputs rounded once.
// J2's force density kappa_ref (u_ref - U) is a small difference of the fluid
// velocity, which the Brinkman term drives to the transferred rigid velocity,
// and U, so single-precision weights and sums would show in it at the scale of
// U; the objective J1 does not need them, and its kernels are built without.
template <class R, bool J2F = false>
__device__ __forceinline__ void map2d_row(const Geo& g, const R* kref, Mot m, Box box,
                                          const StepInfo* si, R* bk, R* bu, int full_grid,
                                          int bx_blk, int by_blk) {
  apply_step(box, m, si);
  const int i = bx_blk * MAP2_TX + (int)threadIdx.x % MAP2_TX;
  const int j = by_blk * MAP2_TY + (int)threadIdx.x / MAP2_TX;
  if (i >= box.ext[0] || j >= box.ext[1]) return;
  const int bx = box.lo[0] + i, by = box.lo[1] + j;
  int x = bx, y = by;
  const bool inside = wrap_axis(g, 0, x) && wrap_axis(g, 1, y);
  const bool wall = inside && is_wall(g, x, y, 0);
  R k = R(0), usx = R(0), usy = R(0);
  if (inside && !wall) {
    if (J2F) {
      double kd, ud, vd;
      map2d_sums<R, double>(g, kref, m, bx, by, kd, ud, vd);
      k = (R)kd;
      usx = (R)ud;
      usy = (R)vd;
    } else {
      map2d_sums<R, R>(g, kref, m, bx, by, k, usx, usy);
    }
  }
  if (full_grid) {
    if (!inside || wall) return;
    const long long n = nidx(g, x, y, 0);
    bk[n] = k;
    bu[n] = usx;
    bu[g.N + n] = usy;
  } else {
    const long long bi = i + (long long)box.sx * j;
    bk[bi] = k;
    bu[bi] = usx;
    bu[box.vol + bi] = usy;
  }
}

template <class R, bool J2F>
__global__ __launch_bounds__(MAP2_TX * MAP2_TY) void k_map2d(Geo g, const R* kref, Mot m,
                                                             Box box, const StepInfo* si, R* bk,
                                                             R* bu, int full_grid) {
  map2d_row<R, J2F>(g, kref, m, box, si, bk, bu, full_grid, blockIdx.x, blockIdx.y);
}

// 3D transfer.  The z factor of the kernel is axis aligned and its 4 weights
// are the same for every design column and every analysis z (design levels
// and analysis planes are one node apart), so with kappa_ref stored z-fastest
// (krefT, built once per run, zero-padded by KZ_PAD levels below and
// MAP_ZC + KZ_PAD above) a thread first sums the W_xy-weighted columns of its
// rotated xy candidates over MAP_ZC + 3 consecutive levels and then applies
// the z filter once.  One thread per analysis column and MAP_ZC z values.
template <class R>
__global__ __launch_bounds__(256) void k_kref_t(Geo g, const R* kref, R* kt, int lz) {
  const long long cols = (long long)g.D[0] * g.D[1];
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= cols * lz) return;
  const long long col = idx / lz;
  const int e2 = (int)(idx % lz) - KZ_PAD;
  kt[idx] = (e2 >= 0 && e2 < g.D[2]) ? kref[col + cols * e2] : R(0);
}

template <class R>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 8 : 4) void k_map3d(Geo g, const R* kt, int lz, Mot m, Box box,
                                               const StepInfo* si, R* bk, R* bu, int full_grid,
                                               long long bstride) {
  // blockIdx.y: step within a batch of consecutive steps (per-step table rows
  // and body slots bstride values apart)
  if (si) si += blockIdx.y;
  bk += blockIdx.y * bstride;
  bu += blockIdx.y * bstride;
  constexpr int ZPL = MAP_ZPL;  // z values per lane
  static_assert(ZPL <= MAP_ZC, "the z-fastest copy is padded for ZPL values per lane");
  constexpr int NS = 36;         // candidate window: at most 6 x 6 design columns
  __shared__ R cw[8][NS], cr0[8][NS], cr1[8][NS];  // weight, design offsets r0, r1
  __shared__ int ci[8][NS];                         // design column index
  // outputs of the block's 8 columns (consecutive along x) for one z pass,
  // stored from here with lanes along x so a store covers 8 nodes of a row
  constexpr int ZB = 32 * ZPL;
  __shared__ R ost[4][ZB][8];
  apply_step(box, m, si);
  const int hw = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int ncol = box.ext[0] * box.ext[1];
  const int colid = blockIdx.x * 8 + hw;
  const bool cok = colid < ncol;
  const int i = cok ? colid % box.ext[0] : 0, j = cok ? colid / box.ext[0] : 0;
  const int bx = box.lo[0] + i, by = box.lo[1] + j;
  int x = bx, y = by;
  const bool col_inside = cok && wrap_axis(g, 0, x) && wrap_axis(g, 1, y);
  const bool col_wall = col_inside && (on_wall(g, 0, x) || on_wall(g, 1, y));
  const bool col_live = col_inside && !col_wall;
  // candidate slots of this column's window (e1 outer, e0 inner), lanes in
  // parallel; the half-wave then walks the valid ones in slot order
  const double rx = bx - m.xg[0], ry = by - m.xg[1];
  const double q0 = m.c * rx + m.s * ry + g.xiG[0];
  const double q1 = -m.s * rx + m.c * ry + g.xiG[1];
  const double h = 2.0 * (fabs(m.c) + fabs(m.s));
  const int i0 = max(0, (int)ceil(q0 - h)), i1 = min(g.D[0] - 1, (int)floor(q0 + h));
  const int j0 = max(0, (int)ceil(q1 - h)), j1 = min(g.D[1] - 1, (int)floor(q1 + h));
  unsigned long long mk = 0;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int sl = lane + 32 * r;
    bool ok = false;
    if (col_live && sl < NS) {
      const int e0 = i0 + sl % 6, e1 = j0 + sl / 6;
      if (e0 <= i1 && e1 <= j1) {
        const double r0 = e0 - g.xiG[0], r1 = e1 - g.xiG[1];
        const double d0 = bx - (m.c * r0 - m.s * r1 + m.xg[0]);
        const double d1 = by - (m.s * r0 + m.c * r1 + m.xg[1]);
        if (fabs(d0) < 2.0 && fabs(d1) < 2.0) {
          ok = true;
          cw[hw][sl] = wk((R)d0) * wk((R)d1);
          cr0[hw][sl] = (R)r0;
          cr1[hw][sl] = (R)r1;
          ci[hw][sl] = e0 + g.D[0] * e1;
        }
      }
    }
    const unsigned long long b = __ballot(ok);
    mk |= ((b >> (32 * (hw & 1))) & 0xffffffffull) << (32 * r);
  }
  __syncthreads();
  const double o = g.xiG[2] - m.xg[2];
  const int fo = (int)floor(o);
  const R f = (R)(o - fo);
  R wz[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wz[q] = wk(f + R(1) - R(q));
  const R om = (R)m.om, c = (R)m.c, sn = (R)m.s;
  // the z-fastest kappa_ref copy: each candidate's ZPL + 3 levels in wide loads
  const __amdgpu_buffer_rsrc_t rkt = brsrc(kt, (unsigned)(g.D[0] * g.D[1] * lz) * sizeof(R));
  for (int zblk = 0; zblk < box.ext[2]; zblk += 32 * ZPL) {
    const int zbase = zblk + lane * ZPL;
    const bool zlive = zbase < box.ext[2];
    // analysis z = lo2 + zbase + t uses design levels L0 + t + q (q = 0..3),
    // L0 = lo2 + zbase + floor(xiG2 - xg2) - 1, with weights w(f + 1 - q)
    const int L0 = box.lo[2] + zbase + fo - 1;
    R G[ZPL + 3];
#pragma unroll
    for (int t = 0; t < ZPL + 3; ++t) G[t] = R(0);
    R m0 = R(0), m1 = R(0), m2 = R(0);
    // candidates two at a time: their loads are issued before the sums,
    // which run in slot order (in FP32 this keeps the kernel within 64
    // VGPRs, eight waves per SIMD, which pays more than larger groups)
    constexpr int CG = 2;
    unsigned long long it = mk;
    while (it) {
      int sl[CG];
      bool v[CG];
#pragma unroll
      for (int u = 0; u < CG; ++u) {
        v[u] = it != 0;
        sl[u] = v[u] ? __ffsll((long long)it) - 1 : 0;
        it &= it - 1;
      }
      R W[CG], V[CG][ZPL + 3], a0[CG], a1[CG];
      int cidx[CG];
#pragma unroll
      for (int u = 0; u < CG; ++u) {
        W[u] = v[u] ? cw[hw][sl[u]] : R(0);
        a0[u] = v[u] ? cr0[hw][sl[u]] : R(0);
        a1[u] = v[u] ? cr1[hw][sl[u]] : R(0);
        cidx[u] = v[u] ? ci[hw][sl[u]] : 0;
#pragma unroll
        for (int t = 0; t < ZPL + 3; ++t) V[u][t] = R(0);
        if (v[u] && zlive)
          bld_run<R, ZPL + 3>(rkt, (unsigned)(cidx[u] * lz + L0 + KZ_PAD) * sizeof(R), V[u]);
      }
#pragma unroll
      for (int u = 0; u < CG; ++u) {
        if (!v[u]) continue;
        m0 += W[u];
        m1 += W[u] * a0[u];
        m2 += W[u] * a1[u];
#pragma unroll
        for (int t = 0; t < ZPL + 3; ++t) G[t] += W[u] * V[u][t];
      }
    }
    const R vx = om * (-sn * m1 - c * m2) + (R)m.ug[0] * m0;
    const R vy = om * (c * m1 - sn * m2) + (R)m.ug[1] * m0;
    const R vz = (R)m.ug[2] * m0;
#pragma unroll
    for (int t = 0; t < ZPL; ++t) {
      const int kk = zbase + t;
      int z = box.lo[2] + kk;
      const bool inside = col_inside && wrap_axis(g, 2, z);
      const bool wall = !inside || col_wall || on_wall(g, 2, z);
      // z weight sum over the design levels that exist
      R zs = R(0), kv = R(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e2 = L0 + t + q;
        if (e2 >= 0 && e2 < g.D[2]) zs += wz[q];
        kv += wz[q] * G[t + q];
      }
      if (wall) kv = R(0);
      const int zz = lane * ZPL + t;
      ost[0][zz][hw] = kv;
      ost[1][zz][hw] = wall ? R(0) : zs * vx;
      ost[2][zz][hw] = wall ? R(0) : zs * vy;
      ost[3][zz][hw] = wall ? R(0) : zs * vz;
    }
    __syncthreads();
    if (!full_grid) {
      // thread: column c of the block (fixed), staging rows r + 32 t; eight
      // lanes in a row store eight consecutive x of one z level
      const int c = threadIdx.x & 7, r = threadIdx.x >> 3;
      const int cid = blockIdx.x * 8 + c;
      if (cid < ncol) {
        const int ic = cid % box.ext[0], jc = cid / box.ext[0];
        const unsigned vb = (unsigned)box.vol * sizeof(R);
        const __amdgpu_buffer_rsrc_t rbk = brsrc(bk, vb), rbu = brsrc(bu, 3u * vb);
        const unsigned plane = (unsigned)(box.sx * box.sy) * sizeof(R);
        const unsigned cb = (unsigned)(ic + box.sx * jc) * sizeof(R);
#pragma unroll
        for (int t = 0; t < ZPL; ++t) {
          const int zz = r + 32 * t, kk = zblk + zz;
          if (kk < box.ext[2]) {
            const unsigned vo = cb + plane * (unsigned)kk;
            bst<R>(ost[0][zz][c], rbk, vo, 0u);
            bst<R>(ost[1][zz][c], rbu, vo, 0u);
            bst<R>(ost[2][zz][c], rbu, vo, vb);
            bst<R>(ost[3][zz][c], rbu, vo, 2u * vb);
          }
        }
      }
    } else
    // element e: column e % 8 (fastest), z e / 8 % ZB, field e / (8 ZB)
    for (int e = threadIdx.x; e < 4 * ZB * 8; e += 256) {
      const int c = e & 7, zz = (e >> 3) % ZB, q = e / (8 * ZB);
      const int kk = zblk + zz;
      const int cid = blockIdx.x * 8 + c;
      if (cid >= ncol || kk >= box.ext[2]) continue;
      const int ic = cid % box.ext[0], jc = cid / box.ext[0];
      const R v = ost[q][zz][c];
      R* dst = q == 0 ? bk : bu;
      if (full_grid) {
        int xc = box.lo[0] + ic, yc = box.lo[1] + jc, zc = box.lo[2] + kk;
        if (!wrap_axis(g, 0, xc) || !wrap_axis(g, 1, yc) || !wrap_axis(g, 2, zc)) continue;
        if (on_wall(g, 0, xc) || on_wall(g, 1, yc) || on_wall(g, 2, zc)) continue;
        dst[(q == 0 ? 0 : (long long)(q - 1) * g.N) + nidx(g, xc, yc, zc)] = v;
      } else {
        dst[(q == 0 ? 0 : (long long)(q - 1) * box.vol) + ic +
            (long long)box.sx * (jc + (long long)box.sy * kk)] = v;
      }
    }
    __syncthreads();  // before the next pass rewrites the staging array
  }
}


// A value every lane of the wave holds, moved to a scalar register.
__device__ __forceinline__ float uniform(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// 3D transfer transpose.  A block takes an 8 x 8 patch of design columns and
// a chunk of LCH design levels; its four waves take the four body-adjoint
// fields (dJ/dkappa and the three components of dJ/du_s), one lane per
// design column.  The z factor is the same 4-tap kernel for every level and
// consecutive levels are one node apart, so the block marches the analysis
// planes once.  The xy taps of the whole patch lie in a 16 x 16 window of
// the analysis plane (the rotated patch spans at most 7 sqrt(2) nodes, the
// taps 4 more), so each plane's window is staged in LDS with one coalesced
// load per field and thread, and every lane reads its 4 x 4 taps from there.
// Each plane is reduced to its sums weighted by W_xy, dW/dx and dW/dy, and a
// window of the last four planes gives each level its z-weighted sums.  The
// motion partials are linear in those sums: each field accumulates its share
// over the levels and the block adds the four.
constexpr int MAW = 16;  // staged window side (analysis nodes)
template <class R, int LCH>
__global__ __launch_bounds__(MAPADJ_THREADS, sizeof(R) == 4 ? 5 : 2) void k_mapadj3d(Geo g, const R* kref, Mot m, Box box,
                                                             const StepInfo* si, const R* bkbar,
                                                             const R* bubar, double* kref_bar,
                                                             int overwrite, double* mpart,
                                                             StepBatch sb) {
  {
    const int st = blockIdx.y;  // step within a batch of consecutive steps
    if (si) si += st;
    bkbar += st * sb.body;
    bubar += st * sb.body;
    kref_bar += st * sb.kref;
    mpart += st * sb.mpart;
  }
  apply_step(box, m, si);
  constexpr unsigned BAD = 0x80000000u;  // byte offset past every buffer: loads read 0
  constexpr unsigned es = sizeof(R);
  constexpr int WIN = MAW * MAW;
  static_assert(MAPADJ_THREADS == 256 && WIN == MAPADJ_THREADS,
                "four waves, one per field; one window node per thread");
  __shared__ R win[2][4][WIN];  // two planes in turn, four fields
  const int f = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // field of this wave
  const int lane = threadIdx.x & 63;
  const int npx = (g.D[0] + 7) >> 3, npy = (g.D[1] + 7) >> 3;
  const int nch = (g.D[2] + LCH - 1) / LCH;
  // XCD-aware: each XCD takes a contiguous run of patches (x fastest), so
  // the overlapping windows of neighbouring patches meet in the same L2
  int px, py, ch;
  const int bi = xcd_tile_of(blockIdx.x, g.nxcd, npx, npy, nch, px, py, ch);
  const int e0 = px * 8 + (lane & 7), e1 = py * 8 + (lane >> 3);
  const bool active = e0 < g.D[0] && e1 < g.D[1];
  const int cols = g.D[0] * g.D[1];
  const int col = active ? e0 + g.D[0] * e1 : 0;
  const int l0 = ch * LCH, l1 = min(l0 + LCH, g.D[2]);
  const double r0 = e0 - g.xiG[0], r1 = e1 - g.xiG[1];
  const double X0 = m.c * r0 - m.s * r1 + m.xg[0];
  const double X1 = m.s * r0 + m.c * r1 + m.xg[1];
  // window origin: the patch's rotated positions are linear in (e0, e1), so
  // their least floor is at a corner; one node of margin covers rounding
  int wx0, wy0;
  {
    double mx = 1e300, my = 1e300;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double q0 = px * 8 + 7 * (k & 1) - g.xiG[0], q1 = py * 8 + 7 * (k >> 1) - g.xiG[1];
      mx = fmin(mx, m.c * q0 - m.s * q1 + m.xg[0]);
      my = fmin(my, m.s * q0 + m.c * q1 + m.xg[1]);
    }
    wx0 = (int)floor(mx) - 2;
    wy0 = (int)floor(my) - 2;
  }
  R wx[4], dx[4], wy[4], dy[4];
  unsigned tap[16];  // LDS byte offset of tap (row cy, column cx) at 4 cy + cx, field plane 0
  {
    const int lx = (int)floor(X0) - 1 - wx0, ly = (int)floor(X1) - 1 - wy0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const R rx = (R)((double)(lx + wx0 + q) - X0), ry = (R)((double)(ly + wy0 + q) - X1);
      // lanes past the design grid weight their taps by 0
      wx[q] = active ? wk(rx) : R(0);
      dx[q] = active ? wkd(rx) : R(0);
      wy[q] = wk(ry);
      dy[q] = wkd(ry);
    }
    // (lx, ly) in [1, MAW - 5] by the choice of the window: clamped only so
    // that a lane past the design grid cannot address outside the window
    const int cx0 = min(max(lx, 0), MAW - 4), cy0 = min(max(ly, 0), MAW - 4);
#pragma unroll
    for (int cy = 0; cy < 4; ++cy)
#pragma unroll
      for (int cx = 0; cx < 4; ++cx)
        tap[4 * cy + cx] = (unsigned)((f * WIN + (cy0 + cy) * MAW + cx0 + cx) * es);
  }
  const double o2 = m.xg[2] - g.xiG[2];
  const int fo = (int)floor(o2);
  const R fr = (R)(o2 - fo);
  // the z weights are the same for every lane: keep them in scalar registers
  R wz[4], dz[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    wz[q] = uniform(wk(R(q) - R(1) - fr));
    dz[q] = uniform(wkd(R(q) - R(1) - fr));
  }
  // this thread stages window node threadIdx.x of every field: its byte
  // offset within a box plane, or BAD outside the box or on a wall
  const int bvol = (int)box.vol, bplane = box.sx * box.sy;
  unsigned noff = BAD;
  {
    int vx = wx0 + (int)(threadIdx.x % MAW), vy = wy0 + (int)(threadIdx.x / MAW);
    if (wrap_axis(g, 0, vx) && wrap_axis(g, 1, vy) && !on_wall(g, 0, vx) && !on_wall(g, 1, vy)) {
      int b0 = vx - box.lo[0], b1 = vy - box.lo[1];
      if (g.bc[0] == 0) { b0 %= g.n[0]; if (b0 < 0) b0 += g.n[0]; }
      if (g.bc[1] == 0) { b1 %= g.n[1]; if (b1 < 0) b1 += g.n[1]; }
      if (b0 >= 0 && b0 < box.ext[0] && b1 >= 0 && b1 < box.ext[1])
        noff = (unsigned)(b0 + box.sx * b1) * es;
    }
  }
  const unsigned fbytes = (unsigned)bvol * es;
  const __amdgpu_buffer_rsrc_t rk = brsrc(bkbar, fbytes);
  const __amdgpu_buffer_rsrc_t ru0 = brsrc(bubar, fbytes);
  const __amdgpu_buffer_rsrc_t ru1 = brsrc(bubar + bvol, fbytes);
  const __amdgpu_buffer_rsrc_t ru2 = brsrc(bubar + 2LL * bvol, fbytes);
  // the analysis planes are visited in order (z is periodic in 3D); planes
  // outside the box read 0 (offset BAD for every thread)
  int r2 = (l0 + fo - 1 - box.lo[2]) % g.n[2];  // box plane of the next fetch
  if (r2 < 0) r2 += g.n[2];
  auto fetch = [&](R* S) {
    const bool in = r2 < box.ext[2];
    const unsigned vo = in ? noff : BAD;
    const unsigned so = in ? (unsigned)(bplane * r2) * es : 0u;
    S[0] = bld<R>(rk, vo, so);
    S[1] = bld<R>(ru0, vo, so);
    S[2] = bld<R>(ru1, vo, so);
    S[3] = bld<R>(ru2, vo, so);
    r2 = r2 + 1 == g.n[2] ? 0 : r2 + 1;
  };
  auto stage = [&](int buf, const R* S) {
#pragma unroll
    for (int q = 0; q < 4; ++q) win[buf][q][threadIdx.x] = S[q];
  };
  // a plane's sums: (W_xy, dW/dx W_y, W_x dW/dy) weighted
  auto reduce = [&](int buf, R* P) {
    const char* wb = (const char*)&win[buf][0][0];
    R V[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) V[k] = *(const R*)(wb + tap[k]);
    R s[4], d[4];
#pragma unroll
    for (int cy = 0; cy < 4; ++cy) {
      s[cy] = wx[0] * V[4 * cy] + wx[1] * V[4 * cy + 1] + wx[2] * V[4 * cy + 2] +
              wx[3] * V[4 * cy + 3];
      d[cy] = dx[0] * V[4 * cy] + dx[1] * V[4 * cy + 1] + dx[2] * V[4 * cy + 2] +
              dx[3] * V[4 * cy + 3];
    }
    P[0] = wy[0] * s[0] + wy[1] * s[1] + wy[2] * s[2] + wy[3] * s[3];
    P[1] = wy[0] * d[0] + wy[1] * d[1] + wy[2] * d[2] + wy[3] * d[3];
    P[2] = dy[0] * s[0] + dy[1] * s[1] + dy[2] * s[2] + dy[3] * s[3];
  };
  // Plane p (p = 0 .. LCH + 2, analysis plane zb + p, zb = l0 + fo - 1) sits
  // in win[p & 1] while it is reduced; the registers hold the next two
  // planes' values in flight.  Level l0 + t uses planes t .. t + 3.
  constexpr int NP = LCH + 3;
  R S0[4], S1[4];
  fetch(S0);
  stage(0, S0);
  fetch(S0);  // plane 1
  fetch(S1);  // plane 2
  __syncthreads();
  R Wp[4][3];
  // field 0 writes dJ/dkappa_ref and weights its sums by kappa_ref; the
  // velocity fields' weights (U) are constant over the column and applied at
  // the end.  kappa_ref, the previous dJ/dkappa_ref and the stores go through
  // buffer resources: lanes that take no part get an offset past the buffer
  // (loads read 0, stores are dropped), levels past the chunk a resource of
  // size 0, and the level offset is uniform.
  const unsigned mcount = (unsigned)(cols * g.D[2]);
  const __amdgpu_buffer_rsrc_t rkr = brsrc(kref, mcount * es);
  const __amdgpu_buffer_rsrc_t rkb = brsrc(kref_bar, mcount * 8u);
  const __amdgpu_buffer_rsrc_t rk0 = brsrc(kref_bar, 0u);
  const bool own = f == 0 && active;
  const unsigned kro = own ? (unsigned)col * es : BAD;
  const unsigned kbo = own ? (unsigned)col * 8u : BAD;
  const unsigned kbl = own && !overwrite ? kbo : BAD;
  double T[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int t = p - 3;  // level finished after this plane (t >= 0)
    const int L = l0 + t;
    const bool lv = t >= 0 && L < l1;
    const unsigned lo = lv ? (unsigned)(cols * L) : 0u;  // uniform level offset (elements)
    R kr = R(0);
    double kb = 0.0;
    if (t >= 0) {
      kr = bld<R>(lv ? rkr : rk0, kro, lo * es);
      kb = bld<double>(lv ? rkb : rk0, kbl, lo * 8u);
    }
    reduce(p & 1, Wp[p & 3]);
    if (p + 1 < NP) {
      // plane p + 1 enters the other buffer, plane p + 3 is fetched
      R* S = (p & 1) ? S1 : S0;
      stage((p + 1) & 1, S);
      if (p + 3 < NP) fetch(S);
      __syncthreads();
    }
    if (t >= 0) {
      const R* P0 = Wp[t & 3];
      const R* P1 = Wp[(t + 1) & 3];
      const R* P2 = Wp[(t + 2) & 3];
      const R* P3 = Wp[(t + 3) & 3];
      const R aS = wz[0] * P0[0] + wz[1] * P1[0] + wz[2] * P2[0] + wz[3] * P3[0];
      const R aX = wz[0] * P0[1] + wz[1] * P1[1] + wz[2] * P2[1] + wz[3] * P3[1];
      const R aY = wz[0] * P0[2] + wz[1] * P1[2] + wz[2] * P2[2] + wz[3] * P3[2];
      const R aZ = dz[0] * P0[0] + dz[1] * P1[0] + dz[2] * P2[0] + dz[3] * P3[0];
      bst<double>(kb + (double)aS, lv ? rkb : rk0, kbo, lo * 8u);
      if (lv) {  // uniform: levels past the design grid add nothing
        const double c = f == 0 ? (double)kr : 1.0;
        T[0] += c * (double)aX;
        T[1] += c * (double)aY;
        T[2] += c * (double)aZ;
        T[3] += (double)aS;
      }
    }
  }
  // motion partials of this lane's field (Eq. dJdchi, dJdpsi via the rigid
  // motion): Xb = dJ/dx^G, then u^G, theta and omega
  double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  {
    const double dX0 = -m.s * r0 - m.c * r1, dX1 = m.c * r0 - m.s * r1;  // R' r
    if (f == 0) {
      part[0] = -T[0];
      part[1] = -T[1];
      part[2] = -T[2];
      part[6] = part[0] * dX0 + part[1] * dX1;
    } else {
      // U = om R' r + u^G and its angle derivative om R'' r
      const double U = f == 1   ? m.om * dX0 + m.ug[0]
                       : f == 2 ? m.om * dX1 + m.ug[1]
                                : m.ug[2];
      part[0] = -U * T[0];
      part[1] = -U * T[1];
      part[2] = -U * T[2];
      part[3] = f == 1 ? T[3] : 0.0;
      part[4] = f == 2 ? T[3] : 0.0;
      part[5] = f == 3 ? T[3] : 0.0;
      part[6] = part[0] * dX0 + part[1] * dX1;
      if (f == 1) {
        part[6] += T[3] * (m.om * (-m.c * r0 + m.s * r1));
        part[7] = T[3] * dX0;
      } else if (f == 2) {
        part[6] += T[3] * (m.om * (-m.s * r0 - m.c * r1));
        part[7] = T[3] * dX1;
      }
    }
  }
  double tot[8];
  block_sum<8, MAPADJ_THREADS>(part, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < 8; ++q) mpart[(long long)bi * 8 + q] = tot[q];
}

// 2D transpose of the transfer for one step.  A block takes a 16 x 16 patch
// of design points, one thread each.  The 4 x 4 taps of the whole patch lie
// in a 28 x 28 window of the analysis grid (the rotated patch spans at most
// 15 sqrt(2) nodes, the taps 4 more), so the window's three body-adjoint
// fields are staged in LDS with loads along x and every thread reads its
// taps from there.  Each point's sums weighted by W, dW/dx and dW/dy give
// dJ/dkappa_ref and its motion terms; the block writes one fixed-order set
// of motion partials.  Weights and tap sums in arithmetic type C: FP64 where
// the transfer itself takes FP64 sums (single-precision states under J2), so
// the transpose stays the transpose of the transfer that ran.
constexpr int MA2_P = 16, MA2_W = 28;
template <class R, class C>
__device__ __forceinline__ void mapadj_block(const Geo& g, const R* kref, Mot m, Box box,
                                             const StepInfo* si, const R* bkbar, const R* bubar,
                                             double* kref_bar, int overwrite, double* mpart,
                                             int bid) {
  apply_step(box, m, si);
  static_assert(MAPADJ_THREADS == MA2_P * MA2_P, "one design point per thread");
  constexpr int WN = MA2_W * MA2_W;
  __shared__ R win[3][WN];
  const int npx = (g.D[0] + MA2_P - 1) / MA2_P;
  const int px = bid % npx, py = bid / npx;
  const int e0 = px * MA2_P + (int)threadIdx.x % MA2_P, e1 = py * MA2_P + (int)threadIdx.x / MA2_P;
  const bool active = e0 < g.D[0] && e1 < g.D[1];
  const long long k = active ? e0 + (long long)g.D[0] * e1 : 0;
  const double r0 = e0 - g.xiG[0], r1 = e1 - g.xiG[1];
  const double X0 = m.c * r0 - m.s * r1 + m.xg[0];
  const double X1 = m.s * r0 + m.c * r1 + m.xg[1];
  // window origin: the rotated positions are linear in (e0, e1), so their
  // least floor is at a corner; one node of margin covers rounding
  int wx0, wy0;
  {
    double mx = 1e300, my = 1e300;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double q0 = px * MA2_P + (MA2_P - 1) * (c & 1) - g.xiG[0];
      const double q1 = py * MA2_P + (MA2_P - 1) * (c >> 1) - g.xiG[1];
      mx = fmin(mx, m.c * q0 - m.s * q1 + m.xg[0]);
      my = fmin(my, m.s * q0 + m.c * q1 + m.xg[1]);
    }
    wx0 = (int)floor(mx) - 2;
    wy0 = (int)floor(my) - 2;
  }
  // stage the window: nodes outside the box or on a wall read 0
  const int bvol = (int)box.vol;
  for (int n = threadIdx.x; n < WN; n += MAPADJ_THREADS) {
    int vx = wx0 + n % MA2_W, vy = wy0 + n / MA2_W;
    R v0 = R(0), v1 = R(0), v2 = R(0);
    if (wrap_axis(g, 0, vx) && wrap_axis(g, 1, vy) && !on_wall(g, 0, vx) && !on_wall(g, 1, vy)) {
      int b0 = vx - box.lo[0], b1 = vy - box.lo[1];
      if (g.bc[0] == 0) { b0 %= g.n[0]; if (b0 < 0) b0 += g.n[0]; }
      if (g.bc[1] == 0) { b1 %= g.n[1]; if (b1 < 0) b1 += g.n[1]; }
      if (b0 >= 0 && b0 < box.ext[0] && b1 >= 0 && b1 < box.ext[1]) {
        const int bi = b0 + box.sx * b1;
        v0 = bkbar[bi];
        v1 = bubar[bi];
        v2 = bubar[bvol + bi];
      }
    }
    win[0][n] = v0;
    win[1][n] = v1;
    win[2][n] = v2;
  }
  __syncthreads();
  C wx[4], dx[4], wy[4], dy[4];
  const int lx = (int)floor(X0) - 1 - wx0, ly = (int)floor(X1) - 1 - wy0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const C rx = (C)((double)(lx + wx0 + q) - X0), ry = (C)((double)(ly + wy0 + q) - X1);
    // points past the design grid weight their taps by 0
    wx[q] = active ? wk(rx) : C(0);
    dx[q] = active ? wkd(rx) : C(0);
    wy[q] = wk(ry);
    dy[q] = wkd(ry);
  }
  // (lx, ly) lie in [0, MA2_W - 4] by the choice of the window; clamped only
  // so that no thread can address outside it
  const int c0 = min(max(lx, 0), MA2_W - 4) + MA2_W * min(max(ly, 0), MA2_W - 4);
  C P[9];  // (W, dW/dx, dW/dy) x (k-bar, u-bar_x, u-bar_y)
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    C S = C(0), Dx = C(0), Dy = C(0);
#pragma unroll
    for (int cy = 0; cy < 4; ++cy) {
      C s = C(0), d = C(0);
#pragma unroll
      for (int cx = 0; cx < 4; ++cx) {
        const C v = (C)win[q][c0 + cy * MA2_W + cx];
        s += wx[cx] * v;
        d += dx[cx] * v;
      }
      S += wy[cy] * s;
      Dx += wy[cy] * d;
      Dy += dy[cy] * s;
    }
    P[q] = S;
    P[3 + q] = Dx;
    P[6 + q] = Dy;
  }
  double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (active) {
    const double kr = (double)kref[k];
    const double U0 = m.om * (-m.s * r0 - m.c * r1) + m.ug[0];
    const double U1 = m.om * (m.c * r0 - m.s * r1) + m.ug[1];
    const double Xb0 = -(kr * P[3] + U0 * P[4] + U1 * P[5]);
    const double Xb1 = -(kr * P[6] + U0 * P[7] + U1 * P[8]);
    kref_bar[k] = (overwrite ? 0.0 : kref_bar[k]) + (double)P[0];
    const double dX0 = -m.s * r0 - m.c * r1, dX1 = m.c * r0 - m.s * r1;                      // R' r
    const double dU0 = m.om * (-m.c * r0 + m.s * r1), dU1 = m.om * (-m.s * r0 - m.c * r1);  // om R'' r
    part[0] = Xb0;
    part[1] = Xb1;
    part[3] = P[1];
    part[4] = P[2];
    part[6] = Xb0 * dX0 + Xb1 * dX1 + (double)P[1] * dU0 + (double)P[2] * dU1;
    part[7] = (double)P[1] * dX0 + (double)P[2] * dX1;
  }
  double tot[8];
  block_sum<8, MAPADJ_THREADS>(part, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < 8; ++q) mpart[(long long)bid * 8 + q] = tot[q];
}

// J2F: built for single-precision states under J2 (launched for those plans
// only; see map2d_row): weights and tap sums in FP64.
template <class R, bool J2F>
__global__ __launch_bounds__(MAPADJ_THREADS) void k_mapadj(Geo g, const R* kref, Mot m, Box box,
                                                           const StepInfo* si, const R* bkbar,
                                                           const R* bubar, double* kref_bar,
                                                           int overwrite, double* mpart,
                                                           StepBatch sb) {
  const int st = blockIdx.y;  // step within a batch of consecutive steps
  if (si) si += st;
  using C = typename std::conditional<J2F, double, R>::type;
  mapadj_block<R, C>(g, kref, m, box, si, bkbar + st * sb.body, bubar + st * sb.body,
                     kref_bar + st * sb.kref, overwrite, mpart + st * sb.mpart, blockIdx.x);
}

// ------------------------------------------------- objective J2 (Sec. 2.6)
// Eq. objective2 on a 2D body.  Design point k of step n sits at
// X = x^G + R(theta) r (r its offset from the design centre, v = R r) and
// moves with U = u^G + omega R'(theta) r.  Its force density is
// f = kappa_ref (u_ref - U), u_ref = sum_x W(x - X) u(x) over the 4 x 4 taps
// of the cosine kernel, wall nodes left out.  Per step: sum f_1 (F_L),
// u^G_2 sum f_2 (F_D), omega sum (v_1 f_2 - v_2 f_1) (T); J2 = F_L + w_D F_D
// + w_T T with the normalisations of Geo::j2s.  dJ2/df = (g_1, g_2),
// g_1 = a_1 - b v_2, g_2 = a_2 + b v_1 with a_1 = 1/(nt M),
// a_2 = w_D u^G_2 / ((x2max - x2min) M), b = w_T omega / (2 pi l_m M), M the
// inner design points: it does not depend on the flow.
struct J2Pt {
  double r0, r1, v0, v1, X0, X1, U0, U1;
};
__device__ __forceinline__ J2Pt j2_point(const Geo& g, const StepInfo& S, int e0, int e1) {
  J2Pt p;
  p.r0 = (double)e0 - g.xiG[0];
  p.r1 = (double)e1 - g.xiG[1];
  p.v0 = S.c * p.r0 - S.s * p.r1;
  p.v1 = S.s * p.r0 + S.c * p.r1;
  p.X0 = p.v0 + S.xg[0];
  p.X1 = p.v1 + S.xg[1];
  p.U0 = S.om * (-S.s * p.r0 - S.c * p.r1) + S.ug[0];
  p.U1 = S.om * (S.c * p.r0 - S.s * p.r1) + S.ug[1];
  return p;
}
__device__ __forceinline__ void j2_coef(const Geo& g, const StepInfo& S, double& a0, double& a1,
                                        double& b) {
  a0 = g.j2s[0];
  a1 = g.j2w[0] * S.ug[1] * g.j2s[1];
  b = g.j2w[1] * S.om * g.j2s[2];
}
// u_ref at X and (DER) its derivatives dur[a][q] = d u_ref_q / d X_a.  The
// kernel factors are taken once per axis and, like the sums, in FP64 for
// either state precision: inside the body u_ref - U is a small difference of
// nearly equal velocities, and single-precision factors would show in it.
template <class R, bool DER>
__device__ __forceinline__ void j2_gather(const Geo& g, const R* st, double X0, double X1,
                                          double ur[2], double dur[2][2]) {
  const long long N = g.N;
  const int lx = (int)floor(X0) - 1, ly = (int)floor(X1) - 1;
  double wx[4], dx[4], wy[4], dy[4];
  int xs[4], ys[4];
  bool okx[4], oky[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    xs[q] = lx + q;
    ys[q] = ly + q;
    const double rx = (double)xs[q] - X0, ry = (double)ys[q] - X1;
    wx[q] = wk(rx);
    wy[q] = wk(ry);
    dx[q] = DER ? wkd(rx) : 0.0;
    dy[q] = DER ? wkd(ry) : 0.0;
    okx[q] = wrap_axis(g, 0, xs[q]) && !on_wall(g, 0, xs[q]);
    oky[q] = wrap_axis(g, 1, ys[q]) && !on_wall(g, 1, ys[q]);
  }
#pragma unroll
  for (int ky = 0; ky < 4; ++ky) {
    if (!oky[ky]) continue;
#pragma unroll
    for (int kx = 0; kx < 4; ++kx) {
      if (!okx[kx]) continue;
      const long long i = nidx(g, xs[kx], ys[ky], 0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double uq = (double)st[(1 + q) * N + i];
        ur[q] += wx[kx] * wy[ky] * uq;
        if constexpr (DER) {
          dur[0][q] -= dx[kx] * wy[ky] * uq;
          dur[1][q] -= wx[kx] * dy[ky] * uq;
        }
      }
    }
  }
}

// Step sums of one step, one thread per design point: each block adds its
// fixed-order partial to its own slot of jacc [blocks][3].
template <class R>
__device__ __forceinline__ void j2_fwd_block(const Geo& g, const R* kref, const StepInfo* si,
                                             const R* st, double* jacc, int bid) {
  const long long k = bid * (long long)J2_THREADS + threadIdx.x;
  double part[3] = {0.0, 0.0, 0.0};
  if (k < g.Mtot) {
    const StepInfo S = *si;
    const int e1 = (int)(k / g.D[0]);
    const J2Pt p = j2_point(g, S, (int)k - e1 * g.D[0], e1);
    double ur[2] = {0.0, 0.0}, dur[2][2];
    j2_gather<R, false>(g, st, p.X0, p.X1, ur, dur);
    const double kr = (double)kref[k];
    const double f0 = kr * (ur[0] - p.U0), f1 = kr * (ur[1] - p.U1);
    part[0] = f0;
    part[1] = S.ug[1] * f1;
    part[2] = S.om * (p.v0 * f1 - p.v1 * f0);
  }
  double tot[3];
  block_sum<3, J2_THREADS>(part, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) jacc[bid * 3 + q] += tot[q];
}

template <class R>
__global__ __launch_bounds__(J2_THREADS) void k_j2_fwd(Geo g, const R* kref, const StepInfo* si,
                                                       const R* st, double* jacc) {
  j2_fwd_block<R>(g, kref, si, st, jacc, blockIdx.x);
}

// 2D: the LKS step n and the transfer of step n + 1 (into another body
// slot) in one launch: both are short, latency-bound kernels and neither
// depends on the other.  Blocks [0, nstep) step, the rest map.
// With J2 (jst non-null) a third range of blocks adds the J2 step sums of
// the step's input state (after step jsi), which the step only reads.
// Single precision is held to eight waves per SIMD (64 VGPRs), and the J2F
// form, whose FP64 transfer sums need more registers, to seven (72 VGPRs, a
// few spilled): its J2 pass ran 2.5 % faster than at the five its registers
// would otherwise allow.
template <class R, bool J2F>
__global__ __launch_bounds__(STEP_THREADS, sizeof(R) == 4 ? (J2F ? 7 : 8) : 4) void k_fwd2d_map(Geo g, FwdArgs a, int nstep,
                                                           const R* kref, Box box,
                                                           const StepInfo* msi, R* bk, R* bu,
                                                           int nbx, int nmap,
                                                           const StepInfo* jsi, const R* jst,
                                                           double* jacc) {
  static_assert(MAP2_TX * MAP2_TY == STEP_THREADS && J2_THREADS == STEP_THREADS,
                "one block size for every part");
  const int b = blockIdx.x;
  if (b < nstep) {
    fwd2d_tile<R>(g, a, b);
    return;
  }
  if (b < nstep + nmap) {
    Mot m{};  // taken from msi
    map2d_row<R, J2F>(g, kref, m, box, msi, bk, bu, 0, (b - nstep) % nbx, (b - nstep) / nbx);
    return;
  }
  j2_fwd_block<R>(g, kref, jsi, jst, jacc, b - nstep - nmap);
}

// The transfer of step n and the J2 step sums of state n - 1 in one launch
// (both are short, latency-bound kernels with no dependence on each other):
// blocks [0, nmap) map, the rest sum.
template <class R, bool J2F>
__global__ __launch_bounds__(J2_THREADS) void k_map2d_j2(Geo g, const R* kref, Box box,
                                                         const StepInfo* si, R* bk, R* bu, int nbx,
                                                         int nmap, const StepInfo* jsi,
                                                         const R* jst, double* jacc) {
  static_assert(MAP2_TX * MAP2_TY == J2_THREADS, "one block size for both parts");
  const int b = blockIdx.x;
  if (b < nmap) {
    Mot m{};  // taken from si
    map2d_row<R, J2F>(g, kref, m, box, si, bk, bu, 0, b % nbx, b / nbx);
    return;
  }
  j2_fwd_block<R>(g, kref, jsi, jst, jacc, b - nmap);
}

// J_out = (J2, F_L, F_D) from the block slots, in a fixed order.
__global__ void k_j2_final(Geo g, const double* jacc, int nblk, double* J3) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < nblk; ++b)
    for (int q = 0; q < 3; ++q) s[q] += jacc[b * 3 + q];
  const double FL = s[0] * g.j2s[0], FD = s[1] * g.j2s[1], T = s[2] * g.j2s[2];
  J3[0] = FL + g.j2w[0] * FD + g.j2w[1] * T;
  J3[1] = FL;
  J3[2] = FD;
}

// Reverse-step seed on the fluid velocity, dJ sum_k W(x - X_k) kappa_ref g,
// on the body box of the step ([2][box.vol], box-indexed like the body
// fields; 0 at wall nodes): one thread per box node gathers the design
// points in its rotated window, as the transfer does, in the state
// precision on offsets relative to the window corner.  With d = X_k - x,
// v = (x - x^G) + d, so the seed needs only sum W kappa_ref and its first
// moments in d.  Consecutive steps in one launch: blockIdx.y = step within
// the batch, its seed in slot y of js.
template <class R>
__global__ __launch_bounds__(J2_THREADS) void k_j2_seed(Geo g, const R* kref, const StepInfo* si,
                                                        Box box, const double* dJ, R* js) {
  si += blockIdx.y;
  js += blockIdx.y * 2 * box.vol;
  apply_step(box, si);
  const long long t = blockIdx.x * (long long)J2_THREADS + threadIdx.x;
  if (t >= (long long)box.ext[0] * box.ext[1]) return;
  const int i = (int)(t % box.ext[0]), j = (int)(t / box.ext[0]);
  const int bx = box.lo[0] + i, by = box.lo[1] + j;
  int x = bx, y = by;
  const StepInfo S = *si;
  R m0 = R(0), m1 = R(0), m2 = R(0);  // sum W kappa_ref, times d_1, times d_2
  if (wrap_axis(g, 0, x) && wrap_axis(g, 1, y) && !is_wall(g, x, y, 0)) {
    const double rx = bx - S.xg[0], ry = by - S.xg[1];
    const double q0 = S.c * rx + S.s * ry + g.xiG[0];
    const double q1 = -S.s * rx + S.c * ry + g.xiG[1];
    const double h = 2.0 * (fabs(S.c) + fabs(S.s));
    const int i0 = max(0, (int)ceil(q0 - h)), i1 = min(g.D[0] - 1, (int)floor(q0 + h));
    const int j0 = max(0, (int)ceil(q1 - h)), j1 = min(g.D[1] - 1, (int)floor(q1 + h));
    const R c = (R)S.c, sn = (R)S.s;
    const R f0 = (R)(q0 - i0), f1 = (R)(q1 - j0);  // q - (window corner)
    for (int e1 = j0; e1 <= j1; ++e1) {
      const R t1 = f1 - (R)(e1 - j0);
      const R* kr = kref + (long long)g.D[0] * e1;
      for (int e0 = i0; e0 <= i1; ++e0) {
        const R t0 = f0 - (R)(e0 - i0);
        const R d0 = sn * t1 - c * t0, d1 = -(sn * t0 + c * t1);  // X_k - x = R (e - q)
        if (fabs(d0) < R(2) && fabs(d1) < R(2)) {
          const R w = wk(d0) * wk(d1) * kr[e0];
          m0 += w;
          m1 += w * d0;
          m2 += w * d1;
        }
      }
    }
  }
  double a0, a1, b;
  j2_coef(g, S, a0, a1, b);
  const double vx = bx - S.xg[0], vy = by - S.xg[1];
  const double sc = dJ[0];
  const double s0 = (a0 - b * vy) * (double)m0 - b * (double)m2;
  const double s1 = (a1 + b * vx) * (double)m0 + b * (double)m1;
  const long long bi = i + (long long)box.sx * j;
  js[bi] = (R)(sc * s0);
  js[box.vol + bi] = (R)(sc * s1);
}

// Direct J2 terms of consecutive reverse steps (blockIdx.y = step within the
// batch, state st0 + y sstride): dJ/dkappa_ref added into the step's
// kappa_ref partial row, and the motion partials (position, velocity, angle,
// angular velocity; the explicit u^G_2 of F_D and omega of T included) into
// block slot slot0 + blockIdx.x of the step's motion-partial row.
template <class R>
__global__ __launch_bounds__(J2_THREADS) void k_j2_adj(Geo g, const R* kref, const StepInfo* si,
                                                       const R* st0, long long sstride,
                                                       const double* dJ, double* kpart,
                                                       long long kstride, double* mpart,
                                                       long long mstride, int slot0) {
  const int y = blockIdx.y;
  const StepInfo S = si[y];
  const R* st = st0 + y * sstride;
  const long long k = blockIdx.x * (long long)J2_THREADS + threadIdx.x;
  double part[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (k < g.Mtot) {
    const int k1 = (int)(k / g.D[0]);
    const J2Pt p = j2_point(g, S, (int)k - k1 * g.D[0], k1);
    double ur[2] = {0.0, 0.0}, dur[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    j2_gather<R, true>(g, st, p.X0, p.X1, ur, dur);
    double a0, a1, b;
    j2_coef(g, S, a0, a1, b);
    const double dj = dJ[0], kr = (double)kref[k];
    const double e0 = ur[0] - p.U0, e1 = ur[1] - p.U1;
    const double f0 = kr * e0, f1 = kr * e1;
    const double g0 = a0 - b * p.v1, g1 = a1 + b * p.v0;
    kpart[y * kstride + k] += dj * (g0 * e0 + g1 * e1);
    const double dX0 = -S.s * p.r0 - S.c * p.r1, dX1 = S.c * p.r0 - S.s * p.r1;  // R' r
    const double dU0 = S.om * (-S.c * p.r0 + S.s * p.r1);                        // omega R'' r
    const double dU1 = S.om * (-S.s * p.r0 - S.c * p.r1);
    const double Xb0 = dj * kr * (g0 * dur[0][0] + g1 * dur[0][1]);
    const double Xb1 = dj * kr * (g0 * dur[1][0] + g1 * dur[1][1]);
    const double Ub0 = -dj * kr * g0, Ub1 = -dj * kr * g1;
    part[0] = Xb0;
    part[1] = Xb1;
    part[3] = Ub0;
    part[4] = Ub1 + dj * g.j2w[0] * g.j2s[1] * f1;
    part[6] = Xb0 * dX0 + Xb1 * dX1 + Ub0 * dU0 + Ub1 * dU1 + dj * b * (dX0 * f1 - dX1 * f0);
    part[7] = Ub0 * dX0 + Ub1 * dX1 + dj * g.j2w[1] * g.j2s[2] * (p.v0 * f1 - p.v1 * f0);
  }
  double tot[8];
  block_sum<8, J2_THREADS>(part, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < 8; ++q) mpart[y * mstride + (long long)(slot0 + blockIdx.x) * 8 + q] = tot[q];
}

// ----------------------------------------------------------- prelude
__device__ double filter_den(int t, int nt, int R) {
  double den = 0.0;
  const int a = max(0, t - R + 1), b = min(nt - 1, t + R - 1);
  for (int tau = a; tau <= b; ++tau) den += (double)(R - abs(t - tau)) / (double)R;
  return den;
}

// Temporal filter and bound map (Eqs. chi_filtered, x_g, psi_filtered, theta).
// Motion component c (0..2 translation, 3.. the angles: one about z, or
// three with rot = 1): its column of the position and of the rate in a
// motion row, and its range.
__host__ __device__ inline int mpos_col(const Geo& g, int c) { return c < 3 ? c : 6 + (c - 3); }
__host__ __device__ inline int mrate_col(const Geo& g, int c) {
  return c < 3 ? 3 + c : (g.rot ? 9 + (c - 3) : 7);
}
__host__ __device__ inline double mspan(const Geo& g, int c) {
  if (c < 3) return g.xmax[c] - g.xmin[c];
  const int k = c - 3;
  if (g.rot && k < 2) return g.tmax[k] - g.tmin[k];
  return g.thmax - g.thmin;
}
__host__ __device__ inline double mlow(const Geo& g, int c) {
  if (c < 3) return g.xmin[c];
  const int k = c - 3;
  if (g.rot && k < 2) return g.tmin[k];
  return g.thmin;
}

__global__ void k_motion_pos(Geo g, const double* chi, const double* psi, double* mot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int comp = blockIdx.y;  // 0..2 translation, 3.. the angles
  if (t >= g.nt) return;
  if (comp < 3 && comp >= g.d) {
    mot[t * g.mw + comp] = 0.0;
    return;
  }
  const int R = comp < 3 ? g.r_t : g.r_w;
  const double* src = comp < 3 ? chi + comp : psi + (g.rot ? comp - 3 : 0);
  const int stride = comp < 3 ? 3 : (g.rot ? 3 : 1);
  double num = 0.0, den = 0.0;
  const int a = max(0, t - R + 1), b = min(g.nt - 1, t + R - 1);
  for (int tau = a; tau <= b; ++tau) {
    const double w = (double)(R - abs(t - tau)) / (double)R;
    num += w * src[(long long)tau * stride];
    den += w;
  }
  const double f = num / den;
  mot[t * g.mw + mpos_col(g, comp)] = mspan(g, comp) * f + mlow(g, comp);
}

// Time derivative of the filtered motion (Eqs. u_g, omega).
__global__ void k_motion_rate(Geo g, double* mot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int comp = blockIdx.y;
  if (t >= g.nt) return;
  const int pc = mpos_col(g, comp), vc = mrate_col(g, comp);
  const int nt = g.nt, W = g.mw;
  double v;
  if (nt == 1)
    v = 0.0;
  else if (t == 0)
    v = mot[W + pc] - mot[pc];
  else if (t == nt - 1)
    v = mot[(nt - 1) * W + pc] - mot[(nt - 2) * W + pc];
  else
    v = 0.5 * (mot[(t + 1) * W + pc] - mot[(t - 1) * W + pc]);
  mot[t * W + vc] = v;
}

// Support box per step and the domain check.  boxes[t] = lo[3], ext[3], flag, 0.
__host__ __device__ void body_box(const Geo& g, const double* m8, int* out) {
  const double c = cos(m8[6]), s = sin(m8[6]);
  double Rg[9], Rdg[9];
  if (g.rot) row_rotation(g.mw, m8, Rg, Rdg);
  int lo[3], hi[3];
  int flag = 0;
  for (int pass = 0; pass < 2; ++pass) {  // 0: inner design points, 1: incl. margin
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    // three angles: the eight corners of the rotated design block
    for (int corner = 0; g.rot && corner < 8; ++corner) {
      double r[3];
      for (int a = 0; a < 3; ++a) {
        const bool up = (corner >> a) & 1;
        const double e = pass == 0 ? (up ? g.margin + g.m[a] - 1 : g.margin) : (up ? g.D[a] - 1 : 0);
        r[a] = e - g.xiG[a];
      }
      for (int a = 0; a < 3; ++a) {
        const double X = Rg[a * 3] * r[0] + Rg[a * 3 + 1] * r[1] + Rg[a * 3 + 2] * r[2] + m8[a];
        mn[a] = fmin(mn[a], X);
        mx[a] = fmax(mx[a], X);
      }
    }
    for (int corner = 0; !g.rot && corner < 4; ++corner) {
      double e0, e1;
      if (pass == 0) {
        e0 = (corner & 1) ? g.margin + g.m[0] - 1 : g.margin;
        e1 = (corner & 2) ? g.margin + g.m[1] - 1 : g.margin;
      } else {
        e0 = (corner & 1) ? g.D[0] - 1 : 0;
        e1 = (corner & 2) ? g.D[1] - 1 : 0;
      }
      const double r0 = e0 - g.xiG[0], r1 = e1 - g.xiG[1];
      const double X0 = c * r0 - s * r1 + m8[0], X1 = s * r0 + c * r1 + m8[1];
      mn[0] = fmin(mn[0], X0);
      mx[0] = fmax(mx[0], X0);
      mn[1] = fmin(mn[1], X1);
      mx[1] = fmax(mx[1], X1);
    }
    if (g.d == 3 && !g.rot) {
      const double lo2 = (pass == 0 ? g.margin : 0) - g.xiG[2];
      const double hi2 = (pass == 0 ? g.margin + g.m[2] - 1 : g.D[2] - 1) - g.xiG[2];
      mn[2] = lo2 + m8[2];
      mx[2] = hi2 + m8[2];
    }
    _Pragma("unroll") for (int a = 0; a < 3; ++a) if (a < g.d) {
      lo[a] = (int)floor(mn[a]) - 1;
      hi[a] = (int)floor(mx[a]) + 2;
      if (pass == 0 && g.bc[a] == 1 && (lo[a] < 1 || hi[a] > g.n[a] - 2)) flag = 1;
    }
    if (pass == 0) {
      bool empty = false;
      _Pragma("unroll") for (int a = 0; a < 3; ++a) if (a < g.d) empty = empty || g.m[a] == 0;
      if (empty) flag = 0;
    }
  }
  for (int a = 0; a < 3; ++a) {
    if (a >= g.d) {
      out[a] = 0;
      out[3 + a] = 1;
      continue;
    }
    int l = lo[a], h = hi[a];
    if (g.bc[a] == 1) {
      l = l < 0 ? 0 : l;
      h = h > g.n[a] - 1 ? g.n[a] - 1 : h;
    } else if (h - l + 1 > g.n[a]) {
      flag = flag ? flag : 2;
    }
    out[a] = l;
    out[3 + a] = h >= l ? h - l + 1 : 0;
  }
  out[6] = flag;
  out[7] = 0;
}

__host__ __device__ void step_info(const Geo& g, const double* m, StepInfo& si) {
  for (int k = 0; k < 3; ++k) {
    si.xg[k] = m[k];
    si.ug[k] = m[3 + k];
  }
  row_angles(g.mw, m, si.th, si.om3);
  si.c = cos(si.th[2]);
  si.s = sin(si.th[2]);
  si.om = si.om3[2];
  row_rotation(g.mw, m, si.R, si.Rd);
  int b[8];
  body_box(g, m, b);
  for (int k = 0; k < 3; ++k) {
    si.lo[k] = b[k];
    si.ext[k] = b[3 + k];
  }
  si.flag = b[6];
  si.pad = 0;
}

__global__ void k_steps(Geo g, const double* mot, StepInfo* tab, int* info) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nt) return;
  StepInfo si;
  step_info(g, mot + t * g.mw, si);
  tab[t] = si;
  if (si.flag) atomicMax(info, si.flag);
}

__global__ void k_boxes(Geo g, const double* mot, int* boxes) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nt) return;
  body_box(g, mot + t * g.mw, boxes + t * 8);
}

// Eq. kappa_ref on the design grid incl. margin.
template <class R>
__global__ void k_kref(Geo g, const double* gamma, R* kref) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= g.Mtot) return;
  const int e[3] = {(int)(k % g.D[0]), (int)((k / g.D[0]) % g.D[1]),
                    (int)(k / ((long long)g.D[0] * g.D[1]))};
  bool inner = true;
  int j[3] = {0, 0, 0};
  _Pragma("unroll") for (int a = 0; a < 3; ++a) if (a < g.d) {
    j[a] = e[a] - g.margin;
    inner = inner && j[a] >= 0 && j[a] < g.m[a];
  }
  if (!inner) {
    kref[k] = R(0);
    return;
  }
  const double gm = gamma[j[0] + (long long)g.m[0] * (j[1] + (long long)g.m[1] * j[2])];
  kref[k] = (R)(g.kmax * g.q * gm / ((1.0 - gm) + g.q));
}

// ---------------------------------------------------------- epilogue
__global__ void k_obj_final(Geo g, const double* opart, int nblk, double* J3) {
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256) {
    v[0] += opart[2 * b];
    v[1] += opart[2 * b + 1];
  }
  double tot[2];
  block_sum<2, 256>(v, tot);
  if (threadIdx.x == 0) {
    const double E = tot[0] * g.NTinv;
    const double V = tot[1] * g.NTinv - E * E;
    J3[0] = E - g.phi * V;
    J3[1] = E;
    J3[2] = V;
  }
}

// dJ/dgamma through Eq. kappa_ref.
__global__ void k_sens_gamma(Geo g, const double* gamma, const double* kref_bar, double* dg) {
  const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  long long M = 1;
  _Pragma("unroll") for (int a = 0; a < 3; ++a) if (a < g.d) M *= g.m[a];
  if (j >= M) return;
  const int i0 = (int)(j % g.m[0]);
  const int i1 = (int)((j / g.m[0]) % g.m[1]);
  const int i2 = (g.d == 3) ? (int)(j / ((long long)g.m[0] * g.m[1])) : 0;
  const int e2 = (g.d == 3) ? i2 + g.margin : 0;
  const long long k =
      (i0 + g.margin) + (long long)g.D[0] * ((i1 + g.margin) + (long long)g.D[1] * e2);
  const double gm = gamma[j];
  const double den = (1.0 - gm) + g.q;
  dg[j] = kref_bar[k] * g.kmax * g.q * (1.0 + g.q) / (den * den);
}

// Per-step motion partials: fixed-order sum over map-transpose blocks.  Lane
// (j, q) of the 256 sums component q over blocks j, j+32, ...; the 32 partial
// sums are then added in index order.
constexpr int SENS_MBAR_THREADS = 256;
__global__ __launch_bounds__(SENS_MBAR_THREADS) void k_sens_mbar(Geo g, const double* mpart,
                                                                  int nblk, double* mbar) {
  __shared__ double red[SENS_MBAR_THREADS];
  const int t = blockIdx.x;
  const int W = g.mw, G = SENS_MBAR_THREADS / W;  // G lane groups of W
  const int j = threadIdx.x / W, q = threadIdx.x % W;
  double s = 0.0;
  if (t < g.nt && j < G) {
    const double* p = mpart + (long long)t * nblk * W;
    for (int b = j; b < nblk; b += G) s += p[b * W + q];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (t < g.nt && j == 0) {
    double a = 0.0;
    for (int i = 0; i < G; ++i) a += red[i * W + q];
    mbar[t * W + q] = a;
  }
}

// tot[t][c] = span_c * (xbar(t) + (D_t^T vbar)(t)); den_t, den_w filter normalisers.
__global__ void k_sens_tot(Geo g, const double* mbar, double* tot, double* den_t, double* den_w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;  // 0..2 translation, 3.. the angles
  const int nt = g.nt, W = g.mw;
  if (t >= nt) return;
  if (c == 0) {
    den_t[t] = filter_den(t, nt, g.r_t);
    den_w[t] = filter_den(t, nt, g.r_w);
  }
  const int pc = mpos_col(g, c), vc = mrate_col(g, c);
  double v = mbar[t * W + pc];
  if (nt >= 2) {
    auto vb = [&](int tt) { return mbar[tt * W + vc]; };
    if (t == 0) v -= vb(0);
    if (t == 1) v += vb(0);
    if (t == nt - 1) v += vb(nt - 1);
    if (t == nt - 2) v -= vb(nt - 1);
    if (t - 1 >= 1 && t - 1 <= nt - 2) v += 0.5 * vb(t - 1);
    if (t + 1 >= 1 && t + 1 <= nt - 2) v -= 0.5 * vb(t + 1);
  }
  tot[t * g.nmc + c] = (c < 3 && c >= g.d) ? 0.0 : mspan(g, c) * v;
}

// Transposed temporal filter -> dJ/dchi, dJ/dpsi.
__global__ void k_sens_filter(Geo g, const double* tot, const double* den_t, const double* den_w,
                              double* dchi, double* dpsi) {
  const int tau = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const int nt = g.nt;
  if (tau >= nt) return;
  const int R = c < 3 ? g.r_t : g.r_w;
  const double* den = c < 3 ? den_t : den_w;
  double s = 0.0;
  if (!(c < 3 && c >= g.d)) {
    const int a = max(0, tau - R + 1), b = min(nt - 1, tau + R - 1);
    for (int t = a; t <= b; ++t) s += ((double)(R - abs(t - tau)) / (double)R / den[t]) * tot[t * g.nmc + c];
  }
  if (c < 3)
    dchi[tau * 3 + c] = s;
  else if (g.rot)
    dpsi[tau * 3 + (c - 3)] = s;
  else
    dpsi[tau] = s;
}

template <class R>
__global__ void k_wall_fixup(Geo g, R* st) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const int x = (int)(i % g.n[0]);
  const int y = (int)((i / g.n[0]) % g.n[1]);
  const int z = (int)(i / ((long long)g.n[0] * g.n[1]));
  if (is_wall(g, x, y, z)) st[i] = st[wall_src(g, x, y, z)];
}

// The adjoint state an ALKS reverse sweep starts from when it carries a
// state (p~, u~, s~) into its last level (Sec. 3.3, Algorithm 1): the
// level's adjoint equilibrium p~ + c_i . V with
// V = 3 (u~ + 3 s~ u - p~ u) + 2 A sum_a D_a^T s~_ab (the divergence read as
// minus the transpose of the forward's difference operator), u that level's
// flow velocity.  In the sweep's form: lam = (-3 p~, -V), X = -3 u~.  One
// thread per node; neighbours are read from global memory (it runs once per
// sweep).  carry: [1 + d + d(d+1)/2][N], symmetric s~ as (xx, yy[, zz], xy
// [, xz, yz]).
template <class R>
__global__ void k_alks_carry_in(Geo g, const R* carry, const R* st, R* lam, R* X) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const int d = g.d;
  const long long N = g.N;
  const int c[3] = {(int)(i % g.n[0]), (int)((i / g.n[0]) % g.n[1]),
                    (int)(i / ((long long)g.n[0] * g.n[1]))};
  // plane of s~_ab in the carry
  auto splane = [&](int a, int b) -> int {
    if (a == b) return 1 + d + a;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return 1 + d + d + (lo == 0 ? hi - 1 : 2);
  };
  const R pt = carry[i];
  R u[3] = {R(0), R(0), R(0)};
  for (int a = 0; a < d; ++a) u[a] = st[(1 + a) * N + i];
  lam[i] = R(-3) * pt;
  const R A2 = R(2) * (R)g.A;
  for (int b = 0; b < d; ++b) {
    R v = R(3) * carry[(1 + b) * N + i] - R(3) * pt * u[b];
    for (int a = 0; a < d; ++a) {
      const R* sab = carry + (long long)splane(a, b) * N;
      v += R(9) * sab[i] * u[a];
      R k[5];
      dnumT_taps(g, a, c[a], k);
      R t = R(0);
      for (int q = 0; q < 5; ++q) {
        if (k[q] == R(0)) continue;
        int cc[3] = {c[0], c[1], c[2]};
        cc[a] += q - 2;
        wrap_axis(g, a, cc[a]);
        t += k[q] * sab[nidx(g, cc[0], cc[1], cc[2])];
      }
      v += A2 * t;
    }
    lam[(1 + b) * N + i] = -v;
    X[b * N + i] = R(-3) * carry[(1 + b) * N + i];
  }
}

__global__ void k_zero(uint32_t* p, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ------------------------------------------ design prelude and constraints
// Optimiser side of the loop (Sec. 3.1, Sec. 2.6), once per design
// iteration, all in FP64 on the inner design grid (gamma is [m2][m1][m0],
// design spacing 1).  One thread per design point walks the cone stencil of
// Eq. filtering: weights (R - |x_i - x_j|) / R for distances below R,
// restricted to the grid; the filter normalises by their sum at i.
struct DesignGrid {
  int m[3], d, r;
  double R;
};
__device__ __forceinline__ void design_point(const DesignGrid& G, long long k, int i[3]) {
  i[0] = (int)(k % G.m[0]);
  i[1] = (int)((k / G.m[0]) % G.m[1]);
  i[2] = (int)(k / ((long long)G.m[0] * G.m[1]));
}
// fn(j, w) over the stencil of point i
template <class F>
__device__ __forceinline__ void design_walk(const DesignGrid& G, const int i[3], F fn) {
  const int rz = G.d == 3 ? G.r : 0;
  const int z0 = max(i[2] - rz, 0), z1 = min(i[2] + rz, G.m[2] - 1);
  const int y0 = max(i[1] - G.r, 0), y1 = min(i[1] + G.r, G.m[1] - 1);
  const int x0 = max(i[0] - G.r, 0), x1 = min(i[0] + G.r, G.m[0] - 1);
  for (int z = z0; z <= z1; ++z)
    for (int y = y0; y <= y1; ++y) {
      const int dz = z - i[2], dy = y - i[1];
      const long long row = (long long)G.m[0] * (y + (long long)G.m[1] * z);
      for (int x = x0; x <= x1; ++x) {
        const int dx = x - i[0];
        const double w = (G.R - sqrt((double)(dx * dx + dy * dy + dz * dz))) / G.R;
        if (w > 0.0) fn(row + x, w);
      }
    }
}
// Eq. projection and its derivative (beta <= 0: the identity).
__device__ __forceinline__ double project(double x, double beta, double eta) {
  if (beta <= 0.0) return x;
  const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
  return (tanh(beta * eta) + tanh(beta * (x - eta))) / den;
}
__device__ __forceinline__ double project_d(double x, double beta, double eta) {
  if (beta <= 0.0) return 1.0;
  const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
  const double c = cosh(beta * (x - eta));
  return beta / (c * c) / den;
}
// phys = P(filter(gamma))
__global__ void k_design_fwd(DesignGrid G, long long M, const double* gamma, double beta,
                             double eta, double* phys) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= M) return;
  int i[3];
  design_point(G, k, i);
  double a = 0.0, W = 0.0;
  design_walk(G, i, [&](long long j, double w) {
    a += w * gamma[j];
    W += w;
  });
  phys[k] = project(a / W, beta, eta);
}
// Chain rule, first half: h_i = P'(filtered gamma_i) gbar_i / W_i.
__global__ void k_design_bwd1(DesignGrid G, long long M, const double* gamma, double beta,
                              double eta, const double* gbar, double* h) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= M) return;
  int i[3];
  design_point(G, k, i);
  double a = 0.0, W = 0.0;
  design_walk(G, i, [&](long long j, double w) {
    a += w * gamma[j];
    W += w;
  });
  h[k] = project_d(a / W, beta, eta) * gbar[k] / W;
}
// Second half: dJ/dgamma_j = sum_i w_ij h_i (the weights are symmetric, so
// the transposed stencil is the same walk).
__global__ void k_design_bwd2(DesignGrid G, long long M, const double* h, double* out) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= M) return;
  int i[3];
  design_point(G, k, i);
  double a = 0.0;
  design_walk(G, i, [&](long long j, double w) { a += w * h[j]; });
  out[k] = a;
}
// Eqs. constraint1, constraint2 on the projected density, fixed-order sum.
__global__ __launch_bounds__(256) void k_con_volume(long long M, const double* phys, double vmax,
                                                    double* Gout) {
  double v[2] = {0.0, 0.0};
  for (long long k = threadIdx.x; k < M; k += 256) {
    v[0] += phys[k];
    v[1] += 1.0 - phys[k];
  }
  double tot[2];
  block_sum<2, 256>(v, tot);
  if (threadIdx.x == 0) {
    Gout[0] = tot[0] / (vmax * (double)M) - 1.0;
    Gout[1] = tot[1] / (vmax * (double)M) - 1.0;
  }
}
__global__ void k_fill(double* p, long long n, double v) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}
// Eq. constraint3 over the steps (dt = 1), |omega| to the power p; writes
// G3 and, into the motion-partial table, dG3/domega_n (all other partials 0)
// for the prelude's chain rule.
__global__ __launch_bounds__(256) void k_con_omega(Geo g, const double* mot, double omax,
                                                   double pw, double* Gout, double* mbar) {
  __shared__ double S_all;
  double v[1] = {0.0};
  // the rate of the angle about z (Eq. constraint3)
  const int oc = mrate_col(g, g.nmc - 1), W = g.mw;
  for (int t = threadIdx.x; t < g.nt; t += 256) v[0] += pow(fabs(mot[t * W + oc] / omax), pw);
  double tot[1];
  block_sum<1, 256>(v, tot);
  if (threadIdx.x == 0) {
    S_all = tot[0];
    Gout[2] = pow(tot[0], 1.0 / pw) - 1.0;
  }
  __syncthreads();
  const double S = S_all;
  for (int t = threadIdx.x; t < g.nt; t += 256) {
    const double om = mot[t * W + oc];
    const double a = fabs(om / omax);
    const double gb = S > 0.0 ? pow(S, 1.0 / pw - 1.0) * pow(a, pw - 1.0) * (om < 0.0 ? -1.0 : 1.0) / omax
                              : 0.0;
    for (int q = 0; q < W; ++q) mbar[t * W + q] = q == oc ? gb : 0.0;
  }
}

// ------------------------------------------------------------ launchers
static dim3 step_grid(const Geo& g) {
  const int bx = (g.n[0] - g.org[0] + TILE_X - 1) / TILE_X;
  const int by = (g.n[1] - g.org[1] + g.ty3 - 1) / g.ty3;
  const int bz = g.d == 3 ? (g.n[2] + g.zseg - 1) / g.zseg : 1;
  return dim3(bx * by * bz);
}
// The 3D forward step runs with its own z-segment length.
static Geo fwd_geo(const Geo& g) {
  Geo f = g;
  if (g.d == 3) f.zseg = g.zseg_f;
  return f;
}
int step_blocks(const Geo& g) {
  dim3 d = step_grid(fwd_geo(g));
  return d.x * d.y * d.z;
}

// ------------------------------------------------------ batched 2D launches
__device__ __forceinline__ int batch_instance(const int* start, int count, int b) {
  int k = 0;
#pragma unroll
  for (int q = 1; q < BATCH_MAX; ++q)
    if (q < count && b >= start[q]) k = q;
  return k;
}

template <class R>
__global__ __launch_bounds__(STEP_THREADS) void k_fwd2d_batch(Batch<FwdArgs> b) {
  const int k = batch_instance(b.start, b.count, blockIdx.x);
  const int bid = blockIdx.x - b.start[k];
  const Geo& g = *b.geo[k];
  if (bid >= tiles_x(g) * tiles_y(g)) return;
  fwd2d_tile<R>(g, b.a[k], bid);
}

// Batched forward march with a body slot per step: step n of every instance
// and the transfer of step n + 1 in one launch, as k_fwd2d_map does for one
// plan (both parts are short and latency-bound, neither depends on the
// other).  Blocks [0, fb.start[count]) step, the rest map.
template <class R>
__global__ __launch_bounds__(STEP_THREADS, sizeof(R) == 4 ? 8 : 4) void k_fwd2d_map_batch(
    Batch<FwdArgs> fb, Batch<MapArgs> mb) {
  static_assert(MAP2_TX * MAP2_TY == STEP_THREADS, "one block size for both parts");
  const int nfwd = fb.start[fb.count];
  if ((int)blockIdx.x < nfwd) {
    const int k = batch_instance(fb.start, fb.count, blockIdx.x);
    const int bid = blockIdx.x - fb.start[k];
    const Geo& g = *fb.geo[k];
    if (bid >= tiles_x(g) * tiles_y(g)) return;
    fwd2d_tile<R>(g, fb.a[k], bid);
    return;
  }
  const int b = (int)blockIdx.x - nfwd;
  const int k = batch_instance(mb.start, mb.count, b);
  const int bid = b - mb.start[k];
  const MapArgs& a = mb.a[k];
  if (bid >= a.bxn * ((a.box.ext[1] + MAP2_TY - 1) / MAP2_TY)) return;
  Mot m;
  memset(&m, 0, sizeof m);
  map2d_row<R>(*mb.geo[k], (const R*)a.kref, m, a.box, a.si, (R*)a.bk, (R*)a.bu, 0, bid % a.bxn,
               bid / a.bxn);
}

template <class R, bool ALK>
__global__ __launch_bounds__(ADJ2D_THREADS, 2) void k_adj2d_batch(Batch<AdjArgs> b) {
  const int k = batch_instance(b.start, b.count, blockIdx.x);
  const int bid = blockIdx.x - b.start[k];
  const Geo& g = *b.geo[k];
  if (bid >= tiles_x(g) * adj2d_tiles_y(g)) return;
  adj2d_tile<R, ALK>(g, b.a[k], bid);
}

// J2 plans never join a batched launch (lks_batch_run runs them as graph
// branches), so the batched transfers take the J1 form.
template <class R>
__global__ __launch_bounds__(MAP2_TX * MAP2_TY) void k_map2d_batch(Batch<MapArgs> b) {
  const int k = batch_instance(b.start, b.count, blockIdx.x);
  const int bid = blockIdx.x - b.start[k];
  const MapArgs& a = b.a[k];
  if (bid >= a.bxn * ((a.box.ext[1] + MAP2_TY - 1) / MAP2_TY)) return;
  Mot m;
  memset(&m, 0, sizeof m);
  map2d_row<R>(*b.geo[k], (const R*)a.kref, m, a.box, a.si, (R*)a.bk, (R*)a.bu, 0, bid % a.bxn,
               bid / a.bxn);
}

template <class R>
__global__ __launch_bounds__(MAPADJ_THREADS) void k_mapadj_batch(Batch<MapAdjArgs> b) {
  const int k = batch_instance(b.start, b.count, blockIdx.x);
  const int bid = blockIdx.x - b.start[k];
  const Geo& g = *b.geo[k];
  if (bid >= mapadj_blocks_2d(g)) return;
  const MapAdjArgs& a = b.a[k];
  Mot m;
  memset(&m, 0, sizeof m);
  const int st = blockIdx.y;  // step within a batch of consecutive steps
  mapadj_block<R, R>(g, (const R*)a.kref, m, a.box, a.si ? a.si + st : nullptr,
                     (const R*)a.bkbar + st * a.sb.body, (const R*)a.bubar + st * a.sb.body,
                     a.kref_bar + st * a.sb.kref, a.overwrite, a.mpart + st * a.sb.mpart, bid);
}

LaunchEvents& launch_events() {
  static thread_local LaunchEvents e;
  return e;
}

// Launch that carries the pending profiling event pair, if any.
// ------------------------------------ map and transpose, three rotation angles
// With a general rotation R = Rz(th3) Ry(th2) Rx(th1) the kernel window has
// no axis-aligned factor.  Each analysis node of the box gathers over the
// design points whose rotated position lies within its kernel support: with
// q = R^T (x - x^G) + xi^G the node in design coordinates, x - X(e) =
// R (q - e), and the candidates e are the integer points of the box
// |e_a - q_a| <= 2 sum_b |R_ba| (the preimage of the support cube's bounding
// box).  Geometry in FP64, kernel weights in the state precision.  One
// thread per box node.  sv is the step's data when si is null.
template <class R>
__global__ __launch_bounds__(256) void k_map3r(Geo g, const R* kref, StepInfo sv,
                                               const StepInfo* si, Box box, R* bk, R* bu,
                                               int full_grid) {
  const StepInfo& S = si ? *si : sv;
  const int e0 = S.ext[0], e1 = S.ext[1], e2 = S.ext[2];
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= (long long)e0 * e1 * e2) return;
  const int i = (int)(idx % e0), j = (int)((idx / e0) % e1), kk = (int)(idx / ((long long)e0 * e1));
  const int bx = S.lo[0] + i, by = S.lo[1] + j, bz = S.lo[2] + kk;
  int x = bx, y = by, z = bz;
  const bool inside = wrap_axis(g, 0, x) && wrap_axis(g, 1, y) && wrap_axis(g, 2, z);
  const bool wall = !inside || is_wall(g, x, y, z);
  R kv = R(0), m0 = R(0), m1[3] = {R(0), R(0), R(0)};
  if (!wall) {
    const double v[3] = {bx - S.xg[0], by - S.xg[1], bz - S.xg[2]};
    double q[3];
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      q[a] = S.R[a] * v[0] + S.R[3 + a] * v[1] + S.R[6 + a] * v[2] + g.xiG[a];
      const double h = 2.0 * (fabs(S.R[a]) + fabs(S.R[3 + a]) + fabs(S.R[6 + a]));
      lo[a] = max(0, (int)ceil(q[a] - h));
      hi[a] = min(g.D[a] - 1, (int)floor(q[a] + h));
    }
    for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
      for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
        for (int c0 = lo[0]; c0 <= hi[0]; ++c0) {
          const double r[3] = {c0 - g.xiG[0], c1 - g.xiG[1], c2 - g.xiG[2]};
          double d[3];
          bool in = true;
          for (int a = 0; a < 3; ++a) {
            d[a] = v[a] - (S.R[a * 3] * r[0] + S.R[a * 3 + 1] * r[1] + S.R[a * 3 + 2] * r[2]);
            in = in && fabs(d[a]) < 2.0;
          }
          if (!in) continue;
          const R W = wk((R)d[0]) * wk((R)d[1]) * wk((R)d[2]);
          kv += W * kref[c0 + (long long)g.D[0] * (c1 + (long long)g.D[1] * c2)];
          m0 += W;
          for (int a = 0; a < 3; ++a) m1[a] += W * (R)r[a];
        }
  }
  // u_s = sum W (Rd r + u^G) = Rd m1 + u^G m0
  R us[3];
  for (int a = 0; a < 3; ++a)
    us[a] = (R)S.Rd[a * 3] * m1[0] + (R)S.Rd[a * 3 + 1] * m1[1] + (R)S.Rd[a * 3 + 2] * m1[2] +
            (R)S.ug[a] * m0;
  if (full_grid) {
    if (wall) return;
    const long long n = nidx(g, x, y, z);
    bk[n] = kv;
    for (int a = 0; a < 3; ++a) bu[a * g.N + n] = us[a];
  } else {
    const long long bi = i + (long long)box.sx * (j + (long long)box.sy * kk);
    bk[bi] = kv;
    for (int a = 0; a < 3; ++a) bu[a * box.vol + bi] = wall ? R(0) : us[a];
  }
}

// Transpose of k_map3r at one step per blockIdx.y (a segment's steps in one
// launch, strides sb): one thread per design point e gathers the body
// adjoint (dJ/dkappa, dJ/du_s) of the 64 analysis nodes of its kernel
// support and forms kappa_ref-bar(e) = sum W kbar, U-bar = sum W usbar,
// X-bar = sum dW/dX (kappa_ref kbar + U . usbar); then the step's motion
// partials: x^G-bar += X-bar, u^G-bar += U-bar, for each angle
// th_k-bar += X-bar . (dR/dth_k) r + U-bar . sum_j om_j (d2R/dth_k dth_j) r and
// om_k-bar += U-bar . (dR/dth_k) r, summed over the block in a fixed order
// into mpart [blocks][12].  Accumulations in FP64.
template <class R>
__global__ __launch_bounds__(MAPADJ_THREADS) void k_mapadj3r(Geo g, const R* kref, StepInfo sv,
                                                             const StepInfo* si, Box box,
                                                             const R* bkbar, const R* bubar,
                                                             double* kref_bar, int overwrite,
                                                             double* mpart, StepBatch sb) {
  const int y = blockIdx.y;
  if (si) si += y;
  bkbar += (long long)y * sb.body;
  bubar += (long long)y * sb.body;
  kref_bar += (long long)y * sb.kref;
  mpart += (long long)y * sb.mpart;
  const StepInfo& S = si ? *si : sv;
  // dR/dth_k and sum_j om_j d2R/dth_k dth_j, once per block
  __shared__ double dR[3][9], dW[3][9];
  if (threadIdx.x < 6) {
    const int k = threadIdx.x % 3;
    if (threadIdx.x < 3) {
      int o[3] = {0, 0, 0};
      o[k] = 1;
      euler_mat(S.th, o, dR[k]);
    } else {
      double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int jj = 0; jj < 3; ++jj) {
        int o[3] = {0, 0, 0};
        o[k] += 1;
        o[jj] += 1;
        double M[9];
        euler_mat(S.th, o, M);
        for (int q = 0; q < 9; ++q) acc[q] += S.om3[jj] * M[q];
      }
      for (int q = 0; q < 9; ++q) dW[k][q] = acc[q];
    }
  }
  __syncthreads();
  Box b = box;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = S.lo[a];
    b.ext[a] = S.ext[a];
  }
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double mp[12];
  for (int q = 0; q < 12; ++q) mp[q] = 0.0;
  if (e < g.Mtot) {
    const int c0 = (int)(e % g.D[0]), c1 = (int)((e / g.D[0]) % g.D[1]),
              c2 = (int)(e / ((long long)g.D[0] * g.D[1]));
    const double r[3] = {c0 - g.xiG[0], c1 - g.xiG[1], c2 - g.xiG[2]};
    double X[3], U[3];
    for (int a = 0; a < 3; ++a) {
      X[a] = S.R[a * 3] * r[0] + S.R[a * 3 + 1] * r[1] + S.R[a * 3 + 2] * r[2] + S.xg[a];
      U[a] = S.Rd[a * 3] * r[0] + S.Rd[a * 3 + 1] * r[1] + S.Rd[a * 3 + 2] * r[2] + S.ug[a];
    }
    const double kr = (double)kref[e];
    int lo[3];
    for (int a = 0; a < 3; ++a) lo[a] = (int)floor(X[a]) - 1;
    double kb = 0.0, Ub[3] = {0.0, 0.0, 0.0}, Xb[3] = {0.0, 0.0, 0.0};
    for (int t2 = 0; t2 < 4; ++t2)
      for (int t1 = 0; t1 < 4; ++t1)
        for (int t0 = 0; t0 < 4; ++t0) {
          int xx[3] = {lo[0] + t0, lo[1] + t1, lo[2] + t2};
          double d[3];
          for (int a = 0; a < 3; ++a) d[a] = xx[a] - X[a];
          if (!(wrap_axis(g, 0, xx[0]) && wrap_axis(g, 1, xx[1]) && wrap_axis(g, 2, xx[2])))
            continue;
          if (is_wall(g, xx[0], xx[1], xx[2])) continue;
          const long long bi = box_index(g, b, xx[0], xx[1], xx[2]);
          if (bi < 0) continue;
          double w[3], dw[3];
          for (int a = 0; a < 3; ++a) {
            w[a] = (double)wk((R)d[a]);
            dw[a] = (double)wkd((R)d[a]);
          }
          const double W = w[0] * w[1] * w[2];
          const double kbv = (double)bkbar[bi];
          const double ub[3] = {(double)bubar[bi], (double)bubar[b.vol + bi],
                                (double)bubar[2 * b.vol + bi]};
          kb += W * kbv;
          const double gsum = kr * kbv + U[0] * ub[0] + U[1] * ub[1] + U[2] * ub[2];
          for (int a = 0; a < 3; ++a) Ub[a] += W * ub[a];
          Xb[0] += -dw[0] * w[1] * w[2] * gsum;
          Xb[1] += -w[0] * dw[1] * w[2] * gsum;
          Xb[2] += -w[0] * w[1] * dw[2] * gsum;
        }
    if (overwrite)
      kref_bar[e] = kb;
    else
      kref_bar[e] += kb;
    for (int a = 0; a < 3; ++a) {
      mp[a] = Xb[a];
      mp[3 + a] = Ub[a];
    }
    for (int k = 0; k < 3; ++k) {
      double dv[3], wv[3];
      for (int a = 0; a < 3; ++a) {
        dv[a] = dR[k][a * 3] * r[0] + dR[k][a * 3 + 1] * r[1] + dR[k][a * 3 + 2] * r[2];
        wv[a] = dW[k][a * 3] * r[0] + dW[k][a * 3 + 1] * r[1] + dW[k][a * 3 + 2] * r[2];
      }
      mp[6 + k] = Xb[0] * dv[0] + Xb[1] * dv[1] + Xb[2] * dv[2] + Ub[0] * wv[0] + Ub[1] * wv[1] +
                  Ub[2] * wv[2];
      mp[9 + k] = Ub[0] * dv[0] + Ub[1] * dv[1] + Ub[2] * dv[2];
    }
  }
  double tot[12];
  block_sum<12, MAPADJ_THREADS>(mp, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < 12; ++q) mpart[(long long)blockIdx.x * 12 + q] = tot[q];
}

#define LKS_LAUNCH(K, GRID, BLOCK, SHMEM, STREAM, ...)                                    \
  do {                                                                                   \
    LaunchEvents& le_ = launch_events();                                                 \
    if (le_.start) {                                                                     \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, le_.start, le_.stop, 0,        \
                            __VA_ARGS__);                                                \
      le_.start = le_.stop = nullptr;                                                    \
    } else {                                                                             \
      hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                   \
    }                                                                                    \
  } while (0)

hipError_t launch_forward_step(const Geo& g, int precision, const FwdArgs& a, hipStream_t s) {
  if (g.d == 2) {
    dim3 grid = step_grid(g);
    if (precision == 0)
      LKS_LAUNCH(k_fwd2d<float>, grid, dim3(STEP_THREADS), 0, s, g, a);
    else
      LKS_LAUNCH(k_fwd2d<double>, grid, dim3(STEP_THREADS), 0, s, g, a);
  } else {
    const Geo f = fwd_geo(g);
    dim3 grid = step_grid(f);
    if (precision == 0)
      LKS_LAUNCH(k_fwd3d<float>, grid, dim3(Tile3<float>::NT), 0, s, f, a);
    else
      LKS_LAUNCH(k_fwd3d<double>, grid, dim3(Tile3<double>::NT), 0, s, f, a);
  }
  return hipGetLastError();
}

template <bool ALK>
static void launch_adjoint_step_t(const Geo& g, int precision, const AdjArgs& a, hipStream_t s) {
  if (g.d == 2) {
    const dim3 grid(adj2d_blocks(g));
    if (precision == 0) {
      auto k = &k_adj2d<float, ALK>;
      LKS_LAUNCH(k, grid, dim3(ADJ2D_THREADS), 0, s, g, a);
    } else {
      auto k = &k_adj2d<double, ALK>;
      LKS_LAUNCH(k, grid, dim3(ADJ2D_THREADS), 0, s, g, a);
    }
  } else {
    const dim3 grid = step_grid(g);
    if (precision == 0) {
      auto k = &k_adj3d<float, ALK>;
      LKS_LAUNCH(k, grid, dim3(Tile3<float>::NT), 0, s, g, a);
    } else {
      auto k = &k_adj3d<double, ALK>;
      LKS_LAUNCH(k, grid, dim3(Tile3<double>::NT), 0, s, g, a);
    }
  }
}
hipError_t launch_adjoint_step(const Geo& g, int precision, const AdjArgs& a, hipStream_t s) {
  if (a.xin)
    launch_adjoint_step_t<true>(g, precision, a, s);
  else
    launch_adjoint_step_t<false>(g, precision, a, s);
  return hipGetLastError();
}

int kz_levels(const Geo& g) { return g.D[2] + MAP_ZC + 2 * KZ_PAD; }
size_t kz_bytes(const Geo& g, int ext2max, int precision) {
  (void)ext2max;
  if (g.d != 3) return 0;
  return (size_t)g.D[0] * g.D[1] * kz_levels(g) * (precision == 0 ? 4 : 8);
}

hipError_t launch_kref_t(const Geo& g, int precision, const void* kref, void* kt, hipStream_t s) {
  if (g.d != 3) return hipSuccess;
  const int lz = kz_levels(g);
  const long long n = (long long)g.D[0] * g.D[1] * lz;
  dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 0)
    hipLaunchKernelGGL(k_kref_t<float>, grid, dim3(256), 0, s, g, (const float*)kref, (float*)kt, lz);
  else
    hipLaunchKernelGGL(k_kref_t<double>, grid, dim3(256), 0, s, g, (const double*)kref,
                       (double*)kt, lz);
  return hipGetLastError();
}

hipError_t launch_map(const Geo& g, int precision, const void* kref, void* kzbuf, int ext2max,
                      const double* mot8_host, const StepInfo* si, const Box& box, void* bk,
                      void* bu, int full_grid, hipStream_t s, int nsteps, long long bstride) {
  (void)ext2max;
  if (box.ext[0] <= 0 || box.ext[1] <= 0 || box.ext[2] <= 0) return hipSuccess;
  // several steps per launch: the 3D map about z with table rows only
  if (nsteps > 1 && (g.d != 3 || g.rot || !si)) return hipErrorInvalidValue;
  if (g.rot) {
    StepInfo sv;
    memset(&sv, 0, sizeof sv);
    if (mot8_host) step_info(g, mot8_host, sv);
    if (mot8_host && !si)
      for (int a = 0; a < 3; ++a) {  // the caller's box (a stand-alone map)
        sv.lo[a] = box.lo[a];
        sv.ext[a] = box.ext[a];
      }
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    dim3 grid((unsigned)((n + 255) / 256));
    if (precision == 0)
      LKS_LAUNCH(k_map3r<float>, grid, dim3(256), 0, s, g, (const float*)kref, sv, si, box,
                 (float*)bk, (float*)bu, full_grid);
    else
      LKS_LAUNCH(k_map3r<double>, grid, dim3(256), 0, s, g, (const double*)kref, sv, si, box,
                 (double*)bk, (double*)bu, full_grid);
    return hipGetLastError();
  }
  Mot m;
  if (mot8_host)
    m = make_mot(mot8_host);
  else
    memset(&m, 0, sizeof m);
  if (g.d == 2) {
    dim3 grid((box.ext[0] + MAP2_TX - 1) / MAP2_TX, (box.ext[1] + MAP2_TY - 1) / MAP2_TY);
    if (precision == 0) {
      auto k = g.obj == 1 ? &k_map2d<float, true> : &k_map2d<float, false>;
      LKS_LAUNCH(k, grid, dim3(MAP2_TX * MAP2_TY), 0, s, g, (const float*)kref, m, box, si,
                 (float*)bk, (float*)bu, full_grid);
    } else {
      auto k = &k_map2d<double, false>;
      LKS_LAUNCH(k, grid, dim3(MAP2_TX * MAP2_TY), 0, s, g, (const double*)kref, m, box, si,
                 (double*)bk, (double*)bu, full_grid);
    }
  } else {
    const int lz = kz_levels(g);
    dim3 grid((unsigned)((box.ext[0] * box.ext[1] + 7) / 8), (unsigned)nsteps);
    if (precision == 0)
      LKS_LAUNCH(k_map3d<float>, grid, dim3(256), 0, s, g, (const float*)kzbuf, lz, m, box, si,
                 (float*)bk, (float*)bu, full_grid, bstride);
    else
      LKS_LAUNCH(k_map3d<double>, grid, dim3(256), 0, s, g, (const double*)kzbuf, lz, m, box,
                 si, (double*)bk, (double*)bu, full_grid, bstride);
  }
  return hipGetLastError();
}

// Design levels per lane group of the 3D map transpose: long chunks reuse
// more of the sliding z window, short ones give more waves.  FP64 keeps the
// short chunks (the long ones exceed its register file).
static int mapadj_lch(const Geo& g) {
  return g.prec == 0 && g.D[2] >= 3 * MAPADJ_LCH_LONG ? MAPADJ_LCH_LONG : MAPADJ_LCH;
}

int mapadj_blocks(const Geo& g) {
  if (g.rot) return (int)((g.Mtot + MAPADJ_THREADS - 1) / MAPADJ_THREADS);
  if (g.d == 3) {
    // 8 x 8 design columns per block, times the level chunks
    const int lch = mapadj_lch(g);
    return (int)((long long)((g.D[0] + 7) / 8) * ((g.D[1] + 7) / 8) * ((g.D[2] + lch - 1) / lch));
  }
  return mapadj_blocks_2d(g);
}

hipError_t launch_map_adjoint(const Geo& g, int precision, const void* kref,
                              const double* mot8_host, const StepInfo* si, const Box& box,
                              const void* bkbar, const void* bubar, double* kref_bar, int overwrite,
                              double* mpart, hipStream_t s, int nsteps, StepBatch sb) {
  if (g.rot) {
    StepInfo sv;
    memset(&sv, 0, sizeof sv);
    if (mot8_host) step_info(g, mot8_host, sv);
    if (mot8_host && !si)
      for (int a = 0; a < 3; ++a) {
        sv.lo[a] = box.lo[a];
        sv.ext[a] = box.ext[a];
      }
    const dim3 grid(mapadj_blocks(g), nsteps);
    if (precision == 0)
      LKS_LAUNCH(k_mapadj3r<float>, grid, dim3(MAPADJ_THREADS), 0, s, g, (const float*)kref, sv,
                 si, box, (const float*)bkbar, (const float*)bubar, kref_bar, overwrite, mpart, sb);
    else
      LKS_LAUNCH(k_mapadj3r<double>, grid, dim3(MAPADJ_THREADS), 0, s, g, (const double*)kref,
                 sv, si, box, (const double*)bkbar, (const double*)bubar, kref_bar, overwrite,
                 mpart, sb);
    return hipGetLastError();
  }
  Mot m;
  if (mot8_host)
    m = make_mot(mot8_host);
  else
    memset(&m, 0, sizeof m);
  const dim3 grid(mapadj_blocks(g), nsteps);
  if (g.d == 3) {
    const bool lng = mapadj_lch(g) == MAPADJ_LCH_LONG;
    if (precision == 0) {
      if (lng)
        LKS_LAUNCH((k_mapadj3d<float, MAPADJ_LCH_LONG>), grid, dim3(MAPADJ_THREADS), 0, s, g,
                   (const float*)kref, m, box, si, (const float*)bkbar, (const float*)bubar,
                   kref_bar, overwrite, mpart, sb);
      else
        LKS_LAUNCH((k_mapadj3d<float, MAPADJ_LCH>), grid, dim3(MAPADJ_THREADS), 0, s, g,
                   (const float*)kref, m, box, si, (const float*)bkbar, (const float*)bubar,
                   kref_bar, overwrite, mpart, sb);
    } else {
      LKS_LAUNCH((k_mapadj3d<double, MAPADJ_LCH>), grid, dim3(MAPADJ_THREADS), 0, s, g,
                 (const double*)kref, m, box, si, (const double*)bkbar, (const double*)bubar,
                 kref_bar, overwrite, mpart, sb);
    }
    return hipGetLastError();
  }
  if (precision == 0) {
    auto k = g.obj == 1 ? &k_mapadj<float, true> : &k_mapadj<float, false>;
    LKS_LAUNCH(k, grid, dim3(MAPADJ_THREADS), 0, s, g, (const float*)kref, m, box, si,
               (const float*)bkbar, (const float*)bubar, kref_bar, overwrite, mpart, sb);
  } else {
    auto k = &k_mapadj<double, false>;
    LKS_LAUNCH(k, grid, dim3(MAPADJ_THREADS), 0, s, g, (const double*)kref, m, box, si,
               (const double*)bkbar, (const double*)bubar, kref_bar, overwrite, mpart, sb);
  }
  return hipGetLastError();
}

// The steps' partials join the accumulator one at a time, last step first:
// the order (and rounding) of a transpose per step run in reverse.
__global__ void k_kref_accum(long long M, int n, const double* part, double* kref_bar) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= M) return;
  double a = kref_bar[k];
  for (int j = n - 1; j >= 0; --j) a += part[j * M + k];
  kref_bar[k] = a;
}
hipError_t launch_kref_accum(long long M, int n, const double* part, double* kref_bar,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_kref_accum, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, n, part,
                     kref_bar);
  return hipGetLastError();
}

int j2_blocks(const Geo& g) { return (int)((g.Mtot + J2_THREADS - 1) / J2_THREADS); }

hipError_t launch_j2_forward(const Geo& g, int precision, const void* kref, const StepInfo* si,
                             const void* st, double* jacc, hipStream_t s) {
  const dim3 grid(j2_blocks(g));
  if (precision == 0)
    LKS_LAUNCH(k_j2_fwd<float>, grid, dim3(J2_THREADS), 0, s, g, (const float*)kref, si,
               (const float*)st, jacc);
  else
    LKS_LAUNCH(k_j2_fwd<double>, grid, dim3(J2_THREADS), 0, s, g, (const double*)kref, si,
               (const double*)st, jacc);
  return hipGetLastError();
}

hipError_t launch_forward_step_map(const Geo& g, int precision, const FwdArgs& a,
                                  const void* kref, const StepInfo* msi, const Box& box, void* bk,
                                  void* bu, const StepInfo* jsi, const void* jst, double* jacc,
                                  hipStream_t s) {
  const dim3 sg = step_grid(g);
  const int nstep = (int)(sg.x * sg.y * sg.z);
  const int nbx = msi ? (box.ext[0] + MAP2_TX - 1) / MAP2_TX : 0;
  const int nmap = msi ? nbx * ((box.ext[1] + MAP2_TY - 1) / MAP2_TY) : 0;
  const dim3 grid(nstep + nmap + (jst ? j2_blocks(g) : 0));
  if (precision == 0) {
    auto k = g.obj == 1 ? &k_fwd2d_map<float, true> : &k_fwd2d_map<float, false>;
    LKS_LAUNCH(k, grid, dim3(STEP_THREADS), 0, s, g, a, nstep, (const float*)kref, box, msi,
               (float*)bk, (float*)bu, nbx, nmap, jsi, (const float*)jst, jacc);
  } else {
    auto kd = &k_fwd2d_map<double, false>;
    LKS_LAUNCH(kd, grid, dim3(STEP_THREADS), 0, s, g, a, nstep,
               (const double*)kref, box, msi, (double*)bk, (double*)bu, nbx, nmap, jsi,
               (const double*)jst, jacc);
  }
  return hipGetLastError();
}

hipError_t launch_map_j2(const Geo& g, int precision, const void* kref, const StepInfo* si,
                         const Box& box, void* bk, void* bu, const StepInfo* jsi, const void* jst,
                         double* jacc, hipStream_t s) {
  const int nbx = (box.ext[0] + MAP2_TX - 1) / MAP2_TX, nby = (box.ext[1] + MAP2_TY - 1) / MAP2_TY;
  const dim3 grid(nbx * nby + j2_blocks(g));
  if (precision == 0) {
    auto k = g.obj == 1 ? &k_map2d_j2<float, true> : &k_map2d_j2<float, false>;
    LKS_LAUNCH(k, grid, dim3(J2_THREADS), 0, s, g, (const float*)kref, box, si, (float*)bk,
               (float*)bu, nbx, nbx * nby, jsi, (const float*)jst, jacc);
  } else {
    auto kd = &k_map2d_j2<double, false>;
    LKS_LAUNCH(kd, grid, dim3(J2_THREADS), 0, s, g, (const double*)kref, box, si,
               (double*)bk, (double*)bu, nbx, nbx * nby, jsi, (const double*)jst, jacc);
  }
  return hipGetLastError();
}

hipError_t launch_j2_final(const Geo& g, const double* jacc, double* J3, hipStream_t s) {
  LKS_LAUNCH(k_j2_final, dim3(1), dim3(64), 0, s, g, jacc, j2_blocks(g), J3);
  return hipGetLastError();
}

hipError_t launch_j2_seed(const Geo& g, int precision, const void* kref, const StepInfo* si,
                          const Box& box, const double* dJ, void* js, int nsteps, hipStream_t s) {
  // box: the largest step box (strides, volume and launch extents)
  const long long nodes = (long long)box.ext[0] * box.ext[1];
  const dim3 grid((unsigned)((nodes + J2_THREADS - 1) / J2_THREADS), nsteps);
  if (precision == 0)
    LKS_LAUNCH(k_j2_seed<float>, grid, dim3(J2_THREADS), 0, s, g, (const float*)kref, si, box,
               dJ, (float*)js);
  else
    LKS_LAUNCH(k_j2_seed<double>, grid, dim3(J2_THREADS), 0, s, g, (const double*)kref, si, box,
               dJ, (double*)js);
  return hipGetLastError();
}

hipError_t launch_j2_adjoint(const Geo& g, int precision, const void* kref, const StepInfo* si,
                             const void* st0, long long sstride, const double* dJ, double* kpart,
                             long long kstride, double* mpart, long long mstride, int slot0,
                             int nsteps, hipStream_t s) {
  const dim3 grid(j2_blocks(g), nsteps);
  if (precision == 0)
    LKS_LAUNCH(k_j2_adj<float>, grid, dim3(J2_THREADS), 0, s, g, (const float*)kref, si,
               (const float*)st0, sstride, dJ, kpart, kstride, mpart, mstride, slot0);
  else
    LKS_LAUNCH(k_j2_adj<double>, grid, dim3(J2_THREADS), 0, s, g, (const double*)kref, si,
               (const double*)st0, sstride, dJ, kpart, kstride, mpart, mstride, slot0);
  return hipGetLastError();
}

hipError_t launch_kappa_ref(const Geo& g, int precision, const double* gamma, void* kref,
                            hipStream_t s) {
  dim3 grid((unsigned)((g.Mtot + 255) / 256));
  if (precision == 0)
    hipLaunchKernelGGL(k_kref<float>, grid, dim3(256), 0, s, g, gamma, (float*)kref);
  else
    hipLaunchKernelGGL(k_kref<double>, grid, dim3(256), 0, s, g, gamma, (double*)kref);
  return hipGetLastError();
}

hipError_t launch_motion(const Geo& g, const double* chi, const double* psi, double* mot,
                         hipStream_t s) {
  dim3 grid((g.nt + 255) / 256, g.nmc);
  hipLaunchKernelGGL(k_motion_pos, grid, dim3(256), 0, s, g, chi, psi, mot);
  hipLaunchKernelGGL(k_motion_rate, grid, dim3(256), 0, s, g, mot);
  return hipGetLastError();
}

hipError_t launch_boxes(const Geo& g, const double* mot, int* boxes, int* info, hipStream_t s) {
  (void)info;
  hipLaunchKernelGGL(k_boxes, dim3((g.nt + 255) / 256), dim3(256), 0, s, g, mot, boxes);
  return hipGetLastError();
}

hipError_t launch_steps(const Geo& g, const double* mot, StepInfo* tab, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_steps, dim3((g.nt + 255) / 256), dim3(256), 0, s, g, mot, tab, info);
  return hipGetLastError();
}

hipError_t launch_objective_final(const Geo& g, const double* opart, int nblk, double* J3,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_obj_final, dim3(1), dim3(256), 0, s, g, opart, nblk, J3);
  return hipGetLastError();
}

hipError_t launch_sens(const Geo& g, int precision, const double* gamma, const double* kref_bar,
                       const double* mpart, int nblk, double* mbar, double* den_t, double* den_w,
                       double* dgamma, double* dchi, double* dpsi, hipStream_t s) {
  (void)precision;
  long long M = 1;
  for (int a = 0; a < g.d; ++a) M *= g.m[a];
  if (M > 0)
    hipLaunchKernelGGL(k_sens_gamma, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, g, gamma,
                       kref_bar, dgamma);
  hipLaunchKernelGGL(k_sens_mbar, dim3(g.nt), dim3(SENS_MBAR_THREADS), 0, s, g, mpart, nblk, mbar);
  // tot buffer follows den_w (nt * nmc doubles) -- see workspace layout
  double* tot = den_w + g.nt;
  dim3 grid((g.nt + 255) / 256, g.nmc);
  hipLaunchKernelGGL(k_sens_tot, grid, dim3(256), 0, s, g, mbar, tot, den_t, den_w);
  hipLaunchKernelGGL(k_sens_filter, grid, dim3(256), 0, s, g, tot, den_t, den_w, dchi, dpsi);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const Geo& g, const double* part, int nblk, double* out8,
                              hipStream_t s) {
  Geo g1 = g;
  g1.nt = 1;
  hipLaunchKernelGGL(k_sens_mbar, dim3(1), dim3(SENS_MBAR_THREADS), 0, s, g1, part, nblk, out8);
  return hipGetLastError();
}

hipError_t launch_alks_carry_in(const Geo& g, int precision, const void* carry, const void* st,
                                void* lam, void* X, hipStream_t s) {
  dim3 grid((unsigned)((g.N + 255) / 256));
  if (precision == 0)
    hipLaunchKernelGGL(k_alks_carry_in<float>, grid, dim3(256), 0, s, g, (const float*)carry,
                       (const float*)st, (float*)lam, (float*)X);
  else
    hipLaunchKernelGGL(k_alks_carry_in<double>, grid, dim3(256), 0, s, g, (const double*)carry,
                       (const double*)st, (double*)lam, (double*)X);
  return hipGetLastError();
}

hipError_t launch_wall_fixup(const Geo& g, int precision, void* st, hipStream_t s) {
  dim3 grid((unsigned)((g.N + 255) / 256));
  if (precision == 0)
    hipLaunchKernelGGL(k_wall_fixup<float>, grid, dim3(256), 0, s, g, (float*)st);
  else
    hipLaunchKernelGGL(k_wall_fixup<double>, grid, dim3(256), 0, s, g, (double*)st);
  return hipGetLastError();
}

static DesignGrid design_grid(const Geo& g, double radius) {
  DesignGrid G;
  for (int a = 0; a < 3; ++a) G.m[a] = a < g.d ? g.m[a] : 1;
  G.d = g.d;
  G.R = radius;
  G.r = (int)floor(radius);
  return G;
}
static long long design_points(const Geo& g) {
  long long M = 1;
  for (int a = 0; a < g.d; ++a) M *= g.m[a];
  return M;
}
hipError_t launch_design_filter(const Geo& g, const double* gamma, double radius, double beta,
                                double eta, double* phys, hipStream_t s) {
  const long long M = design_points(g);
  hipLaunchKernelGGL(k_design_fwd, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                     design_grid(g, radius), M, gamma, beta, eta, phys);
  return hipGetLastError();
}
hipError_t launch_design_filter_adjoint(const Geo& g, const double* gamma, double radius,
                                        double beta, double eta, const double* gbar, double* work,
                                        double* out, hipStream_t s) {
  const long long M = design_points(g);
  const DesignGrid G = design_grid(g, radius);
  const dim3 grid((unsigned)((M + 255) / 256));
  hipLaunchKernelGGL(k_design_bwd1, grid, dim3(256), 0, s, G, M, gamma, beta, eta, gbar, work);
  hipLaunchKernelGGL(k_design_bwd2, grid, dim3(256), 0, s, G, M, (const double*)work, out);
  return hipGetLastError();
}

// ---- the design chain rule without allocation: its scratch h (one double
// per inner design point) lives in a fixed device array of this file.  Each
// device holds its own copy until the process ends; calls on one device share
// it, so calls that overlap on a device race.
static __device__ __align__(256) double scratch[NOALLOC_MAX_POINTS];

// Device address of `scratch` on the current device, looked up once per
// device (the array's name is not a device address in host code).
hipError_t noalloc_scratch(double** out) {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static double* addr[MAX_DEV] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_constraints(const Geo& g, const double* phys, const double* chi,
                              const double* psi, double vmax, double omax, double pw,
                              double* Gout, double* dG1, double* dG2, double* dG3_dpsi, double* mot,
                              double* mbar, double* den, double* dchi_scratch, hipStream_t s) {
  const long long M = design_points(g);
  hipLaunchKernelGGL(k_con_volume, dim3(1), dim3(256), 0, s, M, phys, vmax, Gout);
  const dim3 gm((unsigned)((M + 255) / 256));
  if (dG1) hipLaunchKernelGGL(k_fill, gm, dim3(256), 0, s, dG1, M, 1.0 / (vmax * (double)M));
  if (dG2) hipLaunchKernelGGL(k_fill, gm, dim3(256), 0, s, dG2, M, -1.0 / (vmax * (double)M));
  if (hipError_t e = launch_motion(g, chi, psi, mot, s)) return e;
  hipLaunchKernelGGL(k_con_omega, dim3(1), dim3(256), 0, s, g, (const double*)mot, omax, pw, Gout,
                     mbar);
  if (dG3_dpsi) {
    // the motion prelude's chain rule, as for the adjoint's motion partials
    double* den_t = den;
    double* den_w = den + g.nt;
    double* tot = den_w + g.nt;
    const dim3 grid((g.nt + 255) / 256, g.nmc);
    hipLaunchKernelGGL(k_sens_tot, grid, dim3(256), 0, s, g, (const double*)mbar, tot, den_t, den_w);
    hipLaunchKernelGGL(k_sens_filter, grid, dim3(256), 0, s, g, (const double*)tot,
                       (const double*)den_t, (const double*)den_w, dchi_scratch, dG3_dpsi);
  }
  return hipGetLastError();
}

// flag[0] = 1 if the n doubles of a and b differ in any bit.
__global__ void k_differ(const unsigned long long* a, const unsigned long long* b, long long n,
                         int* flag) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n && a[i] != b[i]) flag[0] = 1;
}
hipError_t launch_differ(const double* a, const double* b, long long n, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_differ, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     (const unsigned long long*)a, (const unsigned long long*)b, n, flag);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_state_init(const Geo& g, int precision, void* st, hipStream_t s) {
  return launch_zero(st, (size_t)(g.d + 1) * g.N * (precision == 0 ? 4 : 8), s);
}


// ------------------------------------------------------ batched launchers
int step_blocks_2d(const Geo& g) {
  return ((g.n[0] - g.org[0] + TILE_X - 1) / TILE_X) * ((g.n[1] - g.org[1] + TILE_Y - 1) / TILE_Y);
}
int adj2d_blocks(const Geo& g) {
  return ((g.n[0] - g.org[0] + TILE_X - 1) / TILE_X) * adj2d_tiles_y(g);
}

int map_blocks_2d(const Box& bmax, int* bxn) {
  *bxn = (bmax.ext[0] + MAP2_TX - 1) / MAP2_TX;
  return *bxn * ((bmax.ext[1] + MAP2_TY - 1) / MAP2_TY);
}

hipError_t launch_forward_step_batch(int precision, const Batch<FwdArgs>& b, hipStream_t s) {
  dim3 grid(b.start[b.count]);
  if (precision == 0)
    LKS_LAUNCH(k_fwd2d_batch<float>, grid, dim3(STEP_THREADS), 0, s, b);
  else
    LKS_LAUNCH(k_fwd2d_batch<double>, grid, dim3(STEP_THREADS), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_forward_step_map_batch(int precision, const Batch<FwdArgs>& fb,
                                        const Batch<MapArgs>& mb, hipStream_t s) {
  const dim3 grid(fb.start[fb.count] + mb.start[mb.count]);
  if (precision == 0)
    LKS_LAUNCH(k_fwd2d_map_batch<float>, grid, dim3(STEP_THREADS), 0, s, fb, mb);
  else
    LKS_LAUNCH(k_fwd2d_map_batch<double>, grid, dim3(STEP_THREADS), 0, s, fb, mb);
  return hipGetLastError();
}

hipError_t launch_adjoint_step_batch(int precision, const Batch<AdjArgs>& b, hipStream_t s) {
  // the instances of one batch share the adjoint scheme
  const dim3 grid(b.start[b.count]);
  const bool alk = b.a[0].xin != nullptr;
  using KB = void (*)(Batch<AdjArgs>);
  KB k = precision == 0 ? (alk ? &k_adj2d_batch<float, true> : &k_adj2d_batch<float, false>)
                        : (alk ? &k_adj2d_batch<double, true> : &k_adj2d_batch<double, false>);
  LKS_LAUNCH(k, grid, dim3(ADJ2D_THREADS), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_map_batch(int precision, const Batch<MapArgs>& b, hipStream_t s) {
  dim3 grid(b.start[b.count]);
  if (precision == 0)
    LKS_LAUNCH(k_map2d_batch<float>, grid, dim3(MAP2_TX * MAP2_TY), 0, s, b);
  else
    LKS_LAUNCH(k_map2d_batch<double>, grid, dim3(MAP2_TX * MAP2_TY), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_map_adjoint_batch(int precision, const Batch<MapAdjArgs>& b, hipStream_t s,
                                    int nsteps) {
  dim3 grid(b.start[b.count], nsteps);
  if (precision == 0)
    LKS_LAUNCH(k_mapadj_batch<float>, grid, dim3(MAPADJ_THREADS), 0, s, b);
  else
    LKS_LAUNCH(k_mapadj_batch<double>, grid, dim3(MAPADJ_THREADS), 0, s, b);
  return hipGetLastError();
}

}  // namespace lks
