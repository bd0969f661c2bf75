// gfx950 kernels of one SMPC plan step (ParaMaP, arXiv:2512.22575, Sec. IV, Algorithm 1).
//
// K1 rollout_cost_kernel: one block holds R whole rollouts, one thread per
//    (rollout m, step k).  It stages the block's disturbances in LDS, integrates
//    the controls (eq. 7), evaluates forward kinematics (eq. 6) and the running /
//    terminal cost of its step (eqs. 16-25) in registers, sums each rollout's
//    cost over k in double (eq. 28) and reduces the block's rollouts to a
//    softmax partial (block minimum, sum of exponentials, exponential-weighted
//    sum of disturbances) so that eqs. 29-30 need no second pass over eps.
// K2 merge_kernel: merges the per-block partials into S_min, Z and
//    U* = Ubar + sum w eps (eqs. 29-30) and writes per-rollout weights and costs.
//
// Thread k of a rollout charges the control terms of u_k and the state terms
// of state k+1 (running terms for k+1 < H, terminal pose term for k+1 = H).
// The state terms of state 0 are the same for every rollout; K2 computes them
// once and adds them to the reported costs (the weights are invariant to a common
// shift of the costs).
#include <hip/hip_runtime.h>
#include <math.h>

#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>

#include "smpc_internal.h"

namespace smpc {
namespace {

constexpr int kWave = 64;

// Rotation columns (x, y, z axes) and translation of a link frame.
struct Frame {
  float xx, xy, xz;
  float yx, yy, yz;
  float zx, zy, zz;
  float tx, ty, tz;
};

__device__ __forceinline__ Frame identity_frame() {
  Frame T;
  T.xx = 1.f; T.xy = 0.f; T.xz = 0.f;
  T.yx = 0.f; T.yy = 1.f; T.yz = 0.f;
  T.zx = 0.f; T.zy = 0.f; T.zz = 1.f;
  T.tx = 0.f; T.ty = 0.f; T.tz = 0.f;
  return T;
}

// T <- T RotX(alpha) TransX(a) RotZ(theta) TransZ(d), given cos/sin of alpha and theta.
__device__ __forceinline__ void mdh_step(Frame& T, float ca, float sa, float a, float d,
                                         float ct, float st) {
  // TransX(a): RotX leaves the x axis unchanged, so the offset is along T's x axis.
  T.tx = fmaf(a, T.xx, T.tx);
  T.ty = fmaf(a, T.xy, T.ty);
  T.tz = fmaf(a, T.xz, T.tz);
  // RotX(alpha): y' = ca y + sa z, z' = ca z - sa y.
  const float y0 = fmaf(ca, T.yx, sa * T.zx);
  const float y1 = fmaf(ca, T.yy, sa * T.zy);
  const float y2 = fmaf(ca, T.yz, sa * T.zz);
  const float z0 = fmaf(ca, T.zx, -sa * T.yx);
  const float z1 = fmaf(ca, T.zy, -sa * T.yy);
  const float z2 = fmaf(ca, T.zz, -sa * T.yz);
  // RotZ(theta): x'' = ct x + st y', y'' = ct y' - st x.
  const float x0 = fmaf(ct, T.xx, st * y0);
  const float x1 = fmaf(ct, T.xy, st * y1);
  const float x2 = fmaf(ct, T.xz, st * y2);
  const float w0 = fmaf(ct, y0, -st * T.xx);
  const float w1 = fmaf(ct, y1, -st * T.xy);
  const float w2 = fmaf(ct, y2, -st * T.xz);
  T.xx = x0; T.xy = x1; T.xz = x2;
  T.yx = w0; T.yy = w1; T.yz = w2;
  T.zx = z0; T.zy = z1; T.zz = z2;
  // TransZ(d) along the new z axis.
  T.tx = fmaf(d, z0, T.tx);
  T.ty = fmaf(d, z1, T.ty);
  T.tz = fmaf(d, z2, T.tz);
}

__device__ __forceinline__ void transform_point(const Frame& T, float cx, float cy, float cz,
                                                float& px, float& py, float& pz) {
  px = fmaf(cx, T.xx, fmaf(cy, T.yx, fmaf(cz, T.zx, T.tx)));
  py = fmaf(cx, T.xy, fmaf(cy, T.yy, fmaf(cz, T.zy, T.ty)));
  pz = fmaf(cx, T.xz, fmaf(cy, T.yz, fmaf(cz, T.zz, T.tz)));
}

// sin and cos of r for |r| <= pi/4 by Taylor polynomials (sin to r^9, cos to r^10);
// truncation error < 2e-9.
__device__ __forceinline__ void sincos_poly(float r, float& sr, float& cr) {
  const float r2 = r * r;
  float ps = fmaf(r2, 1.f / 362880.f, -1.f / 5040.f);
  ps = fmaf(ps, r2, 1.f / 120.f);
  ps = fmaf(ps, r2, -1.f / 6.f);
  sr = fmaf(ps * r2, r, r);
  float pc = fmaf(r2, -1.f / 3628800.f, 1.f / 40320.f);
  pc = fmaf(pc, r2, -1.f / 720.f);
  pc = fmaf(pc, r2, 1.f / 24.f);
  pc = fmaf(pc, r2, -0.5f);
  cr = fmaf(pc, r2, 1.f);
}

// Rotate (sin r, cos r) by q quarter turns: sin/cos of r + q pi/2.
__device__ __forceinline__ void quadrant(int q, float sr, float cr, float& s, float& c) {
  const float s1 = (q & 1) ? cr : sr;
  const float c1 = (q & 1) ? sr : cr;
  s = (q & 2) ? -s1 : s1;
  c = ((q + 1) & 2) ? -c1 : c1;
}

// sin and cos of x: Cody-Waite reduction by pi/2 (three-part constant, fused
// multiply-adds) to r in [-pi/4, pi/4], then sincos_poly and the quadrant.  The
// result is within ~1.2 * 2^-24 of the true values for |x| < 60.
__device__ __forceinline__ void sincos_cw(float x, float& s, float& c) {
  const float n = rintf(x * 0.636619772f);
  float r = fmaf(-n, 1.57079637050628662f, x);
  r = fmaf(-n, -4.37113882867379e-08f, r);
  r = fmaf(-n, -1.77635683940025e-15f, r);
  float sr, cr;
  sincos_poly(r, sr, cr);
  quadrant((int)n, sr, cr, s, c);
}

// sin and cos of 2 pi t: the quarter-turn count q = rint(4t) is removed exactly in
// turns (t - q/4 is exact for t with at most 24 significant bits), then the
// remaining angle, at most pi/4, goes through sincos_poly.
__device__ __forceinline__ void sincos_turns(float t, float& s, float& c) {
  const float q = rintf(4.f * t);
  const float a = fmaf(-0.25f, q, t) * 6.28318530717958648f;
  float sr, cr;
  sincos_poly(a, sr, cr);
  quadrant((int)q, sr, cr, s, c);
}

// ---------------------------------------------------------------------------
// Counter-based sampling of the disturbances (Algorithm 1, sampling step) when
// the caller passes no noise buffer: Philox4x32-10 (Salmon et al., SC'11), key =
// the 64-bit seed, counter n = 2 (m H + k) + b as (n_lo, n_hi, 0, 0); 23-bit
// uniforms u = ((w >> 9) + 1/2) 2^-23; Box-Muller pairs; counter b = 0 gives
// joints 0..3, b = 1 joints 4..6.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ float uniform23(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-07f;  // 2^-23
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& za, float& zb) {
  const float r = sqrtf(-2.f * logf(uniform23(wa)));
  float s, c;
  sincos_turns(uniform23(wb), s, c);
  za = r * c;
  zb = r * s;
}

// Normals of item (m, k) with n0 = 2 (m H + k): z[0..6] are used, z[7] is spare;
// w receives the 8 raw words.
__device__ __forceinline__ void step_normals(uint64_t n0, uint32_t k0, uint32_t k1,
                                             float (&z)[8], uint32_t (&w)[8]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const uint64_t n = n0 + (uint64_t)b;
    const uint4 v = philox4x32_10(make_uint4((uint32_t)n, (uint32_t)(n >> 32), 0u, 0u), k0, k1);
    w[4 * b + 0] = v.x;
    w[4 * b + 1] = v.y;
    w[4 * b + 2] = v.z;
    w[4 * b + 3] = v.w;
    box_muller(v.x, v.y, z[4 * b + 0], z[4 * b + 1]);
    box_muller(v.z, v.w, z[4 * b + 2], z[4 * b + 3]);
  }
}

__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// exp(-d / lambda) for d >= 0 (weights and softmax rescaling, eq. 29) as
// 2^(-d * log2(e) / lambda) on the hardware exp2, with k = log2(e) / lambda.  Rounding
// the product costs at most |d / lambda| * 2^-24 relative, below 1e-6 for every factor
// larger than e^-16; smaller factors carry no weight that matters.
__device__ __forceinline__ float softmax_factor(float d, float k) {
  return __builtin_amdgcn_exp2f(-d * k);
}

// Cross-lane combines without the LDS: xor 1 and xor 2 by quad permutations (DPP),
// then the half-row and row mirrors -- once the lanes of each quad (then of each
// half-row) agree, a mirror pairs the same groups as xor 4 (xor 8) would -- and the
// four row values combined in scalar registers in a fixed order, so every lane of
// wave_min_f64 / wave_sum_f32 returns the same value.  All 64 lanes must be active.
template <int kCtrl>
__device__ __forceinline__ int dpp_move(int x) {
  return __builtin_amdgcn_update_dpp(x, x, kCtrl, 0xF, 0xF, false);
}
constexpr int kDppSwap1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppSwap2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;   // lane i <-> 7 - i within each 8
constexpr int kDppMirror = 0x140;       // lane i <-> 15 - i within each row of 16

template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(dpp_move<kCtrl>(__float_as_int(x)));
}
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = dpp_move<kCtrl>((int)v), hi = dpp_move<kCtrl>((int)(v >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}
__device__ __forceinline__ float readlane_f32(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ double wave_min_f64(double x) {
  x = fmin(x, dpp_f64<kDppSwap1>(x));
  x = fmin(x, dpp_f64<kDppSwap2>(x));
  x = fmin(x, dpp_f64<kDppHalfMirror>(x));
  x = fmin(x, dpp_f64<kDppMirror>(x));
  return fmin(fmin(readlane_f64(x, 0), readlane_f64(x, 16)),
              fmin(readlane_f64(x, 32), readlane_f64(x, 48)));
}
__device__ __forceinline__ float wave_sum_f32(float x) {
  x += dpp_f32<kDppSwap1>(x);
  x += dpp_f32<kDppSwap2>(x);
  x += dpp_f32<kDppHalfMirror>(x);
  x += dpp_f32<kDppMirror>(x);
  return (readlane_f32(x, 0) + readlane_f32(x, 16)) + (readlane_f32(x, 32) + readlane_f32(x, 48));
}

// g(theta) = (x^2 - sin^2 x) / (2 sin^4 x), x = theta / 2, for theta in [0, pi].
// With it |v|^2 = |t|^2 + g(theta) t^T (I - R) t for the translational part v of
// log(T) (eqs. 12-14): V(theta) acts as the identity along the rotation axis and
// scales the orthogonal plane by sin(x)/x, and t^T (I - R) t = 2 sin^2(x) |t_perp|^2.
__device__ __forceinline__ float log_norm_gain(float theta) {
  const float x = 0.5f * theta;
  const float x2 = x * x;
  if (x < 1e-3f) return fmaf(x2, 4.f / 45.f, 1.f / 6.f);
  float s, c_unused;
  sincos_cw(x, s, c_unused);
  float xms;  // x - sin x, by its Taylor series where the subtraction would cancel
  if (x < 0.75f) {
    xms = x * x2 * (1.f / 6.f + x2 * (-1.f / 120.f + x2 * (1.f / 5040.f +
          x2 * (-1.f / 362880.f + x2 * (1.f / 39916800.f)))));
  } else {
    xms = x - s;
  }
  const float s2 = s * s;
  return xms * (x + s) / (2.f * s2 * s2);
}

// 1/2 xi^T Q xi for Delta T = T_g^{-1} T (eqs. 11-16, 25) with Q = diag(wt I3, wr I3).
// |omega|^2 = theta^2 with theta = atan2(|vee(R - R^T)|/2, (tr R - 1)/2).
__device__ __forceinline__ float pose_cost(const Frame& T, const StepParams& p, float wt,
                                           float wr) {
  const float* G = p.RgT;
  // R_Delta = R_g^T R; R's column c holds (T.cx, T.cy, T.cz).
  const float d00 = fmaf(G[0], T.xx, fmaf(G[1], T.xy, G[2] * T.xz));
  const float d01 = fmaf(G[0], T.yx, fmaf(G[1], T.yy, G[2] * T.yz));
  const float d02 = fmaf(G[0], T.zx, fmaf(G[1], T.zy, G[2] * T.zz));
  const float d10 = fmaf(G[3], T.xx, fmaf(G[4], T.xy, G[5] * T.xz));
  const float d11 = fmaf(G[3], T.yx, fmaf(G[4], T.yy, G[5] * T.yz));
  const float d12 = fmaf(G[3], T.zx, fmaf(G[4], T.zy, G[5] * T.zz));
  const float d20 = fmaf(G[6], T.xx, fmaf(G[7], T.xy, G[8] * T.xz));
  const float d21 = fmaf(G[6], T.yx, fmaf(G[7], T.yy, G[8] * T.yz));
  const float d22 = fmaf(G[6], T.zx, fmaf(G[7], T.zy, G[8] * T.zz));
  // t_Delta = R_g^T (t - t_g) = R_g^T t - R_g^T t_g.
  const float t0 = fmaf(G[0], T.tx, fmaf(G[1], T.ty, fmaf(G[2], T.tz, -p.tgr[0])));
  const float t1 = fmaf(G[3], T.tx, fmaf(G[4], T.ty, fmaf(G[5], T.tz, -p.tgr[1])));
  const float t2 = fmaf(G[6], T.tx, fmaf(G[7], T.ty, fmaf(G[8], T.tz, -p.tgr[2])));
  const float c = 0.5f * (d00 + d11 + d22 - 1.f);
  const float sx = 0.5f * (d21 - d12);
  const float sy = 0.5f * (d02 - d20);
  const float sz = 0.5f * (d10 - d01);
  const float sn = sqrt_hw(fmaf(sx, sx, fmaf(sy, sy, sz * sz)));
  const float theta = atan2f(sn, c);
  const float n = fmaf(t0, t0, fmaf(t1, t1, t2 * t2));
  const float r0 = fmaf(d00, t0, fmaf(d01, t1, d02 * t2));
  const float r1 = fmaf(d10, t0, fmaf(d11, t1, d12 * t2));
  const float r2 = fmaf(d20, t0, fmaf(d21, t1, d22 * t2));
  const float tRt = fmaf(t0, r0, fmaf(t1, r1, t2 * r2));
  const float v2 = fmaf(log_norm_gain(theta), fmaxf(n - tRt, 0.f), n);
  return 0.5f * fmaf(wt, v2, wr * theta * theta);
}

// delta(x) of eq. 21 for a tightened interval [lo, hi] (lo <= hi): x minus x clamped to
// the interval, which for finite x is bitwise max(x - hi, 0) + min(x - lo, 0) (x - hi
// above, x - lo below, +0 inside), in two instructions instead of five.
__device__ __forceinline__ float limit_violation(float x, float lo, float hi) {
  return x - __builtin_amdgcn_fmed3f(x, lo, hi);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t grid_resource(const void* grid,
                                                                uint32_t bytes) {
  // Raw byte-addressed buffer (stride 0): loads past `bytes` return 0 instead of faulting.
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(grid), 0, (int)bytes, 0x00020000);
}

// One grid element at byte offset off + soff: float32, or float16 widened to float32.
template <int kElemBytes>
__device__ __forceinline__ float load_grid(__amdgpu_buffer_rsrc_t rsrc, uint32_t off,
                                           uint32_t soff) {
  if constexpr (kElemBytes == 4) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)off, (int)soff, 0));
  } else {
    const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(rsrc, (int)off, (int)soff, 0);
    return (float)__builtin_bit_cast(_Float16, h);
  }
}

// Trilinear phi(p) between voxel centres, query clamped to the grid (edge extension),
// in two halves: esdf_locate finds the lower corner and the fractions
// (u = p / voxel + (-origin / voxel - 1/2) per axis, clamped to [0, n - 1]; corner
// min(floor(u), n - 2)), esdf_blend_at loads the 8 corners and interpolates.
struct GridLoc {
  uint32_t ix, iy, iz;
  float fx, fy, fz;
};

__device__ __forceinline__ GridLoc esdf_locate(const StepParams& p, float px, float py,
                                               float pz) {
  const float fx_hi = (float)(p.nx - 1), fy_hi = (float)(p.ny - 1), fz_hi = (float)(p.nz - 1);
  const float ux = __builtin_amdgcn_fmed3f(fmaf(px, p.inv_voxel, p.gcx), 0.f, fx_hi);
  const float uy = __builtin_amdgcn_fmed3f(fmaf(py, p.inv_voxel, p.gcy), 0.f, fy_hi);
  const float uz = __builtin_amdgcn_fmed3f(fmaf(pz, p.inv_voxel, p.gcz), 0.f, fz_hi);
  const float bx = fminf(floorf(ux), fx_hi - 1.f);
  const float by = fminf(floorf(uy), fy_hi - 1.f);
  const float bz = fminf(floorf(uz), fz_hi - 1.f);
  GridLoc g;
  g.fx = ux - bx;
  g.fy = uy - by;
  g.fz = uz - bz;
  g.ix = (uint32_t)bx;
  g.iy = (uint32_t)by;
  g.iz = (uint32_t)bz;
  return g;
}

template <int kElemBytes>
__device__ __forceinline__ float esdf_blend_at(__amdgpu_buffer_rsrc_t rsrc, const StepParams& p,
                                               const GridLoc& g) {
  constexpr uint32_t e = kElemBytes;
  const uint32_t sy = (uint32_t)p.nx * e;
  const uint32_t sz = (uint32_t)p.nx * (uint32_t)p.ny * e;
  const uint32_t off = ((g.iz * (uint32_t)p.ny + g.iy) * (uint32_t)p.nx + g.ix) * e;
  const float v000 = load_grid<kElemBytes>(rsrc, off, 0u);
  const float v100 = load_grid<kElemBytes>(rsrc, off + e, 0u);
  const float v010 = load_grid<kElemBytes>(rsrc, off, sy);
  const float v110 = load_grid<kElemBytes>(rsrc, off + e, sy);
  const float v001 = load_grid<kElemBytes>(rsrc, off, sz);
  const float v101 = load_grid<kElemBytes>(rsrc, off + e, sz);
  const float v011 = load_grid<kElemBytes>(rsrc, off, sy + sz);
  const float v111 = load_grid<kElemBytes>(rsrc, off + e, sy + sz);
  const float c00 = fmaf(g.fx, v100 - v000, v000);
  const float c10 = fmaf(g.fx, v110 - v010, v010);
  const float c01 = fmaf(g.fx, v101 - v001, v001);
  const float c11 = fmaf(g.fx, v111 - v011, v011);
  const float c0 = fmaf(g.fy, c10 - c00, c00);
  const float c1 = fmaf(g.fy, c11 - c01, c01);
  return fmaf(g.fz, c1 - c0, c0);
}

template <int kElemBytes>
__device__ __forceinline__ float esdf_lookup(__amdgpu_buffer_rsrc_t rsrc, const StepParams& p,
                                             float px, float py, float pz) {
  return esdf_blend_at<kElemBytes>(rsrc, p, esdf_locate(p, px, py, pz));
}

// Coarse lower bound of the cell holding the lookup corner of p (0-filled past the
// buffer, which only ever happens without bounds, and then it is not consulted).  The
// corner is i0 = min(floor(u), n - 2) per axis with u clamped to [0, n - 1] (as in
// esdf_locate), and its cell i0 >> 3 equals floor(u / 8) clamped to [0, nc - 1]:
// u / 8 is exact, floor(u / 8) = floor(floor(u) / 8) for u >= 0, and the clamped ends
// agree because nc - 1 = floor((n - 2) / 8) <= floor((n - 1) / 8).  The cell index is
// formed in float (exact below 2^24).  u / 8 is taken as fma(p, inv_voxel / 8,
// gc / 8), which equals fma(p, inv_voxel, gc) / 8 exactly (a power-of-two scaling
// commutes with rounding; away from the subnormal range, where floor only sees the sign).
__device__ __forceinline__ float coarse_bound(__amdgpu_buffer_rsrc_t crsrc, const StepParams& p,
                                              float px, float py, float pz) {
  const float cx = __builtin_amdgcn_fmed3f(floorf(fmaf(px, p.inv_voxel8, p.gc8[0])), 0.f,
                                           p.cmax[0]);
  const float cy = __builtin_amdgcn_fmed3f(floorf(fmaf(py, p.inv_voxel8, p.gc8[1])), 0.f,
                                           p.cmax[1]);
  const float cz = __builtin_amdgcn_fmed3f(floorf(fmaf(pz, p.inv_voxel8, p.gc8[2])), 0.f,
                                           p.cmax[2]);
  const uint32_t cell = (uint32_t)fmaf(cz, p.cstride[1], fmaf(cy, p.cstride[0], cx));
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(crsrc, cell * 4u, 0, 0));
}

// Forward kinematics (eq. 6) of q0 + dq with sin/cos of q0 + dq by angle addition,
// so the large common angle q0 enters exactly once and only the small dq is
// rounded; writes the sphere slot centres and returns the end-effector frame.
__device__ __forceinline__ Frame fk_spheres(const DevRobot* __restrict__ rob, const float* sc0,
                                            const float (&dq)[kNdof], float (&px)[kSlots],
                                            float (&py)[kSlots], float (&pz)[kSlots]) {
  Frame T = identity_frame();
#pragma unroll
  for (int i = 0; i < kNdof; ++i) {
    float s1, c1;
    sincos_cw(dq[i], s1, c1);
    const float s0 = sc0[i], c0 = sc0[kNdof + i];
    const float st = fmaf(s0, c1, c0 * s1);
    const float ct = fmaf(c0, c1, -s0 * s1);
    mdh_step(T, rob->ca[i], rob->sa[i], rob->a[i], rob->d[i], ct, st);
#pragma unroll
    for (int j = 0; j < kSpl; ++j) {
      const int s = i * kSpl + j;
      transform_point(T, rob->sc[s][0], rob->sc[s][1], rob->sc[s][2], px[s], py[s], pz[s]);
    }
  }
  return T;
}

// Position / velocity limits (eq. 22) and null-space term (eq. 24) of one state
// q0 + dq, qd.
__device__ __forceinline__ float state_limit_cost(const StepParams& p, const float (&q0)[kNdof],
                                                  const float (&dq)[kNdof],
                                                  const float (&qd)[kNdof]) {
  float c_q = 0.f, c_qd = 0.f, c_ns = 0.f;
#pragma unroll
  for (int j = 0; j < kNdof; ++j) {
    const float q = q0[j] + dq[j];
    const float vq = limit_violation(q, p.qlo[j], p.qhi[j]);
    const float vqd = limit_violation(qd[j], p.qdlo[j], p.qdhi[j]);
    const float e = q - p.qref[j];
    c_q = fmaf(vq, vq, c_q);
    c_qd = fmaf(vqd, vqd, c_qd);
    c_ns = fmaf(e, e, c_ns);
  }
  return fmaf(p.w_q, c_q, fmaf(p.w_qd, c_qd, p.w_ns * c_ns));
}

// Cost charged by thread (m, k): control terms of u_k and state terms of state k+1.
//   q0 : start positions (wave-uniform);  dq, qd : q_{k+1} - q0 and qd_{k+1};  u : u_k;
//   sc0 : sin(q0) then cos(q0) (LDS).
//   kFar: the robot's self-collision pairs all join links two or more apart (the usual
//   sphere model), so the groups of a link with itself and with its neighbour, which
//   then hold no pair, are left out of the code (a smaller kernel, fewer instruction
//   fetches); otherwise every group is tested at run time.
template <int kElemBytes, bool kFar>
__device__ __forceinline__ float step_cost(const DevRobot* __restrict__ rob, const StepParams& p,
                                           __amdgpu_buffer_rsrc_t rsrc,
                                           __amdgpu_buffer_rsrc_t crsrc, const float* sc0,
                                           const float (&q0)[kNdof],
                                           const float (&dq)[kNdof], const float (&qd)[kNdof],
                                           const float (&u)[kNdof], bool terminal) {
  // Smoothness (eq. 23) and acceleration limit (eq. 22) on u_k.
  float c_u2 = 0.f, c_ulim = 0.f;
#pragma unroll
  for (int j = 0; j < kNdof; ++j) {
    c_u2 = fmaf(u[j], u[j], c_u2);
    const float v = limit_violation(u[j], p.qddlo[j], p.qddhi[j]);
    c_ulim = fmaf(v, v, c_ulim);
  }
  float cost = fmaf(p.w_smooth, c_u2, p.w_qdd * c_ulim);
  if (!terminal) cost += state_limit_cost(p, q0, dq, qd);

  float px[kSlots], py[kSlots], pz[kSlots];
  const Frame T = fk_spheres(rob, sc0, dq, px, py, pz);
  // Pose tracking (eq. 16) or terminal (eq. 25) cost.
  cost += pose_cost(T, p, terminal ? p.w_term_t : p.w_pose_t, terminal ? p.w_term_r : p.w_pose_r);

  if (terminal) return cost;

  // Environment collision (eqs. 17, 19, 20), with the self-collision terms evaluated
  // while the coarse bounds are in flight.  With coarse bounds, all spheres first
  // fetch the bound of their lookup cell (one load each, issued together); a sphere
  // whose bound clears its threshold has phi >= threshold, i.e. a hinge of exactly 0,
  // and skips the trilinear lookup.
  const uint32_t active = rob->slot_active;
  uint32_t need = active;
  float bound[kSlots];
  if (p.coarse_bytes != 0u) {
#pragma unroll
    for (int s = 0; s < kSlots; ++s) bound[s] = coarse_bound(crsrc, p, px[s], py[s], pz[s]);
  }

  // Self collision (eqs. 18-20), grouped by link pair.  When no lane's link bounding
  // spheres overlap, no pair of the two links can overlap and the group is skipped
  // (its hinges are exactly 0); otherwise each sphere of the first link is tested
  // against the second link's bounding sphere the same way, and each remaining pair
  // takes a squared-distance test, with a square root only on overlap.
  float c_self = 0.f;
#pragma unroll
  for (int la = 0; la < kNdof; ++la) {
#pragma unroll
    for (int lb = kFar ? la + 2 : la; lb < kNdof; ++lb) {
      const LinkPair& G = rob->lp[la * kNdof + lb];
      const uint32_t mask = G.mask;
      if (mask == 0u) continue;
      bool near = true;
      if (la != lb) {
        // A link's bounding sphere is centred on the sphere in its first slot.
        const int ca = la * kSpl, cb = lb * kSpl;
        const float dx = px[ca] - px[cb], dy = py[ca] - py[cb], dz = pz[ca] - pz[cb];
        near = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < G.bthr;
      }
      if (near) {
        // The group's constants, fetched together before any of them is used.
        float sthr[kSpl], rr2[kSpl * kSpl], rs[kSpl * kSpl];
#pragma unroll
        for (int i = 0; i < kSpl; ++i) sthr[i] = G.sthr[i];
#pragma unroll
        for (int b = 0; b < kSpl * kSpl; ++b) {
          rr2[b] = G.rr2[b];
          rs[b] = G.rs[b];
        }
#pragma unroll
        for (int i = 0; i < kSpl; ++i) {
          if (!(mask & (0xFu << (i * kSpl)))) continue;
          // Sphere i of la against lb's bounding sphere: when clear, so is each of
          // its pairs with lb (exactly, by the same margin as the link test).
          if (la != lb) {
            const int sa = la * kSpl + i, cb = lb * kSpl;
            const float dx = px[sa] - px[cb], dy = py[sa] - py[cb], dz = pz[sa] - pz[cb];
            if (!(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < sthr[i])) continue;
          }
#pragma unroll
          for (int j = 0; j < kSpl; ++j) {
            const int bit = i * kSpl + j;
            if (!(mask & (1u << bit))) continue;
            const int sa = la * kSpl + i, sb = lb * kSpl + j;
            const float dx = px[sa] - px[sb], dy = py[sa] - py[sb], dz = pz[sa] - pz[sb];
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (d2 < rr2[bit]) {
              const float h = rs[bit] - sqrt_hw(d2);
              c_self = fmaf(h, h, c_self);
            }
          }
        }
      }
    }
  }
  if (p.coarse_bytes != 0u) {
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
      if (bound[s] >= p.env_thr[s]) need &= ~(1u << s);
  }
  float c_env = 0.f;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    if (need & (1u << s)) {
      const float phi = esdf_lookup<kElemBytes>(rsrc, p, px[s], py[s], pz[s]);
      const float h = fmaxf(p.env_thr[s] - phi, 0.f);
      c_env = fmaf(h, h, c_env);
    }
  }
  return cost + fmaf(p.w_env, c_env, p.w_self * c_self);
}

// State terms of state 0 (pose, environment, self, q/qd limits, null space) are the
// same for every rollout (reading of eq. 28 at k = 0); they are evaluated once, by
// one whole block: one thread runs the forward-kinematics chain, one thread per
// sphere transforms the centres, the lookups and the pairs are spread over the
// block.  Every thread of the block must call this; all get the value.
template <int kElemBytes>
__device__ __forceinline__ float state0_cost(const DevRobot* __restrict__ rob,
                                             const StepParams& p, const void* grid,
                                             const float* __restrict__ state_in) {
  __shared__ float centres[kSlots * 4];
  __shared__ Frame frames[kNdof];
  __shared__ float sc0[2 * kNdof];
  __shared__ float red[1024 / kWave];
  __shared__ float pose0;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), nthreads = blockDim.x;
  if (tid < kNdof) {
    float s_, c_;
    sincosf(state_in ? state_in[tid] : p.q0[tid], &s_, &c_);
    sc0[tid] = s_;
    sc0[kNdof + tid] = c_;
  }
  __syncthreads();
  if (tid == kWave) {  // wave 0 stays free for the caller's independent loads
    float zero[kNdof], q0[kNdof], qd0[kNdof];
#pragma unroll
    for (int j = 0; j < kNdof; ++j) {
      zero[j] = 0.f;
      q0[j] = state_in ? state_in[j] : p.q0[j];
      qd0[j] = state_in ? state_in[kNdof + j] : p.qd0[j];
    }
    Frame T = identity_frame();
#pragma unroll
    for (int i = 0; i < kNdof; ++i) {
      mdh_step(T, rob->ca[i], rob->sa[i], rob->a[i], rob->d[i], sc0[kNdof + i], sc0[i]);
      frames[i] = T;
    }
    pose0 = pose_cost(T, p, p.w_pose_t, p.w_pose_r) + state_limit_cost(p, q0, zero, qd0);
  }
  __syncthreads();
  if (tid < kSlots) {
    float px, py, pz;
    transform_point(frames[tid / kSpl], rob->sc[tid][0], rob->sc[tid][1], rob->sc[tid][2], px,
                    py, pz);
    centres[tid * 4 + 0] = px;
    centres[tid * 4 + 1] = py;
    centres[tid * 4 + 2] = pz;
  }
  __syncthreads();
  float part = 0.f;
  if (tid < kSlots && (rob->slot_active & (1u << tid))) {
    const __amdgpu_buffer_rsrc_t rsrc = grid_resource(grid, p.grid_bytes);
    const float phi = esdf_lookup<kElemBytes>(rsrc, p, centres[tid * 4], centres[tid * 4 + 1],
                                              centres[tid * 4 + 2]);
    const float h = fmaxf(p.env_thr[tid] - phi, 0.f);
    part = p.w_env * h * h;
  }
  for (int i = tid; i < rob->n_pairs; i += nthreads) {
    const float4 pr = rob->pair_rec[i];
    const int a = __float_as_int(pr.x), c = __float_as_int(pr.y);
    const float dx = centres[a * 4] - centres[c * 4];
    const float dy = centres[a * 4 + 1] - centres[c * 4 + 1];
    const float dz = centres[a * 4 + 2] - centres[c * 4 + 2];
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (d2 < pr.z) {
      const float h = pr.w - sqrt_hw(d2);
      part = fmaf(p.w_self * h, h, part);
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, kWave);
  if (lane == 0) red[tid / kWave] = part;
  __syncthreads();
  float c0 = pose0;
  for (int w = 0; w < nthreads / kWave; ++w) c0 += red[w];
  return c0;
}

// LDS layout of K1 (floats unless noted), for R rollouts of H steps.
struct K1Lds {
  float* eps;    // [R*H*7]
  float* dq;     // [R*H*7]  q_{k+1} - q0
  float* qd;     // [R*H*7]  qd_{k+1}
  float* ubar;   // [H*7]
  float* cost;   // [R*H]
  float* sc0;    // [16]     sin(q0), cos(q0)
  float* x0;     // [16]     q0, qd0
  float* e;      // [R]      exp(-(S - m_b)/lambda)
  float* seg;    // [R*7*nseg*2 + 2*kSeg] velocity / displacement increments of 8-step
                 //          segments (the tail pads reads of absent segments)
  double* sr;    // [R]      per-rollout cost sums
};

constexpr int kSeg = 8;  // integration segment length

__host__ __device__ constexpr int k1_segments(int H) { return (H + kSeg - 1) / kSeg; }

__device__ __forceinline__ K1Lds k1_lds(unsigned char* base, int R, int H) {
  K1Lds L;
  const int rh7 = R * H * kNdof;
  L.eps = reinterpret_cast<float*>(base);
  L.dq = L.eps + rh7;
  L.qd = L.dq + rh7;
  L.ubar = L.qd + rh7;
  L.cost = L.ubar + H * kNdof;
  L.sc0 = L.cost + R * H;
  L.x0 = L.sc0 + 16;
  L.e = L.x0 + 16;
  // 8-byte aligned (read as float2).
  L.seg = reinterpret_cast<float*>((reinterpret_cast<uintptr_t>(L.e + R) + 7) & ~uintptr_t(7));
  const uintptr_t end = reinterpret_cast<uintptr_t>(L.seg + R * kNdof * k1_segments(H) * 2 + 2 * kSeg);
  L.sr = reinterpret_cast<double*>((end + 7) & ~uintptr_t(7));
  return L;
}

// q / d for 0 <= q < 2^12 and 1 <= d <= 64 by a float reciprocal: (q + 1/2) / d lies at
// least 1/(2d) from an integer and the product's rounding error is far below that.
__device__ __forceinline__ int div_small(int q, float inv_d) {
  return (int)(((float)q + 0.5f) * inv_d);
}

// Rollout-cost work of block b (counted within its request) of request q.
template <int kElemBytes, bool kFar>
__device__ __forceinline__ void rollout_cost_block(const DevRobot* __restrict__ rob,
                                                   const Request& q, int b) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const StepParams& p = q.p;
  const Workspace& ws = q.ws;
  const float* __restrict__ noise = q.noise;
  const float* __restrict__ U_in = q.U_in;
  const int H = p.H, R = p.R, RH = R * H;
  const K1Lds L = k1_lds(lds_raw, R, H);
  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  const int m0 = b * R;
  const int nroll = min(R, p.K - m0);

  // The robot constants the cost phase reads through chains of dependent scalar loads
  // (DH parameters, sphere slots, link-pair records) are touched once here with vector
  // loads, in parallel and beside the disturbances: after a kernel that streamed other
  // data through L2 (a new distance field) they would otherwise come from HBM one chain
  // link at a time.  The words are folded into a value the cost phase overwrites.
  constexpr int kWarm16 = (int)(offsetof(DevRobot, lbound) / 16);
  constexpr int kWarmLoads = (kWarm16 + kK1Threads - 1) / kK1Threads;
  uint4 warm[kWarmLoads];
  {
    const uint4* rw = reinterpret_cast<const uint4*>(rob);
#pragma unroll
    for (int i = 0; i < kWarmLoads; ++i) warm[i] = rw[min(tid + i * kK1Threads, kWarm16 - 1)];
  }

  // Stage this block's disturbances (contiguous [nroll][H][7]) and the nominal sequence:
  // read them, or sample them here (one (rollout, step) item per thread).
  if (noise == nullptr) {
    for (int t = tid; t < RH; t += nthreads) {
      const int r = t / H, k = t - r * H;
      float z[8];
      uint32_t w[8];
      if (r < nroll) {
        step_normals(2ull * ((uint64_t)(m0 + r) * (uint64_t)H + (uint64_t)k), p.seed_lo,
                     p.seed_hi, z, w);
      }
#pragma unroll
      for (int j = 0; j < kNdof; ++j) L.eps[t * kNdof + j] = r < nroll ? p.sigma[j] * z[j] : 0.f;
    }
  } else {
    // All loads of a thread are issued before any is stored (indices clamped into
    // range, so no load sits behind a branch); 16 bytes per load when the block's
    // disturbances start on a 16-byte boundary and both counts are multiples of 4
    // (at H = 40 every block), else 4.
    const float* src = noise + (size_t)m0 * H * kNdof;
    const int n_eps = nroll * H * kNdof;
    if ((reinterpret_cast<uintptr_t>(src) & 15u) == 0 && (n_eps & 3) == 0 &&
        ((RH * kNdof) & 3) == 0) {
      const float4* src4 = reinterpret_cast<const float4*>(src);
      float4* dst4 = reinterpret_cast<float4*>(L.eps);
      const int n4 = n_eps >> 2, t4 = (RH * kNdof) >> 2;
      constexpr int kLoads4 = 2;
      for (int i0 = tid; i0 < t4; i0 += nthreads * kLoads4) {
        float4 v[kLoads4];
#pragma unroll
        for (int c = 0; c < kLoads4; ++c) v[c] = src4[min(i0 + c * nthreads, n4 - 1)];
#pragma unroll
        for (int c = 0; c < kLoads4; ++c) {
          const int i = i0 + c * nthreads;
          if (i < t4) dst4[i] = i < n4 ? v[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
    } else {
      constexpr int kLoads = 8;
      for (int i0 = tid; i0 < RH * kNdof; i0 += nthreads * kLoads) {
        float v[kLoads];
#pragma unroll
        for (int c = 0; c < kLoads; ++c) v[c] = src[min(i0 + c * nthreads, n_eps - 1)];
#pragma unroll
        for (int c = 0; c < kLoads; ++c) {
          const int i = i0 + c * nthreads;
          if (i < RH * kNdof) L.eps[i] = i < n_eps ? v[c] : 0.f;
        }
      }
    }
  }
  for (int i = tid; i < H * kNdof; i += nthreads) L.ubar[i] = U_in[i];
  // Start state (q0, qd0): read from the device when the request carries it there.
  if (tid < 2 * kNdof) {
    const float x = q.state_in ? q.state_in[tid] : (tid < kNdof ? p.q0[tid] : p.qd0[tid - kNdof]);
    L.x0[tid] = x;
    if (tid < kNdof) {
      float s, c;
      sincosf(x, &s, &c);
      L.sc0[tid] = s;
      L.sc0[kNdof + tid] = c;
    }
  }
  {
    uint32_t x = 0u;
#pragma unroll
    for (int i = 0; i < kWarmLoads; ++i) x ^= warm[i].x ^ warm[i].y ^ warm[i].z ^ warm[i].w;
    L.cost[min(tid, RH - 1)] = __uint_as_float(x);
  }
  __syncthreads();

  // Roll out eq. 7 (semi-implicit Euler) per (rollout, joint), relative to (q0, qd0),
  // in segments of kSeg steps so that the dependent chain stays short: every
  // (rollout, joint, segment) item first integrates its segment from a zero start
  // (velocity increment dv, displacement dx), then starts from the state the earlier
  // segments reach (a segment of n steps entered with velocity offset v moves
  // dx + n dt v) and replays its steps.
  const int nseg = k1_segments(H);
  const int n_items = R * kNdof * nseg;
  const float inv_nseg = 1.f / (float)nseg;
  // Item w = ((r * 7 + j) * nseg + sg): rollout r, joint j, segment sg.  Its controls are
  // read at a constant stride from the segment's first row (rows past H - 1 read padding
  // or the next rollout and are never used).  A thread keeps its items' controls in
  // registers for the second pass (at most kMaxItems items per thread).
  constexpr int kMaxItems = 2;
  float uk[kMaxItems][kSeg];
#pragma unroll
  for (int it = 0; it < kMaxItems; ++it) {
    const int w = tid + it * nthreads;
    const int rj = div_small(w, inv_nseg), sg = w - rj * nseg;
    const int r = div_small(rj, 1.f / 7.f), j = rj - r * kNdof;
    if (w < n_items && r < nroll) {
      const float dt = p.dt, qd0 = L.x0[kNdof + j];
      const int k0 = sg * kSeg;
      const float* e_p = L.eps + (__mul24(r, H) + k0) * kNdof + j;
      const float* u_p = L.ubar + k0 * kNdof + j;
#pragma unroll
      for (int c = 0; c < kSeg; ++c) uk[it][c] = u_p[c * kNdof] + e_p[c * kNdof];  // eq. 27
      float dv = 0.f, dx = 0.f;
#pragma unroll
      for (int c = 0; c < kSeg; ++c) {
        if (k0 + c < H) {
          dv = fmaf(uk[it][c], dt, dv);
          dx = fmaf(qd0 + dv, dt, dx);
        }
      }
      L.seg[2 * w] = dv;
      L.seg[2 * w + 1] = dx;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kMaxItems; ++it) {
    const int w = tid + it * nthreads;
    const int rj = div_small(w, inv_nseg), sg = w - rj * nseg;
    const int r = div_small(rj, 1.f / 7.f), j = rj - r * kNdof;
    if (w < n_items && r < nroll) {
      const float dt = p.dt, qd0 = L.x0[kNdof + j];
      const int k0 = sg * kSeg;
      const float2* sp = reinterpret_cast<const float2*>(L.seg) + rj * nseg;
      float2 pvx[kSeg - 1];
#pragma unroll
      for (int c = 0; c < kSeg - 1; ++c) pvx[c] = sp[c];  // earlier segments (c < sg used)
      float dqd = 0.f, dq = 0.f;
      const float full = (float)kSeg * dt;
#pragma unroll
      for (int c = 0; c < kSeg - 1; ++c) {  // earlier segments are full
        if (c < sg) {
          dq = fmaf(full, dqd, dq + pvx[c].y);
          dqd += pvx[c].x;
        }
      }
      float* dq_r = L.dq + (__mul24(r, H) + k0) * kNdof + j;
      float* qd_r = L.qd + (__mul24(r, H) + k0) * kNdof + j;
#pragma unroll
      for (int c = 0; c < kSeg; ++c) {
        if (k0 + c < H) {
          dqd = fmaf(uk[it][c], dt, dqd);
          const float qd = qd0 + dqd;
          dq = fmaf(qd, dt, dq);
          dq_r[c * kNdof] = dq;
          qd_r[c * kNdof] = qd;
        }
      }
    }
  }
  __syncthreads();

  // Per-(rollout, step) cost.
  if (tid < RH) {
    const int r = div_small(tid, 1.f / (float)H), k = tid - __mul24(r, H);
    float cost = 0.f;
    if (r < nroll) {
      const int base = tid * kNdof;
      float dq[kNdof], qd[kNdof], u[kNdof];
#pragma unroll
      for (int j = 0; j < kNdof; ++j) {
        dq[j] = L.dq[base + j];
        qd[j] = L.qd[base + j];
        u[j] = L.ubar[k * kNdof + j] + L.eps[base + j];
      }
      float q0[kNdof];  // wave-uniform: moved to scalar registers
#pragma unroll
      for (int j = 0; j < kNdof; ++j)
        q0[j] = __builtin_bit_cast(
            float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, L.x0[j])));
      const __amdgpu_buffer_rsrc_t rsrc = grid_resource(q.grid, p.grid_bytes);
      const __amdgpu_buffer_rsrc_t crsrc = grid_resource(q.coarse, p.coarse_bytes);
      cost = step_cost<kElemBytes, kFar>(rob, p, rsrc, crsrc, L.sc0, q0, dq, qd, u, k == H - 1);
    }
    L.cost[tid] = cost;
  }
  __syncthreads();

  // S^(m) without the k = 0 state terms (eq. 28), summed over k in double, and the
  // block's softmax partial (eqs. 29-30 regrouped per block), by wave 0: G = 64 / R
  // (rounded down to a power of 2) lanes per rollout, lane j of rollout r summing
  // steps k = j, j + G, ... in order, then a butterfly over the G lanes.  The block
  // minimum and the sums of exponentials then run over the rollouts in order, every lane
  // reading the per-rollout values back from LDS (one wave's LDS accesses complete in
  // program order, so no barrier is needed).  The global stores come last, so that no
  // wait for them delays the exchange.
  if (tid < kWave) {
    int G = 1;
    while (G * 2 * R <= kWave) G *= 2;
    const int r = tid / G, j = tid - r * G;
    double s = 0.0;
    if (r < nroll) {
      const float* c_r = L.cost + r * H;
      for (int c0 = 0; j + c0 * G < H; c0 += 8) {
        float cv[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) cv[c] = c_r[min(j + (c0 + c) * G, H - 1)];
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (j + (c0 + c) * G < H) s += (double)cv[c];
      }
    }
    for (int off = G / 2; off > 2; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (G >= 4) s += dpp_f64<kDppSwap2>(s);  // the same pairs as xor 2 and xor 1
    if (G >= 2) s += dpp_f64<kDppSwap1>(s);
    if (r < nroll && j == 0) L.sr[r] = s;
    __builtin_amdgcn_wave_barrier();
    constexpr int kBatch = 8;  // LDS reads in flight at once
    double mn = __builtin_inf();
    for (int r0 = 0; r0 < nroll; r0 += kBatch) {
      double v[kBatch];
#pragma unroll
      for (int c = 0; c < kBatch; ++c) v[c] = L.sr[min(r0 + c, nroll - 1)];
#pragma unroll
      for (int c = 0; c < kBatch; ++c)
        if (isfinite(v[c])) mn = fmin(mn, v[c]);  // a repeated last value changes nothing
    }
    const bool fin = r < nroll && j == 0 && isfinite(s);
    const float e = (fin && isfinite(mn)) ? softmax_factor((float)(s - mn), p.k_lambda) : 0.f;
    if (r < R && j == 0) L.e[r] = e;
    __builtin_amdgcn_wave_barrier();
    float Z = 0.f, Z2 = 0.f;
    for (int r0 = 0; r0 < nroll; r0 += kBatch) {
      float v[kBatch];
#pragma unroll
      for (int c = 0; c < kBatch; ++c) v[c] = L.e[min(r0 + c, nroll - 1)];
#pragma unroll
      for (int c = 0; c < kBatch; ++c) {
        if (r0 + c < nroll) {
          Z += v[c];
          Z2 = fmaf(v[c], v[c], Z2);
        }
      }
    }
    if (r < nroll && j == 0) ws.S[m0 + r] = s;
    if (tid == 0) {
      ws.part_m[b] = mn;
      ws.part_Z[b] = Z;
      ws.part_Z2[b] = Z2;
    }
  }
  __syncthreads();
  // N_b[o] = sum_r e_r eps_r[o], two consecutive outputs per thread, stored by output
  // chunk: the kOutPerBlock outputs of chunk o / kOutPerBlock of all blocks are
  // contiguous ([chunk][block][kOutPerBlock]), so a merge block reads whole lines.
  const int HO = H * kNdof, HO8 = (HO + kOutPerBlock - 1) & ~(kOutPerBlock - 1);
  for (int o = 2 * tid; o < HO8; o += 2 * nthreads) {
    float acc0 = 0.f, acc1 = 0.f;
    const int o1 = min(o + 1, HO - 1);
    if (o < HO) {
      for (int r0 = 0; r0 < nroll; r0 += 8) {
        float ev[8], xv0[8], xv1[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int r = min(r0 + c, nroll - 1);
          ev[c] = L.e[r];
          xv0[c] = L.eps[r * HO + o];
          xv1[c] = L.eps[r * HO + o1];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {  // weight-0 rollouts excluded
          if (r0 + c < nroll && ev[c] > 0.f) {
            acc0 = fmaf(ev[c], xv0[c], acc0);
            acc1 = fmaf(ev[c], xv1[c], acc1);
          }
        }
      }
    }
    float* dst = ws.part_N + ((size_t)(o / kOutPerBlock) * p.P + b) * kOutPerBlock +
                 o % kOutPerBlock;
    dst[0] = acc0;
    dst[1] = o + 1 < HO ? acc1 : 0.f;
  }
}

// Register budget: at most 128 VGPRs (4 waves per SIMD), so that a CU holds a third
// block next to two rollout blocks -- the extra state-0 block of a plan step runs
// alongside them instead of waiting for a rollout block to finish.
//
// One plan step: the request travels by value in the kernel arguments.
//
// With the state-0 terms requested, block 0 evaluates them and the rollout blocks
// follow: the dispatcher places blocks in index order and fills each CU with two
// rollout blocks, so an extra block at the end would only start when one of them ends.
template <int kElemBytes, bool kFar>
__device__ __forceinline__ void plan_rollout_block(const DevRobot* __restrict__ rob,
                                                   const Request& q, int bi) {
  const int b = bi - q.c0_in_ws;
  if (b < 0) {
    const float c0 = state0_cost<kElemBytes>(rob, q.p, q.grid, q.state_in);
    if (threadIdx.x == 0) q.ws.c0[0] = c0;
    return;
  }
  rollout_cost_block<kElemBytes, kFar>(rob, q, b);
}

template <int kElemBytes, bool kFar>
__global__ __launch_bounds__(kK1Threads) __attribute__((amdgpu_waves_per_eu(4))) void
rollout_cost_kernel(const DevRobot* __restrict__ rob, const Request q) {
  plan_rollout_block<kElemBytes, kFar>(rob, q, (int)blockIdx.x);
}

// A batch of plan steps: block_req maps each block to its request.
template <int kElemBytes, bool kFar>
__global__ __launch_bounds__(kK1Threads) __attribute__((amdgpu_waves_per_eu(4))) void
rollout_cost_batch_kernel(const DevRobot* __restrict__ rob, const Request* __restrict__ reqs,
                          const int32_t* __restrict__ block_req) {
  const Request& q = reqs[block_req[blockIdx.x]];
  rollout_cost_block<kElemBytes, kFar>(rob, q, (int)blockIdx.x - q.k1_begin);
}

// ---------------------------------------------------------------------------
// K2: merge
// ---------------------------------------------------------------------------


// Global statistics of the block partials, computed by one whole wave:
// m = min_b m_b over finite m_b, then with c_b = exp(-(m_b - m)/lambda),
// Z = sum_b Z_b c_b and Z2 = sum_b Z2_b c_b^2 (eqs. 29-30 regrouped).  Lane l folds
// rows b = l + 64 c in order and the lanes combine in a fixed order (DPP moves, then
// readlanes), so every wave that calls this (in any block) gets bitwise the same
// result, with no barrier; all 64 lanes of the wave take part.  The first kStatRows
// rows per lane are loaded in one round and kept; larger P reloads the rest.
// m = +inf when no cost is finite.
struct GlobalStats {
  double m;
  float Z, Z2;
};
constexpr int kStatRows = 12;

// Rows of the first round, loaded by stats_load and folded by stats_finish (so a
// caller can issue the loads early and overlap their latency with other work).
struct StatRows {
  double m[kStatRows];
  float z[kStatRows], z2[kStatRows];
};

__device__ __forceinline__ void stats_load(const Workspace& ws, int P, int lane, StatRows& r) {
#pragma unroll
  for (int c = 0; c < kStatRows; ++c) {
    const int b = min(lane + kWave * c, P - 1);
    r.m[c] = ws.part_m[b];
    r.z[c] = ws.part_Z[b];
    r.z2[c] = ws.part_Z2[b];
  }
}

__device__ __forceinline__ GlobalStats stats_finish(const Workspace& ws, int P, float k_lambda,
                                                    int lane, const StatRows& r) {
  double mn = __builtin_inf();
#pragma unroll
  for (int c = 0; c < kStatRows; ++c)
    if (lane + kWave * c < P) mn = fmin(mn, r.m[c]);
  for (int b = lane + kWave * kStatRows; b < P; b += kWave) mn = fmin(mn, ws.part_m[b]);
  mn = wave_min_f64(mn);
  float Z = 0.f, Z2 = 0.f;
  if (isfinite(mn)) {
#pragma unroll
    for (int c = 0; c < kStatRows; ++c) {
      if (lane + kWave * c >= P || !isfinite(r.m[c])) continue;
      const float e = softmax_factor((float)(r.m[c] - mn), k_lambda);
      Z = fmaf(r.z[c], e, Z);
      Z2 = fmaf(r.z2[c], e * e, Z2);
    }
    for (int b = lane + kWave * kStatRows; b < P; b += kWave) {
      const double mb = ws.part_m[b];
      if (!isfinite(mb)) continue;
      const float e = softmax_factor((float)(mb - mn), k_lambda);
      Z = fmaf(ws.part_Z[b], e, Z);
      Z2 = fmaf(ws.part_Z2[b], e * e, Z2);
    }
  }
  return {mn, wave_sum_f32(Z), wave_sum_f32(Z2)};
}

__device__ __forceinline__ GlobalStats wave_stats(const Workspace& ws, int P, float k_lambda,
                                                  int lane) {
  StatRows r;
  stats_load(ws, P, lane, r);
  return stats_finish(ws, P, k_lambda, lane, r);
}

// State terms of state 0 (pose, environment, self, q/qd limits, null space) are the
// same for every rollout (reading of eq. 28 at k = 0); K2's block 0 evaluates them
// once: one thread runs the forward kinematics, then the sphere centres, lookups
// and pairs are spread over the block.
//
// Grid of K2: block 0 as above (costs and statistics); then one block per
// kOutPerBlock outputs o in [0, 7H) merges the block partials into U*[o]: thread t
// folds partial rows b = t / kOutPerBlock (mod kRowGroups) of output t % kOutPerBlock;
// the partials are stored chunk-major, so one load instruction of a wave reads 256
// contiguous bytes (8 rows x 8 outputs); then one
// block per kWeightsPerBlock rollouts writes the weights.
constexpr int kCostsPerThread = 32;   // costs per thread per later pass
constexpr int kCostsAhead = 16;       // costs per thread loaded before c0 (K <= 4096)
constexpr int kRowGroups = kK2Threads / kOutPerBlock;
constexpr int kRowsAhead = 24;  // partial rows per thread loaded before the statistics
constexpr int kWeightsPerThread = kWeightsPerBlock / kK2Threads;

template <int kElemBytes>
__device__ __forceinline__ void merge_block(const DevRobot* __restrict__ rob, const Request& q,
                                            int kb) {
  const StepParams& p = q.p;
  const Workspace& ws = q.ws;
  const void* grid = q.grid;
  const float* U_in = q.U_in;
  float* U_out = q.U_out;
  float* __restrict__ costs_out = q.costs_out;
  float* __restrict__ weights_out = q.weights_out;
  float* __restrict__ stats_out = q.stats_out;
  __shared__ float red[kK2Threads];
  const int lane = threadIdx.x & (kWave - 1);
  const int tid = threadIdx.x;
  const int K = p.K, P = p.P, HO = p.H * kNdof;
  const int n_out_blocks = (HO + kOutPerBlock - 1) / kOutPerBlock;

  if (kb == 0) {
    if (!costs_out && !stats_out) return;
    // --- independent fetches first: the statistics rows (wave 0) and the first
    // pass of costs to shift
    StatRows rows;
    if (stats_out && tid < kWave) stats_load(ws, P, lane, rows);
    double sv0[kCostsAhead];
    if (costs_out) {
#pragma unroll
      for (int c = 0; c < kCostsAhead; ++c) sv0[c] = ws.S[min(tid + kK2Threads * c, K - 1)];
    }
    const float c0 = q.c0_in_ws ? ws.c0[0] : state0_cost<kElemBytes>(rob, p, grid, q.state_in);
    // --- costs S = S' + c0 (eq. 28) and statistics
    if (costs_out) {
#pragma unroll
      for (int c = 0; c < kCostsAhead; ++c) {
        const int i = tid + kK2Threads * c;
        if (i < K) costs_out[i] = (float)(sv0[c] + (double)c0);
      }
      for (int base = kK2Threads * kCostsAhead; base < K; base += kK2Threads * kCostsPerThread) {
        double sv[kCostsPerThread];
#pragma unroll
        for (int c = 0; c < kCostsPerThread; ++c) {
          const int i = base + tid + kK2Threads * c;
          sv[c] = i < K ? ws.S[i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kCostsPerThread; ++c) {
          const int i = base + tid + kK2Threads * c;
          if (i < K) costs_out[i] = (float)(sv[c] + (double)c0);
        }
      }
    }
    GlobalStats st{__builtin_inf(), 0.f, 0.f};
    if (stats_out && tid < kWave) st = stats_finish(ws, P, p.k_lambda, lane, rows);
    if (stats_out && tid == 0) {
      const bool ok = isfinite(st.m);
      stats_out[0] = ok ? (float)(st.m + (double)c0) : __builtin_nanf("");
      stats_out[1] = ok ? st.Z : 0.f;
      stats_out[2] = ok ? st.Z * st.Z / st.Z2 : 0.f;
      stats_out[3] = ok ? 0.f : (float)SMPC_E_NUMERIC;
    }
    return;
  }

  const int ob = kb - 1;  // output block, or weight block after them
  if (ob >= n_out_blocks && !weights_out) return;
  // The loads of this block's partial rows (or costs) are issued before the
  // statistics, which they do not depend on, so both memory rounds overlap.
  const int oi = tid % kOutPerBlock, g = tid / kOutPerBlock;
  const int o = ob * kOutPerBlock + oi;
  const bool is_out = ob < n_out_blocks;
  // This block's chunk of the block partials: [block][kOutPerBlock], contiguous.
  const float* chunk = ws.part_N + (size_t)min(ob, n_out_blocks - 1) * P * kOutPerBlock + oi;
  float nv[kRowsAhead];
  double mv[kRowsAhead];
  const int lo = (ob - n_out_blocks) * kWeightsPerBlock;
  double sv[kWeightsPerThread];
  if (is_out) {
#pragma unroll
    for (int c = 0; c < kRowsAhead; ++c) {
      const int b = min(g + kRowGroups * c, P - 1);
      nv[c] = chunk[(size_t)b * kOutPerBlock];
      mv[c] = ws.part_m[b];
    }
  } else {
#pragma unroll
    for (int c = 0; c < kWeightsPerThread; ++c) sv[c] = ws.S[min(lo + tid + kK2Threads * c, K - 1)];
  }
  const GlobalStats st = wave_stats(ws, P, p.k_lambda, lane);
  const bool ok = isfinite(st.m);

  if (is_out) {
    // U*[o] = Ubar[o] + sum_b N_b[o] c_b / Z   (eq. 30)
    float acc = 0.f;
    if (ok && o < HO) {
#pragma unroll
      for (int c = 0; c < kRowsAhead; ++c) {
        if (g + kRowGroups * c < P && isfinite(mv[c]))
          acc = fmaf(nv[c], softmax_factor((float)(mv[c] - st.m), p.k_lambda), acc);
      }
      constexpr int kBatch = 8;
      for (int b0 = g + kRowGroups * kRowsAhead; b0 < P; b0 += kRowGroups * kBatch) {
        float nb[kBatch];
        double mb[kBatch];
#pragma unroll
        for (int c = 0; c < kBatch; ++c) {
          const int b = min(b0 + kRowGroups * c, P - 1);
          nb[c] = chunk[(size_t)b * kOutPerBlock];
          mb[c] = ws.part_m[b];
        }
#pragma unroll
        for (int c = 0; c < kBatch; ++c) {
          if (b0 + kRowGroups * c < P && isfinite(mb[c]))
            acc = fmaf(nb[c], softmax_factor((float)(mb[c] - st.m), p.k_lambda), acc);
        }
      }
    }
    red[tid] = acc;
    __syncthreads();
    if (g == 0 && o < HO) {
      float n = 0.f;
#pragma unroll
      for (int r = 0; r < kRowGroups; ++r) n += red[r * kOutPerBlock + oi];
      const float u = ok ? U_in[o] + n / st.Z : U_in[o];
      if (o < kNdof) {
        if (q.u0_out) q.u0_out[o] = u;
        if (q.state_out) {
          // Execute u*_0 for one period with the rollouts' integrator (eq. 7):
          // qd' = qd0 + u*_0 dt, q' = q0 + qd' dt.
          const float q0 = q.state_in ? q.state_in[o] : p.q0[o];
          const float qd0 = q.state_in ? q.state_in[kNdof + o] : p.qd0[o];
          const float qd1 = fmaf(u, p.dt, qd0);
          q.state_out[o] = fmaf(qd1, p.dt, q0);
          q.state_out[kNdof + o] = qd1;
        }
      }
      if (q.U_star_out) q.U_star_out[o] = u;
      if (!q.shift_out) {
        U_out[o] = u;
      } else {
        // Receding-horizon warm start: U_out = [u*_1 .. u*_{H-1}, 0].
        if (o >= kNdof) U_out[o - kNdof] = u;
        if (o >= HO - kNdof) U_out[o] = 0.f;
      }
    }
    return;
  }
  // w^(m) (eq. 29) for this block's rollouts.
  const float invZ = ok ? 1.f / st.Z : 0.f;
#pragma unroll
  for (int c = 0; c < kWeightsPerThread; ++c) {
    const int i = lo + tid + kK2Threads * c;
    if (i >= K) continue;
    float w = 0.f;
    if (ok && isfinite(sv[c])) w = softmax_factor((float)(sv[c] - st.m), p.k_lambda) * invZ;
    weights_out[i] = w;
  }
}

template <int kElemBytes>
__global__ __launch_bounds__(kK2Threads) void merge_kernel(const DevRobot* __restrict__ rob,
                                                           const Request q) {
  merge_block<kElemBytes>(rob, q, blockIdx.x);
}

template <int kElemBytes>
__global__ __launch_bounds__(kK2Threads) void merge_batch_kernel(
    const DevRobot* __restrict__ rob, const Request* __restrict__ reqs,
    const int32_t* __restrict__ block_req) {
  const Request& q = reqs[block_req[blockIdx.x]];
  merge_block<kElemBytes>(rob, q, (int)blockIdx.x - q.k2_begin);
}

// The disturbances of the sampling mode, for inspection: eps [K][H][7] and the raw
// Philox words [K][H][8] (either output may be null).  One thread per item.
__global__ __launch_bounds__(256) void sample_noise_kernel(uint32_t k0, uint32_t k1, int K, int H,
                                                           SigmaArg sigma, float* eps,
                                                           uint32_t* words) {
  const long long item = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= (long long)K * H) return;
  float z[8];
  uint32_t w[8];
  step_normals(2ull * (uint64_t)item, k0, k1, z, w);
  if (eps) {
#pragma unroll
    for (int j = 0; j < kNdof; ++j) eps[item * kNdof + j] = sigma.v[j] * z[j];
  }
  if (words) {
#pragma unroll
    for (int j = 0; j < 8; ++j) words[item * 8 + j] = w[j];
  }
}

// float32 -> float16 grid: clamp to [-clamp, clamp], round to nearest even.
// Coarse lower bounds (smpc_grid_coarse_min): one block per row (cy, cz) of cells.
// Each thread folds one x column of the rows y in [8 cy, 8 cy + 8], z in
// [8 cz, 8 cz + 8] (clamped to the grid) -- minimum, largest |phi|, any non-finite
// value -- with a batch of loads in flight; then each cell combines its 9 columns
// [8 cx, 8 cx + 8] through LDS.  The x axis is covered in chunks of 31 cells (249
// columns).  A non-finite value anywhere in a cell's window makes its bound -inf.
// A ball of query points in continuous-index units (u = (p - origin) / voxel - 1/2
// per axis): centre c and radius r; r = inf takes every cell.  Cell k along an axis
// (nk cells) holds the lookups with u in [8k, 8k + 8), extended to -inf for k = 0 and
// to +inf for k = nk - 1 by the clamping of the lookup (R5).
struct CoarseBall {
  float c[3];
  float r2;
};

// Squared distance, along one axis, from the ball centre to the u-range of cells
// [k0, k1].
__device__ __forceinline__ float coarse_axis_gap(float c, int k0, int k1, int nk) {
  const float lo = k0 == 0 ? -__builtin_inff() : 8.f * (float)k0;
  const float hi = k1 == nk - 1 ? __builtin_inff() : 8.f * (float)(k1 + 1);
  const float d = fmaxf(fmaxf(lo - c, c - hi), 0.f);
  return d * d;
}

constexpr int kCoarseThreads = 256;
constexpr int kCellsPerChunk = (kCoarseThreads - 1) / kCoarseCell;  // 31

template <int kElemBytes>
__global__ __launch_bounds__(kCoarseThreads) void grid_coarse_min_kernel(
    const void* __restrict__ grid, uint32_t grid_bytes, int nx, int ny, int nz, int ncx,
    int ncy, int ncz, CoarseBall ball, float* __restrict__ out) {
  __shared__ float col_min[kCoarseThreads], col_max[kCoarseThreads];
  __shared__ int col_bad[kCoarseThreads];
  const int cy = blockIdx.x % ncy, cz = blockIdx.x / ncy;
  const int y0 = cy * kCoarseCell, z0 = cz * kCoarseCell;
  const int wy = min(y0 + kCoarseCell, ny - 1) - y0 + 1;
  const int wz = min(z0 + kCoarseCell, nz - 1) - z0 + 1;
  const int rows = wy * wz;
  const __amdgpu_buffer_rsrc_t rsrc = grid_resource(grid, grid_bytes);
  const int tid = threadIdx.x;
  if (coarse_axis_gap(ball.c[0], 0, ncx - 1, ncx) + coarse_axis_gap(ball.c[1], cy, cy, ncy) +
          coarse_axis_gap(ball.c[2], cz, cz, ncz) > ball.r2) {
    // No lookup from the ball reaches this row of cells: no bound (never skips).
    for (int cx = tid; cx < ncx; cx += kCoarseThreads)
      out[((long long)cz * ncy + cy) * ncx + cx] = -__builtin_inff();
    return;
  }
  for (int cx0 = 0; cx0 < ncx; cx0 += kCellsPerChunk) {
    const int x0 = cx0 * kCoarseCell;
    const int x = min(x0 + tid, nx - 1);
    float mn = __builtin_inff(), mx = 0.f;
    bool bad = false;
    constexpr int kBatch = 27;
    for (int r0 = 0; r0 < rows; r0 += kBatch) {
      float v[kBatch];
#pragma unroll
      for (int c = 0; c < kBatch; ++c) {
        const int r = min(r0 + c, rows - 1);
        const int y = y0 + r % wy, z = z0 + r / wy;
        const uint32_t off = (uint32_t)(((long long)z * ny + y) * nx + x) * kElemBytes;
        v[c] = load_grid<kElemBytes>(rsrc, off, 0u);
      }
#pragma unroll
      for (int c = 0; c < kBatch; ++c) {
        bad |= !isfinite(v[c]);
        mn = fminf(mn, v[c]);
        mx = fmaxf(mx, fabsf(v[c]));
      }
    }
    col_min[tid] = mn;
    col_max[tid] = mx;
    col_bad[tid] = bad;
    __syncthreads();
    const int cx = cx0 + tid;
    if (tid < kCellsPerChunk && cx < ncx) {
      const int c_lo = tid * kCoarseCell;
      const int c_hi = min(x0 + c_lo + kCoarseCell, nx - 1) - x0;  // last column, chunk-relative
      float cmn = __builtin_inff(), cmx = 0.f;
      bool cbad = false;
      for (int c = c_lo; c <= c_hi; ++c) {
        cmn = fminf(cmn, col_min[c]);
        cmx = fmaxf(cmx, col_max[c]);
        cbad |= col_bad[c] != 0;
      }
      out[((long long)cz * ncy + cy) * ncx + cx] =
          cbad ? -__builtin_inff() : cmn - (1e-5f + cmx * 0x1p-18f);
    }
    __syncthreads();
  }
}

// Coarse lower bounds, wide path: rows whose byte length is a multiple of 16 in a
// 16-byte-aligned grid.  A block covers one row (cy, cz) of cells and a chunk of
// kCoarseChunkGroups - 1 sixteen-byte groups of columns (31 cells of float32, 63 of
// float16) plus the next group, whose first column closes the chunk's last window.
// Wave s of a block of kWaves waves loads group g (its lane) of the 9 rows of planes
// s, s + kWaves, ... of the cell row's window (all loads issued at once, at
// wave-uniform row starts; plane, row and group indices are clamped instead of masked,
// since a repeated value changes neither a minimum nor a maximum) and folds, per group,
// the minimum and the largest |phi| (with non-finite values flagged) of all its columns
// and of its first column alone.  The waves' partial results meet in LDS, then
// each cell combines its groups: the window [8 cx, 8 cx + 8] is two whole groups of
// float32 (one of float16) plus the first column of the next one, or ends at the
// last column of the row.  Blocks are laid out by XCD (block b runs on XCD b mod 8,
// and takes work item (b mod 8) * per + b / 8), so windows that share rows or
// planes are read through the same L2.
constexpr int kCoarseChunkGroups = 64;
constexpr int kCoarseSubsets = 5;
constexpr int kCoarseWideThreads = kCoarseChunkGroups * kCoarseSubsets;  // 320
constexpr int kXcds = 8;
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));

// One wide-path bounds job: the grid, its cell counts, the work items (chunks x cell
// rows) and the ball the bounds are restricted to.
struct CoarseJob {
  const unsigned char* grid;
  int nx, ny, nz, ncx, ncy, ncz, nchunks, nwork;
  CoarseBall ball;
  float* out;
};

// Wave s of a bounds block: loads group `lane_off` of the 9 rows of the kP planes s,
// s + kWaves, ... of the window (plane and row indices clamped to it: a repeated row
// changes nothing), all issued at once at wave-uniform row starts, and folds them into
// the minimum and the largest |phi| as the bits of |phi|, over all columns of the group
// and over its first column alone.  For a float the bits with the sign cleared order like
// |phi| when finite and are >= 0x7f800000 for +-inf and NaN, so one unsigned maximum
// gives max |phi| and flags any non-finite value.
struct CoarseFold {
  float mn, fmn;
  uint32_t mxb, fmxb;
};

template <int kElemBytes, int kP>
__device__ __forceinline__ CoarseFold coarse_fold(const unsigned char* __restrict__ grid,
                                                  size_t plane_bytes, size_t row_bytes, int z0,
                                                  int wz, int y0, int wy, int s, int kWaves,
                                                  uint32_t lane_off) {
  constexpr int kCols = 16 / kElemBytes;
  // Non-temporal loads: the grid streams through once and does not displace what the
  // plan step that follows keeps in L2 (robot constants, instructions).
  U32x4 v[kP][kCoarseCell + 1];
#pragma unroll
  for (int zi = 0; zi < kP; ++zi) {
    const int z = z0 + min(s + kWaves * zi, wz - 1);
#pragma unroll
    for (int yy = 0; yy <= kCoarseCell; ++yy) {
      const int y = y0 + min(yy, wy - 1);
      const unsigned char* row = grid + (size_t)z * plane_bytes + (size_t)y * row_bytes;
      v[zi][yy] = __builtin_nontemporal_load(reinterpret_cast<const U32x4*>(row + lane_off));
    }
  }
  CoarseFold f{__builtin_inff(), __builtin_inff(), 0u, 0u};
#pragma unroll
  for (int j = 0; j < kP * (kCoarseCell + 1); ++j) {
    const U32x4& vj = v[j / (kCoarseCell + 1)][j % (kCoarseCell + 1)];
    const uint32_t wd[4] = {vj[0], vj[1], vj[2], vj[3]};
#pragma unroll
    for (int c = 0; c < kCols; ++c) {
      float x;
      if constexpr (kElemBytes == 4) {
        x = __uint_as_float(wd[c]);
      } else {
        const unsigned short h = (unsigned short)(wd[c >> 1] >> ((c & 1) * 16));
        x = (float)__builtin_bit_cast(_Float16, h);
      }
      const uint32_t ab = __float_as_uint(x) & 0x7fffffffu;
      f.mn = fminf(f.mn, x);
      f.mxb = max(f.mxb, ab);
      if (c == 0) {
        f.fmn = fminf(f.fmn, x);
        f.fmxb = max(f.fmxb, ab);
      }
    }
  }
  return f;
}

// Block b (b mod 8 = the XCD it runs on) of a wide-path job, with kWaves waves.
template <int kElemBytes, int kWaves>
__device__ __forceinline__ void coarse_wide_block(const CoarseJob& J, int b) {
  constexpr int kCols = 16 / kElemBytes;                               // columns per group
  constexpr int kCells = (kCoarseChunkGroups - 1) * kCols / kCoarseCell;  // cells per chunk
  static_assert(kWaves >= 2 && kWaves <= kCoarseCell + 1, "2 to 9 waves per block");
  __shared__ float s_mn[kWaves][kCoarseChunkGroups];
  __shared__ uint32_t s_mx[kWaves][kCoarseChunkGroups];
  __shared__ float s_fmn[kWaves][kCoarseChunkGroups];
  __shared__ uint32_t s_fmx[kWaves][kCoarseChunkGroups];
  const int nx = J.nx, ny = J.ny, nz = J.nz, ncx = J.ncx, ncy = J.ncy, nchunks = J.nchunks;
  const int per = (J.nwork + kXcds - 1) / kXcds;
  const int w = (b % kXcds) * per + b / kXcds;
  if (w >= J.nwork) return;
  const int cyz = w / nchunks, ch = w - cyz * nchunks;
  const int cz = cyz / ncy, cy = cyz - cz * ncy;
  const int y0 = cy * kCoarseCell, z0 = cz * kCoarseCell;
  const int wy = min(y0 + kCoarseCell, ny - 1) - y0 + 1;
  const int wz = min(z0 + kCoarseCell, nz - 1) - z0 + 1;
  const int x0 = ch * kCells * kCoarseCell;                     // first column of the chunk
  const int n_groups = nx / kCols;                              // groups per grid row
  const int tid = threadIdx.x;
  const int cx_last = min(ch * kCells + kCells, ncx) - 1;
  if (coarse_axis_gap(J.ball.c[0], ch * kCells, cx_last, ncx) +
          coarse_axis_gap(J.ball.c[1], cy, cy, ncy) +
          coarse_axis_gap(J.ball.c[2], cz, cz, J.ncz) >
      J.ball.r2) {
    // No lookup from the ball reaches these cells: no bound (never skips), no loads.
    if (tid <= cx_last - ch * kCells)
      J.out[((size_t)cz * ncy + cy) * ncx + ch * kCells + tid] = -__builtin_inff();
    return;
  }
  // Wave s takes planes s, s + kWaves, ... of the cell row's window and all 9 of its rows,
  // so every address is a wave-uniform row start plus the lane's 16-byte group.
  const int s = __builtin_amdgcn_readfirstlane(tid / kCoarseChunkGroups);
  const int g = tid & (kCoarseChunkGroups - 1);
  const int gg = min(x0 / kCols + g, n_groups - 1);             // clamped group of the row
  const uint32_t lane_off = (uint32_t)gg * 16u;
  const size_t row_bytes = (size_t)nx * kElemBytes, plane_bytes = row_bytes * (size_t)ny;
  // The 9 planes of the window are dealt to the waves in turn: the first 9 mod kWaves
  // waves take one plane more than the others, so no plane is loaded twice.
  constexpr int kLo = (kCoarseCell + 1) / kWaves, kExtra = (kCoarseCell + 1) % kWaves;
  const CoarseFold f =
      s < kExtra ? coarse_fold<kElemBytes, kLo + 1>(J.grid, plane_bytes, row_bytes, z0, wz, y0,
                                                    wy, s, kWaves, lane_off)
                 : coarse_fold<kElemBytes, kLo>(J.grid, plane_bytes, row_bytes, z0, wz, y0, wy,
                                                s, kWaves, lane_off);
  const float mn = f.mn, fmn = f.fmn;
  const uint32_t mxb = f.mxb, fmxb = f.fmxb;
  s_mn[s][g] = mn;
  s_mx[s][g] = mxb;
  s_fmn[s][g] = fmn;
  s_fmx[s][g] = fmxb;
  __syncthreads();
  const int cx = ch * kCells + tid;
  if (tid < kCells && cx < ncx) {
    const int c_lo = tid * kCoarseCell;                          // chunk-relative columns
    const int c_hi = min(c_lo + kCoarseCell, nx - 1 - x0);
    // Whole groups [c_lo / kCols, g_end); the window's last column opens group g_end
    // when it is a group's first column (c_hi = c_lo + 8), else it closes g_end - 1.
    const bool first_only = (c_hi % kCols) == 0;
    const int g_end = first_only ? c_hi / kCols : c_hi / kCols + 1;
    float cmn = __builtin_inff();
    uint32_t cmxb = 0u;
    for (int gi = c_lo / kCols; gi < g_end; ++gi) {
#pragma unroll
      for (int t = 0; t < kWaves; ++t) {
        cmn = fminf(cmn, s_mn[t][gi]);
        cmxb = max(cmxb, s_mx[t][gi]);
      }
    }
    if (first_only) {
#pragma unroll
      for (int t = 0; t < kWaves; ++t) {
        cmn = fminf(cmn, s_fmn[t][g_end]);
        cmxb = max(cmxb, s_fmx[t][g_end]);
      }
    }
    J.out[((size_t)cz * ncy + cy) * ncx + cx] =
        cmxb >= 0x7f800000u ? -__builtin_inff()
                            : cmn - (1e-5f + __uint_as_float(cmxb) * 0x1p-18f);
  }
}

template <int kElemBytes>
__global__ __launch_bounds__(kCoarseWideThreads) void grid_coarse_min_wide_kernel(CoarseJob J) {
  coarse_wide_block<kElemBytes, kCoarseSubsets>(J, (int)blockIdx.x);
}

// A plan step's merge blocks (the first n_k2 blocks) and the wide-path bounds of another
// grid (from block n_k2p on; n_k2p is n_k2 rounded up to a multiple of 8, so that the
// bounds blocks keep their XCD layout) in one launch.  The merge blocks leave most of
// the device idle, and neither part reads what the other writes (the merge never reads
// bounds).
template <int kElemBytes>
__global__ __launch_bounds__(kK2Threads) void merge_bounds_kernel(const DevRobot* __restrict__ rob,
                                                                  const Request q, int n_k2,
                                                                  int n_k2p, CoarseJob J) {
  const int b = (int)blockIdx.x;
  if (b < n_k2)
    merge_block<kElemBytes>(rob, q, b);
  else if (b >= n_k2p)
    coarse_wide_block<kElemBytes, kK2Threads / kCoarseChunkGroups>(J, b - n_k2p);
}

// A plan step's rollout blocks (the first n_k1 blocks, as rollout_cost_kernel) and the
// wide-path bounds of another grid (from block n_k1p on; n_k1p is n_k1 rounded up to a
// multiple of 8, for the bounds blocks' XCD layout) in one launch: the bounds load while
// the rollouts, which leave HBM mostly idle, compute.  The table written must not be the
// one the rollouts read.
template <int kElemBytes, bool kFar>
__global__ __launch_bounds__(kK1Threads) __attribute__((amdgpu_waves_per_eu(4))) void
rollout_bounds_kernel(const DevRobot* __restrict__ rob, const Request q, int n_k1, int n_k1p,
                      CoarseJob J) {
  const int b = (int)blockIdx.x;
  if (b < n_k1)
    plan_rollout_block<kElemBytes, kFar>(rob, q, b);
  else if (b >= n_k1p) {
    // Hold the bounds loads back for about 2.7 us (100 x 64 clocks): every rollout block
    // first waits on its disturbances from HBM, and those loads go first (29.0 against
    // 30.2 us per period at K = 4096, H = 40 on 200^3; waiting twice as long lets the
    // bounds blocks dispatched later finish after the rollouts).
    __builtin_amdgcn_s_sleep(100);
    coarse_wide_block<kElemBytes, kK1Threads / kCoarseChunkGroups>(J, b - n_k1p);
  }
}

// ---------------------------------------------------------------------------
// Occupancy update by voxel projection (Sec. III-A) with the robot mask (Remark 2)
// ---------------------------------------------------------------------------
constexpr int kOgmThreads = 256;
constexpr int kOgmPerThread = 4;  // pixels or voxels per thread, kOgmThreads apart
constexpr int kOgmTile = kOgmThreads * kOgmPerThread;

// Robot data one thread needs for the sphere table, fetched before anything else so
// that its latency overlaps the caller's own loads: the DH constants (wave-uniform,
// scalar loads), this lane's joint angle (lanes below kNdof) and sphere slot (lanes
// below kSlots; radius -1 when the slot is empty).
struct OgmRobotFetch {
  float ca[kNdof], sa[kNdof], a[kNdof], d[kNdof];
  float q;
  float4 slot;
};

__device__ __forceinline__ OgmRobotFetch ogm_fetch_robot(const DevRobot* __restrict__ rob,
                                                         const OgmArgs& a) {
  OgmRobotFetch f;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kNdof; ++i) {
    f.ca[i] = rob->ca[i];
    f.sa[i] = rob->sa[i];
    f.a[i] = rob->a[i];
    f.d[i] = rob->d[i];
  }
  f.q = a.q[0];
#pragma unroll
  for (int i = 1; i < kNdof; ++i) f.q = tid == i ? a.q[i] : f.q;
  f.slot = make_float4(0.f, 0.f, 0.f, -1.f);
  if (tid < kSlots && (rob->slot_active & (1u << tid)))
    f.slot = *reinterpret_cast<const float4*>(rob->sc[tid]);
  return f;
}

// The robot's collision spheres at joint positions q, padded: centres and squared
// padded radii in sph[4 s .. 4 s + 3] (inactive slots get radius^2 = -1, which no
// point is within), bounding box of the padded spheres in sph[kOgmBox .. + 5] (min x,
// y, z, then max x, y, z) and in voxel indices in sph[kOgmIndexBox .. + 5].  Called
// by every thread of the block.
__device__ __forceinline__ void ogm_robot_spheres(const OgmRobotFetch& f, const OgmArgs& a,
                                                  float* sph) {
  __shared__ float sincos_q[2 * kNdof];
  __shared__ Frame frames[kNdof];
  const int tid = threadIdx.x;
  if (tid < kNdof) sincosf(f.q, &sincos_q[tid], &sincos_q[kNdof + tid]);
  __syncthreads();
  if (tid == 0) {
    Frame T = identity_frame();
#pragma unroll
    for (int i = 0; i < kNdof; ++i) {
      mdh_step(T, f.ca[i], f.sa[i], f.a[i], f.d[i], sincos_q[kNdof + i], sincos_q[i]);
      frames[i] = T;
    }
  }
  __syncthreads();
  if (tid < kWave) {
    // lanes 0..kSlots-1 hold one slot each; the box is reduced over the first 32 lanes
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    if (tid < kSlots) {
      float p[3] = {0.f, 0.f, 0.f}, r2 = -1.f;
      if (f.slot.w >= 0.f) {
        transform_point(frames[tid / kSpl], f.slot.x, f.slot.y, f.slot.z, p[0], p[1], p[2]);
        const float r = f.slot.w + a.robot_pad;
        r2 = r * r;
        const float rb = r * 1.0001f + 1e-6f;  // slack over the rounding of r^2 and |p - c|^2
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          lo[k] = p[k] - rb;
          hi[k] = p[k] + rb;
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) sph[4 * tid + k] = p[k];
      sph[4 * tid + 3] = r2;
    }
    static_assert(kSlots <= 32, "box reduction covers 32 lanes");
#pragma unroll
    for (int off = 16; off > 0; off >>= 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lo[k] = fminf(lo[k], __shfl_xor(lo[k], off, kWave));
        hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off, kWave));
      }
    if (tid == 0)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sph[kOgmBox + k] = lo[k];
        sph[kOgmBox + 3 + k] = hi[k];
        // voxel indices whose centre origin + (i + 1/2) voxel may lie in the box
        const float il = floorf((lo[k] - a.origin[k]) / a.voxel - 0.5f) - 1.f;
        const float ih = ceilf((hi[k] - a.origin[k]) / a.voxel - 0.5f) + 1.f;
        sph[kOgmIndexBox + k] = __int_as_float((int32_t)fminf(fmaxf(il, -2.f), 2.0e9f));
        sph[kOgmIndexBox + 3 + k] = __int_as_float((int32_t)fminf(fmaxf(ih, -2.f), 2.0e9f));
      }
  }
  __syncthreads();
}

// Whether p lies in a padded robot sphere (entries read at uniform addresses).
__device__ __forceinline__ bool in_robot_spheres(const float* sph, float x, float y, float z) {
  bool in = false;
#pragma unroll 4
  for (int s = 0; s < kSlots; ++s) {
    const float dx = x - sph[4 * s], dy = y - sph[4 * s + 1], dz = z - sph[4 * s + 2];
    in |= fmaf(dx, dx, fmaf(dy, dy, dz * dz)) <= sph[4 * s + 3];
  }
  return in;
}

// The same, first tested against the table's bounding box: the sphere entries are
// read only when some lane of the wave is inside the box.
__device__ __forceinline__ bool in_robot(const float* sph, float x, float y, float z) {
  const float* box = sph + kOgmBox;
  const bool in_box = (x >= box[0]) & (y >= box[1]) & (z >= box[2]) & (x <= box[3]) &
                      (y <= box[4]) & (z <= box[5]);
  return in_box && in_robot_spheres(sph, x, y, z);
}

// Pass 1: valid returns not inside the robot, others 0.  Each block takes a tile of
// kOgmTile pixels; block 0 also publishes the sphere table after the image.
__global__ __launch_bounds__(kOgmThreads) void ogm_pixel_kernel(
    const DevRobot* __restrict__ rob, const OgmArgs a, const float* __restrict__ depth,
    float* __restrict__ work) {
  __shared__ float sph[kOgmSphereFloats];
  const uint32_t npix = (uint32_t)a.width * (uint32_t)a.height;
  const uint32_t base = blockIdx.x * (uint32_t)kOgmTile + threadIdx.x;
  OgmRobotFetch rf;
  if (a.use_mask) rf = ogm_fetch_robot(rob, a);
  float d[kOgmPerThread];
#pragma unroll
  for (int k = 0; k < kOgmPerThread; ++k) {
    const uint32_t i = base + k * kOgmThreads;
    d[k] = i < npix ? depth[i] : 0.f;
  }
  if (a.use_mask) {
    ogm_robot_spheres(rf, a, sph);
    if (blockIdx.x == 0 && threadIdx.x < kOgmSphereFloats)
      work[npix + threadIdx.x] = sph[threadIdx.x];
  }
#pragma unroll
  for (int k = 0; k < kOgmPerThread; ++k) {
    const uint32_t i = base + k * kOgmThreads;
    if (i >= npix) break;
    bool keep = isfinite(d[k]) && d[k] >= a.min_depth && d[k] <= a.max_depth;
    if (keep && a.use_mask) {
      const uint32_t v = i / (uint32_t)a.width, u = i - v * (uint32_t)a.width;
      const float xc = ((float)u + 0.5f - a.cx) * d[k] / a.fx;
      const float yc = ((float)v + 0.5f - a.cy) * d[k] / a.fy;
      const float wx = fmaf(a.R[0], xc, fmaf(a.R[1], yc, fmaf(a.R[2], d[k], a.t[0])));
      const float wy = fmaf(a.R[3], xc, fmaf(a.R[4], yc, fmaf(a.R[5], d[k], a.t[1])));
      const float wz = fmaf(a.R[6], xc, fmaf(a.R[7], yc, fmaf(a.R[8], d[k], a.t[2])));
      keep = !in_robot(sph, wx, wy, wz);
    }
    work[i] = keep ? d[k] : 0.f;
  }
}

// n / d for n < 2^31 and 1 <= d < 2^31: the double quotient is within one of the
// truth, and one correction step makes it exact.
__device__ __forceinline__ uint32_t ogm_div(uint32_t n, uint32_t d, double inv_d) {
  const uint32_t q = (uint32_t)((double)n * inv_d);
  const int64_t r = (int64_t)n - (int64_t)q * d;
  return r < 0 ? q - 1u : (r >= (int64_t)d ? q + 1u : q);
}

// Raw buffer over `bytes` bytes at p: accesses past the end read 0 and write nothing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ogm_buffer(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

// Pass 2: a block takes kOgmTile consecutive voxels (x fastest), each wave 64 of them
// per step, kOgmThreads apart over kOgmPerThread steps.  The log-odds and occupancy
// are accessed through buffers bounded at the block's last voxel, so the ragged end
// needs no branch.  A wave's first voxel is split into (x, y, z) on the scalar unit;
// a lane past the end of that row wraps into the next one (at most once, as nx >= 64;
// narrower grids split every voxel).  The centre maps to (X, Y, Z) by the affine map
// M, m: Z is its depth and floor(X / Z), floor(Y / Z) its pixel, read through a
// bounded buffer, so that a voxel out of view reads past the end of the image and
// gets 0 ("no return").  Then the log-odds are updated, voxels inside the robot
// reset and the occupancy written.
__global__ __launch_bounds__(kOgmThreads) void ogm_voxel_kernel(
    const OgmArgs a, const float* __restrict__ work, float* __restrict__ log_odds,
    uint8_t* __restrict__ occ) {
  const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
  const uint32_t plane = nx * ny, nvox = plane * (uint32_t)a.nz;
  const uint32_t width = (uint32_t)a.width, height = (uint32_t)a.height;
  const uint32_t npix = width * height;
  const __amdgpu_buffer_rsrc_t img = ogm_buffer(work, npix * 4u);
  const float* sph = work + npix;
  const uint32_t blk0 = blockIdx.x * (uint32_t)kOgmTile;
  const uint32_t nblk = min(nvox - blk0, (uint32_t)kOgmTile);
  const __amdgpu_buffer_rsrc_t lbuf = ogm_buffer(log_odds + blk0, nblk * 4u);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t loc = wave * kWave + lane;  // voxel blk0 + loc + k kOgmThreads
  // Robot bounding box in voxel indices (empty without the mask).
  int32_t blo[3] = {1, 1, 1}, bhi[3] = {0, 0, 0};
  if (a.use_mask)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = __float_as_int(sph[kOgmIndexBox + k]);
      bhi[k] = __float_as_int(sph[kOgmIndexBox + 3 + k]);
    }
  float L[kOgmPerThread], d[kOgmPerThread], z[kOgmPerThread];
  uint32_t vx[kOgmPerThread], vy[kOgmPerThread], vz[kOgmPerThread];
  bool in_box[kOgmPerThread];
#pragma unroll
  for (int k = 0; k < kOgmPerThread; ++k)
    L[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                         lbuf, (int)((loc + k * kOgmThreads) * 4u), 0, 0));
#pragma unroll
  for (int k = 0; k < kOgmPerThread; ++k) {
    uint32_t ix, iy, iz;
    bool box;
    if (nx >= (uint32_t)kWave) {
      // wave-uniform split of the wave's first voxel (scalar unit)
      const uint32_t w0 = min(blk0 + wave * kWave + k * kOgmThreads, nvox - 1u);
      const uint32_t bz = __umulhi(w0, a.plane_mul) >> a.plane_shift;
      const uint32_t rem = w0 - bz * plane;
      const uint32_t by = __umulhi(rem, a.nx_mul) >> a.nx_shift;
      const uint32_t bx = rem - by * nx;
      const bool last_y = by + 1u >= ny;
      const uint32_t ny1 = last_y ? 0u : by + 1u, nz1 = last_y ? bz + 1u : bz;
      const bool row0 = ((int32_t)by >= blo[1]) & ((int32_t)by <= bhi[1]) &
                        ((int32_t)bz >= blo[2]) & ((int32_t)bz <= bhi[2]);
      const bool row1 = ((int32_t)ny1 >= blo[1]) & ((int32_t)ny1 <= bhi[1]) &
                        ((int32_t)nz1 >= blo[2]) & ((int32_t)nz1 <= bhi[2]);
      ix = bx + lane;
      const bool wrap = ix >= nx;
      ix = wrap ? ix - nx : ix;
      iy = wrap ? ny1 : by;
      iz = wrap ? nz1 : bz;
      box = false;
      if (row0 | row1)
        box = (wrap ? row1 : row0) & ((int32_t)ix >= blo[0]) & ((int32_t)ix <= bhi[0]);
    } else {
      const uint32_t i = min(blk0 + loc + k * kOgmThreads, nvox - 1u);
      iz = ogm_div(i, plane, a.inv_plane);
      iy = ogm_div(i - iz * plane, nx, a.inv_nx);
      ix = i - iz * plane - iy * nx;
      box = ((int32_t)ix >= blo[0]) & ((int32_t)ix <= bhi[0]) & ((int32_t)iy >= blo[1]) &
            ((int32_t)iy <= bhi[1]) & ((int32_t)iz >= blo[2]) & ((int32_t)iz <= bhi[2]);
    }
    const float fx = (float)ix, fy = (float)iy, fz = (float)iz;
    const float X = fmaf(a.M[0], fx, fmaf(a.M[1], fy, fmaf(a.M[2], fz, a.m[0])));
    const float Y = fmaf(a.M[3], fx, fmaf(a.M[4], fy, fmaf(a.M[5], fz, a.m[1])));
    const float Z = fmaf(a.M[6], fx, fmaf(a.M[7], fy, fmaf(a.M[8], fz, a.m[2])));
    // In front: Z above the smallest normal float, so 1 / Z and X / Z stay finite.
    const float inv_z = __builtin_amdgcn_rcpf(Z);
    const int32_t pu = __float2int_rd(X * inv_z), pv = __float2int_rd(Y * inv_z);
    const bool in_view =
        (Z > 1.17549435e-38f) & ((uint32_t)pu < width) & ((uint32_t)pv < height);
    // pixel row and column are below 2^14: a 24-bit multiply is exact
    const uint32_t off = in_view ? __umul24((uint32_t)pv, width) + (uint32_t)pu : npix;
    d[k] = __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(img, (int)(off * 4u), 0, 0));
    z[k] = Z;
    vx[k] = ix;
    vy[k] = iy;
    vz[k] = iz;
    in_box[k] = box;
  }
#pragma unroll
  for (int k = 0; k < kOgmPerThread; ++k) {
    float l = L[k];
    const float e = z[k] - d[k];
    const bool hit = fabsf(e) <= a.tol, free = e < -a.tol;
    if ((d[k] > 0.f) & (hit | free))
      l = fminf(fmaxf(l + (hit ? a.l_hit : a.l_miss), a.l_min), a.l_max);
    if (in_box[k]) {
      const float wx = a.origin[0] + ((float)vx[k] + 0.5f) * a.voxel;
      const float wy = a.origin[1] + ((float)vy[k] + 0.5f) * a.voxel;
      const float wz = a.origin[2] + ((float)vz[k] + 0.5f) * a.voxel;
      if (in_robot_spheres(sph, wx, wy, wz)) l = a.l_min;
    }
    const uint32_t o = loc + k * kOgmThreads;
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, l), lbuf, (int)(o * 4u),
                                          0, 0);
    if (occ)
      __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(l > a.l_occ ? 1 : 0),
                                           ogm_buffer(occ + blk0, nblk), (int)o, 0, 0);
  }
}

// Pass 2 for rows of a multiple of four voxels (16-byte aligned log-odds, 4-byte
// aligned occupancy): each lane takes kOgmGroups groups of four consecutive voxels of
// one row, 16 bytes of log-odds and one occupancy word per group (plain global
// accesses guarded by the group count: groups are whole); the index split and the
// affine map are evaluated once per group (X, Y, Z of the next voxel differ by the
// first column of M).  Otherwise as ogm_voxel_kernel.
constexpr int kOgmGroups = 2;
constexpr int kOgmGroupTile = kOgmThreads * kOgmGroups;  // groups per block

__global__ __launch_bounds__(kOgmThreads) void ogm_voxel4_kernel(
    const OgmArgs a, const float* __restrict__ work, float* __restrict__ log_odds,
    uint8_t* __restrict__ occ) {
  const uint32_t nx = (uint32_t)a.nx, plane = nx * (uint32_t)a.ny;
  const uint32_t ngroups = plane * (uint32_t)a.nz / 4u;
  const uint32_t width = (uint32_t)a.width, height = (uint32_t)a.height;
  const uint32_t npix = width * height;
  const __amdgpu_buffer_rsrc_t img = ogm_buffer(work, npix * 4u);
  const float* sph = work + npix;
  const uint32_t blk_g = blockIdx.x * (uint32_t)kOgmGroupTile;
  float4* __restrict__ L4 = reinterpret_cast<float4*>(log_odds);
  uint32_t* __restrict__ occ4 = reinterpret_cast<uint32_t*>(occ);
  int32_t blo[3] = {1, 1, 1}, bhi[3] = {0, 0, 0};
  if (a.use_mask)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = __float_as_int(sph[kOgmIndexBox + k]);
      bhi[k] = __float_as_int(sph[kOgmIndexBox + 3 + k]);
    }
  const uint32_t tid = threadIdx.x;
  float L[kOgmGroups][4], d[kOgmGroups][4], z[kOgmGroups][4];
  uint32_t gx[kOgmGroups], gy[kOgmGroups], gz[kOgmGroups];
  bool row_box[kOgmGroups];
#pragma unroll
  for (int k = 0; k < kOgmGroups; ++k) {
    const uint32_t g = blk_g + tid + k * kOgmThreads;
    const float4 v = g < ngroups ? L4[g] : make_float4(0.f, 0.f, 0.f, 0.f);
    L[k][0] = v.x;
    L[k][1] = v.y;
    L[k][2] = v.z;
    L[k][3] = v.w;
  }
#pragma unroll
  for (int k = 0; k < kOgmGroups; ++k) {
    const uint32_t i0 = 4u * min(blk_g + tid + k * kOgmThreads, ngroups - 1u);
    const uint32_t iz = __umulhi(i0, a.plane_mul) >> a.plane_shift;
    const uint32_t rem = i0 - iz * plane;
    const uint32_t iy = __umulhi(rem, a.nx_mul) >> a.nx_shift;
    const uint32_t ix = rem - iy * nx;
    gx[k] = ix;
    gy[k] = iy;
    gz[k] = iz;
    row_box[k] = ((int32_t)iy >= blo[1]) & ((int32_t)iy <= bhi[1]) & ((int32_t)iz >= blo[2]) &
                 ((int32_t)iz <= bhi[2]);
    const float fx = (float)ix, fy = (float)iy, fz = (float)iz;
    const float X0 = fmaf(a.M[0], fx, fmaf(a.M[1], fy, fmaf(a.M[2], fz, a.m[0])));
    const float Y0 = fmaf(a.M[3], fx, fmaf(a.M[4], fy, fmaf(a.M[5], fz, a.m[1])));
    const float Z0 = fmaf(a.M[6], fx, fmaf(a.M[7], fy, fmaf(a.M[8], fz, a.m[2])));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float X = fmaf((float)j, a.M[0], X0);
      const float Y = fmaf((float)j, a.M[3], Y0);
      const float Z = fmaf((float)j, a.M[6], Z0);
      // In front: Z above the smallest normal float, so 1 / Z and X / Z stay finite.
      const float inv_z = __builtin_amdgcn_rcpf(Z);
      const int32_t pu = __float2int_rd(X * inv_z), pv = __float2int_rd(Y * inv_z);
      const bool in_view =
          (Z > 1.17549435e-38f) & ((uint32_t)pu < width) & ((uint32_t)pv < height);
      // pixel row and column are below 2^14: a 24-bit multiply is exact
      const uint32_t off = in_view ? __umul24((uint32_t)pv, width) + (uint32_t)pu : npix;
      d[k][j] = __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(img, (int)(off * 4u), 0, 0));
      z[k][j] = Z;
    }
  }
#pragma unroll
  for (int k = 0; k < kOgmGroups; ++k) {
    uint32_t bits = 0u;
    float out[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float l = L[k][j];
      const float e = z[k][j] - d[k][j];
      const bool hit = fabsf(e) <= a.tol, free = e < -a.tol;
      if ((d[k][j] > 0.f) & (hit | free))
        l = fminf(fmaxf(l + (hit ? a.l_hit : a.l_miss), a.l_min), a.l_max);
      const int32_t ix = (int32_t)(gx[k] + j);
      if (row_box[k] & (ix >= blo[0]) & (ix <= bhi[0])) {
        const float wx = a.origin[0] + ((float)ix + 0.5f) * a.voxel;
        const float wy = a.origin[1] + ((float)gy[k] + 0.5f) * a.voxel;
        const float wz = a.origin[2] + ((float)gz[k] + 0.5f) * a.voxel;
        if (in_robot_spheres(sph, wx, wy, wz)) l = a.l_min;
      }
      out[j] = l;
      bits |= (l > a.l_occ ? 1u : 0u) << (8 * j);
    }
    const uint32_t g = blk_g + tid + k * kOgmThreads;
    if (g < ngroups) {
      L4[g] = make_float4(out[0], out[1], out[2], out[3]);
      if (occ) occ4[g] = bits;
    }
  }
}

__global__ __launch_bounds__(256) void grid_to_f16_kernel(const float* __restrict__ src,
                                                          unsigned short* __restrict__ dst,
                                                          long long n, float clamp) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float v = __builtin_amdgcn_fmed3f(src[i], -clamp, clamp);
    dst[i] = __builtin_bit_cast(unsigned short, (_Float16)v);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side launch helpers

// ---------------------------------------------------------------------------

static size_t k1_lds_bytes(int R, int H) {
  const size_t floats = (size_t)R * H * kNdof * 3 + (size_t)H * kNdof + (size_t)R * H + 32 + R +
                        (size_t)R * kNdof * k1_segments(H) * 2 + 2 * kSeg;
  return floats * 4 + 4 + 8 + (size_t)R * 8;  // seg aligned; R doubles 8-byte aligned
}

static_assert(kK1Threads == 256, "the integration keeps at most two items per thread: "
              "R * 7 * ceil(H / 8) <= 512 for R = min(64, 256 / H), 1 <= H <= 64");

LaunchConfig plan_launch_config(int K, int H) {
  // Every block has kK1Threads threads and holds R = kK1Threads / H whole rollouts
  // (at most 64), whatever else shares the launch: a request's arithmetic is the
  // same alone and in a batch.  Four waves put one wave of every block on each SIMD
  // of a CU, so the SIMDs of a CU carry equal work (a five-wave block doubles up on one
  // SIMD, and two such blocks on the same one leave it with twice the others' work).
  // 256 fits H = 16, 32 and 64 exactly and uses 240 lanes at H = 40.
  int R = kK1Threads / H;
  if (R > 64) R = 64;
  if (R < 1) R = 1;
  LaunchConfig lc;
  lc.R = R;
  lc.k1_threads = kK1Threads;
  lc.P = (K + R - 1) / R;
  lc.k1_lds = k1_lds_bytes(R, H);
  lc.k2_blocks = 1 + (H * kNdof + kOutPerBlock - 1) / kOutPerBlock +
                 (K + kWeightsPerBlock - 1) / kWeightsPerBlock;
  return lc;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Outputs 7H padded to whole merge chunks.
static size_t padded_outputs(int H) {
  return ((size_t)H * kNdof + kOutPerBlock - 1) / kOutPerBlock * kOutPerBlock;
}

size_t workspace_bytes(int K, int H, int P) {
  return align256((size_t)K * 8) + align256((size_t)P * 8) + 2 * align256((size_t)P * 4) +
         align256(padded_outputs(H) * P * 4) + 256;
}

Workspace carve_workspace(void* base, int K, int H, int P) {
  unsigned char* b = static_cast<unsigned char*>(base);
  Workspace ws;
  ws.S = reinterpret_cast<double*>(b);
  b += align256((size_t)K * 8);
  ws.part_m = reinterpret_cast<double*>(b);
  b += align256((size_t)P * 8);
  ws.part_Z = reinterpret_cast<float*>(b);
  b += align256((size_t)P * 4);
  ws.part_Z2 = reinterpret_cast<float*>(b);
  b += align256((size_t)P * 4);
  ws.part_N = reinterpret_cast<float*>(b);
  b += align256(padded_outputs(H) * P * 4);
  ws.c0 = reinterpret_cast<float*>(b);
  return ws;
}

// Workspace of the allocation-free plan step: one static array per device, held until
// the process ends.  Host code never hands `scratch` itself to a kernel or a copy (its
// host-side name is not a device address): it uses the address hipGetSymbolAddress
// returns on each device, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kScratchDevices] = {};
  if (device < 0 || device >= kScratchDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!ptr) return (int)hipErrorInvalidSymbol;
    addr[device] = ptr;
  }
  *out = addr[device];
  return 0;
}

int launch_plan_step(const DevRobot* robot, const Request& q, const LaunchConfig& lc,
                     bool f16, void* stream, void* events) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t* ev = static_cast<hipEvent_t*>(events);
  hipError_t e;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return (int)e;
  auto k1 = f16 ? (lc.far_pairs ? rollout_cost_kernel<2, true> : rollout_cost_kernel<2, false>)
                 : (lc.far_pairs ? rollout_cost_kernel<4, true> : rollout_cost_kernel<4, false>);
  hipLaunchKernelGGL(k1, dim3(lc.P + (q.c0_in_ws ? 1 : 0)), dim3(lc.k1_threads), lc.k1_lds, s,
                     robot, q);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return (int)e;
  auto k2 = f16 ? merge_kernel<2> : merge_kernel<4>;
  hipLaunchKernelGGL(k2, dim3(lc.k2_blocks), dim3(kK2Threads), 0, s, robot, q);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return (int)e;
  return 0;
}

namespace {
struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t up = nullptr, k1 = nullptr, k2 = nullptr, down = nullptr;
  bool f16 = false, far = false;
};

hipKernelNodeParams kernel_node(void* func, int blocks, int threads, size_t lds, void** args) {
  hipKernelNodeParams p;
  std::memset(&p, 0, sizeof p);
  p.func = func;
  p.gridDim = dim3((unsigned)blocks);
  p.blockDim = dim3((unsigned)threads);
  p.sharedMemBytes = (unsigned)lds;
  p.kernelParams = args;
  p.extra = nullptr;
  return p;
}
}  // namespace

void destroy_batch_graph(void* handle) {
  BatchGraph* g = static_cast<BatchGraph*>(handle);
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

int launch_batch_graph(void** handle, const DevRobot* robot, void* d_up, const void* h_up,
                       size_t up_bytes, const Request* reqs, const int32_t* k1_map,
                       int k1_blocks, const int32_t* k2_map, int k2_blocks, size_t k1_lds,
                       bool f16, bool far, void* h_res, const void* d_res, size_t res_bytes,
                       void* stream) {
  void* f1 = f16 ? (far ? reinterpret_cast<void*>(rollout_cost_batch_kernel<2, true>)
                       : reinterpret_cast<void*>(rollout_cost_batch_kernel<2, false>))
                 : (far ? reinterpret_cast<void*>(rollout_cost_batch_kernel<4, true>)
                       : reinterpret_cast<void*>(rollout_cost_batch_kernel<4, false>));
  void* f2 = f16 ? reinterpret_cast<void*>(merge_batch_kernel<2>)
                 : reinterpret_cast<void*>(merge_batch_kernel<4>);
  const DevRobot* rob = robot;
  const Request* rq = reqs;
  const int32_t* m1 = k1_map;
  const int32_t* m2 = k2_map;
  void* a1[] = {&rob, &rq, &m1};
  void* a2[] = {&rob, &rq, &m2};
  const hipKernelNodeParams p1 = kernel_node(f1, k1_blocks, kK1Threads, k1_lds, a1);
  const hipKernelNodeParams p2 = kernel_node(f2, k2_blocks, kK2Threads, 0, a2);
  BatchGraph* g = static_cast<BatchGraph*>(*handle);
  hipError_t e;
  if (g && g->far != far) {  // a robot of the other pair kind: the kernel node changes
    destroy_batch_graph(g);
    *handle = nullptr;
    g = nullptr;
  }
  if (!g) {
    g = new (std::nothrow) BatchGraph();
    if (!g) return (int)hipErrorOutOfMemory;
    g->f16 = f16;
    g->far = far;
    if ((e = hipGraphCreate(&g->graph, 0)) != hipSuccess ||
        (e = hipGraphAddMemcpyNode1D(&g->up, g->graph, nullptr, 0, d_up, h_up, up_bytes,
                                     hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipGraphAddKernelNode(&g->k1, g->graph, &g->up, 1, &p1)) != hipSuccess ||
        (e = hipGraphAddKernelNode(&g->k2, g->graph, &g->k1, 1, &p2)) != hipSuccess ||
        (e = hipGraphAddMemcpyNode1D(&g->down, g->graph, &g->k2, 1, h_res, d_res, res_bytes,
                                     hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
      destroy_batch_graph(g);
      return (int)e;
    }
    *handle = g;
  } else {
    if (g->f16 != f16) return (int)hipErrorInvalidValue;
    if ((e = hipGraphExecMemcpyNodeSetParams1D(g->exec, g->up, d_up, h_up, up_bytes,
                                               hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipGraphExecKernelNodeSetParams(g->exec, g->k1, &p1)) != hipSuccess ||
        (e = hipGraphExecKernelNodeSetParams(g->exec, g->k2, &p2)) != hipSuccess ||
        (e = hipGraphExecMemcpyNodeSetParams1D(g->exec, g->down, h_res, d_res, res_bytes,
                                               hipMemcpyDeviceToHost)) != hipSuccess)
      return (int)e;
  }
  return (int)hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
}

int launch_sample_noise(uint64_t seed, int K, int H, const float* sigma, float* eps,
                        uint32_t* words, void* stream) {
  SigmaArg sg;
  for (int j = 0; j < kNdof; ++j) sg.v[j] = sigma[j];
  const long long items = (long long)K * H;
  const int blocks = (int)((items + 255) / 256);
  hipLaunchKernelGGL(sample_noise_kernel, dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), (uint32_t)seed, (uint32_t)(seed >> 32), K,
                     H, sg, eps, words);
  return (int)hipGetLastError();
}

int launch_ogm(const DevRobot* robot, const OgmArgs& a, const float* depth, float* log_odds,
               uint8_t* occ, float* work, hipStream_t stream) {
  const long long npix = (long long)a.width * a.height;
  const long long nvox = (long long)a.nx * a.ny * a.nz;
  hipLaunchKernelGGL(ogm_pixel_kernel, dim3((unsigned)((npix + kOgmTile - 1) / kOgmTile)),
                     dim3(kOgmThreads), 0, stream, robot, a, depth, work);
  const bool grouped = a.nx % 4 == 0 && ((uintptr_t)log_odds & 15u) == 0 &&
                       ((uintptr_t)occ & 3u) == 0;
  if (grouped) {
    const long long ngroups = nvox / 4;
    hipLaunchKernelGGL(ogm_voxel4_kernel,
                       dim3((unsigned)((ngroups + kOgmGroupTile - 1) / kOgmGroupTile)),
                       dim3(kOgmThreads), 0, stream, a, work, log_odds, occ);
  } else {
    hipLaunchKernelGGL(ogm_voxel_kernel, dim3((unsigned)((nvox + kOgmTile - 1) / kOgmTile)),
                       dim3(kOgmThreads), 0, stream, a, work, log_odds, occ);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The wide-path job for a grid, or false when its rows are not a multiple of 16 bytes
// in a 16-byte-aligned grid.
static bool wide_coarse_job(const void* grid, bool f16, int nx, int ny, int nz,
                            const CoarseBall& ball, float* out, CoarseJob& job) {
  const int elem = f16 ? 2 : 4;
  if (((long long)nx * elem) % 16 != 0 || reinterpret_cast<uintptr_t>(grid) % 16 != 0)
    return false;
  job.grid = static_cast<const unsigned char*>(grid);
  job.nx = nx;
  job.ny = ny;
  job.nz = nz;
  job.ncx = coarse_cells_1d(nx);
  job.ncy = coarse_cells_1d(ny);
  job.ncz = coarse_cells_1d(nz);
  const int cells_per_chunk = (kCoarseChunkGroups - 1) * (16 / elem) / kCoarseCell;
  job.nchunks = (job.ncx + cells_per_chunk - 1) / cells_per_chunk;
  job.nwork = (int)((long long)job.nchunks * job.ncy * job.ncz);
  job.ball = ball;
  job.out = out;
  return true;
}

int launch_grid_coarse_min(const void* grid, bool f16, int nx, int ny, int nz,
                           const float* ball_c, float ball_r2, float* out, void* stream) {
  const int ncx = coarse_cells_1d(nx), ncy = coarse_cells_1d(ny), ncz = coarse_cells_1d(nz);
  const long long ncells = (long long)ncx * ncy * ncz;
  const int elem = f16 ? 2 : 4;
  (void)ncells;
  CoarseBall ball;
  for (int a = 0; a < 3; ++a) ball.c[a] = ball_c ? ball_c[a] : 0.f;
  ball.r2 = ball_c ? ball_r2 : __builtin_inff();
  CoarseJob job;
  if (wide_coarse_job(grid, f16, nx, ny, nz, ball, out, job)) {
    const long long blocks = (job.nwork + kXcds - 1) / kXcds * kXcds;
    auto k = f16 ? grid_coarse_min_wide_kernel<2> : grid_coarse_min_wide_kernel<4>;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kCoarseWideThreads), 0,
                       (hipStream_t)stream, job);
  } else {
    const uint32_t bytes = (uint32_t)((long long)nx * ny * nz * elem);
    auto k = f16 ? grid_coarse_min_kernel<2> : grid_coarse_min_kernel<4>;
    hipLaunchKernelGGL(k, dim3((unsigned)((long long)ncy * ncz)), dim3(kCoarseThreads), 0,
                       (hipStream_t)stream, grid, bytes, nx, ny, nz, ncx, ncy, ncz, ball, out);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_plan_step_bounds(const DevRobot* robot, const Request& q, const LaunchConfig& lc,
                            bool f16, const void* grid, bool grid_f16, int nx, int ny, int nz,
                            const float* ball_c, float ball_r2, float* out, void* stream,
                            void* events) {
  CoarseBall ball;
  for (int a = 0; a < 3; ++a) ball.c[a] = ball_c[a];
  ball.r2 = ball_r2;
  CoarseJob job;
  if (grid_f16 != f16 || !wide_coarse_job(grid, grid_f16, nx, ny, nz, ball, out, job)) {
    // Not fusable: the plan step, then the bounds by their own launch (same results).
    const int e = launch_plan_step(robot, q, lc, f16, stream, events);
    if (e != 0) return e;
    return launch_grid_coarse_min(grid, grid_f16, nx, ny, nz, ball_c, ball_r2, out, stream);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t* ev = static_cast<hipEvent_t*>(events);
  hipError_t e;
  const int n_bounds = (job.nwork + kXcds - 1) / kXcds * kXcds;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return (int)e;
  if (out != q.coarse) {
    // Another table than the one the rollouts read: the bounds blocks join the rollout
    // launch, whose blocks leave HBM mostly idle (1.5 us added to it at 200^3, against
    // 3.6 us added to the merge launch).
    const int n_k1 = lc.P + (q.c0_in_ws ? 1 : 0), n_k1p = (n_k1 + kXcds - 1) / kXcds * kXcds;
    auto k1 = f16 ? (lc.far_pairs ? rollout_bounds_kernel<2, true> : rollout_bounds_kernel<2, false>)
                   : (lc.far_pairs ? rollout_bounds_kernel<4, true> : rollout_bounds_kernel<4, false>);
    hipLaunchKernelGGL(k1, dim3((unsigned)(n_k1p + n_bounds)), dim3(lc.k1_threads), lc.k1_lds, s,
                       robot, q, n_k1, n_k1p, job);
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return (int)e;
    auto k2 = f16 ? merge_kernel<2> : merge_kernel<4>;
    hipLaunchKernelGGL(k2, dim3(lc.k2_blocks), dim3(kK2Threads), 0, s, robot, q);
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return (int)e;
    return 0;
  }
  auto k1 = f16 ? (lc.far_pairs ? rollout_cost_kernel<2, true> : rollout_cost_kernel<2, false>)
                 : (lc.far_pairs ? rollout_cost_kernel<4, true> : rollout_cost_kernel<4, false>);
  hipLaunchKernelGGL(k1, dim3(lc.P + (q.c0_in_ws ? 1 : 0)), dim3(lc.k1_threads), lc.k1_lds, s,
                     robot, q);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return (int)e;
  const int n_k2 = lc.k2_blocks, n_k2p = (n_k2 + kXcds - 1) / kXcds * kXcds;
  auto k2 = f16 ? merge_bounds_kernel<2> : merge_bounds_kernel<4>;
  hipLaunchKernelGGL(k2, dim3((unsigned)(n_k2p + n_bounds)), dim3(kK2Threads), 0, s, robot, q,
                     n_k2, n_k2p, job);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return (int)e;
  return 0;
}

int launch_grid_to_f16(const float* src, void* dst, long long n, float clamp, void* stream) {
  const long long want = (n + 255) / 256;
  const int blocks = (int)(want < 65536 ? (want > 0 ? want : 1) : 65536);
  hipLaunchKernelGGL(grid_to_f16_kernel, dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), src, static_cast<unsigned short*>(dst), n,
                     clamp);
  return (int)hipGetLastError();
}

}  // namespace smpc
