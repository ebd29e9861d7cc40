// Exact integer geometry of the cube-map rotation g(w) = f(R w)
// (Sec. V.A: each point p of the rotated map takes the value of the original
// at R p).  Device-side helpers shared by the relight and phase-shift
// kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rrt {

// Rotations of an n x n map are quantised to R_q = rint(R 2^k), k = 22 -
// log2(n).  A texel direction R_q (U eU + V eV + n eN) with |U|, |V| < n, and
// every partial sum of its terms, is then an integer of magnitude below
// 3 n 2^k = 3 2^22 < 2^24: exact in binary32, so directions are formed with
// binary32 adds and fmas and fed to the cube-map instructions unrounded.
__device__ __forceinline__ int scale_bits(int logn) { return 22 - logn; }

// Quantised rotation, row-major int32.
struct IRot {
  int m[9];
};

__device__ __forceinline__ int quantise_entry(float r, int k) {
  return int(rintf(ldexpf(r, k)));
}

// R_fv = (R_q(frame) R_q(vertex) + 2^(k-1)) >> k (flooring shift), or R_q(vertex).
__device__ __forceinline__ IRot frame_vertex_rotation(const float* __restrict__ vrot,
                                                      const float* __restrict__ frot, int k) {
  IRot v, out;
#pragma unroll
  for (int e = 0; e < 9; ++e) v.m[e] = quantise_entry(vrot[e], k);
  if (frot == nullptr) return v;
  int f[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) f[e] = quantise_entry(frot[e], k);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      int64_t acc = int64_t(1) << (k - 1);
#pragma unroll
      for (int m = 0; m < 3; ++m) acc += int64_t(f[3 * i + m]) * int64_t(v.m[3 * m + j]);
      out.m[3 * i + j] = int(acc >> k);
    }
  return out;
}

// Face axes: texel direction = U * eU + V * eV + n * eN with
// faces +X,-X,+Y,-Y,+Z,-Z:
//   +X ( n,-V,-U)  -X (-n,-V, U)  +Y ( U, n, V)
//   -Y ( U,-n,-V)  +Z ( U,-V, n)  -Z (-U,-V,-n).
// Each axis is a signed unit vector: encoded as axis index and sign.  The
// rotated axes hold the integer entries of R_q (|entry| <= 2^k), exactly.
struct FaceAxes {
  float3 mU, mV, mN;  // R * eU, R * eV, R * eN
};

__device__ __forceinline__ int pick3(int a, int b, int c, int axis) {
  return axis == 0 ? a : (axis == 1 ? b : c);
}

// sign * (column `axis` of R), without dynamic register indexing.
__device__ __forceinline__ float3 signed_column(const IRot& R, int axis, int sign) {
  return make_float3(float(sign * pick3(R.m[0], R.m[1], R.m[2], axis)),
                     float(sign * pick3(R.m[3], R.m[4], R.m[5], axis)),
                     float(sign * pick3(R.m[6], R.m[7], R.m[8], axis)));
}

__device__ __forceinline__ FaceAxes face_axes(const IRot& R, int face) {
  // (axis, sign) of eU, eV, eN per face
  const int uax = (face < 2) ? 2 : 0;
  const int usg = (face == 0 || face == 5) ? -1 : 1;
  const int vax = (face == 2 || face == 3) ? 2 : 1;
  const int vsg = (face == 2) ? 1 : -1;
  const int nax = face >> 1;
  const int nsg = (face & 1) ? -1 : 1;
  FaceAxes a;
  a.mU = signed_column(R, uax, usg);
  a.mV = signed_column(R, vax, vsg);
  a.mN = signed_column(R, nax, nsg);
  return a;
}

// Direction a U + b V + c (three components), exact for the integer
// operands described at scale_bits.
__device__ __forceinline__ float3 dir_mad(float3 u, float a, float3 v, float b, float3 c) {
  return make_float3(__builtin_fmaf(u.x, a, __builtin_fmaf(v.x, b, c.x)),
                     __builtin_fmaf(u.y, a, __builtin_fmaf(v.y, b, c.y)),
                     __builtin_fmaf(u.z, a, __builtin_fmaf(v.z, b, c.z)));
}
__device__ __forceinline__ float3 dir_add(float3 u, float a, float3 c) {
  return make_float3(__builtin_fmaf(u.x, a, c.x), __builtin_fmaf(u.y, a, c.y),
                     __builtin_fmaf(u.z, a, c.z));
}

// floor(s * 2^logh / D) exactly, given q0 within one of it (|s| <= D, D >= 1):
// one int64 comparison on each side.
__device__ __forceinline__ int exact_floor(int s, int D, int logh, int q0) {
  const int64_t num = int64_t(s) * (int64_t(1) << logh);
  const int64_t lo = int64_t(q0) * int64_t(D);
  q0 -= int(lo > num);
  q0 += int(lo + D <= num);
  return q0;
}

// Flat source texel (face * n^2 + i * n + j) of the integer direction d.
// Major axis a = argmax |d_k| with ties to the lower axis, face 2a + [d_a < 0],
// in-face coordinates
//   +X (-z,-y)  -X (z,-y)  +Y (x, z)  -Y (x,-z)  +Z (x,-y)  -Z (-x,-y),
// column j = min(n-1, floor(h (sc + D) / D)), h = n / 2, D = |d_a|; row i
// likewise from tc.
//
// Exact form: integer face selection, a binary32 estimate of h sc / D + h
// (float(sc) and float(D) round once each (2^-24), v_rcp_f32 is within one
// ulp (2^-23), the fma rounds once (at most 2h 2^-24): within h 2^-21 of the
// exact value, so its floor is off by at most one) and an int64 test on each
// side of the estimate.  Every output is in [0, 6 n^2).
__device__ __forceinline__ int source_texel_exact(int x, int y, int z, int logn) {
  const int n = 1 << logn;
  const int logh = logn - 1;
  const int h = 1 << logh;
  const int nx = -x, ny = -y, nz = -z;
  const int ax = max(x, nx), ay = max(y, ny), az = max(z, nz);
  const bool px = ax >= max(ay, az);
  const bool py = !px && (ay >= az);
  const int D = max(max(max(ax, ay), az), 1);
  const int da = px ? x : (py ? y : z);
  const bool neg = da < 0;
  const int face = (px ? 0 : (py ? 2 : 4)) + int(neg);
  const int t1 = neg ? z : nz;
  const int t2 = neg ? nx : x;
  const int sc = px ? t1 : (py ? x : t2);
  const int tc = py ? (neg ? nz : z) : ny;
  const float hf = float(h);
  const float hr = hf * __builtin_amdgcn_rcpf(float(D));
  const int j0 = int(floorf(__builtin_fmaf(float(sc), hr, hf)));
  const int i0 = int(floorf(__builtin_fmaf(float(tc), hr, hf)));
  const int j = min(h + exact_floor(sc, D, logh, j0 - h), n - 1);
  const int i = min(h + exact_floor(tc, D, logh, i0 - h), n - 1);
  return (face << (2 * logn)) + (i << logn) + j;
}

// The same map, with a binary32 fast path on the cube-map instructions
// (v_cubeid / v_cubesc / v_cubetc / v_cubema: face, in-face coordinates and
// twice the major component, in the face convention above, ties resolved
// towards z then y), for a direction given as exact binary32 integers.
//
// The fast path works on x = q / n + 1 + e, q = h sc / D + h the exact texel
// coordinate and e = 2^-22, so that x lies in (1, 2) and the bits of its
// significand are q's: the top log2(n) bits are floor(q + n e), the rest its
// fraction.  sc and |ma| = 2 D are exact, v_rcp_f32 is within one ulp
// (2^-23 relative), so sc / |ma| (at most 1/2) is within 2^-24 of the exact
// ratio, and the fma that adds 3/2 + e rounds once (at most 2^-24): x is
// within 2^-23 = e / 2 of its exact value.  If the fraction bits of both
// coordinates are at least 4 (the fraction of n (x - 1) is at least 2 n e),
// the exact q lies strictly between the same two integers, so the top bits
// are the exact floor (in [0, n - 1]); otherwise the exact form replaces the
// result.  An estimate at or above 2 has fraction bits below 4 (x < 2 + 3/2 e)
// and also takes the exact form.
//
// With exact components the binary32 face comparison can differ from the
// exact one only at an exact tie broken the other way; the exact major
// component is then an in-face coordinate equal to +-D, whose x is within
// e / 2 of 1 + e or 2 + e, where the fraction test fails.  A zero direction
// gives NaN, whose fraction bits are zero for n >= 2: the exact form.
// 127 (n^2 + n): the offset that the significand bits of x add to a flat
// index (see source_texel_biased).
__device__ __forceinline__ unsigned texel_bias(int logn) {
  return (127u << (2 * logn)) + (127u << logn);
}

// Strip layout of a source map (n >= 4): global rows R = face n + i are
// grouped in strips of four, each strip stored column by column, so texel
// (R, j) sits at ((R >> 2) << (log2 n + 2)) + 4 j + (R & 3) and a 4-row x
// 8-column patch (32 binary32 values) shares one 128-byte cache line.  A
// rotated 8 x 8 patch of destination texels then touches about half the
// lines it touches in row-major order.
__device__ __forceinline__ unsigned strip_offset(unsigned R, unsigned j, int logn) {
  return ((R >> 2) << (logn + 2)) + (j << 2) + (R & 3u);
}
// 127 n^2: the offset of the strip index built from significand bits.
__device__ __forceinline__ unsigned strip_bias(int logn) { return 127u << (2 * logn); }

// Fast path of the map (see source_texel_biased for the error analysis):
// significands of x for both in-face coordinates, the face, and whether the
// top bits are exact floors.
struct FastTexel {
  unsigned bs, bt, face;
  bool ok;
};
__device__ __forceinline__ FastTexel fast_texel(float fx, float fy, float fz, int logn) {
  const float r = __builtin_amdgcn_rcpf(fabsf(__builtin_amdgcn_cubema(fx, fy, fz)));
  constexpr float kOff = 1.5f + 0x1p-22f;
  FastTexel t;
  t.bs = __float_as_uint(__builtin_fmaf(__builtin_amdgcn_cubesc(fx, fy, fz), r, kOff));
  t.bt = __float_as_uint(__builtin_fmaf(__builtin_amdgcn_cubetc(fx, fy, fz), r, kOff));
  t.face = unsigned(__builtin_amdgcn_cubeid(fx, fy, fz));
  // fraction bits at least 4 in both: some bit of [2, 23 - log2 n) set in each
  const unsigned fr = ((1u << (23 - logn)) - 1u) & ~3u;
  t.ok = min(t.bs & fr, t.bt & fr) != 0u;
  return t;
}

// Flat source texel plus texel_bias(logn), so that the fast path needs no
// subtraction; in [texel_bias, texel_bias + 6 n^2).
__device__ __forceinline__ unsigned source_texel_biased(float fx, float fy, float fz, int logn) {
  const FastTexel t = fast_texel(fx, fy, fz, logn);
  // for x in (1, 2), the bits above the fraction are 127 n + column (or row)
  const int sh = 23 - logn;
  const unsigned rows = (t.face << logn) + (t.bt >> sh);   // face n + 127 n + i
  unsigned at = (rows << logn) + (t.bs >> sh);             // flat + 127 n^2 + 127 n
  if (!t.ok) at = unsigned(source_texel_exact(int(fx), int(fy), int(fz), logn)) + texel_bias(logn);
  return at;
}

// Strip offset (strip_offset) of the source texel plus strip_bias(logn), for
// n >= 4; in [strip_bias, strip_bias + 6 n^2).
__device__ __forceinline__ unsigned source_texel_strip(float fx, float fy, float fz, int logn) {
  const FastTexel t = fast_texel(fx, fy, fz, logn);
  const int sh = 23 - logn;
  // low part 4 j + (i & 3): column bits from bs, the row's two low bits from
  // bt's top part 127 n + i (127 n is a multiple of 4 for n >= 4)
  const unsigned lo = ((t.bt >> sh) & 3u) | ((t.bs >> (sh - 2)) & ~3u);
  // high part (strip (face + 127) n / 4 + (i >> 2)) << (log2 n + 2): the bits
  // of ((face + 127) n + i) n above log2 n + 2 (bt shifted to that scale
  // carries fraction bits below log2 n, which the mask drops)
  const unsigned R = (t.face << (2 * logn)) + (t.bt >> (sh - logn));
  const unsigned hi = ~((4u << logn) - 1u);
  // (R & hi) | (lo & ~hi) in one v_bfi_b32 (the mask is loop-invariant, so the
  // compiler would otherwise not see its complement and emit two operations)
  unsigned at;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(at) : "s"(hi), "v"(R), "v"(lo));
  if (!t.ok) {
    const unsigned q = unsigned(source_texel_exact(int(fx), int(fy), int(fz), logn));
    at = strip_offset(q >> logn, q & ((1u << logn) - 1u), logn) + strip_bias(logn);
  }
  return at;
}

template <int ES>
__device__ __forceinline__ unsigned source_texel_scaled(float fx, float fy, float fz, int logn) {
  return (source_texel_biased(fx, fy, fz, logn) - texel_bias(logn)) << ES;
}

__device__ __forceinline__ int source_texel(float3 d, int logn) {
  return int(source_texel_scaled<0>(d.x, d.y, d.z, logn));
}

}  // namespace rrt
