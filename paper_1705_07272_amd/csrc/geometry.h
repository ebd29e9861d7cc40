// Exact integer geometry of the cube-map rotation g(w) = f(R w)
// (Sec. V.A: each point p of the rotated map takes the value of the original
// at R p).  Device-side helpers shared by the relight and phase-shift
// kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rrt {

constexpr int kScaleBits = 20;  // R_q = rint(R * 2^20)

// Quantised rotation, row-major int32.
struct IRot {
  int m[9];
};

__device__ __forceinline__ int quantise_entry(float r) {
  return int(rintf(r * float(1 << kScaleBits)));
}

// R_fv = (R_q(frame) R_q(vertex) + 2^19) >> 20 (flooring shift), or R_q(vertex).
__device__ __forceinline__ IRot frame_vertex_rotation(const float* __restrict__ vrot,
                                                      const float* __restrict__ frot) {
  IRot v, out;
#pragma unroll
  for (int k = 0; k < 9; ++k) v.m[k] = quantise_entry(vrot[k]);
  if (frot == nullptr) return v;
  int f[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = quantise_entry(frot[k]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      int64_t acc = int64_t(1) << (kScaleBits - 1);
#pragma unroll
      for (int m = 0; m < 3; ++m) acc += int64_t(f[3 * i + m]) * int64_t(v.m[3 * m + j]);
      out.m[3 * i + j] = int(acc >> kScaleBits);
    }
  return out;
}

// Face axes: texel direction = U * eU + V * eV + n * eN with
// faces +X,-X,+Y,-Y,+Z,-Z:
//   +X ( n,-V,-U)  -X (-n,-V, U)  +Y ( U, n, V)
//   -Y ( U,-n,-V)  +Z ( U,-V, n)  -Z (-U,-V,-n).
// Each axis is a signed unit vector: encoded as axis index and sign.
struct FaceAxes {
  int3 mU, mV, mN;  // R * eU, R * eV, R * eN
};

__device__ __forceinline__ int pick3(int a, int b, int c, int axis) {
  return axis == 0 ? a : (axis == 1 ? b : c);
}

// sign * (column `axis` of R), without dynamic register indexing.
__device__ __forceinline__ int3 signed_column(const IRot& R, int axis, int sign) {
  return make_int3(sign * pick3(R.m[0], R.m[1], R.m[2], axis),
                   sign * pick3(R.m[3], R.m[4], R.m[5], axis),
                   sign * pick3(R.m[6], R.m[7], R.m[8], axis));
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

// Modular int32 arithmetic: the true direction components fit in int32 for
// n <= 1024 (|R_q| <= 2^20, |dir| <= n sqrt(3)), so wrapped partial sums still
// give the exact final value.
__device__ __forceinline__ int wrap_mad(int a, int b, int c) {
  return int(unsigned(a) * unsigned(b) + unsigned(c));
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
// towards z then y), returned scaled by 2^ES (a byte offset for elements of
// 2^ES bytes).
//
// The components are converted to binary32 (relative error 2^-24 each; sc
// and D are copies of them, |ma| = 2 D exactly) and q = h sc / D + h + eps
// is estimated as fma(sc, n rcp(|ma|), h + eps): sc / D is off by at most
// 2^-23 relative, v_rcp_f32 by one ulp (2^-23), so the product is within
// h 2^-22 of h sc / D, and the fma rounds once (at most h 2^-23): the error
// is below 1.5 h 2^-22 < eps = h 2^-20 (quotient_margin).  If frac(q) >= 2 eps
// for both coordinates, the exact quotient lies strictly between the same
// two integers as q - eps, so trunc(q) is the exact floor (and lies in
// [0, n - 1]); otherwise the exact form replaces the result.
//
// A face chosen by the binary32 comparison that differs from the exact one
// (a near tie |d_a| ~ |d_b| or an exact tie broken the other way) is always
// caught: the exact major component then appears as an in-face coordinate
// with |a_f| / |b_f| in [1 - 2^-23, 1], so that coordinate's q - eps is
// within h 2^-23 + 1.5 h 2^-22 = h 2^-21 < eps of 0 or 2h and fails the
// margin test.  A zero direction gives NaN and also takes the exact form.
// Every output is in [0, 6 n^2) << ES.
template <int ES>
__device__ __forceinline__ unsigned source_texel_scaled(int x, int y, int z, int logn, float eps) {
  const float fx = float(x), fy = float(y), fz = float(z);
  const float ma = __builtin_amdgcn_cubema(fx, fy, fz);
  const float hr = float(1 << logn) * __builtin_amdgcn_rcpf(fabsf(ma));
  const float off = float(1 << (logn - 1)) + eps;
  const float qs = __builtin_fmaf(__builtin_amdgcn_cubesc(fx, fy, fz), hr, off);
  const float qt = __builtin_fmaf(__builtin_amdgcn_cubetc(fx, fy, fz), hr, off);
  // q > 0, so truncation is the floor; the flat index (face n + i) n + j is
  // below 6 * 2^20 < 2^24 and so exact in binary32 arithmetic
  const float js = __builtin_truncf(qs), it = __builtin_truncf(qt);
  const float es = qs - js, et = qt - it;
  const float nf = float(1 << logn);
  const float flat = __builtin_fmaf(__builtin_amdgcn_cubeid(fx, fy, fz), nf * nf,
                                    __builtin_fmaf(it, nf, js));
  unsigned at = unsigned(flat) << ES;
  if (!(fminf(es, et) >= 2.0f * eps)) at = unsigned(source_texel_exact(x, y, z, logn)) << ES;
  return at;
}

__device__ __forceinline__ int source_texel(int x, int y, int z, int logn, float eps) {
  return int(source_texel_scaled<0>(x, y, z, logn, eps));
}

// Margin of the binary32 quotient estimate (see source_texel).
__device__ __forceinline__ float quotient_margin(int logn) {
  return float(1 << (logn - 1)) * 0x1p-20f;
}

}  // namespace rrt
