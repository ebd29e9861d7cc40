// Relighting: rotate the lighting into each vertex's frame directly in the
// Haar domain and take the sparse inner product with the vertex's transport
// coefficients (Sec. V.A-V.C: rotate the finest level, recurse to the
// coarser levels with 2x2 averaging/downsampling, plug the rotated
// coefficients into the light-transport product; Sec. III: with BRDF,
// cosine and visibility pre-multiplied the product is an inner product).
//
// Exact discrete form of the finest-level rotation: every texel q of the
// local map takes the source value P[pi(q)], pi the exact integer
// nearest-texel map of R_fv q (geometry.h), P = W^T L the pixel-domain
// source map reconstructed once per lighting.  The coarser levels are the
// paper's recursive averaging, done as in-place 2x2 butterflies.
//
// Work decomposition (one wave per vertex, all frames; no workgroup barrier):
//   * the faces touched by the vertex's transport row are processed, each as
//     G x G blocks of Q x Q texels (Q = min(n, 32));
//   * per block, lane (ty, tx) gathers texel (8a + ty, 8b + tx) of each 8 x 8
//     patch (a compact patch per load instruction) into an LDS image, then
//     runs the levels of its own 4 x 4 tile in registers and the levels up to
//     the block with lane shuffles, in place (the coefficient of a block of
//     side B at its corner offset by B/2 for H/V/D);
//   * the transport entries are decoded once per vertex into an LDS list; the
//     entries inside the block read the image, the coarser ones read the FP64
//     block-sum grid after the levels above the blocks; products are
//     accumulated per lane and reduced with lane shuffles;
//   * a block that holds no listed entry only contributes its sum to the
//     levels above it and skips the image, the levels and the entry scan.
//
// Variants of the same kernel: the chain rule for the finest level
// (Sec. V.A-V.B, eq:pde1-eq:pde3), the triple product with a BRDF factor per
// material (Sec. III, eq:tripleSum), and the longitude-latitude map with its
// elevation rotation and exact azimuth shifts (Sec. V.A).
#include <hip/hip_fp16.h>

#include "geometry.h"
#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr int kThreads = 64;  // one wave per vertex
// Block side: a 32 x 32 block is 8 x 8 tiles of 4 x 4 texels, one tile per
// lane, so every Haar level up to the block stays inside the wave.
constexpr int kBlock = 32;
// Transport entries of a vertex listed in LDS; entries past this count are
// decoded from global memory in every block.
constexpr int kMaxListed = 512;
// Chunks of 64 transport entries whose loads the listing issues together.
constexpr int kListChunks = 4;
// LDS for the FP64 block sums of the faces processed together.
constexpr int kGroupBytes = 4096;
// LDS bit mask of the blocks of a face group that hold listed entries (at
// most 1,024 blocks: kGroupBytes / 8, or one face of 32 x 32 blocks)
constexpr int kBlockMaskBytes = 128;

// Gathers from the source map go through a structured buffer resource whose
// stride is the element size: the element index is the whole per-texel
// address computation (no 64-bit arithmetic, no byte scaling), and the
// hardware checks the index against the element count (reads past the map
// return 0).  The structured loads are the LLVM intrinsics themselves.
constexpr int kBufferWord3 = 0x00020000;  // gfx9 buffer: 32-bit data format
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
extern "C" __device__ float rrt_struct_load_f32(__amdgpu_buffer_rsrc_t rsrc, int index, int voffset,
                                                int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.f32");

// Resource over `count` elements at p, addressed with indices offset by
// `bias` (element i of the map is index bias + i; the cube-map gather hands
// texel_bias-offset indices straight to the load, which by construction are
// never below the bias).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t source_resource(const float* p, int count,
                                                                  unsigned bias) {
  const uintptr_t base = reinterpret_cast<uintptr_t>(p) - uintptr_t(bias) * sizeof(float);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(base), short(sizeof(float)),
                                           count + int(bias), kBufferWord3);
}

// Element `at` of the source map.
__device__ __forceinline__ float load_src(__amdgpu_buffer_rsrc_t r, unsigned at) {
  return rrt_struct_load_f32(r, int(at), 0, 0, 0);
}

// Code e of a packed 11-bit row (RRT_S11): bits [11 e, 11 e + 11) of the
// row's word stream, sign-extended.  The second word is read only when the
// code reaches into it, which stays inside the row's RRT_S11_WORDS(nnz).
__device__ __forceinline__ int s11_code(const uint32_t* row, int e) {
  const int b = 11 * e;
  const int wi = b >> 5, sh = b & 31;
  const uint32_t lo = row[wi];
  const uint32_t hi = sh > 21 ? row[wi + 1] : 0u;
  const uint32_t bits = uint32_t(((uint64_t(hi) << 32) | lo) >> sh);
  return int(bits << 21) >> 21;
}

__device__ __forceinline__ float transport_value(const void* val, const float* scale, int dtype,
                                                 int64_t row, int nnz, int e) {
  const int64_t at = row * nnz + e;
  if (dtype == RRT_F32) return static_cast<const float*>(val)[at];
  if (dtype == RRT_BF16)
    return __uint_as_float(unsigned(static_cast<const uint16_t*>(val)[at]) << 16);
  const int nblk = (nnz + RRT_BLOCK - 1) / RRT_BLOCK;
  const float sc = scale[row * nblk + e / RRT_BLOCK];
  if (dtype == RRT_S16) return float(static_cast<const int16_t*>(val)[at]) * sc;
  if (dtype == RRT_S11)
    return float(s11_code(static_cast<const uint32_t*>(val) + row * RRT_S11_WORDS(nnz), e)) * sc;
  // gfx950's FP8 conversion reads the OCP E4M3FN encoding (bias 7,
  // subnormals, 0x7f / 0xff NaN) exactly
  return __builtin_amdgcn_cvt_f32_fp8(int(static_cast<const uint8_t*>(val)[at]), 0) * sc;
}

// Position of a transport entry in the in-place layout of its face.
struct Slot {
  int face;   // -1: invalid index
  int pr, pc; // in-place row / column inside the face
  int logb;   // log2 of the block side of the basis function
};

// nf: faces (squares) of the map, 6 for a cube map, 2 for a lat-long map.
__device__ __forceinline__ Slot decode_slot(int idx, int logn, int nf) {
  Slot s;
  const int n = 1 << logn;
  const int per_face = n << logn;
  if (idx < 0 || idx >= nf * per_face) {
    s.face = -1;
    s.pr = s.pc = s.logb = 0;
    return s;
  }
  s.face = idx >> (2 * logn);
  const int pos = idx & (per_face - 1);
  const int r = pos >> logn, c = pos & (n - 1);
  const int m = r | c;  // same highest bit as max(r, c)
  if (m == 0) {
    s.pr = s.pc = 0;
    s.logb = logn;
    return s;
  }
  const int qb = 31 - __clz(m);
  const int q = 1 << qb;
  s.logb = logn - qb;
  const int half = 1 << (s.logb - 1);
  s.pr = ((r & (q - 1)) << s.logb) + ((r >= q) ? half : 0);
  s.pc = ((c & (q - 1)) << s.logb) + ((c >= q) ? half : 0);
  return s;
}

struct Acc {
  float s, c;
};

// Error-free product and Neumaier sum (contraction would defeat both).
#pragma clang fp contract(off)
__device__ __forceinline__ void acc_add(Acc& a, float x, float y, bool comp) {
  if (!comp) {
    a.s = __builtin_fmaf(x, y, a.s);
    return;
  }
  const float p = x * y;
  const float pe = __builtin_fmaf(x, y, -p);
  const float t = a.s + p;
  const float e = (fabsf(a.s) >= fabsf(p)) ? ((a.s - t) + p) : ((p - t) + a.s);
  a.s = t;
  a.c += e + pe;
}

__device__ __forceinline__ Acc acc_merge(Acc a, Acc b) {
  const float t = a.s + b.s;
  const float bb = t - a.s;
  const float e = (a.s - (t - bb)) + (b.s - bb);
  Acc r;
  r.s = t;
  r.c = (a.c + b.c) + e;
  return r;
}
#pragma clang fp contract(fast)

__device__ __forceinline__ void tile_levels_d(double a, double b, double c, double d, double& S,
                                              double& H, double& V, double& D) {
  S = 0.5 * ((a + b) + (c + d));
  H = 0.5 * ((a - b) + (c - d));
  V = 0.5 * ((a + b) - (c + d));
  D = 0.5 * ((a - b) - (c - d));
}

struct RelightParams {
  const float* src;       // source map (binary32)
  const float* vrot;
  const float* frot;
  const int32_t* tidx;
  const void* tval;
  const float* tscale;
  const int32_t* cluster;
  int nclusters;
  float* out;
  int64_t out_stride;  // frame stride of out (>= nvert)
  int64_t nvert;
  int nnz;
  int nframes;
  int logn;
  int dtype;
  int comp;
  int listed;       // entries of each row listed in LDS: min(nnz, kMaxListed)
  int group_faces;  // faces whose block sums fit in LDS together
  const float4* blocks;  // chain rule: (S, H, V, D) of every 2x2 source block
  const float* brdf;        // triple product: [nmat][6 n^2] texel factor, or NULL
  const int32_t* material;  // [V] row of brdf, or NULL (row 0)
  int nmat;
  const float* ll_elev;     // lat-long: [V][2] (cos b, sin b)
  const int32_t* ll_shift;  // lat-long: [V][2] (s_a, s_c)
  const int32_t* order;     // [V] processing order, or NULL
  const float* ll_grid;     // lat-long: the rule's binary32 tables (7 H floats)
  int ll_tab_off;           // lat-long: byte offset of the tables in LDS
};

// Correctly rounded binary32 square root of x, for x >= 2^-96 (the lat-long
// rule takes it of q_x^2 + q_z^2 >= (sin t sin f)^2 >= sin^4(pi / 2H), far
// above that for every supported H).  The hardware
// square root is within one ulp, so the rounded result is s or one of its two
// neighbours s-, s+; the nearest is decided by the signs of the residuals
// x - s- s and x - s+ s, each exact up to its one rounding in the fma.  A
// midpoint between two floats squared lies at least a quarter of a square
// ulp away from every product of adjacent floats, and x, a float of twice
// the exponent, is a multiple of that grid, so a residual <= 0 (> 0) puts
// the root below (above) the midpoint.
__device__ __forceinline__ float sqrt_rn(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float lo = __int_as_float(__float_as_int(s) - 1);
  const float hi = __int_as_float(__float_as_int(s) + 1);
  float r = s;
  r = __builtin_fmaf(-lo, s, x) <= 0.0f ? lo : r;
  r = __builtin_fmaf(-hi, s, x) > 0.0f ? hi : r;
  return r;
}

// Source texel of destination texel (row i, column jc + ...) of a
// longitude-latitude map with H = 2^logh rows and W = 2H columns, for the
// elevation rotation R_x(b) = (cb, sb) followed by the azimuth shift sa
// (Sec. V.A: p = (sin t sin f, cos t, sin t cos f), g(p) = f(R p)).  jc is the
// destination column already shifted by s_c.  Every operation is one
// binary32 operation in this order (no contraction), so the decision is
// reproducible: q = R_x p, rho = |q_xz| (correctly rounded),
// row = #{k < H : q_y <= C_k}, c = #{k < H : q_z <= C_k rho} (C_k =
// cos(k pi / H), decreasing, so both counts are binary searches), column = c
// for q_x >= 0, else W - 1 - c.
// Returns the flat index over the two H x H squares.
struct LLTab {
  const float* rs;   // [H] sin of row centres
  const float* rc;   // [H] cos of row centres
  const float* cs;   // [2H] sin of column centres
  const float* cc;   // [2H] cos of column centres
  const float* bnd;  // [H] cos(k pi / H)
};

__device__ __forceinline__ unsigned latlong_source(const LLTab& t, int i, int jc, float cb,
                                                   float sb, int logh, int sa) {
#pragma clang fp contract(off)
  const int H = 1 << logh;
  const float px = t.rs[i] * t.cs[jc];
  const float py = t.rc[i];
  const float pz = t.rs[i] * t.cc[jc];
  const float qy = cb * py - sb * pz;
  const float qz = sb * py + cb * pz;
  const float rho = sqrt_rn(px * px + qz * qz);
  int row = 0, c = 0;
  for (int step = H >> 1; step >= 1; step >>= 1) {
    row += (qy <= t.bnd[row + step]) ? step : 0;
    c += (qz <= t.bnd[c + step] * rho) ? step : 0;
  }
  int col = px >= 0.0f ? c : 2 * H - 1 - c;
  col = (col + sa) & (2 * H - 1);
  return (unsigned(col >> logh) << (2 * logh)) + (unsigned(row) << logh) + unsigned(col & (H - 1));
}

// The same rule for a compile-time H = 2^LOGH: the two searches unroll, the
// table offsets become immediates and the searches of a lane's texels can
// be interleaved.
template <int LOGH>
__device__ __forceinline__ unsigned latlong_source_h(const LLTab& t, int i, int jc, float cb,
                                                     float sb, int sa) {
#pragma clang fp contract(off)
  constexpr int H = 1 << LOGH;
  const float px = t.rs[i] * t.cs[jc];
  const float py = t.rc[i];
  const float pz = t.rs[i] * t.cc[jc];
  const float qy = cb * py - sb * pz;
  const float qz = sb * py + cb * pz;
  const float rho = sqrt_rn(px * px + qz * qz);
  int row = 0, c = 0;
#pragma unroll
  for (int step = H >> 1; step >= 1; step >>= 1) {
    row += (qy <= t.bnd[row + step]) ? step : 0;
    c += (qz <= t.bnd[c + step] * rho) ? step : 0;
  }
  int col = px >= 0.0f ? c : 2 * H - 1 - c;
  col = (col + sa) & (2 * H - 1);
  return (unsigned(col >> LOGH) << (2 * LOGH)) + (unsigned(row) << LOGH) + unsigned(col & (H - 1));
}

// A lane's T x T gathered texels of block (by, bx) of square `face` through
// the longitude-latitude rule at H = 2^LOGH.
template <int LOGH, int Q, int TS, int T>
__device__ __forceinline__ void latlong_gather(float (&val)[T][T], const LLTab& tab,
                                               __amdgpu_buffer_rsrc_t src, int face, int by,
                                               int bx, int ty, int tx, float cb, float sb, int sa,
                                               int sc) {
  constexpr int n = 1 << LOGH;
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const int i = by * Q + TS * a + ty;
      const int jc = (face * n + bx * Q + TS * b + tx + sc) & (2 * n - 1);
      val[a][b] = load_src(src, latlong_source_h<LOGH>(tab, i, jc, cb, sb, sa));
    }
}

// Unscaled 2x2 levels with block side 2..T inside a thread's T x T tile, in
// place (S stays at the block corner, H/V/D at the corner + B/2 offsets):
// S' = (a + b) + (c + d), H' = (a - b) + (c - d), V' = (a + b) - (c + d),
// D' = (a - b) - (c - d).  A coefficient of a block of side B is then B
// times the orthonormal one; the factor is a power of two and is removed
// exactly where the coefficient is read.
template <int T>
__device__ __forceinline__ void tile_levels(float (&g)[T][T]) {
#pragma unroll
  for (int B = 2; B <= T; B <<= 1) {
#pragma unroll
    for (int r0 = 0; r0 < T; r0 += B)
#pragma unroll
      for (int c0 = 0; c0 < T; c0 += B) {
        const int h = B / 2;
        const float a = g[r0][c0], b = g[r0][c0 + h], c = g[r0 + h][c0], d = g[r0 + h][c0 + h];
        g[r0][c0] = (a + b) + (c + d);
        g[r0][c0 + h] = (a - b) + (c - d);
        g[r0 + h][c0] = (a + b) - (c + d);
        g[r0 + h][c0 + h] = (a - b) - (c - d);
      }
  }
}

// Row stride of a wave's Q x Q block image in LDS.  Unpadded at Q = 32: a
// wave then needs 6.8 KiB of LDS, and the 20 waves a CU holds (the register
// limit) leave 25 KiB free for the preparation kernels of the next lighting
// to run beside the relight (the image's stores and tile reads take 2- to
// 4-way bank conflicts instead, a small cost on the LDS pipe).  Q = 16 keeps
// 8 floats of padding.
constexpr int image_stride(int Q) { return Q == 16 ? Q + 8 : Q; }
// Key of a block entry: log2 of its block side (3 bits), block number
// (13 bits) and image offset (11 bits, < 32 * 40).
constexpr int kOffBits = 11;
constexpr int kBlockBits = 13;
constexpr int kLogbShift = kOffBits + kBlockBits;

// x of lane (this lane ^ K), K < 32: one ds_swizzle in bit mode (and mask
// 0x1f, xor mask K within each 32-lane half), no address register.
template <int K>
__device__ __forceinline__ float lane_xor(float x) {
  static_assert(K > 0 && K < 32, "swizzle xor masks stay inside 32 lanes");
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), (K << 10) | 0x1f));
}

// One level above the tiles (tiles of side 2 HT form a block of the next
// level): the four tiles are lanes l, l ^ HT, l ^ HT TS, l ^ (HT TS + HT);
// lanes with ((tx | ty) & (2 HT - 1)) == 0 write the level's H, V, D into the
// image and keep the sum.  The last level (2 HT = TS) has one such lane,
// lane 0, which reads its partners as scalars.
template <int HT, int TS, int T, int STRIDE>
__device__ __forceinline__ void tile_level_above(float& s, float* img, int lane, int tx, int ty,
                                                 bool owns_tile) {
  float b, c, d;
  if constexpr (2 * HT == TS) {
    const int si = __float_as_int(s);
    b = __int_as_float(__builtin_amdgcn_readlane(si, HT));
    c = __int_as_float(__builtin_amdgcn_readlane(si, HT * TS));
    d = __int_as_float(__builtin_amdgcn_readlane(si, HT * TS + HT));
  } else {
    b = lane_xor<HT>(s);
    c = lane_xor<HT * TS>(s);
    d = lane_xor<HT * TS + HT>(s);
  }
  if (owns_tile && ((tx | ty) & (2 * HT - 1)) == 0) {
    img[(ty * T) * STRIDE + (tx + HT) * T] = (s - b) + (c - d);
    img[((ty + HT) * T) * STRIDE + tx * T] = (s + b) - (c + d);
    img[((ty + HT) * T) * STRIDE + (tx + HT) * T] = (s - b) - (c - d);
    s = (s + b) + (c + d);
  }
  if constexpr (4 * HT <= TS) tile_level_above<2 * HT, TS, T, STRIDE>(s, img, lane, tx, ty, owns_tile);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Sum over the 64 lanes of a wave (all lanes active), the same value in every
// lane: DPP adds within each 16-lane row (partner in the quad at xor 1 and
// xor 2, then the mirrored quad of the half row, then the mirrored half row),
// then the four row sums read back as scalars.
__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_mov<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_mov<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_mov<0x141>(x);  // row_half_mirror
  x += dpp_mov<0x140>(x);  // row_mirror
  const int xi = __float_as_int(x);
  return (__int_as_float(__builtin_amdgcn_readlane(xi, 0)) +
          __int_as_float(__builtin_amdgcn_readlane(xi, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(xi, 32)) +
          __int_as_float(__builtin_amdgcn_readlane(xi, 48)));
}

// LDS ordering among the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of the k-th set bit of a face mask (k < popcount).
__device__ __forceinline__ int nth_face(unsigned faces, int k) {
  int face = 0;
  for (int f = 0; f < 6; ++f) {
    if ((faces >> f) & 1u) {
      if (k == 0) face = f;
      --k;
    }
  }
  return face;
}

// Sum of a lane's T x T gathered texels, pairwise.
template <int T>
__device__ __forceinline__ float tile_sum(const float (&v)[T][T]) {
  float r[T];
#pragma unroll
  for (int a = 0; a < T; ++a) {
    if constexpr (T == 4) {
      r[a] = (v[a][0] + v[a][1]) + (v[a][2] + v[a][3]);
    } else if constexpr (T == 2) {
      r[a] = v[a][0] + v[a][1];
    } else {
      r[a] = v[a][0];
    }
  }
  if constexpr (T == 4) return (r[0] + r[1]) + (r[2] + r[3]);
  if constexpr (T == 2) return r[0] + r[1];
  return r[0];
}

// Levels with block side From..T of a thread's tile (the smaller ones are
// already in place), unscaled as in tile_levels.
template <int T, int From>
__device__ __forceinline__ void tile_levels_from(float (&g)[T][T]) {
#pragma unroll
  for (int B = From; B <= T; B <<= 1) {
#pragma unroll
    for (int r0 = 0; r0 < T; r0 += B)
#pragma unroll
      for (int c0 = 0; c0 < T; c0 += B) {
        const int h = B / 2;
        const float a = g[r0][c0], b = g[r0][c0 + h], c = g[r0 + h][c0], d = g[r0 + h][c0 + h];
        g[r0][c0] = (a + b) + (c + d);
        g[r0][c0 + h] = (a - b) + (c - d);
        g[r0 + h][c0] = (a + b) - (c + d);
        g[r0 + h][c0 + h] = (a - b) - (c - d);
      }
  }
}

// In-face and major components (sc, tc, D) of v for source face f:
//   +X (-z,-y, x)  -X (z,-y,-x)  +Y (x, z, y)  -Y (x,-z,-y)  +Z (x,-y, z)  -Z (-x,-y,-z)
__device__ __forceinline__ float3 face_components(int f, float x, float y, float z) {
  const int a = f >> 1;
  const bool neg = (f & 1) != 0;
  const float sc = a == 0 ? (neg ? z : -z) : (f == 5 ? -x : x);
  const float tc = a == 1 ? (neg ? -z : z) : -y;
  const float D = a == 0 ? x : (a == 1 ? y : z);
  return make_float3(sc, tc, neg ? -D : D);
}

// Chain-rule rotation of one destination 2x2 block (Sec. V.A-V.B,
// eq:pde1-eq:pde3): c = (S, H, V, D) of its source block (face sf), d the
// block centre's direction and ex, ey its change per texel step in x and y
// (all in the same units).  Returns the unscaled level-1 coefficients
// (2 S, 2 H, 2 V, 2 D) of the destination block.
__device__ __forceinline__ float4 chain_block(float4 c, int sf, float3 d, float3 ex, float3 ey,
                                              float h) {
  const float3 p = face_components(sf, d.x, d.y, d.z);
  const float3 px = face_components(sf, ex.x, ex.y, ex.z);
  const float3 py = face_components(sf, ey.x, ey.y, ey.z);
  const float iD = __builtin_amdgcn_rcpf(p.z);
  const float iD2 = iD * iD;
  // x' = h (sc / D + 1), y' = h (tc / D + 1)
  const float xx = h * (px.x * p.z - p.x * px.z) * iD2;
  const float xy = h * (py.x * p.z - p.x * py.z) * iD2;
  const float yx = h * (px.y * p.z - p.y * px.z) * iD2;
  const float yy = h * (py.y * p.z - p.y * py.z) * iD2;
  const float xxy = h * (2.0f * p.x * px.z * py.z * iD - (px.x * py.z + py.x * px.z)) * iD2;
  const float yxy = h * (2.0f * p.y * px.z * py.z * iD - (px.y * py.z + py.y * px.z)) * iD2;
  const float fx = -c.y, fy = -c.z, fxy = 2.0f * c.w;
  const float gx = fx * xx + fy * yx;
  const float gy = fx * xy + fy * yy;
  const float gxy = fxy * (xx * yy + xy * yx) + fx * xxy + fy * yxy;
  return make_float4(2.0f * c.x, -2.0f * gx, -2.0f * gy, gxy);
}

// Where a transport entry is consumed when the faces of rank [g0, g0 + FG)
// among `faces` are processed together.  Block gi = (face rank - g0) G^2 +
// block row * G + block column holds every coefficient of a block at most Q
// wide except the face's scaling coefficient: returns 0, key = block side,
// gi and position in the block image (which holds unscaled coefficients).
// The others (blocks wider than Q, and the face's scaling coefficient) are
// "coarse": returns 1, key = index of the group's in-place block-sum grid.
// Returns -1 for entries outside the group or invalid indices.
template <int Q, int NF>
__device__ __forceinline__ int classify(int idx, int logn, int G, unsigned faces, int g0, int FG,
                                        int& key) {
  constexpr int LOGQ = __builtin_ctz(Q);
  constexpr int STRIDE = image_stride(Q);
  const Slot s = decode_slot(idx, logn, NF);
  if (s.face < 0 || !((faces >> s.face) & 1u)) return -1;
  const int rank = __popc(faces & ((1u << s.face) - 1u)) - g0;
  if (rank < 0 || rank >= FG) return -1;
  const int gi = rank * G * G + (s.pr >> LOGQ) * G + (s.pc >> LOGQ);
  if (s.logb <= LOGQ && (s.pr | s.pc) != 0) {
    key = (s.logb << kLogbShift) | (gi << kOffBits) |
          ((s.pr & (Q - 1)) * STRIDE + (s.pc & (Q - 1)));
    return 0;
  }
  key = gi;
  return 1;
}

// Q: block side (min(n, kBlock)); the wave's TS x TS lanes each own a T x T tile.
// CHAIN: the finest level comes from the chain rule on the source blocks
// (Q = 32 only) instead of the exact resampling.  BRDF: triple product, the
// rotated texels are multiplied by the vertex's BRDF factor (not with CHAIN).
// LL: the map is a longitude-latitude map (two squares, one frame, the
// elevation-plus-shift rotation of latlong_source) instead of a cube map.
// The chain-rule variant is held to 5 waves per SIMD (96 VGPRs, a few
// spilled): 0.430 -> 0.411 ms on the benchmark launch against 4 waves
// unspilled; the lat-long variant held to 6 waves spills more and runs
// slower, so it keeps its 5.
template <int Q, bool CHAIN, bool BRDF, bool LL>
__global__ __launch_bounds__(kThreads, CHAIN ? 5 : 1) void relight_kernel(RelightParams p) {
  constexpr int NF = LL ? 2 : 6;  // faces (squares) of the map
  // Blocks holding no listed entry of their own only feed the levels above
  // them through their sum: with SUM_ONLY such a block skips the image, the
  // levels inside it and the entry scan (with CHAIN it also skips the chain
  // rule: a 2x2 block's texels sum to twice its scaling coefficient, which
  // the rule takes from the source block unchanged; not for BRDF, whose
  // factor applies in the tile phase).
  constexpr bool SUM_ONLY = !BRDF;
  constexpr int TS = Q >= 8 ? 8 : Q;  // tiles per block side
  constexpr int T = Q / TS;           // texels per tile side
  constexpr int LOGQ = __builtin_ctz(Q);
  constexpr int LOGTS = __builtin_ctz(TS);
  constexpr int STRIDE = image_stride(Q);
  constexpr int IMG = Q * STRIDE;
  extern __shared__ __align__(16) unsigned char dyn_lds[];

  const int lane = threadIdx.x;
  const int64_t v = p.order ? int64_t(p.order[blockIdx.x]) : int64_t(blockIdx.x);
  if (v < 0 || v >= p.nvert) return;  // not a permutation entry: skipped (uniform)
  const int logn = p.logn;
  const int n = 1 << logn;
  const int G = n >> LOGQ;  // blocks per face side
  const int G2 = G * G;
  const int FG = p.group_faces;
  // the cube map's source map is in strips of four rows for n >= 4 (Q >= 4)
  constexpr bool STRIPS = Q >= 4 && !LL;
  const __amdgpu_buffer_rsrc_t src = source_resource(
      p.src, NF * (n << logn),
      LL ? 0u : (STRIPS ? strip_bias(logn) : texel_bias(logn)));
  const bool comp = p.comp != 0;

  float* img = reinterpret_cast<float*>(dyn_lds);  // the block image
  int* lkey = reinterpret_cast<int*>(dyn_lds + IMG * 4);
  float* lval = reinterpret_cast<float*>(lkey + p.listed);
  double* gS = reinterpret_cast<double*>(dyn_lds + ((IMG * 4 + 8 * p.listed + 7) & ~7));
  // one bit per block of the face group: the block has listed entries
  unsigned* bmask = reinterpret_cast<unsigned*>(gS + FG * G2);
  const int bwords = (FG * G2 + 31) >> 5;

  // index row of this vertex: its own, or its cluster's support row
  const int32_t* idx_row = nullptr;
  bool row_valid = true;
  if (p.tidx) {
    if (p.cluster) {
      const int c = p.cluster[v];
      row_valid = c >= 0 && c < p.nclusters;
      idx_row = p.tidx + int64_t(row_valid ? c : 0) * p.nnz;
    } else {
      idx_row = p.tidx + v * p.nnz;
    }
  }
  // triple product: this vertex's BRDF factor (its material's row)
  const float* brdf_row = nullptr;
  if (BRDF) {
    const int mat = p.material ? p.material[v] : 0;
    if (mat >= 0 && mat < p.nmat)
      brdf_row = p.brdf + int64_t(mat) * 6 * (n << logn);
    else
      row_valid = false;
  }
  const int nnz = row_valid ? p.nnz : 0;
  const int listed = row_valid ? p.listed : 0;

  // faces touched by this vertex's transport row
  unsigned m = 0;
#pragma unroll 4
  for (int e = lane; e < nnz; e += kThreads) {
    const int idx = idx_row ? idx_row[e] : e;
    if (idx >= 0 && idx < NF * (n << logn)) m |= 1u << (idx >> (2 * logn));
  }
  unsigned faces = 0;
#pragma unroll
  for (int f = 0; f < NF; ++f) faces |= (__ballot((m >> f) & 1u) ? 1u : 0u) << f;
  const int nf = __popc(faces);
  const int ngroups = (nf + FG - 1) / FG;

  const bool owns_tile = lane < TS * TS;
  const int ty = lane >> LOGTS, tx = lane & (TS - 1);  // tile of this lane, and its texel in
                                                        // each TS x TS patch of the gather
  const uint64_t lanes_below = (uint64_t(1) << lane) - 1;
  int nfine = 0, ncoarse = 0;

  // lat-long: the rule's tables into LDS, this vertex's rotation
  LLTab tab = {};
  float llcb = 0.0f, llsb = 0.0f;
  int llsa = 0, llsc = 0;
  if constexpr (LL) {
    float* t = reinterpret_cast<float*>(dyn_lds + p.ll_tab_off);
    for (int k = lane; k < 7 * n; k += kThreads) t[k] = p.ll_grid[k];
    tab = {t, t + n, t + 2 * n, t + 4 * n, t + 6 * n};
    llcb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(p.ll_elev[2 * v])));
    llsb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(p.ll_elev[2 * v + 1])));
    llsa = __builtin_amdgcn_readfirstlane(p.ll_shift[2 * v]) & (2 * n - 1);
    llsc = __builtin_amdgcn_readfirstlane(p.ll_shift[2 * v + 1]) & (2 * n - 1);
    wave_sync();
  }

  for (int f = 0; f < p.nframes; ++f) {
    IRot R = {};
    if constexpr (!LL) {
      R = frame_vertex_rotation(p.vrot + v * 9, p.frot ? p.frot + f * 9 : nullptr, scale_bits(logn));
#pragma unroll
      for (int k = 0; k < 9; ++k) R.m[k] = __builtin_amdgcn_readfirstlane(R.m[k]);
    }
    Acc acc = {0.0f, 0.0f};

    for (int grp = 0; grp < ngroups; ++grp) {
      const int g0 = grp * FG;
      const int nfg = min(FG, nf - g0);

      if (f == 0 || ngroups > 1) {
        // List the first `listed` entries in entry order: block entries from
        // the front, coarse entries from the back.
        nfine = 0;
        ncoarse = 0;
        if (SUM_ONLY) {
          for (int k = lane; k < bwords; k += kThreads) bmask[k] = 0u;
          wave_sync();
        }
        for (int c0 = 0; c0 < listed; c0 += kListChunks * kThreads) {
          // the entries of kListChunks chunks of 64 are loaded first, so
          // that their loads are in flight together, then each chunk is
          // classified and listed (a chunk past `listed` lists nothing)
          int ix[kListChunks];
          float vx[kListChunks];
#pragma unroll
          for (int u = 0; u < kListChunks; ++u) {
            const int e = c0 + u * kThreads + lane;
            ix[u] = e < listed ? (idx_row ? idx_row[e] : e) : -1;
            vx[u] = e < listed ? transport_value(p.tval, p.tscale, p.dtype, v, p.nnz, e) : 0.0f;
          }
#pragma unroll
          for (int u = 0; u < kListChunks; ++u) {
            const int e = c0 + u * kThreads + lane;
            int key = 0, kind = -1;
            if (e < listed) kind = classify<Q, NF>(ix[u], logn, G, faces, g0, FG, key);
            const uint64_t bf = __ballot(kind == 0), bc = __ballot(kind == 1);
            if (kind >= 0) {
              const int at = kind == 0 ? nfine + __popcll(bf & lanes_below)
                                       : listed - 1 - (ncoarse + __popcll(bc & lanes_below));
              lkey[at] = key;
              lval[at] = vx[u];
              if (SUM_ONLY && kind == 0) {
                const int gb = (key >> kOffBits) & ((1 << kBlockBits) - 1);
                atomicOr(&bmask[gb >> 5], 1u << (gb & 31));
              }
            }
            nfine += __popcll(bf);
            ncoarse += __popcll(bc);
          }
        }
        wave_sync();
      }

      for (int r = 0, gi = 0; r < nfg; ++r) {
        const int face = nth_face(faces, g0 + r);
        const FaceAxes ax = face_axes(R, face);
        // this lane's direction at texel (ty, tx) of block (0, 0); a block
        // (by, bx) adds the uniform 2 Q (bx R e_U + by R e_V)
        // (exact binary32 integers throughout, see scale_bits)
        const float3 zero3 = make_float3(0.0f, 0.0f, 0.0f);
        const float3 l0 = dir_mad(ax.mU, float(2 * tx + 1 - n), ax.mV, float(2 * ty + 1 - n),
                                  dir_add(ax.mN, float(n), zero3));
        // chain rule: the lane's destination block (ty, tx) at half resolution
        const int hn = n >> 1;
        const float3 h0 = dir_mad(ax.mU, float(2 * tx + 1 - hn), ax.mV, float(2 * ty + 1 - hn),
                                  dir_add(ax.mN, float(hn), zero3));
        for (int by = 0; by < G; ++by) {
          for (int bx = 0; bx < G; ++bx, ++gi) {
            // entries past the list may fall in any block: then every block is full
            bool full = true;
            if constexpr (SUM_ONLY)
              full = nnz > listed ||
                     ((__builtin_amdgcn_readfirstlane(bmask[gi >> 5]) >> (gi & 31)) & 1u) != 0u;
            float lane_sum = 0.0f;  // sum-only blocks: this lane's gathered texels
            if constexpr (LL) {
              // the same compact patches, through the lat-long rule
              if (owns_tile) {
                float val[T][T];
                // H below 32 has Q = H; from 32 on, Q = 32 and H = 32 .. 512
                if constexpr (Q < 32) {
                  latlong_gather<LOGQ, Q, TS, T>(val, tab, src, face, by, bx, ty, tx, llcb,
                                                       llsb, llsa, llsc);
                } else {
                  switch (logn) {
#define RRT_LL_CASE(L)                                                                         \
  case L:                                                                                      \
    latlong_gather<L, Q, TS, T>(val, tab, src, face, by, bx, ty, tx, llcb, llsb, llsa, \
                                      llsc);                                                   \
    break;
                    RRT_LL_CASE(5)
                    RRT_LL_CASE(6)
                    RRT_LL_CASE(7)
                    RRT_LL_CASE(8)
                    RRT_LL_CASE(9)
#undef RRT_LL_CASE
                    default:
#pragma unroll
                      for (int a = 0; a < T; ++a)
#pragma unroll
                        for (int b = 0; b < T; ++b) {
                          const int i = by * Q + TS * a + ty;
                          const int jc = (face * n + bx * Q + TS * b + tx + llsc) & (2 * n - 1);
                          val[a][b] = load_src(
                              src, latlong_source(tab, i, jc, llcb, llsb, logn, llsa));
                        }
                  }
                }
                if (full) {
#pragma unroll
                  for (int a = 0; a < T; ++a)
#pragma unroll
                    for (int b = 0; b < T; ++b) img[(TS * a + ty) * STRIDE + TS * b + tx] = val[a][b];
                } else {
                  lane_sum = tile_sum<T>(val);
                }
              }
            } else if constexpr (CHAIN) {
              // Destination 2x2 blocks (8 a + ty, 8 b + tx) of the 16 x 16 in
              // this block: the source block by the exact map at n / 2, then
              // the chain rule; level-1 coefficients go straight to the image.
              const __amdgpu_buffer_rsrc_t blk = __builtin_amdgcn_make_buffer_rsrc(
                  const_cast<float4*>(p.blocks), short(0), 6 * hn * hn * 16, kBufferWord3);
              const float3 rb = dir_mad(ax.mU, float(2 * (Q / 2) * bx), ax.mV, float(2 * (Q / 2) * by), h0);
              if (SUM_ONLY && !full) {
                // only the block's sum: twice the source blocks' S
                float sv[2][2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                  for (int b = 0; b < 2; ++b) {
                    const float3 d = dir_mad(ax.mU, float(16 * b), ax.mV, float(16 * a), rb);
                    const unsigned at = source_texel_scaled<4>(d.x, d.y, d.z, logn - 1);
                    sv[a][b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(blk, int(at), 0, 0));
                  }
                lane_sum = 2.0f * ((sv[0][0] + sv[0][1]) + (sv[1][0] + sv[1][1]));
              } else {
              float4 cf[2][2];
              int sf[2][2];
#pragma unroll
              for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                  const float3 d = dir_mad(ax.mU, float(16 * b), ax.mV, float(16 * a), rb);
                  const unsigned at = source_texel_scaled<4>(d.x, d.y, d.z, logn - 1);
                  sf[a][b] = int(at >> (2 * (logn - 1) + 4));
                  const u32x4_t raw = __builtin_amdgcn_raw_buffer_load_b128(blk, int(at), 0, 0);
                  cf[a][b] = make_float4(__uint_as_float(raw.x), __uint_as_float(raw.y),
                                         __uint_as_float(raw.z), __uint_as_float(raw.w));
                }
              const float3 ex = make_float3(2.0f * ax.mU.x, 2.0f * ax.mU.y, 2.0f * ax.mU.z);
              const float3 ey = make_float3(2.0f * ax.mV.x, 2.0f * ax.mV.y, 2.0f * ax.mV.z);
#pragma unroll
              for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                  // the block centre at full resolution: twice the half-resolution direction
                  const float3 d = dir_mad(ax.mU, float(16 * b), ax.mV, float(16 * a), rb);
                  const float3 dc = make_float3(2.0f * d.x, 2.0f * d.y, 2.0f * d.z);
                  const float4 o = chain_block(cf[a][b], sf[a][b], dc, ex, ey, float(hn));
                  const int r0 = 2 * (8 * a + ty), c0 = 2 * (8 * b + tx);
                  img[r0 * STRIDE + c0] = o.x;
                  img[r0 * STRIDE + c0 + 1] = o.y;
                  img[(r0 + 1) * STRIDE + c0] = o.z;
                  img[(r0 + 1) * STRIDE + c0 + 1] = o.w;
                }
              }
            } else if (owns_tile) {
            // Gather in TS x TS patches of adjacent texels (one load instruction
            // covers a compact patch, which the L1 serves with few cache lines):
            // lane (ty, tx) takes texel (TS a + ty, TS b + tx) of every patch
            // (a, b) and stores it raw into the block image.
              float3 rw = dir_mad(ax.mU, float(2 * Q * bx), ax.mV, float(2 * Q * by), l0);
              // all T^2 loads are issued before the first store, so that they
              // are in flight together
              float val[T][T];
#pragma unroll
              for (int a = 0; a < T; ++a) {
                float3 d = rw;
#pragma unroll
                for (int b = 0; b < T; ++b) {
                  val[a][b] = load_src(
                      src, STRIPS ? source_texel_strip(d.x, d.y, d.z, logn)
                             : source_texel_biased(d.x, d.y, d.z, logn));
                  d = dir_add(ax.mU, float(2 * TS), d);
                }
                rw = dir_add(ax.mV, float(2 * TS), rw);
              }
              if (full) {
#pragma unroll
                for (int a = 0; a < T; ++a)
#pragma unroll
                  for (int b = 0; b < T; ++b) img[(TS * a + ty) * STRIDE + TS * b + tx] = val[a][b];
              } else {
                lane_sum = tile_sum<T>(val);
              }
            }
            if (SUM_ONLY && !full) {
              // the block's sum for the levels above it; nothing else reads it
              const float bsum = wave_sum(lane_sum);
              if (lane == 0) gS[gi] = double(bsum) * (1.0 / Q);
              wave_sync();
              continue;
            }
            wave_sync();
            float s = 0.0f;  // unscaled sum of this lane's tile, then of its block
            if (owns_tile) {
              // the lane's T x T tile: levels up to side T in registers, in place
              float g[T][T];
#pragma unroll
              for (int rr = 0; rr < T; ++rr)
#pragma unroll
                for (int cc = 0; cc < T; ++cc)
                  g[rr][cc] = img[(ty * T + rr) * STRIDE + tx * T + cc];
              if constexpr (BRDF) {
                {
                  // triple product: times the BRDF factor at each destination texel
                  const float* br =
                      brdf_row + ((face * n + by * Q + ty * T) << logn) + bx * Q + tx * T;
#pragma unroll
                  for (int rr = 0; rr < T; ++rr) {
                    if constexpr (T == 4) {
                      const float4 f4 = *reinterpret_cast<const float4*>(br + (rr << logn));
                      g[rr][0] *= f4.x;
                      g[rr][1] *= f4.y;
                      g[rr][2] *= f4.z;
                      g[rr][3] *= f4.w;
                    } else {
#pragma unroll
                      for (int cc = 0; cc < T; ++cc) g[rr][cc] *= br[(rr << logn) + cc];
                    }
                  }
                }
              }
              if constexpr (CHAIN) {
                tile_levels_from<T, 4>(g);
              } else {
                tile_levels<T>(g);
              }
#pragma unroll
              for (int rr = 0; rr < T; ++rr)
#pragma unroll
                for (int cc = 0; cc < T; ++cc)
                  img[(ty * T + rr) * STRIDE + tx * T + cc] = g[rr][cc];
              s = g[0][0];
            }
            // levels above the tile, unscaled
            if constexpr (TS > 1) tile_level_above<1, TS, T, STRIDE>(s, img, lane, tx, ty, owns_tile);
            // the block's orthonormal scaling coefficient, for the levels above
            if (lane == 0) gS[gi] = double(s) * (1.0 / Q);
            wave_sync();
            // listed entries of this block: four keys per lane and LDS read
            for (int k0 = 4 * lane; k0 < nfine; k0 += 4 * kThreads) {
              const int4 keys = *reinterpret_cast<const int4*>(&lkey[k0]);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int key = q == 0 ? keys.x : (q == 1 ? keys.y : (q == 2 ? keys.z : keys.w));
                if (k0 + q < nfine && ((key >> kOffBits) & ((1 << kBlockBits) - 1)) == gi)
                  acc_add(acc, lval[k0 + q],
                          ldexpf(img[key & ((1 << kOffBits) - 1)], -(key >> kLogbShift)), comp);
              }
            }
            // entries past the list
            for (int e = listed + lane; e < nnz; e += kThreads) {
              int key = 0;
              const int kind = classify<Q, NF>(idx_row ? idx_row[e] : e, logn, G, faces, g0, FG, key);
              if (kind == 0 && ((key >> kOffBits) & ((1 << kBlockBits) - 1)) == gi)
                acc_add(acc, transport_value(p.tval, p.tscale, p.dtype, v, p.nnz, e),
                        ldexpf(img[key & ((1 << kOffBits) - 1)], -(key >> kLogbShift)), comp);
            }
            wave_sync();
          }
        }
      }
      // levels above the blocks, per face of the group (FP64, in place)
      if (G > 1) {
        for (int r = 0; r < nfg; ++r) {
          double* gf = gS + r * G2;
          for (int Bg = 2; Bg <= G; Bg <<= 1) {
            const int hg = Bg / 2, nb = G / Bg;
            for (int t = lane; t < nb * nb; t += kThreads) {
              const int r0 = (t / nb) * Bg, c0 = (t % nb) * Bg;
              double S, H, V, D;
              tile_levels_d(gf[r0 * G + c0], gf[r0 * G + c0 + hg], gf[(r0 + hg) * G + c0],
                            gf[(r0 + hg) * G + c0 + hg], S, H, V, D);
              gf[r0 * G + c0] = S;
              gf[r0 * G + c0 + hg] = H;
              gf[(r0 + hg) * G + c0] = V;
              gf[(r0 + hg) * G + c0 + hg] = D;
            }
            wave_sync();
          }
        }
      }
      // coarse entries: blocks wider than Q and the faces' scaling coefficients
      for (int k = lane; k < ncoarse; k += kThreads) {
        const int at = listed - 1 - k;
        acc_add(acc, lval[at], float(gS[lkey[at]]), comp);
      }
      for (int e = listed + lane; e < nnz; e += kThreads) {
        int key = 0;
        if (classify<Q, NF>(idx_row ? idx_row[e] : e, logn, G, faces, g0, FG, key) == 1)
          acc_add(acc, transport_value(p.tval, p.tscale, p.dtype, v, p.nnz, e), float(gS[key]),
                  comp);
      }
      wave_sync();
    }

    // reduction across the wave
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      Acc other;
      other.s = __shfl_xor(acc.s, o, 64);
      other.c = __shfl_xor(acc.c, o, 64);
      if (comp) {
        acc = acc_merge(acc, other);
      } else {
        acc.s += other.s;
      }
    }
    if (lane == 0) p.out[int64_t(f) * p.out_stride + v] = comp ? (acc.s + acc.c) : acc.s;
  }
}

__global__ void fill_zero(float* __restrict__ x, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) x[i] = 0.0f;
}

__global__ void scatter_light(const int32_t* __restrict__ idx, const void* __restrict__ val,
                              int f16, int k, int total, float* __restrict__ dense) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int at = idx[i];
  if (at < 0 || at >= total) return;
  dense[at] = f16 ? __half2float(static_cast<const __half*>(val)[i])
                  : static_cast<const float*>(val)[i];
}

// Orthonormal (S, H, V, D) of every 2x2 block of the source map, for the
// chain-rule rotation: blocks[face][bi][bj].
__global__ void source_blocks_kernel(const float* __restrict__ src, int logn,
                                     float4* __restrict__ blocks) {
  const int hl = logn - 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 6 << (2 * hl)) return;
  const int f = q >> (2 * hl), bi = (q >> hl) & ((1 << hl) - 1), bj = q & ((1 << hl) - 1);
  // the source map is in strips of four rows (n >= 32 here): the block's
  // two rows share a strip, its columns are four elements apart
  const unsigned at = strip_offset(unsigned((f << logn) + 2 * bi), unsigned(2 * bj), logn);
  const float a = src[at], b = src[at + 4];
  const float c = src[at + 1], d = src[at + 5];
  blocks[q] = make_float4(0.5f * ((a + b) + (c + d)), 0.5f * ((a - b) + (c - d)),
                          0.5f * ((a + b) - (c + d)), 0.5f * ((a - b) - (c - d)));
}

// The lat-long rule's tables: binary32 roundings of sin / cos of the row and
// column centres ((k + 1/2) pi / H) and of the boundary cosines cos(k pi / H),
// evaluated in double precision.
__global__ void latlong_grid_kernel(int H, float* __restrict__ grid) {
  constexpr double kPi = 3.141592653589793;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double centre = (k + 0.5) * kPi / H;
  if (k < H) {
    grid[k] = float(sin(centre));
    grid[H + k] = float(cos(centre));
    grid[6 * H + k] = float(cos(k * kPi / H));
  }
  if (k < 2 * H) {
    grid[2 * H + k] = float(sin(centre));
    grid[4 * H + k] = float(cos(centre));
  }
}

// Heavy-first order, pass 1 (one wave per vertex): the number of faces the
// vertex's row touches.
__global__ __launch_bounds__(kThreads) void order_faces_kernel(
    const int32_t* __restrict__ idx, const int32_t* __restrict__ cluster, int nclusters,
    int nnz, int logn, unsigned char* __restrict__ faces) {
  const int64_t v = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t* row = nullptr;
  if (cluster) {
    const int c = cluster[v];
    if (c >= 0 && c < nclusters) row = idx + int64_t(c) * nnz;
  } else {
    row = idx + v * nnz;
  }
  unsigned m = 0;
  if (row) {
    for (int e = lane; e < nnz; e += kThreads) {
      const int i = row[e];
      if (i >= 0 && i < 6 * (1 << (2 * logn))) m |= 1u << (i >> (2 * logn));
    }
  }
  int nf = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f) nf += __ballot((m >> f) & 1u) ? 1 : 0;
  if (lane == 0) faces[v] = static_cast<unsigned char>(nf);
}

// Pass 2 (256 vertices per block): vertex count of every bucket 6 - faces,
// an LDS histogram per block and one global add per block and bucket.
__global__ __launch_bounds__(256) void order_hist_kernel(const unsigned char* __restrict__ faces,
                                                         int64_t nvert,
                                                         unsigned* __restrict__ counts) {
  __shared__ unsigned h[7];
  if (threadIdx.x < 7) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < nvert) atomicAdd(&h[6 - faces[v]], 1u);
  __syncthreads();
  if (threadIdx.x < 7 && h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

// Pass 3 (256 vertices per block): each block reserves a range of every
// bucket with one global add, then places its vertices in it (the order
// inside a bucket does not affect any result).
__global__ __launch_bounds__(256) void order_place_kernel(const unsigned char* __restrict__ faces,
                                                          int64_t nvert,
                                                          unsigned* __restrict__ counts,
                                                          int32_t* __restrict__ order) {
  __shared__ unsigned h[7], base[7], cur[7];
  if (threadIdx.x < 7) {
    h[threadIdx.x] = 0u;
    cur[threadIdx.x] = 0u;
  }
  __syncthreads();
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int b = v < nvert ? 6 - faces[v] : -1;
  if (b >= 0) atomicAdd(&h[b], 1u);
  __syncthreads();
  if (threadIdx.x < 7) {
    unsigned off = 0;
    for (int k = 0; k < int(threadIdx.x); ++k) off += counts[k];
    base[threadIdx.x] = off + (h[threadIdx.x] ? atomicAdd(&counts[7 + threadIdx.x], h[threadIdx.x]) : 0u);
  }
  __syncthreads();
  if (b >= 0) order[base[b] + atomicAdd(&cur[b], 1u)] = int32_t(v);
}

__global__ void iota_kernel(int32_t* __restrict__ out, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = int32_t(i);
}

__global__ void order_clear_kernel(unsigned* __restrict__ counts) {
  if (threadIdx.x < 14) counts[threadIdx.x] = 0u;
}

// Index of coefficient idx at resolution n in the map n >> levels, or -1 for
// the `levels` finest levels (Mallat layout: the coarse levels are the
// top-left corner of each face).
__global__ void coarsen_indices(const int32_t* __restrict__ idx, int64_t count, int logn,
                                int levels, int32_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int n = 1 << logn;
  const int per_face = n << logn;
  const int v = idx[i];
  int r = -1;
  if (v >= 0 && v < 6 * per_face) {
    const int face = v >> (2 * logn), pos = v & (per_face - 1);
    const int row = pos >> logn, col = pos & (n - 1);
    const int lc = logn - levels;
    if ((row >> lc) == 0 && (col >> lc) == 0) r = (face << (2 * lc)) + (row << lc) + col;
  }
  out[i] = r;
}

// dst[r][q] = src[pi_r(q)] for every texel q of the local map, r < nrot.
__global__ void rotate_pixels(const float* __restrict__ src, const float* __restrict__ rot,
                              int logn, float* __restrict__ dst) {
  const int n = 1 << logn;
  const int per_face = n << logn;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (q >= 6 * per_face) return;
  const IRot R = frame_vertex_rotation(rot + int64_t(r) * 9, nullptr, scale_bits(logn));
  const int face = q >> (2 * logn);
  const int i = (q >> logn) & (n - 1), j = q & (n - 1);
  const FaceAxes ax = face_axes(R, face);
  const int U = 2 * j + 1 - n, V = 2 * i + 1 - n;
  const float3 d = dir_mad(ax.mU, float(U), ax.mV, float(V),
                           dir_add(ax.mN, float(n), make_float3(0.0f, 0.0f, 0.0f)));
  // the map stays in [0, 6 n^2) by construction; the clamp keeps this plain
  // pointer read in bounds whatever the rotation holds
  const unsigned at = unsigned(source_texel(d, logn));
  dst[int64_t(r) * 6 * per_face + q] = src[min(at, unsigned(6 * per_face - 1))];
}

template <int Q, bool CHAIN = false, bool BRDF = false, bool LL = false>
int launch_q(const RelightParams& prm_in, int64_t nvert, hipStream_t s) {
  RelightParams prm = prm_in;
  const int G = (1 << prm.logn) / Q;
  size_t lds = ((size_t(Q) * image_stride(Q) * 4 + 8 * size_t(prm.listed) + 7) & ~size_t(7)) +
               size_t(prm.group_faces) * G * G * 8 + kBlockMaskBytes;
  if (LL) {
    prm.ll_tab_off = int(lds);
    lds += size_t(latlong_grid_floats(1 << prm.logn)) * 4;
  }
  hipLaunchKernelGGL((relight_kernel<Q, CHAIN, BRDF, LL>), dim3(unsigned(nvert)),
                     dim3(kThreads), lds, s, prm);
  return check_launch("relight_kernel");
}

template <bool BRDF>
int launch_size(const RelightParams& prm, int n, int64_t nvert, hipStream_t s) {
  switch (n < kBlock ? n : kBlock) {
    case 2: return launch_q<2, false, BRDF>(prm, nvert, s);
    case 4: return launch_q<4, false, BRDF>(prm, nvert, s);
    case 8: return launch_q<8, false, BRDF>(prm, nvert, s);
    case 16: return launch_q<16, false, BRDF>(prm, nvert, s);
    default: return launch_q<kBlock, false, BRDF>(prm, nvert, s);
  }
}

int launch_latlong(const RelightParams& prm, int n, int64_t nvert, hipStream_t s) {
  switch (n < kBlock ? n : kBlock) {
    case 4: return launch_q<4, false, false, true>(prm, nvert, s);
    case 8: return launch_q<8, false, false, true>(prm, nvert, s);
    case 16: return launch_q<16, false, false, true>(prm, nvert, s);
    default: return launch_q<kBlock, false, false, true>(prm, nvert, s);
  }
}

int launch_variant(const RelightParams& prm, int n, int64_t nvert, bool chain, bool latlong,
                   hipStream_t s) {
  if (latlong) return launch_latlong(prm, n, nvert, s);
  if (chain) return launch_q<kBlock, true>(prm, nvert, s);
  return prm.brdf ? launch_size<true>(prm, n, nvert, s) : launch_size<false>(prm, n, nvert, s);
}

}  // namespace

int launch_relight(const RelightLaunch& a, hipStream_t s) {
  if (a.nvert == 0) return RRT_OK;
  RelightParams p;
  p.src = a.src;
  p.vrot = a.vert_rot;
  p.frot = a.frame_rot;
  p.tidx = a.t_idx;
  p.tval = a.t_val;
  p.tscale = a.t_scale;
  p.cluster = a.cluster;
  p.nclusters = a.nclusters;
  p.out = a.out;
  p.out_stride = a.out_stride > 0 ? a.out_stride : a.nvert;
  p.nvert = a.nvert;
  p.nnz = a.nnz;
  p.nframes = a.nframes;
  p.logn = ilog2(a.n);
  p.dtype = a.t_dtype;
  p.comp = (a.flags & RRT_COMPENSATED) ? 1 : 0;
  p.listed = a.nnz < kMaxListed ? a.nnz : kMaxListed;
  const int G = a.n < kBlock ? 1 : a.n / kBlock;
  const int fit = kGroupBytes / (G * G * 8);
  const int nf = a.latlong ? 2 : 6;
  p.group_faces = fit < 1 ? 1 : (fit > nf ? nf : fit);
  p.blocks = static_cast<const float4*>(a.blocks);
  p.brdf = a.brdf;
  p.material = a.material;
  p.nmat = a.nmaterials;
  p.ll_elev = a.ll_elev;
  p.ll_shift = a.ll_shift;
  p.ll_grid = a.ll_grid;
  p.ll_tab_off = 0;
  p.order = a.order;
  const bool chain = (a.flags & RRT_CHAIN_RULE) != 0;
  return launch_variant(p, a.n, a.nvert, chain, a.latlong, s);
}

int launch_scatter_light(const int32_t* idx, const void* val, int dtype, int k, int n, int squares,
                         float* dense, hipStream_t s) {
  const int64_t total = int64_t(squares) * n * n;
  hipLaunchKernelGGL(fill_zero, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, dense, total);
  int st = check_launch("fill_zero");
  if (st) return st;
  hipLaunchKernelGGL(scatter_light, dim3(unsigned((k + 255) / 256)), dim3(256), 0, s, idx, val,
                     dtype == RRT_F16 ? 1 : 0, k, int(total), dense);
  return check_launch("scatter_light");
}

int launch_source_blocks(const float* src, int n, float* blocks, hipStream_t s) {
  const int total = 6 * (n / 2) * (n / 2);
  hipLaunchKernelGGL(source_blocks_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s,
                     src, ilog2(n), reinterpret_cast<float4*>(blocks));
  return check_launch("source_blocks");
}

int launch_iota(int32_t* out, int64_t count, hipStream_t s) {
  if (count == 0) return RRT_OK;
  hipLaunchKernelGGL(iota_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, out, count);
  return check_launch("iota");
}

size_t relight_order_workspace_bytes(int64_t nvert) {
  return ((size_t(nvert) + 255) & ~size_t(255)) + 256;
}

int launch_relight_order(const int32_t* idx, const int32_t* cluster, int nclusters, int nnz,
                         int64_t nvert, int n, int32_t* order, void* ws, hipStream_t s) {
  if (nvert == 0) return RRT_OK;
  unsigned char* faces = static_cast<unsigned char*>(ws);
  unsigned* counts =
      reinterpret_cast<unsigned*>(faces + ((size_t(nvert) + 255) & ~size_t(255)));
  hipLaunchKernelGGL(order_clear_kernel, dim3(1), dim3(64), 0, s, counts);
  int st = check_launch("order_clear");
  if (st) return st;
  hipLaunchKernelGGL(order_faces_kernel, dim3(unsigned(nvert)), dim3(kThreads), 0, s, idx,
                     cluster, nclusters, nnz, ilog2(n), faces);
  if ((st = check_launch("order_faces"))) return st;
  const unsigned blocks = unsigned((nvert + 255) / 256);
  hipLaunchKernelGGL(order_hist_kernel, dim3(blocks), dim3(256), 0, s, faces, nvert, counts);
  if ((st = check_launch("order_hist"))) return st;
  hipLaunchKernelGGL(order_place_kernel, dim3(blocks), dim3(256), 0, s, faces, nvert, counts,
                     order);
  return check_launch("order_place");
}

int launch_latlong_grid(int H, float* grid, hipStream_t s) {
  hipLaunchKernelGGL(latlong_grid_kernel, dim3(unsigned((2 * H + 255) / 256)), dim3(256), 0, s, H,
                     grid);
  return check_launch("latlong_grid");
}

int launch_coarsen_indices(const int32_t* idx, int64_t count, int n, int levels, int32_t* out,
                           hipStream_t s) {
  if (count == 0) return RRT_OK;
  hipLaunchKernelGGL(coarsen_indices, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, idx,
                     count, ilog2(n), levels, out);
  return check_launch("coarsen_indices");
}

int launch_rotate_pixels(const float* src, const float* rot, int nrot, int n, float* dst,
                         hipStream_t s) {
  const int total = 6 * n * n;
  hipLaunchKernelGGL(rotate_pixels, dim3(unsigned((total + 255) / 256), unsigned(nrot)), dim3(256),
                     0, s, src, rot, ilog2(n), dst);
  return check_launch("rotate_pixels");
}

}  // namespace rrt
