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
// Work decomposition (one 256-thread workgroup per vertex, all frames):
//   * only the faces touched by the vertex's transport row are processed;
//   * a face is processed in Q x Q regions (Q = min(n, 64)); each of the
//     16 x 16 threads owns a T x T tile (T = Q / 16): it computes T^2 source
//     indices (incremental along a row, d += 2 R e_U), gathers the source
//     texels (L2-resident map) and runs the tile's levels in registers;
//   * tile results go to an in-place LDS image of the region (coefficient of
//     a block of side B at its corner offset by B/2 for H/V/D); the levels
//     above the tile run on the 16 x 16 tile sums in FP64 in LDS, and the
//     levels above the region on the region sums (FP64);
//   * the transport row is matched against the LDS image (each entry's Mallat
//     index maps to one in-place position); products are accumulated per
//     thread and reduced across the workgroup with wave shuffles.
#include <hip/hip_fp16.h>

#include "geometry.h"
#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr int kThreads = 256;
// Region side for large faces: a 64 x 64 region (16 KiB LDS image, 4 x 4
// texels per thread) leaves room for five 256-thread workgroups per CU,
// which hides the gather latency better than 128 x 128 regions (64 KiB,
// two workgroups per CU); measured on MI355X at n = 128.
constexpr int kMaxRegion = 64;

// Gathers from the source map go through a raw buffer resource: 32-bit
// offsets (no 64-bit address arithmetic per texel) and hardware range
// checking (reads past the map return 0).
constexpr int kBufferWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format

template <typename SrcT>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t source_resource(const SrcT* p, int count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<SrcT*>(p), short(0),
                                           count * int(sizeof(SrcT)), kBufferWord3);
}

template <typename SrcT>
__device__ __forceinline__ float load_src(__amdgpu_buffer_rsrc_t r, int i);
template <>
__device__ __forceinline__ float load_src<float>(__amdgpu_buffer_rsrc_t r, int i) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, 0));
}
template <>
__device__ __forceinline__ float load_src<__half>(__amdgpu_buffer_rsrc_t r, int i) {
  const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, i * 2, 0, 0);
  return __half2float(__ushort_as_half(b));
}

// OCP E4M3FN: s eeee mmm, bias 7, subnormals, 0x7f/0xff NaN, no infinities.
__device__ __forceinline__ float decode_e4m3(unsigned b) {
  const unsigned e = (b >> 3) & 15u, m = b & 7u;
  float mag = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : float(m) * 0x1p-9f;
  mag = ((b & 0x7fu) == 0x7fu) ? __uint_as_float(0x7fc00000u) : mag;
  return (b & 0x80u) ? -mag : mag;
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
  return decode_e4m3(static_cast<const uint8_t*>(val)[at]) * sc;
}

// Position of a transport entry in the in-place layout of its face.
struct Slot {
  int face;   // -1: invalid index
  int pr, pc; // in-place row / column inside the face
  int logb;   // log2 of the block side of the basis function
};

__device__ __forceinline__ Slot decode_slot(int idx, int logn) {
  Slot s;
  const int n = 1 << logn;
  const int per_face = n << logn;
  if (idx < 0 || idx >= 6 * per_face) {
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
  const void* src;
  const float* vrot;
  const float* frot;
  const int32_t* tidx;
  const void* tval;
  const float* tscale;
  const int32_t* cluster;
  int nclusters;
  float* out;
  int64_t nvert;
  int nnz;
  int nframes;
  int logn;
  int dtype;
  int comp;
};

// 2x2 levels with block side 2..T inside a thread's T x T tile, in place
// (S stays at the block corner, H/V/D at the corner + B/2 offsets).
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
        g[r0][c0] = 0.5f * ((a + b) + (c + d));
        g[r0][c0 + h] = 0.5f * ((a - b) + (c - d));
        g[r0 + h][c0] = 0.5f * ((a + b) - (c + d));
        g[r0 + h][c0 + h] = 0.5f * ((a - b) - (c - d));
      }
  }
}

// General gather of a tile: the full source-texel map per texel.
template <int T, typename SrcT>
__device__ __forceinline__ void gather_general(float (&g)[T][T], int3 d0, const FaceAxes& ax,
                                               __amdgpu_buffer_rsrc_t src, int logn, float eps) {
#pragma unroll
  for (int r = 0; r < T; ++r) {
    int dx = d0.x, dy = d0.y, dz = d0.z;
#pragma unroll
    for (int c = 0; c < T; ++c) {
      g[r][c] = load_src<SrcT>(src, source_texel(dx, dy, dz, logn, eps));
      dx = wrap_mad(ax.mU.x, 2, dx);
      dy = wrap_mad(ax.mU.y, 2, dy);
      dz = wrap_mad(ax.mU.z, 2, dz);
    }
    d0.x = wrap_mad(ax.mV.x, 2, d0.x);
    d0.y = wrap_mad(ax.mV.y, 2, d0.y);
    d0.z = wrap_mad(ax.mV.z, 2, d0.z);
  }
}

// Q: region side (power of two, <= 128); tiles of T x T texels per thread.
template <int Q, typename SrcT>
__global__ __launch_bounds__(kThreads) void relight_kernel(RelightParams p) {
  constexpr int TS = Q >= 16 ? 16 : Q;  // tiles per region side
  constexpr int T = Q / TS;             // texels per tile side
  constexpr int LOGQ = __builtin_ctz(Q);
  constexpr int LOGTS = __builtin_ctz(TS);
  // regions per face side: one below the largest region side, else up to n = 1024
  constexpr int GMAX = Q < kMaxRegion ? 1 : 1024 / Q;
  __shared__ float img[Q * Q];
  __shared__ double tS[TS * TS];
  __shared__ double gS[GMAX * GMAX];
  __shared__ float red_s[kThreads / 64], red_c[kThreads / 64];
  __shared__ unsigned face_mask;

  const int tid = threadIdx.x;
  const int64_t v = blockIdx.x;
  const int logn = p.logn;
  const int n = 1 << logn;
  const int G = n >> LOGQ;                // regions per face side
  const __amdgpu_buffer_rsrc_t src =
      source_resource(static_cast<const SrcT*>(p.src), 6 * (n << logn));
  const float eps = quotient_margin(logn);
  const bool comp = p.comp != 0;
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
  const int nnz = row_valid ? p.nnz : 0;

  // faces touched by this vertex's transport row
  if (tid == 0) face_mask = 0;
  __syncthreads();
  {
    unsigned m = 0;
    for (int e = tid; e < nnz; e += kThreads) {
      const int idx = idx_row ? idx_row[e] : e;
      if (idx >= 0 && idx < 6 * (n << logn)) m |= 1u << (idx >> (2 * logn));
    }
    if (m) atomicOr(&face_mask, m);
  }
  __syncthreads();
  const unsigned faces = face_mask;
  const bool owns_tile = tid < TS * TS;

  for (int f = 0; f < p.nframes; ++f) {
    const IRot R = frame_vertex_rotation(p.vrot + v * 9, p.frot ? p.frot + f * 9 : nullptr);
    Acc acc = {0.0f, 0.0f};

    for (int face = 0; face < 6; ++face) {
      if (!((faces >> face) & 1u)) continue;
      const FaceAxes ax = face_axes(R, face);

      for (int reg = 0; reg < G * G; ++reg) {
        const int gy = reg / G, gx = reg - gy * G;
        if (owns_tile) {
          const int ty = tid >> LOGTS, tx = tid & (TS - 1);
          float g[T][T];
          const int i0 = (gy << LOGQ) + ty * T, j0 = (gx << LOGQ) + tx * T;
          const int U0 = 2 * j0 + 1 - n, V0 = 2 * i0 + 1 - n;
          int3 d0;
          d0.x = wrap_mad(ax.mU.x, U0, wrap_mad(ax.mV.x, V0, wrap_mad(ax.mN.x, n, 0)));
          d0.y = wrap_mad(ax.mU.y, U0, wrap_mad(ax.mV.y, V0, wrap_mad(ax.mN.y, n, 0)));
          d0.z = wrap_mad(ax.mU.z, U0, wrap_mad(ax.mV.z, V0, wrap_mad(ax.mN.z, n, 0)));
          gather_general<T, SrcT>(g, d0, ax, src, logn, eps);
          tile_levels<T>(g);
#pragma unroll
          for (int r = 0; r < T; ++r)
#pragma unroll
            for (int c = 0; c < T; ++c) img[((ty * T + r) << LOGQ) + tx * T + c] = g[r][c];
          tS[ty * TS + tx] = double(g[0][0]);
        }
        __syncthreads();
        // levels above the tile, inside the region (FP64 block sums)
#pragma unroll
        for (int Bt = 2; Bt <= TS; Bt <<= 1) {
          const int nb = TS / Bt, ht = Bt / 2;
          if (tid < nb * nb) {
            const int br = tid / nb, bc = tid - br * nb;
            const int r0 = br * Bt, c0 = bc * Bt;
            double S, H, V, D;
            tile_levels_d(tS[r0 * TS + c0], tS[r0 * TS + c0 + ht], tS[(r0 + ht) * TS + c0],
                          tS[(r0 + ht) * TS + c0 + ht], S, H, V, D);
            tS[r0 * TS + c0] = S;
            img[((r0 * T) << LOGQ) + (c0 + ht) * T] = float(H);
            img[(((r0 + ht) * T) << LOGQ) + c0 * T] = float(V);
            img[(((r0 + ht) * T) << LOGQ) + (c0 + ht) * T] = float(D);
          }
          __syncthreads();
        }
        if (tid == 0) gS[reg] = tS[0];
        // entries whose basis function lies inside this region
        for (int e = tid; e < nnz; e += kThreads) {
          const int idx = idx_row ? idx_row[e] : e;
          const Slot s = decode_slot(idx, logn);
          if (s.face != face || s.logb > LOGQ || (s.pr | s.pc) == 0) continue;
          if ((s.pr >> LOGQ) != gy || (s.pc >> LOGQ) != gx) continue;
          const float coef = img[((s.pr & (Q - 1)) << LOGQ) + (s.pc & (Q - 1))];
          acc_add(acc, transport_value(p.tval, p.tscale, p.dtype, v, p.nnz, e), coef, comp);
        }
        __syncthreads();
      }
      // levels above the regions (region sums in FP64)
      if (G > 1 && tid == 0) {
        for (int Bg = 2; Bg <= G; Bg <<= 1) {
          const int hg = Bg / 2;
          for (int r0 = 0; r0 < G; r0 += Bg)
            for (int c0 = 0; c0 < G; c0 += Bg) {
              double S, H, V, D;
              tile_levels_d(gS[r0 * G + c0], gS[r0 * G + c0 + hg], gS[(r0 + hg) * G + c0],
                            gS[(r0 + hg) * G + c0 + hg], S, H, V, D);
              gS[r0 * G + c0] = S;
              gS[r0 * G + c0 + hg] = H;
              gS[(r0 + hg) * G + c0] = V;
              gS[(r0 + hg) * G + c0 + hg] = D;
            }
        }
      }
      __syncthreads();
      for (int e = tid; e < nnz; e += kThreads) {
        const int idx = idx_row ? idx_row[e] : e;
        const Slot s = decode_slot(idx, logn);
        if (s.face != face) continue;
        if (s.logb <= LOGQ && (s.pr | s.pc) != 0) continue;
        const float coef = float(gS[(s.pr >> LOGQ) * G + (s.pc >> LOGQ)]);
        acc_add(acc, transport_value(p.tval, p.tscale, p.dtype, v, p.nnz, e), coef, comp);
      }
      __syncthreads();
    }

    // workgroup reduction
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
    if ((tid & 63) == 0) {
      red_s[tid >> 6] = acc.s;
      red_c[tid >> 6] = acc.c;
    }
    __syncthreads();
    if (tid == 0) {
      Acc t = {red_s[0], red_c[0]};
      for (int w = 1; w < kThreads / 64; ++w) {
        Acc o = {red_s[w], red_c[w]};
        if (comp) {
          t = acc_merge(t, o);
        } else {
          t.s += o.s;
        }
      }
      p.out[int64_t(f) * p.nvert + v] = comp ? (t.s + t.c) : t.s;
    }
    __syncthreads();
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

// dst[r][q] = src[pi_r(q)] for every texel q of the local map, r < nrot.
__global__ void rotate_pixels(const float* __restrict__ src, const float* __restrict__ rot,
                              int logn, float* __restrict__ dst) {
  const int n = 1 << logn;
  const int per_face = n << logn;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (q >= 6 * per_face) return;
  const IRot R = frame_vertex_rotation(rot + int64_t(r) * 9, nullptr);
  const int face = q >> (2 * logn);
  const int i = (q >> logn) & (n - 1), j = q & (n - 1);
  const FaceAxes ax = face_axes(R, face);
  const int U = 2 * j + 1 - n, V = 2 * i + 1 - n;
  const int dx = wrap_mad(ax.mU.x, U, wrap_mad(ax.mV.x, V, wrap_mad(ax.mN.x, n, 0)));
  const int dy = wrap_mad(ax.mU.y, U, wrap_mad(ax.mV.y, V, wrap_mad(ax.mN.y, n, 0)));
  const int dz = wrap_mad(ax.mU.z, U, wrap_mad(ax.mV.z, V, wrap_mad(ax.mN.z, n, 0)));
  // the map stays in [0, 6 n^2) by construction; the clamp keeps this plain
  // pointer read in bounds whatever the rotation holds
  const unsigned at = unsigned(source_texel(dx, dy, dz, logn, quotient_margin(logn)));
  dst[int64_t(r) * 6 * per_face + q] = src[min(at, unsigned(6 * per_face - 1))];
}

template <int Q, typename SrcT>
int launch_q(const RelightParams& prm, int64_t nvert, hipStream_t s) {
  hipLaunchKernelGGL((relight_kernel<Q, SrcT>), dim3(unsigned(nvert)), dim3(kThreads), 0, s, prm);
  return check_launch("relight_kernel");
}

template <typename SrcT>
int launch_src(const RelightParams& prm, int n, int64_t nvert, hipStream_t s) {
  switch (n < kMaxRegion ? n : kMaxRegion) {
    case 2: return launch_q<2, SrcT>(prm, nvert, s);
    case 4: return launch_q<4, SrcT>(prm, nvert, s);
    case 8: return launch_q<8, SrcT>(prm, nvert, s);
    case 16: return launch_q<16, SrcT>(prm, nvert, s);
    case 32: return launch_q<32, SrcT>(prm, nvert, s);
    default: return launch_q<kMaxRegion, SrcT>(prm, nvert, s);
  }
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
  p.nvert = a.nvert;
  p.nnz = a.nnz;
  p.nframes = a.nframes;
  p.logn = ilog2(a.n);
  p.dtype = a.t_dtype;
  p.comp = (a.flags & RRT_COMPENSATED) ? 1 : 0;
  return a.src_f16 ? launch_src<__half>(p, a.n, a.nvert, s) : launch_src<float>(p, a.n, a.nvert, s);
}

int launch_scatter_light(const int32_t* idx, const void* val, int dtype, int k, int n,
                         float* dense, hipStream_t s) {
  const int64_t total = int64_t(6) * n * n;
  hipLaunchKernelGGL(fill_zero, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, dense, total);
  int st = check_launch("fill_zero");
  if (st) return st;
  hipLaunchKernelGGL(scatter_light, dim3(unsigned((k + 255) / 256)), dim3(256), 0, s, idx, val,
                     dtype == RRT_F16 ? 1 : 0, k, int(total), dense);
  return check_launch("scatter_light");
}

int launch_rotate_pixels(const float* src, const float* rot, int nrot, int n, float* dst,
                         hipStream_t s) {
  const int total = 6 * n * n;
  hipLaunchKernelGGL(rotate_pixels, dim3(unsigned((total + 255) / 256), unsigned(nrot)), dim3(256),
                     0, s, src, rot, ilog2(n), dst);
  return check_launch("rotate_pixels");
}

}  // namespace rrt
