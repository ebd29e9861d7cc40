// Learned transport decoder (not part of the paper): positional encoding,
// BF16 MFMA GEMMs with fused bias / GELU epilogues for the forward and
// backward passes, MSE loss, bias-gradient column sums and Adam.
//
// GEMM: C[M][N] = sum_k A(m, k) B(k, n), A and B in bfloat16, FP32
// accumulation on the matrix cores (v_mfma_f32_32x32x16_bf16, wave64).  A is
// stored [M][K] (row-major) or, transposed, [K][M]; B is stored [K][N] or,
// transposed, [N][K]; the contiguous dimension of each is a multiple of 8.
// A 256-thread workgroup computes a (64 TM) x (64 TM) tile of C, each of its
// four waves a TM x TM grid of 32 x 32 MFMA tiles.  Each 32-deep k-slice of A
// and B is loaded with 16-byte vector loads (the next slice is in flight
// while the matrix cores consume the current one) and staged in LDS in
// k-contiguous rows (row stride 40 bf16), from which every lane reads its 8
// k-consecutive operands with one 16-byte LDS read.  Rows, columns and k
// beyond the matrix read as zero and are not stored.
#include <hip/hip_fp16.h>

#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr int kBK = 32;
constexpr int kLdsStride = kBK + 8;  // bf16 elements per LDS row (16-byte rows, staggered banks)
constexpr float kSqrt2OverPi = 0.7978845608028654f;
constexpr float kGeluC = 0.044715f;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));

// Two values rounded to bfloat16 (nearest, ties to even) by one
// v_cvt_pk_bf16_f32: a in the low half, b in the high half.
__device__ __forceinline__ unsigned bf16x2_bits(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((float2_t){a, b}, bf16x2_t));
}
__device__ __forceinline__ uint16_t bf16_bits(float x) { return uint16_t(bf16x2_bits(x, 0.0f)); }
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(unsigned(h) << 16); }

// GELU with the tanh approximation, written with the identity
// (1 + tanh u) / 2 = 1 / (1 + exp(-2u)): gelu(z) = z sigma(2u),
// u = sqrt(2/pi) (z + 0.044715 z^3); its derivative is
// sigma + 2 z sigma (1 - sigma) du/dz.  exp(-2u) is evaluated as
// 2^(t kGeluExp2), t = z + 0.044715 z^3, with the three constant factors
// folded into one (one product and the hardware 2^x).
constexpr float kGeluExp2 = -2.302208198144325f;  // -2 sqrt(2/pi) log2(e)
__device__ __forceinline__ float gelu_sigma(float z) {
  const float t = z + kGeluC * z * z * z;
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t * kGeluExp2));
}
__device__ __forceinline__ float gelu_f(float z) { return z * gelu_sigma(z); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float sg = gelu_sigma(z);
  const float du = kSqrt2OverPi * (1.0f + 3.0f * kGeluC * z * z);
  return sg + 2.0f * z * sg * (1.0f - sg) * du;
}

enum Epilogue {
  kEpiHidden = 0,   // z = acc + bias -> store z (FP32) and gelu(z) (BF16)
  kEpiOutput = 1,   // out = acc + bias -> FP32
  kEpiGeluGrad = 2, // dz = acc * gelu'(zprev) -> BF16
  kEpiPlain = 3     // acc -> FP32
};

struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K;
  int k_chunk;         // split over k: workgroup z takes [z k_chunk, (z + 1) k_chunk) (a
                       // multiple of kBK) and writes its partial sums to out_f32 + z M N
                       // (kEpiPlain only); 0 = the whole K in one workgroup
  const float* bias;   // [N] (kEpiHidden / kEpiOutput)
  const float* zprev;  // [M][N] (kEpiGeluGrad)
  float* out_f32;      // [M][N]
  uint16_t* out_bf16;  // [M][N]
};

// 8 consecutive bf16 of a row-major [rows][cols] matrix from (r, c), or zeros
// outside it (c and cols are multiples of 8).
__device__ __forceinline__ u32x4_t load8(const uint16_t* base, int rows, int cols, int r, int c) {
  u32x4_t v = {0u, 0u, 0u, 0u};
  if (r < rows && c < cols) v = *reinterpret_cast<const u32x4_t*>(base + int64_t(r) * cols + c);
  return v;
}

// One operand's k-slice: R rows x kBK k, from a k-contiguous ([rows][K]) or
// row-contiguous ([K][rows]) matrix, 16 bytes per vector, R / 64 per thread.
template <int R, bool KCONTIG>
struct Slice {
  static constexpr int kPer = R * kBK / 8 / 256;
  u32x4_t v[kPer];
  __device__ __forceinline__ void load(const uint16_t* base, int rows, int K, int r0, int k0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = i * 256 + int(threadIdx.x);
      if (KCONTIG) {
        v[i] = load8(base, rows, K, r0 + (e >> 2), k0 + (e & 3) * 8);
      } else {
        v[i] = load8(base, K, rows, k0 + e / (R / 8), r0 + (e % (R / 8)) * 8);
      }
    }
  }
  __device__ __forceinline__ void store(uint16_t* lds) const {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = i * 256 + int(threadIdx.x);
      if (KCONTIG) {
        *reinterpret_cast<u32x4_t*>(lds + (e >> 2) * kLdsStride + (e & 3) * 8) = v[i];
      } else {
        const int k = e / (R / 8), r = (e % (R / 8)) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          lds[(r + j) * kLdsStride + k] = uint16_t(v[i][j / 2] >> (16 * (j & 1)));
      }
    }
  }
};

template <bool AT, bool BT, int EPI, int TM>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
  constexpr int BM = 64 * TM, BN = 64 * TM;
  __shared__ __align__(16) uint16_t As[BM * kLdsStride];
  __shared__ __align__(16) uint16_t Bs[BN * kLdsStride];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32 * TM, wn = (wave & 1) * 32 * TM;
  float16_t acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = float16_t{};

  const int kb = g.k_chunk ? int(blockIdx.z) * g.k_chunk : 0;
  const int ke = g.k_chunk ? min(g.K, kb + g.k_chunk) : g.K;
  Slice<BM, !AT> sa;
  Slice<BN, BT> sb;
  sa.load(g.A, g.M, g.K, m0, kb);
  sb.load(g.B, g.N, g.K, n0, kb);
  for (int k0 = kb; k0 < ke; k0 += kBK) {
    sa.store(As);
    sb.store(Bs);
    __syncthreads();
    if (k0 + kBK < ke) {
      sa.load(g.A, g.M, g.K, m0, k0 + kBK);
      sb.load(g.B, g.N, g.K, n0, k0 + kBK);
    }
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      // lane l: operand row l % 32, k = kk + 8 (l / 32) .. + 7
      const int ko = kk + 8 * (lane >> 5);
      bf16x8_t a[TM], b[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = *reinterpret_cast<const bf16x8_t*>(&As[(wm + 32 * i + (lane & 31)) * kLdsStride + ko]);
#pragma unroll
      for (int j = 0; j < TM; ++j)
        b[j] = *reinterpret_cast<const bf16x8_t*>(&Bs[(wn + 32 * j + (lane & 31)) * kLdsStride + ko]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TM; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[m][n]: register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn + 32 * j + (lane & 31);
        if (m >= g.M || n >= g.N) continue;
        const int64_t at = int64_t(m) * g.N + n;
        float x = acc[i][j][r];
        if (EPI == kEpiPlain && g.k_chunk) {
          g.out_f32[int64_t(blockIdx.z) * g.M * g.N + at] = x;
          continue;
        }
        if (EPI == kEpiHidden) {
          x += g.bias[n];
          g.out_f32[at] = x;
          g.out_bf16[at] = bf16_bits(gelu_f(x));
        } else if (EPI == kEpiOutput) {
          g.out_f32[at] = x + g.bias[n];
        } else if (EPI == kEpiGeluGrad) {
          g.out_bf16[at] = bf16_bits(x * gelu_grad_f(g.zprev[at]));
        } else {
          g.out_f32[at] = x;
        }
      }
}

// Band q of gamma(x) = (x, sin(2^k pi x), cos(2^k pi x), k = 0..7) of the 6
// inputs at `in`, rounded to bfloat16 into the feature row `row`: the six
// sines (features 6 + 12 q + i) and cosines (6 + 12 q + 6 + i), band 0 also
// the inputs themselves (features 0..5); band q writes the zero padding of
// features 102 + 4 q .. 102 + 4 q + 3 below 128.  The six inputs are loaded
// together.  2^q pi x is r = 2^(q-1) x revolutions (an exact power-of-two
// product); r - rint(r) is exact and within half a revolution, and the
// hardware sine and cosine of revolutions take it from there (absolute
// error far below the bfloat16 rounding of the features).
constexpr int kEncBands = 8;
static_assert(6 + 12 * kEncBands + 4 * (kEncBands - 1) >= RRT_MLP_IN, "padding per band");

__device__ __forceinline__ void encode_band(const float* __restrict__ in, int q,
                                            uint16_t* __restrict__ row) {
  float x[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] = in[i];
  const float rev = 0.5f * float(1 << q);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float r = x[i] * rev;
    const float f = r - __builtin_rintf(r);
    row[6 + 12 * q + i] = bf16_bits(__builtin_amdgcn_sinf(f));
    row[6 + 12 * q + 6 + i] = bf16_bits(__builtin_amdgcn_cosf(f));
  }
  if (q == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) row[i] = bf16_bits(x[i]);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int f = 6 + 12 * kEncBands + 4 * q + e;
    if (f < RRT_MLP_IN) row[f] = 0;
  }
}

// One thread per (row, band).
__global__ void encode_kernel(const float* __restrict__ in, uint16_t* __restrict__ out,
                              int64_t B) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= B * kEncBands) return;
  const int64_t r = t / kEncBands;
  encode_band(in + r * 6, int(t - r * kEncBands), out + r * RRT_MLP_IN);
}

// Decoder weight layout (rrt_mlp_pack): layer l keeps its offset and size
// of the row-major packing (256 rows of K = 128 or 256 inputs); inside it
// the MFMA operand of feature tile t (rows 32 t .. 32 t + 31) at k-step s
// (k = 16 s .. 16 s + 15) is 512 values at (t * K / 16 + s) * 512, lane
// m + 32 h of the 64 holding W[32 t + m][16 s + 8 h + e], e = 0..7, at
// 8 (m + 32 h) + e.  One thread per 8-value piece (16-byte copies).
__global__ void pack_kernel(const uint16_t* __restrict__ w, uint16_t* __restrict__ out) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= RRT_MLP_WEIGHT_COUNT / 8) return;
  int64_t base = 0;
  int K = RRT_MLP_IN;
  for (int l = 0; l < RRT_MLP_WEIGHTS; ++l) {
    K = l == 0 ? RRT_MLP_IN : RRT_MLP_HIDDEN;
    const int64_t pieces = int64_t(RRT_MLP_HIDDEN) * K / 8;
    if (p < pieces) break;
    p -= pieces;
    base += int64_t(RRT_MLP_HIDDEN) * K;
  }
  const int S = K / 16;
  const int lane = int(p % 64), s = int((p / 64) % S), t = int(p / 64 / S);
  const int m = lane & 31, h = lane >> 5;
  const uint4 v = *reinterpret_cast<const uint4*>(w + base + int64_t(32 * t + m) * K + 16 * s + 8 * h);
  *reinterpret_cast<uint4*>(out + base + p * 8) = v;
}

// The whole decoder for a tile of kDecRows = 64 vertices in one 512-thread
// workgroup (8 waves): encoding, the four hidden layers and the output
// layer, with the tile's activations kept in LDS (one bfloat16 buffer of
// k-contiguous rows, 33.8 KB, rewritten in place between two barriers after
// each layer's products, so that three workgroups share a CU) and the
// weights read from global memory in the decoder layout (592 KB shared by
// every tile: an L2-resident stream).
// Wave w computes output features [32 w, 32 w + 32) of every layer for the
// tile's 64 vertices as the transposed product W A^T: 1 x 2 tiles of
// 32 x 32 MFMAs with the weights as the first operand, so that each lane
// ends with four consecutive features of one vertex per register group and
// stores them with one 8-byte LDS write.  The output layer goes through
// LDS as float rows, 32 vertices at a time, so that each wave writes whole
// 1 KiB rows of the result.  The k steps, the products and their order are those of gemm_bf16
// (a product of two operands is the same either way round), and so are
// the epilogues (bias + GELU rounded to bfloat16; bias, then the per-slot
// scale of the vertex's cluster for the output): the values are
// bit-identical to encode + five gemm_bf16 launches + the per-slot scaling
// in binary32.
constexpr int kDecRows = 64;
constexpr int kDecTiles = kDecRows / 32;  // 32-vertex MFMA tiles per workgroup
constexpr int kDecWaves = 8;                // waves per workgroup
constexpr int kDecFeat = RRT_MLP_HIDDEN / 32 / kDecWaves;  // 32-feature tiles per wave
constexpr int kActStride = RRT_MLP_HIDDEN + 8;  // bf16 per LDS row (staggered banks)
constexpr int kOutStride = RRT_MLP_OUT + 4;      // float per LDS output row (staggered banks)
static_assert(32 * kOutStride * 4 <= kDecRows * kActStride * 2,
              "a 32-vertex output tile fits the activation buffer");
static_assert(RRT_MLP_OUT == 4 * 64, "one float4 per lane and output row");

// One layer's products for the tile: acc[i][j] = W rows [n0 + 32 i, +32) x
// the tile's activations of vertices [32 j, +32), over k = 0..K-1 in steps of
// 16.  The weights come from L2 in the decoder layout (one 16-byte load per
// lane, feature tile and step: 1 KiB contiguous per wave, eight whole cache
// lines); they are loaded kDecAhead steps ahead into a register ring, so
// that that many loads are in flight while the products run instead of
// each step waiting for its own.  K is a compile-time constant so that the
// loop and the ring unroll.
constexpr int kDecAhead = 2;

template <int K>
__device__ __forceinline__ void decode_products(const uint16_t* __restrict__ act,
                                                const uint16_t* __restrict__ Wl, int n0, int lane,
                                                float16_t (&acc)[kDecFeat][kDecTiles]) {
  constexpr int kSteps = K / 16;
  constexpr int kAhead = kDecAhead < kSteps ? kDecAhead : kSteps;
  const int ml = lane & 31;
#pragma unroll
  for (int i = 0; i < kDecFeat; ++i)
#pragma unroll
    for (int j = 0; j < kDecTiles; ++j) acc[i][j] = float16_t{};
  const uint16_t* a_base = act + ml * kActStride + 8 * (lane >> 5);
  // fragment (tile n0 / 32 + i, step s) of this lane: 8 values at
  // ((tile * kSteps + s) * 64 + lane) * 8 of the layer's decoder layout
  const uint16_t* w_base = Wl + (int64_t(n0 / 32) * kSteps * 64 + lane) * 8;
  bf16x8_t ring[kAhead][kDecFeat];
#pragma unroll
  for (int s = 0; s < kAhead; ++s)
#pragma unroll
    for (int i = 0; i < kDecFeat; ++i)
      ring[s][i] = *reinterpret_cast<const bf16x8_t*>(w_base + (int64_t(i) * kSteps + s) * 512);
#pragma unroll
  for (int s = 0; s < kSteps; ++s) {
    // keep each step's loads in their step (the scheduler would otherwise
    // sink them next to their use to save registers)
    __builtin_amdgcn_sched_barrier(0);
    bf16x8_t w[kDecFeat], a[kDecTiles];
#pragma unroll
    for (int i = 0; i < kDecFeat; ++i) w[i] = ring[s % kAhead][i];
    if (s + kAhead < kSteps) {
#pragma unroll
      for (int i = 0; i < kDecFeat; ++i)
        ring[s % kAhead][i] = *reinterpret_cast<const bf16x8_t*>(
            w_base + (int64_t(i) * kSteps + s + kAhead) * 512);
    }
#pragma unroll
    for (int j = 0; j < kDecTiles; ++j)
      a[j] = *reinterpret_cast<const bf16x8_t*>(a_base + 32 * j * kActStride + 16 * s);
#pragma unroll
    for (int i = 0; i < kDecFeat; ++i)
#pragma unroll
      for (int j = 0; j < kDecTiles; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[i], a[j], acc[i][j], 0, 0, 0);
  }
}

__global__ __launch_bounds__(64 * kDecWaves, 6) void decode_kernel(const float* __restrict__ pos_nrm, int64_t B,
                                                     const uint16_t* __restrict__ W,
                                                     const float* __restrict__ bias,
                                                     const int32_t* __restrict__ cluster,
                                                     const float* __restrict__ scale, int C,
                                                     float* __restrict__ out) {
  __shared__ __align__(16) uint16_t act[kDecRows * kActStride];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = int64_t(blockIdx.x) * kDecRows;
  static_assert(kDecRows * kEncBands == 64 * kDecWaves, "one thread per (row, band)");
  {
    const int row = threadIdx.x / kEncBands, q = threadIdx.x % kEncBands;
    uint16_t* dst = act + row * kActStride;
    if (r0 + row < B) {
      encode_band(pos_nrm + (r0 + row) * 6, q, dst);
    } else {
      for (int f = q; f < RRT_MLP_IN; f += kEncBands) dst[f] = 0;
    }
  }
  __syncthreads();
  const int n0 = 32 * kDecFeat * wave;
  // register r of tile (i, j): feature n0 + 32 i + 8 (r / 4) + 4 (lane / 32) + r % 4,
  // vertex 32 j + lane % 32
  const int fl = 4 * (lane >> 5), ml = lane & 31;
  const uint16_t* Wl = W;
  const float* bl = bias;
#pragma unroll 1
  for (int l = 0; l < RRT_MLP_WEIGHTS; ++l) {
    const int K = l == 0 ? RRT_MLP_IN : RRT_MLP_HIDDEN;
    float16_t acc[kDecFeat][kDecTiles];
    if (l == 0)
      decode_products<RRT_MLP_IN>(act, Wl, n0, lane, acc);
    else
      decode_products<RRT_MLP_HIDDEN>(act, Wl, n0, lane, acc);
    __syncthreads();  // every wave has read its operands: the buffer is free
    if (l < RRT_MLP_WEIGHTS - 1) {
#pragma unroll
      for (int i = 0; i < kDecFeat; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int n = n0 + 32 * i + 8 * g + fl;
          const float4 b4 = *reinterpret_cast<const float4*>(bl + n);
#pragma unroll
          for (int j = 0; j < kDecTiles; ++j) {
            const int m = 32 * j + ml;
            uint2 v;
            v.x = bf16x2_bits(gelu_f(acc[i][j][4 * g] + b4.x), gelu_f(acc[i][j][4 * g + 1] + b4.y));
            v.y = bf16x2_bits(gelu_f(acc[i][j][4 * g + 2] + b4.z),
                              gelu_f(acc[i][j][4 * g + 3] + b4.w));
            *reinterpret_cast<uint2*>(act + m * kActStride + n) = v;
          }
        }
      __syncthreads();
    } else {
      // output layer, one 32-vertex tile at a time: acc + bias into LDS
      // (float rows of kOutStride), then each wave writes whole 1 KiB rows,
      // scaled by the row's cluster (one cluster per row: a uniform load)
      float* outl = reinterpret_cast<float*>(act);
#pragma unroll
      for (int j = 0; j < kDecTiles; ++j) {
#pragma unroll
        for (int i = 0; i < kDecFeat; ++i)
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int n = n0 + 32 * i + 8 * g + fl;
            const float4 b4 = *reinterpret_cast<const float4*>(bl + n);
            *reinterpret_cast<float4*>(outl + ml * kOutStride + n) =
                make_float4(acc[i][j][4 * g] + b4.x, acc[i][j][4 * g + 1] + b4.y,
                            acc[i][j][4 * g + 2] + b4.z, acc[i][j][4 * g + 3] + b4.w);
          }
        __syncthreads();
        const int64_t rj = r0 + 32 * j;
        for (int row = wave; row < 32 && rj + row < B; row += kDecWaves) {
          const int c = cluster[rj + row];
          const float4 v = *reinterpret_cast<const float4*>(outl + row * kOutStride + 4 * lane);
          float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          if (c >= 0 && c < C) {
            const float4 s4 = *reinterpret_cast<const float4*>(scale + int64_t(c) * RRT_MLP_OUT + 4 * lane);
            o = make_float4(v.x * s4.x, v.y * s4.y, v.z * s4.z, v.w * s4.w);
          }
          *reinterpret_cast<float4*>(out + (rj + row) * RRT_MLP_OUT + 4 * lane) = o;
        }
        if (j + 1 < kDecTiles) __syncthreads();
      }
    }
    Wl += int64_t(K) * RRT_MLP_HIDDEN;
    bl += RRT_MLP_HIDDEN;
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ in, uint16_t* __restrict__ out,
                               int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) out[t] = bf16_bits(in[t]);
}

// part[c][n] = sum over rows [c R, c R + R) of dz[m][n] (BF16 gradient
// rows); the chunks' partial sums are then added in chunk order
// (sum_splits_kernel), so the bias gradient is deterministic.
__global__ void colsum_kernel(const uint16_t* __restrict__ dz, int64_t M, int N, int R,
                              float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t r0 = int64_t(blockIdx.y) * R;
  const int64_t r1 = r0 + R < M ? r0 + R : M;
  float s = 0.0f;
#pragma unroll 8
  for (int64_t m = r0; m < r1; ++m) s += bf16_value(dz[m * N + n]);
  part[int64_t(blockIdx.y) * N + n] = s;
}

// dout = 2 (out - target) / count; loss += sum (out - target)^2 / count (FP64).
// A grid-stride loop over at most 256 workgroups: one FP64 atomic each.
__global__ void mse_kernel(const float* __restrict__ out, const float* __restrict__ tgt,
                           int64_t count, float* __restrict__ dout, double* __restrict__ loss) {
  __shared__ double part[256];
  double sq = 0.0;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < count;
       t += int64_t(gridDim.x) * blockDim.x) {
    const float d = out[t] - tgt[t];
    dout[t] = 2.0f * d / float(count);
    sq += double(d) * double(d);
  }
  part[threadIdx.x] = sq;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, part[0] / double(count));
}

__global__ void adam_kernel(float* __restrict__ p, uint16_t* __restrict__ p_bf16,
                            float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.0f - b1) * gt;
  const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  const float pt = p[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
  p[t] = pt;
  if (p_bf16) p_bf16[t] = bf16_bits(pt);
}

// out[i] = sum over z < S of part[z count + i], in order of z.
__global__ void sum_splits_kernel(const float* __restrict__ part, int S, int64_t count,
                                  float* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float acc = 0.0f;
  for (int z = 0; z < S; ++z) acc += part[int64_t(z) * count + i];
  out[i] = acc;
}

// out[i] += sum over z < S of part[z count + i], in order of z.
__global__ void sum_splits_acc_kernel(const float* __restrict__ part, int S, int64_t count,
                                      float* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float acc = 0.0f;
  for (int z = 0; z < S; ++z) acc += part[int64_t(z) * count + i];
  out[i] += acc;
}

// 128 x 128 tiles when they still give every CU a workgroup, else 64 x 64.
template <bool AT, bool BT, int EPI>
int gemm(const GemmArgs& a, hipStream_t s) {
  // the contiguous dimension of each stored operand must allow 16-byte loads
  if ((AT ? a.M : a.K) % 8 || (BT ? a.K : a.N) % 8) return RRT_ERR_UNSUPPORTED;
  const int64_t big = int64_t((a.N + 127) / 128) * ((a.M + 127) / 128);
  if (big >= 512) {
    const dim3 grid(unsigned((a.N + 127) / 128), unsigned((a.M + 127) / 128));
    hipLaunchKernelGGL((gemm_bf16<AT, BT, EPI, 2>), grid, dim3(256), 0, s, a);
  } else {
    const dim3 grid(unsigned((a.N + 63) / 64), unsigned((a.M + 63) / 64));
    hipLaunchKernelGGL((gemm_bf16<AT, BT, EPI, 1>), grid, dim3(256), 0, s, a);
  }
  return check_launch("gemm_bf16");
}

inline unsigned blocks(int64_t n, int per = 256) { return unsigned((n + per - 1) / per); }

// Splits of the weight-gradient GEMM's reduction over a batch of B rows:
// 256-row chunks, at most kMaxSplits, so that the 16 (or 8) 64 x 64 output
// tiles of a layer become 256 (or 128) workgroups.
constexpr int kMaxSplits = 16;
// 64-row chunks of the bias gradient's column sums per pass: their partials
// (kColsumChunks x 256 floats) fit in the weight gradient's partial space.
constexpr int kColsumChunks = kMaxSplits * RRT_MLP_HIDDEN / 64;
inline int dw_splits(int64_t B) {
  const int64_t s = (B + 255) / 256;
  return int(s < 1 ? 1 : (s > kMaxSplits ? kMaxSplits : s));
}

// C[M][N] = A^T B over K with the k range split in `splits` (partials in
// `part`, S M N floats), then summed in split order into out.
int gemm_dw_split(GemmArgs a, int splits, float* part, hipStream_t s) {
  if (a.M % 8 || a.N % 8) return RRT_ERR_UNSUPPORTED;
  float* out = a.out_f32;
  const int chunk = ((a.K + splits - 1) / splits + kBK - 1) / kBK * kBK;
  splits = (a.K + chunk - 1) / chunk;
  a.k_chunk = chunk;
  a.out_f32 = part;
  const dim3 grid(unsigned((a.N + 63) / 64), unsigned((a.M + 63) / 64), unsigned(splits));
  hipLaunchKernelGGL((gemm_bf16<true, false, kEpiPlain, 1>), grid, dim3(256), 0, s, a);
  int st = check_launch("gemm_bf16 split");
  if (st) return st;
  const int64_t count = int64_t(a.M) * a.N;
  hipLaunchKernelGGL(sum_splits_kernel, dim3(blocks(count)), dim3(256), 0, s, part, splits, count,
                     out);
  return check_launch("sum_splits");
}

}  // namespace

// Layer geometry: W_l is [out_l][in_l] (row-major), packed in order.
static const int kIn[RRT_MLP_WEIGHTS] = {RRT_MLP_IN, RRT_MLP_HIDDEN, RRT_MLP_HIDDEN,
                                         RRT_MLP_HIDDEN, RRT_MLP_HIDDEN};
static const int kOut[RRT_MLP_WEIGHTS] = {RRT_MLP_HIDDEN, RRT_MLP_HIDDEN, RRT_MLP_HIDDEN,
                                          RRT_MLP_HIDDEN, RRT_MLP_OUT};

int64_t mlp_weight_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += int64_t(kIn[i]) * kOut[i];
  return o;
}
int64_t mlp_bias_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += kOut[i];
  return o;
}

// Activation workspace for a batch of B rows:
//   z_l  FP32 [B][256] for the 4 hidden layers,
//   a_l  BF16 [B][256] for the 4 hidden layers,
//   dz   BF16 [B][256] x 2 (ping-pong, backward only),
//   dout BF16 [B][256] (backward only),
//   the weight-gradient GEMM's split partial sums, FP32 [S][256][256].
size_t mlp_workspace_bytes(int64_t B) {
  const size_t rows = size_t(B) * RRT_MLP_HIDDEN;
  return align256(rows * 4) * 4 + align256(rows * 2) * 4 + align256(rows * 2) * 2 +
         align256(size_t(B) * RRT_MLP_OUT * 2) +
         align256(size_t(dw_splits(B)) * RRT_MLP_HIDDEN * RRT_MLP_HIDDEN * 4);
}

struct MlpWs {
  float* z[4];
  uint16_t* a[4];
  uint16_t* dz[2];
  uint16_t* dout_bf16;
  float* dw_part;
};

static MlpWs carve(void* ws, int64_t B) {
  const size_t rows = size_t(B) * RRT_MLP_HIDDEN;
  char* p = static_cast<char*>(ws);
  MlpWs w;
  for (int l = 0; l < 4; ++l) {
    w.z[l] = reinterpret_cast<float*>(p);
    p += align256(rows * 4);
  }
  for (int l = 0; l < 4; ++l) {
    w.a[l] = reinterpret_cast<uint16_t*>(p);
    p += align256(rows * 2);
  }
  for (int l = 0; l < 2; ++l) {
    w.dz[l] = reinterpret_cast<uint16_t*>(p);
    p += align256(rows * 2);
  }
  w.dout_bf16 = reinterpret_cast<uint16_t*>(p);
  p += align256(size_t(B) * RRT_MLP_OUT * 2);
  w.dw_part = reinterpret_cast<float*>(p);
  return w;
}

int launch_mlp_decode(const void* w, const float* b, const float* scale, int C,
                      const float* pos_nrm, const int32_t* cluster, int64_t B, float* out,
                      hipStream_t s) {
  if (B == 0) return RRT_OK;
  hipLaunchKernelGGL(decode_kernel, dim3(unsigned((B + kDecRows - 1) / kDecRows)),
                     dim3(64 * kDecWaves), 0, s,
                     pos_nrm, B, static_cast<const uint16_t*>(w), b, cluster, scale, C, out);
  return check_launch("decode");
}

int launch_mlp_pack(const void* w, void* out, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(blocks(RRT_MLP_WEIGHT_COUNT / 8)), dim3(256), 0, s,
                     static_cast<const uint16_t*>(w), static_cast<uint16_t*>(out));
  return check_launch("mlp_pack");
}

int launch_mlp_encode(const float* in, int64_t B, void* out, hipStream_t s) {
  hipLaunchKernelGGL(encode_kernel, dim3(blocks(B * kEncBands)), dim3(256), 0, s, in,
                     static_cast<uint16_t*>(out), B);
  return check_launch("encode");
}

int launch_mlp_forward(const void* w, const float* b, const void* x, int64_t B, float* out,
                       void* ws, hipStream_t s) {
  const uint16_t* W = static_cast<const uint16_t*>(w);
  MlpWs k = carve(ws, B);
  const uint16_t* a_in = static_cast<const uint16_t*>(x);
  for (int l = 0; l < RRT_MLP_WEIGHTS; ++l) {
    GemmArgs g = {};
    g.A = a_in;
    g.B = W + mlp_weight_offset(l);
    g.M = int(B);
    g.N = kOut[l];
    g.K = kIn[l];
    g.bias = b + mlp_bias_offset(l);
    int st;
    if (l < RRT_MLP_WEIGHTS - 1) {
      g.out_bf16 = k.a[l];
      g.out_f32 = k.z[l];
      st = gemm<false, true, kEpiHidden>(g, s);
      a_in = k.a[l];
    } else {
      g.out_f32 = out;
      st = gemm<false, true, kEpiOutput>(g, s);
    }
    if (st) return st;
  }
  return RRT_OK;
}

int launch_mlp_backward(const void* w, const void* x, int64_t B, const float* dout, float* dw,
                        float* db, void* ws, hipStream_t s) {
  const uint16_t* W = static_cast<const uint16_t*>(w);
  MlpWs k = carve(ws, B);
  const int64_t nout = B * RRT_MLP_OUT;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(nout)), dim3(256), 0, s, dout, k.dout_bf16, nout);
  int st = check_launch("to_bf16");
  if (st) return st;
  const uint16_t* dz = k.dout_bf16;
  for (int l = RRT_MLP_WEIGHTS - 1; l >= 0; --l) {
    const uint16_t* a_in = l == 0 ? static_cast<const uint16_t*>(x) : k.a[l - 1];
    // dW_l = dz^T a_in : [out][in], reduction over the batch
    GemmArgs gw = {};
    gw.A = dz;          // stored [B][out] = [K][M] -> transposed A
    gw.B = a_in;        // stored [B][in]  = [K][N]
    gw.M = kOut[l];
    gw.N = kIn[l];
    gw.K = int(B);
    gw.out_f32 = dw + mlp_weight_offset(l);
    if ((st = gemm_dw_split(gw, dw_splits(B), k.dw_part, s))) return st;
    // bias gradient: column sums of dz in chunks of 64 rows (the weight
    // gradient's partials are already summed, so their space is free)
    const int nch = int((B + 63) / 64);
    for (int c0 = 0; c0 < nch; c0 += kColsumChunks) {
      const int nc = nch - c0 < kColsumChunks ? nch - c0 : kColsumChunks;
      const int64_t rows = (int64_t(c0) + nc) * 64 < B ? int64_t(nc) * 64 : B - int64_t(c0) * 64;
      hipLaunchKernelGGL(colsum_kernel, dim3(blocks(kOut[l], 64), unsigned(nc)), dim3(64), 0, s,
                         dz + int64_t(c0) * 64 * kOut[l], rows, kOut[l], 64, k.dw_part);
      if ((st = check_launch("colsum"))) return st;
      float* dst = db + mlp_bias_offset(l);
      if (c0 == 0) {
        hipLaunchKernelGGL(sum_splits_kernel, dim3(blocks(kOut[l])), dim3(256), 0, s, k.dw_part,
                           nc, int64_t(kOut[l]), dst);
      } else {
        hipLaunchKernelGGL(sum_splits_acc_kernel, dim3(blocks(kOut[l])), dim3(256), 0, s,
                           k.dw_part, nc, int64_t(kOut[l]), dst);
      }
      if ((st = check_launch("colsum sum"))) return st;
    }
    if (l == 0) break;
    // dz_{l-1} = (dz W_l) * gelu'(z_{l-1})
    GemmArgs gx = {};
    gx.A = dz;                           // [B][out]
    gx.B = W + mlp_weight_offset(l);     // [out][in] = [K][N]
    gx.M = int(B);
    gx.N = kIn[l];
    gx.K = kOut[l];
    gx.zprev = k.z[l - 1];
    uint16_t* next = k.dz[l & 1];
    gx.out_bf16 = next;
    if ((st = gemm<false, false, kEpiGeluGrad>(gx, s))) return st;
    dz = next;
  }
  return RRT_OK;
}

int launch_mse(const float* out, const float* tgt, int64_t count, float* dout, double* loss,
               hipStream_t s) {
  const int64_t nb = (count + 255) / 256;
  hipLaunchKernelGGL(mse_kernel, dim3(unsigned(nb < 256 ? nb : 256)), dim3(256), 0, s, out, tgt,
                     count, dout, loss);
  return check_launch("mse");
}

int launch_adam(float* p, void* p_bf16, float* m, float* v, const float* g, int64_t n, float lr,
                float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, float(step));
  const float c2 = 1.0f - powf(b2, float(step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(n)), dim3(256), 0, s, p,
                     static_cast<uint16_t*>(p_bf16), m, v, g, n, lr, b1, b2, eps, c1, c2);
  return check_launch("adam");
}

}  // namespace rrt
