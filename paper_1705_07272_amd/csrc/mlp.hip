// Learned transport decoder (not part of the paper): positional encoding,
// BF16 MFMA GEMMs with fused bias / GELU epilogues for the forward and
// backward passes, MSE loss, bias-gradient column sums and Adam.
//
// GEMM: C[M][N] = sum_k A(m, k) B(k, n), A and B in bfloat16, FP32
// accumulation on the matrix cores (v_mfma_f32_32x32x8_bf16, wave64).  A is
// stored [M][K] (row-major) or, transposed, [K][M]; B is stored [K][N] or,
// transposed, [N][K].  A 256-thread workgroup computes a 64 x 64 tile of C:
// each k-step stages a 64 x 32 slice of A and a 32 x 64 slice of B in LDS in
// k-contiguous order, and each of the four waves runs four 32x32x8 MFMAs on
// its 32 x 32 quadrant.  Rows, columns and k beyond the matrix read as zero
// and are not stored, so any M, N, K work.
#include <hip/hip_fp16.h>

#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdsStride = kBK + 8;  // bf16 elements per LDS row (padding vs bank conflicts)
constexpr float kSqrt2OverPi = 0.7978845608028654f;
constexpr float kGeluC = 0.044715f;

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  const unsigned b = __float_as_uint(x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return uint16_t((b >> 16) | 0x40u);
  return uint16_t((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(unsigned(h) << 16); }

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + tanhf(kSqrt2OverPi * (z + kGeluC * z * z * z)));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float t = tanhf(kSqrt2OverPi * (z + kGeluC * z * z * z));
  const float du = kSqrt2OverPi * (1.0f + 3.0f * kGeluC * z * z);
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * du;
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
  const float* bias;   // [N] (kEpiHidden / kEpiOutput)
  const float* zprev;  // [M][N] (kEpiGeluGrad)
  float* out_f32;      // [M][N]
  uint16_t* out_bf16;  // [M][N]
};

template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
  __shared__ uint16_t As[kBM * kLdsStride];
  __shared__ uint16_t Bs[kBN * kLdsStride];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  float16_t acc = {};

  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    // stage A(m0.., k0..) as As[m][k]
#pragma unroll
    for (int it = 0; it < (kBM * kBK) / 256; ++it) {
      const int e = it * 256 + tid;
      int m, k;
      if (!AT) {        // [M][K]: k fastest
        m = e / kBK;
        k = e % kBK;
      } else {          // [K][M]: m fastest
        k = e / kBM;
        m = e % kBM;
      }
      const int gm = m0 + m, gk = k0 + k;
      uint16_t val = 0;
      if (gm < g.M && gk < g.K) val = AT ? g.A[int64_t(gk) * g.M + gm] : g.A[int64_t(gm) * g.K + gk];
      As[m * kLdsStride + k] = val;
    }
    // stage B(k0.., n0..) as Bs[n][k]
#pragma unroll
    for (int it = 0; it < (kBN * kBK) / 256; ++it) {
      const int e = it * 256 + tid;
      int n, k;
      if (BT) {         // [N][K]: k fastest
        n = e / kBK;
        k = e % kBK;
      } else {          // [K][N]: n fastest
        k = e / kBN;
        n = e % kBN;
      }
      const int gn = n0 + n, gk = k0 + k;
      uint16_t val = 0;
      if (gn < g.N && gk < g.K) val = BT ? g.B[int64_t(gn) * g.K + gk] : g.B[int64_t(gk) * g.N + gn];
      Bs[n * kLdsStride + k] = val;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 8) {
      const int kq = kk + 4 * (lane >> 5);
      const uint16_t* pa = &As[(wm + (lane & 31)) * kLdsStride + kq];
      const uint16_t* pb = &Bs[(wn + (lane & 31)) * kLdsStride + kq];
      short4_t a, b;
      a[0] = short(pa[0]); a[1] = short(pa[1]); a[2] = short(pa[2]); a[3] = short(pa[3]);
      b[0] = short(pb[0]); b[1] = short(pb[1]); b[2] = short(pb[2]); b[3] = short(pb[3]);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // D[m][n]: register j of lane l holds row 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int m = m0 + wm + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    const int n = n0 + wn + (lane & 31);
    if (m >= g.M || n >= g.N) continue;
    const int64_t at = int64_t(m) * g.N + n;
    float x = acc[j];
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

// gamma(x) = (x, sin(2^k pi x), cos(2^k pi x), k = 0..7), zero-padded to 128.
__global__ void encode_kernel(const float* __restrict__ in, uint16_t* __restrict__ out,
                              int64_t B) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= B * RRT_MLP_IN) return;
  const int64_t row = t / RRT_MLP_IN;
  const int f = int(t - row * RRT_MLP_IN);
  float v = 0.0f;
  if (f < 6) {
    v = in[row * 6 + f];
  } else if (f < 6 + 6 * 2 * 8) {
    const int band = (f - 6) / 12;
    const int r = (f - 6) % 12;
    const float x = in[row * 6 + (r % 6)];
    const float w = float(1 << band) * 3.14159265358979323846f;
    v = (r < 6) ? sinf(w * x) : cosf(w * x);
  }
  out[t] = bf16_bits(v);
}

__global__ void to_bf16_kernel(const float* __restrict__ in, uint16_t* __restrict__ out,
                               int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) out[t] = bf16_bits(in[t]);
}

__global__ void fill_kernel(float* __restrict__ x, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) x[t] = 0.0f;
}

// db[n] += sum over a chunk of rows of dz[m][n] (BF16 gradient rows).
__global__ void colsum_kernel(const uint16_t* __restrict__ dz, int64_t M, int N,
                              float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t r0 = int64_t(blockIdx.y) * 256;
  const int64_t r1 = r0 + 256 < M ? r0 + 256 : M;
  float s = 0.0f;
  for (int64_t m = r0; m < r1; ++m) s += bf16_value(dz[m * N + n]);
  atomicAdd(&db[n], s);
}

// dout = 2 (out - target) / count; loss += sum (out - target)^2 / count (FP64).
__global__ void mse_kernel(const float* __restrict__ out, const float* __restrict__ tgt,
                           int64_t count, float* __restrict__ dout, double* __restrict__ loss) {
  __shared__ double part[256];
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (t < count) {
    const float d = out[t] - tgt[t];
    dout[t] = 2.0f * d / float(count);
    sq = double(d) * double(d);
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

template <bool AT, bool BT, int EPI>
int gemm(const GemmArgs& a, hipStream_t s) {
  const dim3 grid(unsigned((a.N + kBN - 1) / kBN), unsigned((a.M + kBM - 1) / kBM));
  hipLaunchKernelGGL((gemm_bf16<AT, BT, EPI>), grid, dim3(256), 0, s, a);
  return check_launch("gemm_bf16");
}

inline unsigned blocks(int64_t n, int per = 256) { return unsigned((n + per - 1) / per); }

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
//   dz   BF16 [B][256] x 2 (ping-pong, backward only).
size_t mlp_workspace_bytes(int64_t B) {
  const size_t rows = size_t(B) * RRT_MLP_HIDDEN;
  return align256(rows * 4) * 4 + align256(rows * 2) * 4 + align256(rows * 2) * 2 +
         align256(size_t(B) * RRT_MLP_OUT * 2);
}

struct MlpWs {
  float* z[4];
  uint16_t* a[4];
  uint16_t* dz[2];
  uint16_t* dout_bf16;
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
  return w;
}

int launch_mlp_encode(const float* in, int64_t B, void* out, hipStream_t s) {
  hipLaunchKernelGGL(encode_kernel, dim3(blocks(B * RRT_MLP_IN)), dim3(256), 0, s, in,
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
      g.out_f32 = k.z[l];
      g.out_bf16 = k.a[l];
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
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(mlp_bias_offset(RRT_MLP_WEIGHTS))), dim3(256), 0, s,
                     db, mlp_bias_offset(RRT_MLP_WEIGHTS));
  if ((st = check_launch("fill"))) return st;
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
    if ((st = gemm<true, false, kEpiPlain>(gw, s))) return st;
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks(kOut[l], 64), unsigned((B + 255) / 256)),
                       dim3(64), 0, s, dz, B, kOut[l], db + mlp_bias_offset(l));
    if ((st = check_launch("colsum"))) return st;
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
  hipLaunchKernelGGL(mse_kernel, dim3(blocks(count)), dim3(256), 0, s, out, tgt, count, dout, loss);
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
