// Storage conversion of coefficient values for the reduced-precision forms:
// binary16 and bfloat16 (round to nearest even), OCP FP8 E4M3FN, int16 and
// packed 11-bit fixed point, the last three with one float32 scale per
// block of 64 values of a row (scale = max|x| / 448, / 32767, / 1023).
#include <hip/hip_fp16.h>

#include "rrt_internal.h"

namespace rrt {
namespace {

__device__ __forceinline__ uint16_t to_bf16(float x) {
  const unsigned b = __float_as_uint(x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return uint16_t((b >> 16) | 0x40u);  // quiet NaN
  return uint16_t((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

// E4M3FN code of y (|y| <= 448 expected; larger magnitudes saturate to 448).
__device__ __forceinline__ uint8_t to_e4m3(float y) {
  const unsigned b = __float_as_uint(y);
  const unsigned sign = (b >> 24) & 0x80u;
  const float a = fabsf(y);
  unsigned code;
  if (!(a == a)) return uint8_t(sign | 0x7fu);
  if (a < 0x1p-6f) {
    code = unsigned(rintf(a * 512.0f));  // subnormal step 2^-9; 8 carries into 2^-6
  } else {
    const unsigned ab = __float_as_uint(a);
    const int eb = int(ab >> 23) - 127 + 7;  // >= 1 here
    const unsigned m23 = ab & 0x7fffffu;
    const unsigned m = (m23 + 0x7ffffu + ((m23 >> 20) & 1u)) >> 20;  // 0..8, RNE
    code = eb >= 16 ? 0x7fu : (unsigned(eb) << 3) + m;
  }
  if (code > 0x7eu) code = 0x7eu;  // saturate at 448 (0x7f is NaN)
  return uint8_t(sign | code);
}

__global__ void convert_f16(const float* __restrict__ src, __half* __restrict__ dst,
                            int64_t total) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total) dst[i] = __float2half_rn(src[i]);
}

__global__ void convert_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                             int64_t total) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total) dst[i] = to_bf16(src[i]);
}

__device__ __forceinline__ int16_t to_s16(float y) {
  const float r = rintf(fminf(fmaxf(y, -32767.0f), 32767.0f));
  return int16_t(r == r ? r : 0.0f);
}

// One thread per (row, block of 64); codes = round(x * M / max|x|).
template <typename CodeT, int M>
__global__ void convert_blocks(const float* __restrict__ src, CodeT* __restrict__ dst,
                               float* __restrict__ scale, int64_t rows, int cols) {
  const int nblk = (cols + RRT_BLOCK - 1) / RRT_BLOCK;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= rows * nblk) return;
  const int64_t row = t / nblk;
  const int blk = int(t - row * nblk);
  const int c0 = blk * RRT_BLOCK;
  const int c1 = min(cols, c0 + RRT_BLOCK);
  const float* s = src + row * cols;
  float amax = 0.0f;
  for (int c = c0; c < c1; ++c) amax = fmaxf(amax, fabsf(s[c]));
  const float sc = amax > 0.0f ? __fdiv_rn(amax, float(M)) : 1.0f;
  const float inv = amax > 0.0f ? __fdiv_rn(float(M), amax) : 1.0f;
  for (int c = c0; c < c1; ++c) {
    const float y = s[c] * inv;
    if constexpr (M == 448) {
      dst[row * cols + c] = to_e4m3(y);
    } else {
      dst[row * cols + c] = to_s16(y);
    }
  }
  scale[t] = sc;
}

// One thread per (row, block of 64) of the packed 11-bit form: the block's
// 64 codes fill exactly 22 words of the row's bit stream (a shorter last
// block ends inside a word whose remaining bits stay zero), so no two
// threads share a word.
__global__ void convert_s11(const float* __restrict__ src, uint32_t* __restrict__ dst,
                            float* __restrict__ scale, int64_t rows, int cols) {
  const int nblk = (cols + RRT_BLOCK - 1) / RRT_BLOCK;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= rows * nblk) return;
  const int64_t row = t / nblk;
  const int blk = int(t - row * nblk);
  const int c0 = blk * RRT_BLOCK;
  const int c1 = min(cols, c0 + RRT_BLOCK);
  const float* s = src + row * cols;
  float amax = 0.0f;
  for (int c = c0; c < c1; ++c) amax = fmaxf(amax, fabsf(s[c]));
  const float sc = amax > 0.0f ? __fdiv_rn(amax, 1023.0f) : 1.0f;
  const float inv = amax > 0.0f ? __fdiv_rn(1023.0f, amax) : 1.0f;
  const int64_t words = RRT_S11_WORDS(cols);
  uint32_t* w = dst + row * words + int64_t(blk) * 22;
  const int nw = int(min(int64_t(22), words - int64_t(blk) * 22));
  uint64_t acc = 0;  // the block's bit stream not yet written
  int have = 0, out = 0;
  for (int c = c0; c < c1; ++c) {
    const float r = rintf(fminf(fmaxf(s[c] * inv, -1023.0f), 1023.0f));
    const unsigned code = unsigned(int(r == r ? r : 0.0f)) & 0x7ffu;
    acc |= uint64_t(code) << have;
    have += 11;
    if (have >= 32) {
      w[out++] = uint32_t(acc);
      acc >>= 32;
      have -= 32;
    }
  }
  if (out < nw) w[out] = uint32_t(acc);
  scale[t] = sc;
}

}  // namespace

int launch_convert(const float* src, int64_t rows, int cols, int dtype, void* dst, float* scale,
                   hipStream_t s) {
  const int64_t total = rows * cols;
  if (total == 0) return RRT_OK;
  if (dtype == RRT_F16) {
    hipLaunchKernelGGL(convert_f16, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, src,
                       static_cast<__half*>(dst), total);
  } else if (dtype == RRT_BF16) {
    hipLaunchKernelGGL(convert_bf16, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, src,
                       static_cast<uint16_t*>(dst), total);
  } else {
    const int64_t nt = rows * ((cols + RRT_BLOCK - 1) / RRT_BLOCK);
    if (dtype == RRT_E4M3) {
      hipLaunchKernelGGL((convert_blocks<uint8_t, 448>), dim3(unsigned((nt + 255) / 256)),
                         dim3(256), 0, s, src, static_cast<uint8_t*>(dst), scale, rows, cols);
    } else if (dtype == RRT_S11) {
      hipLaunchKernelGGL(convert_s11, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s, src,
                         static_cast<uint32_t*>(dst), scale, rows, cols);
    } else {
      hipLaunchKernelGGL((convert_blocks<int16_t, 32767>), dim3(unsigned((nt + 255) / 256)),
                         dim3(256), 0, s, src, static_cast<int16_t*>(dst), scale, rows, cols);
    }
  }
  return check_launch("convert");
}

}  // namespace rrt
