// Non-linear approximation (Sec. III, Haar-domain methods): keep the k
// entries of largest magnitude of each row, ties to the lower position,
// output in ascending position order.
//
// One workgroup per row (256 threads for many rows, 1024 for a few long
// rows such as one environment map).  The k-th largest key is found by a
// four-pass radix select over the 31 magnitude bits of binary32 (|x| orders
// like its bit pattern): each pass builds a 256-bin histogram of the next
// byte among the keys that share the already-fixed high bytes, one private
// LDS histogram per wave (keys of one map crowd into few bins, so shared
// bins would serialise the atomics), then merged.  A final ordered pass
// keeps every key above the threshold and the first `need` keys equal to it,
// using block-wide prefix sums so that positions come out in ascending
// order.
#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr int kItems = 4;

// Exclusive prefix sum over the workgroup; *total gets the sum.
template <int kWaves>
__device__ __forceinline__ int block_scan(int x, int* total, int* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int v = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) sh[wid] = v;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int s = sh[w];
    base += (w < wid) ? s : 0;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return base + v - x;
}

__device__ __forceinline__ unsigned key_of(float x) { return __float_as_uint(x) & 0x7fffffffu; }

template <int kThreads>
__global__ __launch_bounds__(kThreads) void topk_rows(const float* __restrict__ x, int64_t len,
                                                      int k, int32_t* __restrict__ oidx,
                                                      float* __restrict__ oval) {
  constexpr int kWaves = kThreads / 64;
  __shared__ unsigned hist[kWaves][256];
  __shared__ unsigned s_prefix, s_need;
  __shared__ int sh[kWaves];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const float* row = x + int64_t(blockIdx.x) * len;
  int32_t* ri = oidx + int64_t(blockIdx.x) * k;
  float* rv = oval + int64_t(blockIdx.x) * k;

  unsigned prefix = 0, mask = 0, need = unsigned(k);
  const bool all = int64_t(k) >= len;
  if (!all) {
    for (int pass = 0; pass < 4; ++pass) {
      const int shift = 24 - 8 * pass;
      for (int b = tid; b < kWaves * 256; b += kThreads) (&hist[0][0])[b] = 0;
      __syncthreads();
      int64_t i = tid;
      for (; i + 3 * kThreads < len; i += 4 * kThreads) {
        float v4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v4[j] = row[i + j * kThreads];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const unsigned u = key_of(v4[j]);
          if ((u & mask) == prefix) atomicAdd(&hist[wave][(u >> shift) & 255u], 1u);
        }
      }
      for (; i < len; i += kThreads) {
        const unsigned u = key_of(row[i]);
        if ((u & mask) == prefix) atomicAdd(&hist[wave][(u >> shift) & 255u], 1u);
      }
      __syncthreads();
      for (int b = tid; b < 256; b += kThreads) {
        unsigned t = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += hist[w][b];
        hist[0][b] = t;
      }
      __syncthreads();
      if (tid == 0) {
        unsigned cum = 0;
        int b = 255;
        for (; b > 0; --b) {
          const unsigned c = hist[0][b];
          if (cum + c >= need) break;
          cum += c;
        }
        s_prefix = prefix | (unsigned(b) << shift);
        s_need = need - cum;
      }
      __syncthreads();
      prefix = s_prefix;
      need = s_need;
      mask |= 255u << shift;
    }
  }
  const unsigned thr = prefix;

  int out_base = 0, eq_base = 0;
  for (int64_t c0 = 0; c0 < len; c0 += int64_t(kThreads) * kItems) {
    unsigned gt = 0, eq = 0;
    float v[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t i = c0 + int64_t(tid) * kItems + j;
      v[j] = i < len ? row[i] : 0.0f;
      if (i < len) {
        const unsigned u = key_of(v[j]);
        if (all || u > thr) gt |= 1u << j;
        else if (u == thr) eq |= 1u << j;
      }
    }
    int eq_total;
    const int eq_off = block_scan<kWaves>(__popc(eq), &eq_total, sh);
    // the first `need` equal keys (in position order) are kept
    unsigned sel = gt;
    int rank = eq_base + eq_off;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (eq & (1u << j)) {
        if (unsigned(rank) < need) sel |= 1u << j;
        ++rank;
      }
    }
    int sel_total;
    int pos = out_base + block_scan<kWaves>(__popc(sel), &sel_total, sh);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (sel & (1u << j)) {
        if (pos < k) {
          ri[pos] = int32_t(c0 + int64_t(tid) * kItems + j);
          rv[pos] = v[j];
        }
        ++pos;
      }
    }
    out_base += sel_total;
    eq_base += eq_total;
  }
}

}  // namespace

int launch_topk(const float* x, int64_t rows, int64_t len, int k, int32_t* idx, float* val,
                hipStream_t s) {
  if (rows == 0 || k == 0) return RRT_OK;
  if (rows < 64 && len >= 16384) {
    hipLaunchKernelGGL(topk_rows<1024>, dim3(unsigned(rows)), dim3(1024), 0, s, x, len, k, idx,
                       val);
  } else {
    hipLaunchKernelGGL(topk_rows<256>, dim3(unsigned(rows)), dim3(256), 0, s, x, len, k, idx, val);
  }
  return check_launch("topk_rows");
}

}  // namespace rrt
