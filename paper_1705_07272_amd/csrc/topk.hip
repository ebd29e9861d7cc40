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

// ---------------------------------------------------------------------------
// A few long rows (one environment map): the row is split into chunks
// processed by many workgroups.
//   1. per-chunk histograms of the top 12 key bits;
//   2. per row: the bin holding the k-th largest key and, per chunk, the
//      start of that bin's keys in a candidate list;
//   3. per chunk: the candidates, compacted in position order;
//   4. per row: radix select over the candidates' remaining 19 bits gives the
//      exact threshold key t and how many keys equal to t are kept; the
//      position of the last kept one is the cut;
//   5. per chunk: the number of kept entries (key > t, or key == t at a
//      position up to the cut);
//   6. per chunk: ordered emission at the sum of the preceding chunks' counts.
// ---------------------------------------------------------------------------
constexpr int kBinBits = 12;
constexpr int kBins = 1 << kBinBits;
constexpr int kLowBits = 31 - kBinBits;  // key bits below the bin
constexpr int kMaxChunks = 64;
constexpr int kMinChunk = 4096;
constexpr int kChunkThreads = 256;

// Per-row parameters in the workspace.
enum { P_BIN, P_NEED, P_CAND, P_THR, P_CUT, P_COUNT };

struct ChunkPlan {
  int chunks;
  int64_t chunk_len;
};

ChunkPlan chunk_plan(int64_t len) {
  int64_t chunks = (len + kMinChunk - 1) / kMinChunk;
  if (chunks > kMaxChunks) chunks = kMaxChunks;
  ChunkPlan c;
  c.chunks = int(chunks);
  c.chunk_len = (len + chunks - 1) / chunks;
  return c;
}

struct TopkWs {
  uint32_t* hist;     // [rows][chunks][kBins]
  uint32_t* eq_base;  // [rows][chunks]
  uint32_t* sel_cnt;  // [rows][chunks]
  uint32_t* par;      // [rows][P_COUNT]
  uint32_t* ckey;     // [rows][len]
  int32_t* cidx;      // [rows][len]
};

size_t carve(void* base, int64_t rows, int64_t len, TopkWs* w) {
  const ChunkPlan cp = chunk_plan(len);
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + off : nullptr;
    off += align256(bytes);
    return q;
  };
  TopkWs t;
  t.hist = reinterpret_cast<uint32_t*>(take(size_t(rows) * cp.chunks * kBins * 4));
  t.eq_base = reinterpret_cast<uint32_t*>(take(size_t(rows) * cp.chunks * 4));
  t.sel_cnt = reinterpret_cast<uint32_t*>(take(size_t(rows) * cp.chunks * 4));
  t.par = reinterpret_cast<uint32_t*>(take(size_t(rows) * P_COUNT * 4));
  t.ckey = reinterpret_cast<uint32_t*>(take(size_t(rows) * len * 4));
  t.cidx = reinterpret_cast<int32_t*>(take(size_t(rows) * len * 4));
  if (w) *w = t;
  return off;
}

// Sum over the workgroup; every thread gets the total.
template <int kWaves>
__device__ __forceinline__ int block_sum(int x, int* sh) {
  int total;
  block_scan<kWaves>(x, &total, sh);
  return total;
}

__global__ __launch_bounds__(kChunkThreads) void tk_hist(const float* __restrict__ x, int64_t len,
                                                         int64_t chunk_len, int chunks,
                                                         uint32_t* __restrict__ hist) {
  __shared__ unsigned h[kBins];
  const int tid = threadIdx.x, c = blockIdx.x, row = blockIdx.y;
  for (int b = tid; b < kBins; b += kChunkThreads) h[b] = 0;
  __syncthreads();
  const float* r = x + int64_t(row) * len;
  const int64_t lo = int64_t(c) * chunk_len;
  const int64_t hi = lo + chunk_len < len ? lo + chunk_len : len;
  int64_t i = lo + tid;
  for (; i + 3 * kChunkThreads < hi; i += 4 * kChunkThreads) {
    float v4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v4[j] = r[i + j * kChunkThreads];
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&h[key_of(v4[j]) >> kLowBits], 1u);
  }
  for (; i < hi; i += kChunkThreads) atomicAdd(&h[key_of(r[i]) >> kLowBits], 1u);
  __syncthreads();
  uint32_t* out = hist + (int64_t(row) * chunks + c) * kBins;
  for (int b = tid; b < kBins; b += kChunkThreads) out[b] = h[b];
}

// The single-workgroup steps of a long row run as four waves (one per SIMD)
// of at most 32 VGPRs with dynamic LDS, so that they find room on a CU next
// to other work (a relight kernel holding 5 waves of 96 VGPRs per SIMD
// leaves 32 per SIMD).
constexpr int kSmallThreads = 256;
#define RRT_SMALL_STEP __global__ __launch_bounds__(kSmallThreads)

RRT_SMALL_STEP void tk_bin(const uint32_t* __restrict__ hist, int chunks, int k,
                           uint32_t* __restrict__ eq_base, uint32_t* __restrict__ par) {
  constexpr int kWaves = kSmallThreads / 64;
  constexpr int kPer = kBins / kSmallThreads;
  // per-bin totals in dynamic LDS (kBins words): with a static array the
  // compiler pads the register allocation to the occupancy the LDS allows,
  // which keeps the wave from running beside other kernels
  extern __shared__ unsigned tot[];
  __shared__ int sh[kWaves];
  __shared__ int s_bin, s_need;
  const int tid = threadIdx.x, row = blockIdx.x;
  if (tid == 0) {
    s_bin = 0;
    s_need = 0;
  }
  const uint32_t* h = hist + int64_t(row) * chunks * kBins;
  // per-bin totals over the chunks (each thread owns bins tid + 64 j)
#pragma unroll 1
  for (int b = tid; b < kBins; b += kSmallThreads) {
    unsigned t = 0;
#pragma unroll 4
    for (int c = 0; c < chunks; ++c) t += h[int64_t(c) * kBins + b];
    tot[b] = t;
  }
  __syncthreads();
  // this thread's bins kPer tid .. kPer tid + kPer - 1
  const unsigned* mt = tot + kPer * tid;
  int mine = 0;
#pragma unroll 4
  for (int j = 0; j < kPer; ++j) mine += int(mt[j]);
  int total;
  const int before = block_scan<kWaves>(mine, &total, sh);
  // keys in bins above this thread's bins
  unsigned above = unsigned(total - before - mine);
#pragma unroll 4
  for (int j = kPer - 1; j >= 0; --j) {
    const unsigned c = mt[j];
    if (above < unsigned(k) && above + c >= unsigned(k)) {
      s_bin = kPer * tid + j;
      s_need = int(unsigned(k) - above);
    }
    above += c;
  }
  __syncthreads();
  const int bin = s_bin;
  // start of each chunk's candidates (keys in the bin), in chunk order
  if (tid < 64) {
    int run = 0;
    for (int c0 = 0; c0 < chunks; c0 += 64) {
      const int c = c0 + tid;
      const int cnt = c < chunks ? int(h[int64_t(c) * kBins + bin]) : 0;
      int v = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (tid >= o) v += t;
      }
      if (c < chunks) eq_base[int64_t(row) * chunks + c] = unsigned(run + v - cnt);
      run += __shfl(v, 63, 64);
    }
    if (tid == 0) {
      uint32_t* pr = par + int64_t(row) * P_COUNT;
      pr[P_BIN] = unsigned(bin);
      pr[P_NEED] = unsigned(s_need);
      pr[P_CAND] = unsigned(run);
    }
  }
}

// Ordered compaction helper: the keep flags of kItems consecutive positions
// per thread become positions base + rank in position order.
template <int kThreads, typename Pred, typename Emit>
__device__ __forceinline__ int ordered_pass(int64_t lo, int64_t hi, int base, int* sh, Pred keep,
                                            Emit emit) {
  constexpr int kWaves = kThreads / 64;
  for (int64_t c0 = lo; c0 < hi; c0 += int64_t(kThreads) * kItems) {
    unsigned sel = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t i = c0 + int64_t(threadIdx.x) * kItems + j;
      if (i < hi && keep(i)) sel |= 1u << j;
    }
    int total;
    int pos = base + block_scan<kWaves>(__popc(sel), &total, sh);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (sel & (1u << j)) emit(c0 + int64_t(threadIdx.x) * kItems + j, pos++);
    }
    base += total;
  }
  return base;
}

__global__ __launch_bounds__(kChunkThreads) void tk_cand(const float* __restrict__ x, int64_t len,
                                                         int64_t chunk_len, int chunks,
                                                         const uint32_t* __restrict__ eq_base,
                                                         const uint32_t* __restrict__ par,
                                                         uint32_t* __restrict__ ckey,
                                                         int32_t* __restrict__ cidx) {
  __shared__ int sh[kChunkThreads / 64];
  const int c = blockIdx.x, row = blockIdx.y;
  const float* r = x + int64_t(row) * len;
  const unsigned bin = par[int64_t(row) * P_COUNT + P_BIN];
  const int64_t lo = int64_t(c) * chunk_len;
  const int64_t hi = lo + chunk_len < len ? lo + chunk_len : len;
  uint32_t* kk = ckey + int64_t(row) * len;
  int32_t* ki = cidx + int64_t(row) * len;
  ordered_pass<kChunkThreads>(
      lo, hi, int(eq_base[int64_t(row) * chunks + c]), sh,
      [&](int64_t i) { return (key_of(r[i]) >> kLowBits) == bin; },
      [&](int64_t i, int pos) {
        kk[pos] = key_of(r[i]);
        ki[pos] = int32_t(i);
      });
}

RRT_SMALL_STEP void tk_resolve(int64_t len,
                                                            const uint32_t* __restrict__ ckey,
                                                            const int32_t* __restrict__ cidx,
                                                            uint32_t* __restrict__ par) {
  constexpr int kWaves = kSmallThreads / 64;
  __shared__ unsigned h[1024];
  __shared__ int sh[kWaves];
  __shared__ unsigned s_prefix, s_need;
  __shared__ int s_cut;
  const int tid = threadIdx.x, row = blockIdx.x;
  uint32_t* pr = par + int64_t(row) * P_COUNT;
  const int m = int(pr[P_CAND]);
  const uint32_t* kk = ckey + int64_t(row) * len;
  const int32_t* ki = cidx + int64_t(row) * len;
  unsigned prefix = pr[P_BIN] << kLowBits;
  unsigned mask = ~((1u << kLowBits) - 1u) & 0x7fffffffu;
  unsigned need = pr[P_NEED];
  // two passes: bits 18..9 (1024 bins), then bits 8..0 (512 bins)
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = pass == 0 ? 9 : 0;
    const int nb = pass == 0 ? 1024 : 512;
    if (tid == 0) {
      s_prefix = prefix;
      s_need = need;
    }
    for (int b = tid; b < nb; b += kSmallThreads) h[b] = 0;
    __syncthreads();
    for (int i = tid; i < m; i += kSmallThreads) {
      const unsigned u = kk[i];
      if ((u & mask) == prefix) atomicAdd(&h[(u >> shift) & unsigned(nb - 1)], 1u);
    }
    __syncthreads();
    // bins per * tid .. per * tid + per - 1 of this thread: keys above them,
    // then each bin from the top
    const int per = nb / kSmallThreads;
    int mine = 0;
    for (int j = 0; j < per; ++j) mine += int(h[per * tid + j]);
    int total;
    const int before = block_scan<kWaves>(mine, &total, sh);
    unsigned above = unsigned(total - before - mine);
    for (int j = per - 1; j >= 0; --j) {
      const unsigned c = h[per * tid + j];
      if (above < need && above + c >= need) {
        s_prefix = prefix | (unsigned(per * tid + j) << shift);
        s_need = need - above;
      }
      above += c;
    }
    __syncthreads();
    prefix = s_prefix;
    need = s_need;
    mask |= unsigned(nb - 1) << shift;
    __syncthreads();
  }
  // the need-th key equal to the threshold, in position order
  if (tid == 0) s_cut = -1;
  __syncthreads();
  int base = 0;
  for (int c0 = 0; c0 < m && base < int(need); c0 += kSmallThreads) {
    const int i = c0 + tid;
    const int eq = (i < m && kk[i] == prefix) ? 1 : 0;
    int total;
    const int rank = base + block_scan<kWaves>(eq, &total, sh);
    if (eq && rank == int(need) - 1) s_cut = ki[i];
    base += total;
  }
  __syncthreads();
  if (tid == 0) {
    pr[P_THR] = prefix;
    pr[P_CUT] = unsigned(s_cut);
  }
}

__device__ __forceinline__ bool kept(float v, int64_t i, unsigned thr, int cut) {
  const unsigned u = key_of(v);
  return u > thr || (u == thr && i <= int64_t(cut));
}

__global__ __launch_bounds__(kChunkThreads) void tk_count(const float* __restrict__ x, int64_t len,
                                                          int64_t chunk_len, int chunks,
                                                          const uint32_t* __restrict__ par,
                                                          uint32_t* __restrict__ sel_cnt) {
  __shared__ int sh[kChunkThreads / 64];
  const int c = blockIdx.x, row = blockIdx.y;
  const float* r = x + int64_t(row) * len;
  const unsigned thr = par[int64_t(row) * P_COUNT + P_THR];
  const int cut = int(par[int64_t(row) * P_COUNT + P_CUT]);
  const int64_t lo = int64_t(c) * chunk_len;
  const int64_t hi = lo + chunk_len < len ? lo + chunk_len : len;
  int n = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kChunkThreads) n += kept(r[i], i, thr, cut);
  n = block_sum<kChunkThreads / 64>(n, sh);
  if (threadIdx.x == 0) sel_cnt[int64_t(row) * chunks + c] = unsigned(n);
}

__global__ __launch_bounds__(kChunkThreads) void tk_emit(const float* __restrict__ x, int64_t len,
                                                         int64_t chunk_len, int chunks, int k,
                                                         const uint32_t* __restrict__ par,
                                                         const uint32_t* __restrict__ sel_cnt,
                                                         int32_t* __restrict__ oidx,
                                                         float* __restrict__ oval) {
  __shared__ int sh[kChunkThreads / 64];
  const int c = blockIdx.x, row = blockIdx.y;
  const float* r = x + int64_t(row) * len;
  const unsigned thr = par[int64_t(row) * P_COUNT + P_THR];
  const int cut = int(par[int64_t(row) * P_COUNT + P_CUT]);
  const int64_t lo = int64_t(c) * chunk_len;
  const int64_t hi = lo + chunk_len < len ? lo + chunk_len : len;
  int before = 0;
  for (int c2 = threadIdx.x; c2 < c; c2 += kChunkThreads)
    before += int(sel_cnt[int64_t(row) * chunks + c2]);
  before = block_sum<kChunkThreads / 64>(before, sh);
  int32_t* ri = oidx + int64_t(row) * k;
  float* rv = oval + int64_t(row) * k;
  ordered_pass<kChunkThreads>(
      lo, hi, before, sh, [&](int64_t i) { return kept(r[i], i, thr, cut); },
      [&](int64_t i, int pos) {
        if (pos < k) {
          ri[pos] = int32_t(i);
          rv[pos] = r[i];
        }
      });
}

bool use_chunks(int64_t rows, int64_t len, int k) {
  return rows <= 8 && len >= 16384 && int64_t(k) < len;
}

}  // namespace

size_t topk_workspace_bytes(int64_t rows, int64_t len, int k) {
  return use_chunks(rows, len, k) ? carve(nullptr, rows, len, nullptr) : 0;
}

int launch_topk(const float* x, int64_t rows, int64_t len, int k, int32_t* idx, float* val,
                void* ws, hipStream_t s) {
  if (rows == 0 || k == 0) return RRT_OK;
  if (use_chunks(rows, len, k)) {
    TopkWs w;
    carve(ws, rows, len, &w);
    const ChunkPlan cp = chunk_plan(len);
    const dim3 grid(unsigned(cp.chunks), unsigned(rows));
    hipLaunchKernelGGL(tk_hist, grid, dim3(kChunkThreads), 0, s, x, len, cp.chunk_len, cp.chunks,
                       w.hist);
    hipLaunchKernelGGL(tk_bin, dim3(unsigned(rows)), dim3(kSmallThreads), kBins * sizeof(unsigned), s,
                       w.hist, cp.chunks, k,
                       w.eq_base, w.par);
    hipLaunchKernelGGL(tk_cand, grid, dim3(kChunkThreads), 0, s, x, len, cp.chunk_len, cp.chunks,
                       w.eq_base, w.par, w.ckey, w.cidx);
    hipLaunchKernelGGL(tk_resolve, dim3(unsigned(rows)), dim3(kSmallThreads), 0, s, len, w.ckey,
                       w.cidx, w.par);
    hipLaunchKernelGGL(tk_count, grid, dim3(kChunkThreads), 0, s, x, len, cp.chunk_len, cp.chunks,
                       w.par, w.sel_cnt);
    hipLaunchKernelGGL(tk_emit, grid, dim3(kChunkThreads), 0, s, x, len, cp.chunk_len, cp.chunks,
                       k, w.par, w.sel_cnt, idx, val);
    return check_launch("topk chunks");
  }
  if (rows < 64 && len >= 16384) {
    hipLaunchKernelGGL(topk_rows<1024>, dim3(unsigned(rows)), dim3(1024), 0, s, x, len, k, idx,
                       val);
  } else {
    hipLaunchKernelGGL(topk_rows<256>, dim3(unsigned(rows)), dim3(256), 0, s, x, len, k, idx, val);
  }
  return check_launch("topk_rows");
}

}  // namespace rrt
