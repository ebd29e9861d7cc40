// Orthonormal non-standard 2-D Haar transform of cube faces (Sec. V.B: the
// H/V/D coefficients of every scale are finite differences of 2x2 block
// averages of the next finer scale; Mallat quadrant layout per face).
//
// Each face is cut into Q x Q tiles (Q = min(n, 64)), one 256-thread
// workgroup per tile: the tile is staged in LDS (16 KiB, small enough to run
// beside relight waves that hold most of a CU's LDS), the levels of block
// side 2..Q are computed in place there (S stays at the block's corner), and
// the H/V/D outputs of every level go straight to their Mallat positions,
// which for one tile form contiguous row segments.  For n > 64 the (n/64)^2
// tile sums are combined by a second, tiny launch; the tile sums travel between
// the launches through the top-left corner of the output (forward) or the
// first texel of each output tile (inverse), positions no other coefficient
// or texel of the first launch uses.

#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;
constexpr int kMaxGrid = 1024 / kTile;  // tiles per face side at n = 1024

__device__ __forceinline__ void butterfly(float a, float b, float c, float d, float& S, float& H,
                                          float& V, float& D) {
  S = 0.5f * ((a + b) + (c + d));
  H = 0.5f * ((a - b) + (c - d));
  V = 0.5f * ((a + b) - (c + d));
  D = 0.5f * ((a - b) - (c - d));
}

__device__ __forceinline__ void inverse_butterfly(float S, float H, float V, float D, float& a,
                                                  float& b, float& c, float& d) {
  a = 0.5f * ((S + H) + (V + D));
  b = 0.5f * ((S - H) + (V - D));
  c = 0.5f * ((S + H) - (V + D));
  d = 0.5f * ((S - H) - (V - D));
}

// grid: count * 6 * G * G workgroups (G = n / Q); LDS: Q * Q floats.
__global__ __launch_bounds__(kThreads) void haar_fwd_tiles(const float* __restrict__ pix,
                                                           float* __restrict__ coef, int n,
                                                           int logq, int G) {
  extern __shared__ float lds[];
  const int Q = 1 << logq;
  const int64_t blk = blockIdx.x;
  const int tile = int(blk % (G * G));
  const int64_t face = blk / (G * G);
  const int ty = tile / G, tx = tile % G;
  const float* src = pix + face * int64_t(n) * n;
  float* dst = coef + face * int64_t(n) * n;
  const int row0 = ty * Q, col0 = tx * Q;
  for (int e = threadIdx.x; e < Q * Q; e += kThreads) {
    const int r = e >> logq, c = e & (Q - 1);
    lds[e] = src[int64_t(row0 + r) * n + col0 + c];
  }
  __syncthreads();
  for (int B = 2; B <= Q; B <<= 1) {
    const int nb = Q / B, h = B >> 1, q = n / B;
    for (int e = threadIdx.x; e < nb * nb; e += kThreads) {
      const int br = e / nb, bc = e - br * nb;
      const int r0 = br * B, c0 = bc * B;
      float S, H, V, D;
      butterfly(lds[r0 * Q + c0], lds[r0 * Q + c0 + h], lds[(r0 + h) * Q + c0],
                lds[(r0 + h) * Q + c0 + h], S, H, V, D);
      lds[r0 * Q + c0] = S;
      const int gbr = ty * nb + br, gbc = tx * nb + bc;
      dst[int64_t(gbr) * n + q + gbc] = H;
      dst[int64_t(q + gbr) * n + gbc] = V;
      dst[int64_t(q + gbr) * n + q + gbc] = D;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) dst[int64_t(ty) * n + tx] = lds[0];
}

// Coarse levels above the tiles: the G x G tile sums sit in the top-left
// corner of each face of `coef` (spatial order); they are replaced by their
// own Mallat transform.  grid: count * 6; LDS: G * G floats (G <= kMaxGrid).
__global__ __launch_bounds__(64) void haar_fwd_coarse(float* __restrict__ coef, int n, int G) {
  __shared__ float s[kMaxGrid * kMaxGrid];
  float* f = coef + int64_t(blockIdx.x) * n * n;
  for (int e = threadIdx.x; e < G * G; e += 64) s[e] = f[int64_t(e / G) * n + (e % G)];
  __syncthreads();
  for (int B = 2; B <= G; B <<= 1) {
    const int nb = G / B, h = B >> 1, q = G / B;
    for (int e = threadIdx.x; e < nb * nb; e += 64) {
      const int br = e / nb, bc = e - br * nb;
      const int r0 = br * B, c0 = bc * B;
      float S, H, V, D;
      butterfly(s[r0 * G + c0], s[r0 * G + c0 + h], s[(r0 + h) * G + c0],
                s[(r0 + h) * G + c0 + h], S, H, V, D);
      s[r0 * G + c0] = S;
      f[int64_t(br) * n + q + bc] = H;
      f[int64_t(q + br) * n + bc] = V;
      f[int64_t(q + br) * n + q + bc] = D;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) f[0] = s[0];
}

// Inverse of haar_fwd_coarse: reads the Mallat corner of `coef` and writes
// the tile sum of tile (ty, tx) to stage[face * n * n + ty * rs + tx * cs].
__global__ __launch_bounds__(64) void haar_inv_coarse(const float* coef, float* stage, int n,
                                                      int G, int64_t rs, int64_t cs) {
  __shared__ float s[kMaxGrid * kMaxGrid];
  const float* f = coef + int64_t(blockIdx.x) * n * n;
  float* st = stage + int64_t(blockIdx.x) * n * n;
  if (threadIdx.x == 0) s[0] = f[0];
  __syncthreads();
  for (int B = G; B >= 2; B >>= 1) {
    const int nb = G / B, h = B >> 1, q = G / B;
    for (int e = threadIdx.x; e < nb * nb; e += 64) {
      const int br = e / nb, bc = e - br * nb;
      const int r0 = br * B, c0 = bc * B;
      float a, b, c, d;
      inverse_butterfly(s[r0 * G + c0], f[int64_t(br) * n + q + bc], f[int64_t(q + br) * n + bc],
                        f[int64_t(q + br) * n + q + bc], a, b, c, d);
      s[r0 * G + c0] = a;
      s[r0 * G + c0 + h] = b;
      s[(r0 + h) * G + c0] = c;
      s[(r0 + h) * G + c0 + h] = d;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < G * G; e += 64) st[(e / G) * rs + (e % G) * cs] = s[e];
}

// grid: count * 6 * G * G; the tile sum comes from coef[face][0] when G == 1,
// else from stage[face * n * n + ty * rs + tx * cs].  With `strips` (n >= 4)
// the pixels are written in strips of four rows, each strip column by column:
// row r, column c of a square at ((r >> 2) << (log2 n + 2)) + 4 c + (r & 3).
__global__ __launch_bounds__(kThreads) void haar_inv_tiles(const float* coef, const float* stage,
                                                           float* pix, int n, int logq, int G,
                                                           int64_t rs, int64_t cs, bool strips) {
  extern __shared__ float lds[];
  const int Q = 1 << logq;
  const int64_t blk = blockIdx.x;
  const int tile = int(blk % (G * G));
  const int64_t face = blk / (G * G);
  const int ty = tile / G, tx = tile % G;
  const float* f = coef + face * int64_t(n) * n;
  float* dst = pix + face * int64_t(n) * n;
  if (threadIdx.x == 0)
    lds[0] = (G == 1) ? f[0] : stage[face * int64_t(n) * n + ty * rs + tx * cs];
  __syncthreads();
  for (int B = Q; B >= 2; B >>= 1) {
    const int nb = Q / B, h = B >> 1, q = n / B;
    for (int e = threadIdx.x; e < nb * nb; e += kThreads) {
      const int br = e / nb, bc = e - br * nb;
      const int r0 = br * B, c0 = bc * B;
      const int gbr = ty * nb + br, gbc = tx * nb + bc;
      float a, b, c, d;
      inverse_butterfly(lds[r0 * Q + c0], f[int64_t(gbr) * n + q + gbc],
                        f[int64_t(q + gbr) * n + gbc], f[int64_t(q + gbr) * n + q + gbc], a, b,
                        c, d);
      lds[r0 * Q + c0] = a;
      lds[r0 * Q + c0 + h] = b;
      lds[(r0 + h) * Q + c0] = c;
      lds[(r0 + h) * Q + c0 + h] = d;
    }
    __syncthreads();
  }
  const int row0 = ty * Q, col0 = tx * Q;
  if (strips) {
    // consecutive threads write consecutive elements of a strip
    for (int e = threadIdx.x; e < Q * Q; e += kThreads) {
      const int st = e >> (logq + 2), c = (e >> 2) & (Q - 1), rl = e & 3;
      const int r = 4 * st + rl;
      dst[int64_t((row0 + r) >> 2) * 4 * n + 4 * (col0 + c) + rl] = lds[r * Q + c];
    }
  } else {
    for (int e = threadIdx.x; e < Q * Q; e += kThreads) {
      const int r = e >> logq, c = e & (Q - 1);
      dst[int64_t(row0 + r) * n + col0 + c] = lds[e];
    }
  }
}

}  // namespace

int launch_haar_forward(const float* pix, float* coef, int n, int64_t squares, hipStream_t s) {
  if (squares == 0) return RRT_OK;
  const int Q = n < kTile ? n : kTile;
  const int G = n / Q;
  const int64_t grid = squares * G * G;
  hipLaunchKernelGGL(haar_fwd_tiles, dim3(unsigned(grid)), dim3(kThreads),
                     size_t(Q) * Q * sizeof(float), s, pix, coef, n, ilog2(Q), G);
  int st = check_launch("haar_fwd_tiles");
  if (st || G == 1) return st;
  hipLaunchKernelGGL(haar_fwd_coarse, dim3(unsigned(squares)), dim3(64), 0, s, coef, n, G);
  return check_launch("haar_fwd_coarse");
}

int launch_haar_inverse(const float* coef, float* pix, int n, int64_t squares, hipStream_t s,
                        bool strips) {
  if (squares == 0) return RRT_OK;
  if (n < 4) strips = false;
  const int Q = n < kTile ? n : kTile;
  const int G = n / Q;
  // first texel of each output tile (also in strips: tile rows start strips)
  const int64_t rs = int64_t(Q) * n, cs = strips ? 4 * Q : Q;
  if (G > 1) {
    hipLaunchKernelGGL(haar_inv_coarse, dim3(unsigned(squares)), dim3(64), 0, s, coef, pix, n,
                       G, rs, cs);
    int st = check_launch("haar_inv_coarse");
    if (st) return st;
  }
  const int64_t grid = squares * G * G;
  hipLaunchKernelGGL(haar_inv_tiles, dim3(unsigned(grid)), dim3(kThreads),
                     size_t(Q) * Q * sizeof(float), s, coef, (const float*)pix, pix, n, ilog2(Q),
                     G, rs, cs, strips);
  return check_launch("haar_inv_tiles");
}

}  // namespace rrt
