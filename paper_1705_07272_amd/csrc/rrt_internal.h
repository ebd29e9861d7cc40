// Internal declarations shared by the host entry points and the kernels of
// librrt.so.  Not part of the public ABI (see include/rrt.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rrt.h"

namespace rrt {

// Records a message for rrt_last_error() and returns `status`.
int fail(int status, const char* fmt, ...);
// Maps the last HIP error of a launch to RRT_ERR_DEVICE (or RRT_OK).
int check_launch(const char* what);

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
inline int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace of relight: [dense staging 6n^2 float][source map 6n^2 float]
// (a binary32 map for either lighting dtype); after prepare the staging area
// holds the chain rule's 6 (n/2)^2 float4 blocks.
struct RelightWs {
  size_t dense_off, src_off, total;
};
RelightWs relight_ws(int n);
// Host-side validation of rrt_relight's descriptors and flags (abi.cpp); a
// non-zero return has recorded the message for rrt_last_error().
int validate_relight(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T);
int check_relight_flags(const rrt_light* L, unsigned flags, const rrt_transport* T = nullptr);

// Haar transform launchers (haar.hip).
// squares: number of n x n squares (a cube map is 6, a longitude-latitude map 2)
int launch_haar_forward(const float* pix, float* coef, int n, int64_t squares, hipStream_t s);
// strips: write the pixels in strips of four rows (the cube-map relight's
// source-map layout, n >= 4; see strip_offset in geometry.h) instead of
// row-major order
int launch_haar_inverse(const float* coef, float* pix, int n, int64_t squares, hipStream_t s,
                        bool strips = false);

// Selection (topk.hip).
size_t topk_workspace_bytes(int64_t rows, int64_t len, int k);
int launch_topk(const float* x, int64_t rows, int64_t len, int k, int32_t* idx, float* val,
                void* ws, hipStream_t s);

// Coefficient scatter into a zeroed dense map (relight.hip).
// squares: 6 (cube map) or 2 (longitude-latitude map)
int launch_scatter_light(const int32_t* idx, const void* val, int dtype, int k, int n, int squares,
                         float* dense, hipStream_t s);
// Pixel-domain rotation of one map for a batch of rotations (relight.hip).
int launch_rotate_pixels(const float* src, const float* rot, int nrot, int n, float* dst,
                         hipStream_t s);

struct RelightLaunch {
  const float* src;         // [6][n][n] source map, in strips of four rows for n >= 4
                            // (row-major for n < 4 and for the [2][n][n] lat-long map)
  const float* vert_rot;    // [V][9]
  const float* frame_rot;   // [F][9] or nullptr
  const int32_t* t_idx;     // [V][nnz] or nullptr (dense)
  const void* t_val;        // [V][nnz]
  const float* t_scale;     // [V][nblk] (E4M3 / S16) or nullptr
  const int32_t* cluster;   // [V] or nullptr (then t_idx is [C][nnz])
  int nclusters;
  int t_dtype;
  int nnz;
  int64_t nvert;
  int nframes;
  int n;
  unsigned flags;
  float* out;               // [F][out_stride]: out[f * out_stride + v]
  int64_t out_stride = 0;   // 0: nvert
  const void* blocks;       // chain rule: float4 (S, H, V, D) per 2x2 source block
  const float* brdf;        // triple product: [M][6 n^2] texel factor, or NULL
  const int32_t* material;  // [V] row of brdf, or NULL (row 0)
  int nmaterials;
  const int32_t* order = nullptr;    // [V] processing order, or nullptr
  // longitude-latitude map (then vert_rot, frame_rot, cluster, brdf unused, nframes = 1)
  bool latlong = false;
  const float* ll_elev = nullptr;    // [V][2] (cos b, sin b)
  const int32_t* ll_shift = nullptr; // [V][2] (s_a, s_c)
  const float* ll_grid = nullptr;    // latlong_grid_floats(n) binary32 tables
};
// Tables of the longitude-latitude rule: row sines, row cosines [H], column
// sines, column cosines [2H], boundary cosines [H]; 7 H floats.
inline int latlong_grid_floats(int H) { return 7 * H; }
int launch_latlong_grid(int H, float* grid, hipStream_t s);
int launch_source_blocks(const float* src, int n, float* blocks, hipStream_t s);
int launch_coarsen_indices(const int32_t* idx, int64_t count, int n, int levels, int32_t* out,
                           hipStream_t s);
int launch_relight(const RelightLaunch& a, hipStream_t s);
// Heavy-first processing order (faces touched by each row, most first).
size_t relight_order_workspace_bytes(int64_t nvert);
int launch_iota(int32_t* out, int64_t count, hipStream_t s);
int launch_relight_order(const int32_t* idx, const int32_t* cluster, int nclusters, int nnz,
                         int64_t nvert, int n, int32_t* order, void* ws, hipStream_t s);

// Learned decoder (mlp.hip).
size_t mlp_workspace_bytes(int64_t B);
int launch_mlp_encode(const float* in, int64_t B, void* out, hipStream_t s);
int launch_mlp_pack(const void* w, void* out, hipStream_t s);
// The whole decoder in one kernel (encode, five layers, per-slot scales):
// out [B][256] values, bit-identical to encode + launch_mlp_forward + the
// per-slot scaling in binary32.
int launch_mlp_decode(const void* w, const float* b, const float* scale, int C,
                      const float* pos_nrm, const int32_t* cluster, int64_t B, float* out,
                      hipStream_t s);
// Keeps every layer's pre-activation in ws for a backward pass.
int launch_mlp_forward(const void* w, const float* b, const void* x, int64_t B, float* out,
                       void* ws, hipStream_t s);
int launch_mlp_backward(const void* w, const void* x, int64_t B, const float* dout, float* dw,
                        float* db, void* ws, hipStream_t s);
int launch_mse(const float* out, const float* tgt, int64_t count, float* dout, double* loss,
               hipStream_t s);
int launch_adam(float* p, void* p_bf16, float* m, float* v, const float* g, int64_t n, float lr,
                float b1, float b2, float eps, int step, hipStream_t s);

// Storage conversion (convert.hip).
int launch_convert(const float* src, int64_t rows, int cols, int dtype, void* dst,
                   float* scale, hipStream_t s);

}  // namespace rrt
