// Host side of the C ABI (include/rrt.h): argument validation (always
// before any HIP call), workspace layout and dispatch to the kernels.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "rrt_internal.h"

namespace rrt {

static thread_local char g_last_error[512] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RRT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return RRT_OK;
}

static bool valid_n(int n, int lo) { return n >= lo && n <= 1024 && is_pow2(n); }

static bool block_scaled(int dtype) {
  return dtype == RRT_E4M3 || dtype == RRT_S16 || dtype == RRT_S11;
}
static bool transport_dtype_ok(int dtype) {
  return dtype == RRT_F32 || dtype == RRT_BF16 || block_scaled(dtype);
}

// The coefficient staging buffer and the FP32 source map (for either
// lighting dtype: binary16 lighting is its coefficients' precision; the map
// reconstructed from them is kept in binary32).
RelightWs relight_ws(int n) {
  const size_t cells = size_t(6) * n * n;
  RelightWs w;
  w.dense_off = 0;
  w.src_off = align256(cells * sizeof(float));
  w.total = w.src_off + align256(cells * sizeof(float));
  return w;
}

static int validate_light(const rrt_light* L) {
  if (!L) return fail(RRT_ERR_INVALID, "relight: null lighting descriptor");
  if (!valid_n(L->n, 2)) return fail(RRT_ERR_INVALID, "relight: n=%d not a power of two in [2,1024]", L->n);
  const int64_t cells = int64_t(6) * L->n * L->n;
  if (L->k < 1 || L->k > cells) return fail(RRT_ERR_INVALID, "relight: light k=%d not in [1,%lld]", L->k, (long long)cells);
  if (!L->idx || !L->val) return fail(RRT_ERR_INVALID, "relight: null lighting pointer");
  if (L->dtype != RRT_F32 && L->dtype != RRT_F16)
    return fail(RRT_ERR_UNSUPPORTED, "relight: lighting dtype %d (F32 or F16 only)", L->dtype);
  return RRT_OK;
}

static int check_ws(const void* ws, size_t ws_bytes, size_t need, const char* what) {
  if (!ws || ws_bytes < need)
    return fail(RRT_ERR_WORKSPACE, "%s: workspace %zu < %zu bytes", what, ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(RRT_ERR_INVALID, "%s: workspace not 256-byte aligned", what);
  return RRT_OK;
}

int validate_relight(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T) {
  if (!L || !R || !T) return fail(RRT_ERR_INVALID, "relight: null descriptor");
  const int vs = validate_light(L);
  if (vs) return vs;
  const int64_t cells = int64_t(6) * L->n * L->n;
  if (R->nframes < 1) return fail(RRT_ERR_INVALID, "relight: nframes=%d < 1", R->nframes);
  if (!R->frame_rot && R->nframes != 1)
    return fail(RRT_ERR_INVALID, "relight: frame_rot is NULL but nframes=%d", R->nframes);
  if (T->nvert < 0 || T->nvert > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "relight: nvert=%lld out of range", (long long)T->nvert);
  if (T->nnz < 1 || T->nnz > cells) return fail(RRT_ERR_INVALID, "relight: nnz=%d not in [1,%lld]", T->nnz, (long long)cells);
  if (T->nvert > 0 && !T->idx && T->nnz != cells)
    return fail(RRT_ERR_INVALID, "relight: dense transport (idx NULL) needs nnz = 6 n^2 = %lld", (long long)cells);
  if (T->nvert > 0 && (!T->val || !R->vert_rot))
    return fail(RRT_ERR_INVALID, "relight: null transport values or vertex rotations");
  if (!transport_dtype_ok(T->dtype))
    return fail(RRT_ERR_UNSUPPORTED, "relight: transport dtype %d (F32, BF16, E4M3, S16 or S11)", T->dtype);
  if (block_scaled(T->dtype) && !T->block_scale && T->nvert > 0)
    return fail(RRT_ERR_INVALID, "relight: block-scaled transport needs block_scale");
  if (T->cluster && (T->nclusters < 1 || !T->idx) && T->nvert > 0)
    return fail(RRT_ERR_INVALID, "relight: per-cluster supports need nclusters >= 1 and an idx table");
  if (int64_t(R->nframes) * T->nvert > (int64_t(1) << 40))
    return fail(RRT_ERR_INVALID, "relight: output too large");
  if (T->brdf && T->nmaterials < 1)
    return fail(RRT_ERR_INVALID, "relight: brdf needs nmaterials >= 1");
  if (T->brdf && (reinterpret_cast<uintptr_t>(T->brdf) & 15u))
    return fail(RRT_ERR_INVALID, "relight: brdf not 16-byte aligned");
  if (T->brdf && int64_t(T->nmaterials) * cells > (int64_t(1) << 40))
    return fail(RRT_ERR_INVALID, "relight: brdf table too large");
  return RRT_OK;
}

}  // namespace rrt

using namespace rrt;

extern "C" {

int rrt_abi_version(void) { return RRT_ABI_VERSION; }

const char* rrt_status_string(int status) {
  switch (status) {
    case RRT_OK: return "ok";
    case RRT_ERR_INVALID: return "invalid argument";
    case RRT_ERR_UNSUPPORTED: return "unsupported";
    case RRT_ERR_WORKSPACE: return "workspace too small";
    case RRT_ERR_DEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* rrt_last_error(void) { return g_last_error; }

int rrt_haar_forward(const float* pix, float* coef, int n, int64_t squares, void* stream) {
  if (!valid_n(n, 1)) return fail(RRT_ERR_INVALID, "haar_forward: n=%d not a power of two in [1,1024]", n);
  if (squares < 0) return fail(RRT_ERR_INVALID, "haar_forward: squares=%lld < 0", (long long)squares);
  if (squares == 0) return RRT_OK;
  if (!pix || !coef) return fail(RRT_ERR_INVALID, "haar_forward: null pointer");
  if (pix == coef) return fail(RRT_ERR_INVALID, "haar_forward: in-place transform not supported");
  if (squares * (n / (n < 128 ? n : 128)) * (n / (n < 128 ? n : 128)) > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "haar_forward: too many squares");
  return launch_haar_forward(pix, coef, n, squares, static_cast<hipStream_t>(stream));
}

int rrt_haar_inverse(const float* coef, float* pix, int n, int64_t squares, void* stream) {
  if (!valid_n(n, 1)) return fail(RRT_ERR_INVALID, "haar_inverse: n=%d not a power of two in [1,1024]", n);
  if (squares < 0) return fail(RRT_ERR_INVALID, "haar_inverse: squares=%lld < 0", (long long)squares);
  if (squares == 0) return RRT_OK;
  if (!pix || !coef) return fail(RRT_ERR_INVALID, "haar_inverse: null pointer");
  if (pix == coef) return fail(RRT_ERR_INVALID, "haar_inverse: in-place transform not supported");
  if (squares * (n / (n < 128 ? n : 128)) * (n / (n < 128 ? n : 128)) > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "haar_inverse: too many squares");
  return launch_haar_inverse(coef, pix, n, squares, static_cast<hipStream_t>(stream));
}

int rrt_topk_workspace(int64_t rows, int64_t len, int k, size_t* bytes) {
  if (!bytes) return fail(RRT_ERR_INVALID, "topk_workspace: null bytes");
  if (rows < 0 || len < 0 || k < 0 || k > len) return fail(RRT_ERR_INVALID, "topk_workspace: bad sizes");
  *bytes = topk_workspace_bytes(rows, len, k);
  return RRT_OK;
}

int rrt_topk(const float* x, int64_t rows, int64_t len, int k, int32_t* idx, float* val, void* ws,
             size_t ws_bytes, void* stream) {
  if (rows < 0 || rows > int64_t(0x7fffffff)) return fail(RRT_ERR_INVALID, "topk: rows=%lld out of range", (long long)rows);
  if (len < 0 || len >= (int64_t(1) << 31)) return fail(RRT_ERR_INVALID, "topk: len=%lld out of range", (long long)len);
  if (k < 0 || k > len) return fail(RRT_ERR_INVALID, "topk: k=%d not in [0,len=%lld]", k, (long long)len);
  if (rows == 0 || k == 0) return RRT_OK;
  if (!x || !idx || !val) return fail(RRT_ERR_INVALID, "topk: null pointer");
  const size_t need = topk_workspace_bytes(rows, len, k);
  if (need) {
    const int st = check_ws(ws, ws_bytes, need, "topk");
    if (st) return st;
  }
  return launch_topk(x, rows, len, k, idx, val, ws, static_cast<hipStream_t>(stream));
}

int rrt_coarsen_indices(const int32_t* idx, int64_t count, int n, int levels, int32_t* out,
                        void* stream) {
  if (!valid_n(n, 4)) return fail(RRT_ERR_INVALID, "coarsen: n=%d not a power of two in [4,1024]", n);
  if (levels < 1 || (n >> levels) < 2)
    return fail(RRT_ERR_INVALID, "coarsen: levels=%d needs 1 <= levels and n >> levels >= 2", levels);
  if (count < 0 || count >= (int64_t(1) << 40)) return fail(RRT_ERR_INVALID, "coarsen: bad count");
  if (count == 0) return RRT_OK;
  if (!idx || !out) return fail(RRT_ERR_INVALID, "coarsen: null pointer");
  return launch_coarsen_indices(idx, count, n, levels, out, static_cast<hipStream_t>(stream));
}

int rrt_haar_phase_shift_workspace(int n, int nrot, size_t* bytes) {
  if (!bytes) return fail(RRT_ERR_INVALID, "phase_shift_workspace: null bytes");
  if (!valid_n(n, 2) || nrot < 0) return fail(RRT_ERR_INVALID, "phase_shift_workspace: bad sizes");
  const size_t cells = size_t(6) * n * n;
  *bytes = align256(cells * sizeof(float)) + align256(cells * sizeof(float) * size_t(nrot));
  return RRT_OK;
}

int rrt_haar_phase_shift(const float* coef_in, int n, const float* rot, int nrot, float* coef_out,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!valid_n(n, 2)) return fail(RRT_ERR_INVALID, "phase_shift: n=%d not a power of two in [2,1024]", n);
  if (nrot < 0 || nrot > 65535 || int64_t(nrot) * 6 * n * n > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "phase_shift: nrot=%d out of range", nrot);
  if (nrot == 0) return RRT_OK;
  if (!coef_in || !rot || !coef_out) return fail(RRT_ERR_INVALID, "phase_shift: null pointer");
  size_t need = 0;
  rrt_haar_phase_shift_workspace(n, nrot, &need);
  if (!ws || ws_bytes < need)
    return fail(RRT_ERR_WORKSPACE, "phase_shift: workspace %zu < %zu bytes", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(RRT_ERR_INVALID, "phase_shift: workspace not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t cells = size_t(6) * n * n;
  float* pix = static_cast<float*>(ws);
  float* rotated = reinterpret_cast<float*>(static_cast<char*>(ws) + align256(cells * sizeof(float)));
  int st = launch_haar_inverse(coef_in, pix, n, 6, s);
  if (st) return st;
  st = launch_rotate_pixels(pix, rot, nrot, n, rotated, s);
  if (st) return st;
  return launch_haar_forward(rotated, coef_out, n, int64_t(6) * nrot, s);
}

int rrt_relight_workspace(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T,
                          unsigned flags, size_t* bytes) {
  (void)flags;
  if (!bytes) return fail(RRT_ERR_INVALID, "relight_workspace: null bytes");
  const int st = validate_relight(L, R, T);
  if (st) return st;
  *bytes = relight_ws(L->n).total;
  return RRT_OK;
}

}  // extern "C"

namespace rrt {

int check_relight_flags(const rrt_light* L, unsigned flags, const rrt_transport* T) {
  if (flags & ~(RRT_COMPENSATED | RRT_CHAIN_RULE))
    return fail(RRT_ERR_INVALID, "relight: unknown flags 0x%x", flags);
  if ((flags & RRT_CHAIN_RULE) && L->n < 32)
    return fail(RRT_ERR_UNSUPPORTED, "relight: chain rule needs n >= 32 (n=%d)", L->n);
  if ((flags & RRT_CHAIN_RULE) && T && T->brdf)
    return fail(RRT_ERR_UNSUPPORTED, "relight: chain rule with a brdf (triple product)");
  return RRT_OK;
}

}  // namespace rrt

extern "C" {

int rrt_relight_prepare(const rrt_light* L, unsigned flags, void* ws, size_t ws_bytes,
                        void* stream) {
  int st = validate_light(L);
  if (st) return st;
  st = check_relight_flags(L, flags);
  if (st) return st;
  const RelightWs w = relight_ws(L->n);
  st = check_ws(ws, ws_bytes, w.total, "relight_prepare");
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* dense = reinterpret_cast<float*>(base + w.dense_off);
  float* src = reinterpret_cast<float*>(base + w.src_off);
  st = launch_scatter_light(L->idx, L->val, L->dtype, L->k, L->n, 6, dense, s);
  if (st) return st;
  st = launch_haar_inverse(dense, src, L->n, 6, s, true);
  if (st || !(flags & RRT_CHAIN_RULE)) return st;
  // the staging buffer is free now: it takes the 2x2 block coefficients
  return launch_source_blocks(src, L->n, dense, s);
}

int rrt_relight_prepared(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T,
                         float* radiance, unsigned flags, const void* ws, size_t ws_bytes,
                         void* stream) {
  int st = validate_relight(L, R, T);
  if (st) return st;
  st = check_relight_flags(L, flags, T);
  if (st) return st;
  const RelightWs w = relight_ws(L->n);
  st = check_ws(ws, ws_bytes, w.total, "relight");
  if (st) return st;
  if (T->nvert > 0 && !radiance) return fail(RRT_ERR_INVALID, "relight: null radiance");
  if (T->nvert == 0) return RRT_OK;
  RelightLaunch a;
  a.src = reinterpret_cast<const float*>(static_cast<const char*>(ws) + w.src_off);
  a.vert_rot = R->vert_rot;
  a.frame_rot = R->frame_rot;
  a.t_idx = T->idx;
  a.t_val = T->val;
  a.t_scale = T->block_scale;
  a.cluster = T->cluster;
  a.nclusters = T->cluster ? T->nclusters : 0;
  a.t_dtype = T->dtype;
  a.nnz = T->nnz;
  a.nvert = T->nvert;
  a.nframes = R->nframes;
  a.n = L->n;
  a.flags = flags;
  a.out = radiance;
  a.blocks = static_cast<const char*>(ws) + w.dense_off;
  a.brdf = T->brdf;
  a.material = T->brdf ? T->material : nullptr;
  a.nmaterials = T->brdf ? T->nmaterials : 0;
  a.order = T->order;
  return launch_relight(a, static_cast<hipStream_t>(stream));
}

int rrt_relight_order_workspace(int64_t nvert, size_t* bytes) {
  if (!bytes) return fail(RRT_ERR_INVALID, "relight_order_workspace: null bytes");
  if (nvert < 0 || nvert > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "relight_order_workspace: nvert=%lld out of range", (long long)nvert);
  *bytes = relight_order_workspace_bytes(nvert);
  return RRT_OK;
}

int rrt_relight_order(const rrt_light* L, const rrt_transport* T, int32_t* order, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!L || !T) return fail(RRT_ERR_INVALID, "relight_order: null descriptor");
  if (!valid_n(L->n, 2)) return fail(RRT_ERR_INVALID, "relight_order: n=%d not a power of two in [2,1024]", L->n);
  if (T->nvert < 0 || T->nvert > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "relight_order: nvert=%lld out of range", (long long)T->nvert);
  if (T->nvert == 0) return RRT_OK;
  if (!order) return fail(RRT_ERR_INVALID, "relight_order: null order");
  if (T->nnz < 1) return fail(RRT_ERR_INVALID, "relight_order: nnz=%d < 1", T->nnz);
  if (T->cluster && (T->nclusters < 1 || !T->idx))
    return fail(RRT_ERR_INVALID, "relight_order: per-cluster supports need nclusters >= 1 and an idx table");
  int st = check_ws(ws, ws_bytes, relight_order_workspace_bytes(T->nvert), "relight_order");
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!T->idx) return launch_iota(order, T->nvert, s);   // dense rows: every vertex alike
  return launch_relight_order(T->idx, T->cluster, T->nclusters, T->nnz, T->nvert, L->n, order,
                              ws, s);
}

int rrt_relight(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T, float* radiance,
                unsigned flags, void* ws, size_t ws_bytes, void* stream) {
  // validate everything before enqueueing anything
  int st = validate_relight(L, R, T);
  if (st) return st;
  st = check_relight_flags(L, flags, T);
  if (st) return st;
  st = check_ws(ws, ws_bytes, relight_ws(L->n).total, "relight");
  if (st) return st;
  if (T->nvert > 0 && !radiance) return fail(RRT_ERR_INVALID, "relight: null radiance");
  st = rrt_relight_prepare(L, flags, ws, ws_bytes, stream);
  if (st) return st;
  return rrt_relight_prepared(L, R, T, radiance, flags, ws, ws_bytes, stream);
}

// Workspace of the lat-long relight: [dense staging 2H^2 float][source map
// 2H^2 float|half][rule tables 7H float]
struct LatLongWs {
  size_t dense_off, src_off, grid_off, total;
};

static LatLongWs latlong_ws(int H) {
  const size_t cells = size_t(2) * H * H;
  LatLongWs w;
  w.dense_off = 0;
  w.src_off = align256(cells * sizeof(float));
  w.grid_off = w.src_off + align256(cells * sizeof(float));
  w.total = w.grid_off + align256(size_t(latlong_grid_floats(H)) * sizeof(float));
  return w;
}

static int validate_latlong(const rrt_light* L, const rrt_latlong_rotations* R,
                            const rrt_transport* T) {
  if (!L || !R || !T) return fail(RRT_ERR_INVALID, "relight_latlong: null descriptor");
  if (!valid_n(L->n, 4) || L->n > 512)
    return fail(RRT_ERR_INVALID, "relight_latlong: H=%d not a power of two in [4,512]", L->n);
  const int64_t cells = int64_t(2) * L->n * L->n;
  if (L->k < 1 || L->k > cells)
    return fail(RRT_ERR_INVALID, "relight_latlong: light k=%d not in [1,%lld]", L->k, (long long)cells);
  if (!L->idx || !L->val) return fail(RRT_ERR_INVALID, "relight_latlong: null lighting pointer");
  if (L->dtype != RRT_F32 && L->dtype != RRT_F16)
    return fail(RRT_ERR_UNSUPPORTED, "relight_latlong: lighting dtype %d (F32 or F16 only)", L->dtype);
  if (T->nvert < 0 || T->nvert > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "relight_latlong: nvert=%lld out of range", (long long)T->nvert);
  if (T->nnz < 1 || T->nnz > cells)
    return fail(RRT_ERR_INVALID, "relight_latlong: nnz=%d not in [1,%lld]", T->nnz, (long long)cells);
  if (T->nvert > 0 && !T->idx && T->nnz != cells)
    return fail(RRT_ERR_INVALID, "relight_latlong: dense transport needs nnz = 2 H^2 = %lld", (long long)cells);
  if (T->nvert > 0 && (!T->val || !R->elev || !R->shift))
    return fail(RRT_ERR_INVALID, "relight_latlong: null transport values or rotations");
  if (!transport_dtype_ok(T->dtype))
    return fail(RRT_ERR_UNSUPPORTED, "relight_latlong: transport dtype %d", T->dtype);
  if (block_scaled(T->dtype) && !T->block_scale && T->nvert > 0)
    return fail(RRT_ERR_INVALID, "relight_latlong: block-scaled transport needs block_scale");
  if (T->cluster || T->brdf)
    return fail(RRT_ERR_UNSUPPORTED, "relight_latlong: cluster supports and brdf not supported");
  return RRT_OK;
}

int rrt_relight_latlong_workspace(const rrt_light* L, size_t* bytes) {
  if (!L || !bytes) return fail(RRT_ERR_INVALID, "relight_latlong_workspace: null argument");
  if (!valid_n(L->n, 4) || L->n > 512)
    return fail(RRT_ERR_INVALID, "relight_latlong: H=%d not a power of two in [4,512]", L->n);
  *bytes = latlong_ws(L->n).total;
  return RRT_OK;
}

int rrt_relight_latlong(const rrt_light* L, const rrt_latlong_rotations* R, const rrt_transport* T,
                        float* radiance, unsigned flags, void* ws, size_t ws_bytes, void* stream) {
  int st = validate_latlong(L, R, T);
  if (st) return st;
  if (flags & ~RRT_COMPENSATED)
    return fail(RRT_ERR_INVALID, "relight_latlong: flags 0x%x (only RRT_COMPENSATED)", flags);
  const LatLongWs w = latlong_ws(L->n);
  st = check_ws(ws, ws_bytes, w.total, "relight_latlong");
  if (st) return st;
  if (T->nvert > 0 && !radiance) return fail(RRT_ERR_INVALID, "relight_latlong: null radiance");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* dense = reinterpret_cast<float*>(base + w.dense_off);
  float* src = reinterpret_cast<float*>(base + w.src_off);
  float* grid = reinterpret_cast<float*>(base + w.grid_off);
  st = launch_scatter_light(L->idx, L->val, L->dtype, L->k, L->n, 2, dense, s);
  if (st) return st;
  st = launch_haar_inverse(dense, src, L->n, 2, s);
  if (st) return st;
  st = launch_latlong_grid(L->n, grid, s);
  if (st || T->nvert == 0) return st;
  RelightLaunch a;
  a.src = src;
  a.vert_rot = nullptr;
  a.frame_rot = nullptr;
  a.t_idx = T->idx;
  a.t_val = T->val;
  a.t_scale = T->block_scale;
  a.cluster = nullptr;
  a.nclusters = 0;
  a.t_dtype = T->dtype;
  a.nnz = T->nnz;
  a.nvert = T->nvert;
  a.nframes = 1;
  a.n = L->n;
  a.flags = flags;
  a.out = radiance;
  a.blocks = nullptr;
  a.brdf = nullptr;
  a.material = nullptr;
  a.nmaterials = 0;
  a.latlong = true;
  a.order = T->order;
  a.ll_elev = R->elev;
  a.ll_shift = R->shift;
  a.ll_grid = grid;
  return launch_relight(a, s);
}

int rrt_convert(const float* src, int64_t rows, int cols, int dtype, void* dst, float* block_scale,
                void* stream) {
  if (rows < 0 || cols < 0) return fail(RRT_ERR_INVALID, "convert: negative size");
  if (dtype != RRT_F16 && dtype != RRT_BF16 && !block_scaled(dtype))
    return fail(RRT_ERR_UNSUPPORTED, "convert: dtype %d (F16, BF16, E4M3, S16 or S11)", dtype);
  if (rows * int64_t(cols) > (int64_t(1) << 40)) return fail(RRT_ERR_INVALID, "convert: too large");
  if (rows == 0 || cols == 0) return RRT_OK;
  if (!src || !dst) return fail(RRT_ERR_INVALID, "convert: null pointer");
  if (block_scaled(dtype) && !block_scale)
    return fail(RRT_ERR_INVALID, "convert: block-scaled dtype needs block_scale");
  return launch_convert(src, rows, cols, dtype, dst, block_scale, static_cast<hipStream_t>(stream));
}

int rrt_mlp_encode(const float* pos_nrm, int64_t B, void* x, void* stream) {
  if (B < 0 || B > (int64_t(1) << 31) / RRT_MLP_IN) return fail(RRT_ERR_INVALID, "mlp_encode: B=%lld out of range", (long long)B);
  if (B == 0) return RRT_OK;
  if (!pos_nrm || !x) return fail(RRT_ERR_INVALID, "mlp_encode: null pointer");
  return launch_mlp_encode(pos_nrm, B, x, static_cast<hipStream_t>(stream));
}

int rrt_mlp_workspace(int64_t B, size_t* bytes) {
  if (!bytes) return fail(RRT_ERR_INVALID, "mlp_workspace: null bytes");
  if (B < 0 || B > (int64_t(1) << 31) / RRT_MLP_HIDDEN) return fail(RRT_ERR_INVALID, "mlp_workspace: B=%lld out of range", (long long)B);
  *bytes = mlp_workspace_bytes(B);
  return RRT_OK;
}

static int check_mlp_batch(int64_t B, const char* what) {
  if (B < 0 || B > (int64_t(1) << 31) / RRT_MLP_HIDDEN) return fail(RRT_ERR_INVALID, "%s: B=%lld out of range", what, (long long)B);
  return RRT_OK;
}

int rrt_mlp_pack(const void* w, void* w_dec, void* stream) {
  if (!w || !w_dec) return fail(RRT_ERR_INVALID, "mlp_pack: null pointer");
  const auto a = reinterpret_cast<uintptr_t>(w), b = reinterpret_cast<uintptr_t>(w_dec);
  const uintptr_t n = uintptr_t(RRT_MLP_WEIGHT_COUNT) * 2;
  if (a < b + n && b < a + n) return fail(RRT_ERR_INVALID, "mlp_pack: w and w_dec overlap");
  if ((a | b) % 16) return fail(RRT_ERR_INVALID, "mlp_pack: w and w_dec must be 16-byte aligned");
  return launch_mlp_pack(w, w_dec, static_cast<hipStream_t>(stream));
}

int rrt_mlp_decode(const void* w, const float* bias, const float* scale, int nclusters,
                   const float* pos_nrm, const int32_t* cluster, int64_t B, float* out,
                   void* stream) {
  int st = check_mlp_batch(B, "mlp_decode");
  if (st) return st;
  if (nclusters < 1) return fail(RRT_ERR_INVALID, "mlp_decode: nclusters=%d < 1", nclusters);
  if (B == 0) return RRT_OK;
  if (!w || !bias || !scale || !pos_nrm || !cluster || !out)
    return fail(RRT_ERR_INVALID, "mlp_decode: null pointer");
  if (reinterpret_cast<uintptr_t>(w) % 16) return fail(RRT_ERR_INVALID, "mlp_decode: weights not 16-byte aligned");
  return launch_mlp_decode(w, bias, scale, nclusters, pos_nrm, cluster, B, out,
                           static_cast<hipStream_t>(stream));
}

int rrt_mlp_forward(const void* w, const float* bias, const void* x, int64_t B, float* out,
                    void* ws, size_t ws_bytes, void* stream) {
  int st = check_mlp_batch(B, "mlp_forward");
  if (st) return st;
  if (B == 0) return RRT_OK;
  if (!w || !bias || !x || !out) return fail(RRT_ERR_INVALID, "mlp_forward: null pointer");
  if ((st = check_ws(ws, ws_bytes, mlp_workspace_bytes(B), "mlp_forward"))) return st;
  return launch_mlp_forward(w, bias, x, B, out, ws, static_cast<hipStream_t>(stream));
}

int rrt_mlp_backward(const void* w, const void* x, int64_t B, const float* dout, float* dw,
                     float* db, void* ws, size_t ws_bytes, void* stream) {
  int st = check_mlp_batch(B, "mlp_backward");
  if (st) return st;
  if (B < 1) return fail(RRT_ERR_INVALID, "mlp_backward: empty batch");
  if (!w || !x || !dout || !dw || !db) return fail(RRT_ERR_INVALID, "mlp_backward: null pointer");
  if ((st = check_ws(ws, ws_bytes, mlp_workspace_bytes(B), "mlp_backward"))) return st;
  return launch_mlp_backward(w, x, B, dout, dw, db, ws, static_cast<hipStream_t>(stream));
}

// Workspace of the learned relight, independent of V beyond one chunk:
// [relight workspace][values: one chunk of at most RRT_MLP_CHUNK vertices x
// 256 f32][order of one chunk][its workspace]
struct RelightMlpWs {
  size_t relight_total, values_off, order_off, order_ws_off, total;
};

// Vertices per chunk: the fewest chunks of at most RRT_MLP_CHUNK, equal in
// size (up to one vertex), so that no chunk's launch is a small tail.
static int64_t mlp_chunk(int64_t nvert) {
  if (nvert <= 0) return 0;
  const int64_t nch = (nvert + RRT_MLP_CHUNK - 1) / RRT_MLP_CHUNK;
  return (nvert + nch - 1) / nch;
}

static RelightMlpWs relight_mlp_ws(const rrt_light* L, int64_t nvert) {
  RelightMlpWs w;
  const int64_t chunk = mlp_chunk(nvert);
  w.relight_total = relight_ws(L->n).total;
  w.values_off = w.relight_total;
  w.order_off = w.values_off + align256(size_t(chunk) * RRT_MLP_OUT * sizeof(float));
  w.order_ws_off = w.order_off + align256(size_t(chunk) * sizeof(int32_t));
  w.total = w.order_ws_off + align256(relight_order_workspace_bytes(chunk));
  return w;
}

static int validate_relight_mlp(const rrt_light* L, const rrt_rotations* R, const rrt_mlp* M,
                                int64_t nvert, rrt_transport* T) {
  if (!M) return fail(RRT_ERR_INVALID, "relight_mlp: null decoder");
  if (nvert < 0 || nvert > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "relight_mlp: nvert=%lld out of range", (long long)nvert);
  if (!M->w || !M->bias || !M->support || !M->scale || M->nclusters < 1)
    return fail(RRT_ERR_INVALID, "relight_mlp: decoder needs weights, biases, supports, scales and nclusters >= 1");
  if (reinterpret_cast<uintptr_t>(M->w) % 16)
    return fail(RRT_ERR_INVALID, "relight_mlp: weights not 16-byte aligned");
  T->nvert = nvert;
  T->nnz = RRT_MLP_OUT;
  T->idx = M->support;
  T->val = nullptr;
  T->dtype = RRT_F32;
  T->block_scale = nullptr;
  T->cluster = nullptr;
  T->nclusters = M->nclusters;
  T->brdf = nullptr;
  T->material = nullptr;
  T->nmaterials = 0;
  T->order = nullptr;
  if (!L) return fail(RRT_ERR_INVALID, "relight_mlp: null lighting");
  const int st = validate_light(L);
  if (st) return st;
  if (RRT_MLP_OUT > int64_t(6) * L->n * L->n)
    return fail(RRT_ERR_INVALID, "relight_mlp: n=%d has fewer than %d coefficients", L->n, RRT_MLP_OUT);
  return RRT_OK;
}

int rrt_relight_mlp_workspace(const rrt_light* L, const rrt_rotations* R, int64_t nvert,
                              size_t* bytes) {
  if (!bytes) return fail(RRT_ERR_INVALID, "relight_mlp_workspace: null bytes");
  (void)R;
  if (!L) return fail(RRT_ERR_INVALID, "relight_mlp_workspace: null lighting");
  int st = validate_light(L);
  if (st) return st;
  if (nvert < 0 || nvert > int64_t(0x7fffffff))
    return fail(RRT_ERR_INVALID, "relight_mlp_workspace: nvert=%lld out of range", (long long)nvert);
  *bytes = relight_mlp_ws(L, nvert).total;
  return RRT_OK;
}

int rrt_relight_mlp(const rrt_light* L, const rrt_rotations* R, const rrt_mlp* M,
                    const float* pos_nrm, const int32_t* cluster, int64_t nvert,
                    float* radiance, unsigned flags, void* ws, size_t ws_bytes, void* stream) {
  rrt_transport T;
  int st = validate_relight_mlp(L, R, M, nvert, &T);
  if (st) return st;
  if (nvert > 0 && (!pos_nrm || !cluster))
    return fail(RRT_ERR_INVALID, "relight_mlp: null positions/normals or clusters");
  T.cluster = cluster;
  // validate everything (the values pointer is a placeholder) before enqueueing anything
  T.val = pos_nrm;
  st = validate_relight(L, R, &T);
  if (st) return st;
  st = check_relight_flags(L, flags, &T);
  if (st) return st;
  const RelightMlpWs w = relight_mlp_ws(L, nvert);
  st = check_ws(ws, ws_bytes, w.total, "relight_mlp");
  if (st) return st;
  if (nvert > 0 && !radiance) return fail(RRT_ERR_INVALID, "relight_mlp: null radiance");
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = rrt_relight_prepare(L, flags, ws, w.relight_total, stream);
  if (st || nvert == 0) return st;
  char* base = static_cast<char*>(ws);
  float* values = reinterpret_cast<float*>(base + w.values_off);
  int32_t* order = reinterpret_cast<int32_t*>(base + w.order_off);
  // Chunks of vertices: decode the chunk's values (one kernel: encoding,
  // the five layers, per-slot scales), order it heavy-first from its
  // cluster rows, relight it into its columns of radiance; the next chunk
  // reuses the same values (stream order), so the workspace does not grow
  // with V.
  const int64_t chunk = mlp_chunk(nvert);
  for (int64_t v0 = 0; v0 < nvert; v0 += chunk) {
    const int64_t C = nvert - v0 < chunk ? nvert - v0 : chunk;
    if ((st = launch_mlp_decode(M->w, M->bias, M->scale, M->nclusters, pos_nrm + v0 * 6,
                                cluster + v0, C, values, s)))
      return st;
    if ((st = launch_relight_order(M->support, cluster + v0, M->nclusters, RRT_MLP_OUT, C, L->n,
                                   order, base + w.order_ws_off, s)))
      return st;
    RelightLaunch a;
    a.src = reinterpret_cast<const float*>(base + relight_ws(L->n).src_off);
    a.vert_rot = R->vert_rot + v0 * 9;
    a.frame_rot = R->frame_rot;
    a.t_idx = M->support;
    a.t_val = values;
    a.t_scale = nullptr;
    a.cluster = cluster + v0;
    a.nclusters = M->nclusters;
    a.t_dtype = RRT_F32;
    a.nnz = RRT_MLP_OUT;
    a.nvert = C;
    a.nframes = R->nframes;
    a.n = L->n;
    a.flags = flags;
    a.out = radiance + v0;
    a.out_stride = nvert;
    a.blocks = base + relight_ws(L->n).dense_off;
    a.brdf = nullptr;
    a.material = nullptr;
    a.nmaterials = 0;
    a.order = order;
    if ((st = launch_relight(a, s))) return st;
  }
  return RRT_OK;
}

int rrt_mse(const float* out, const float* target, int64_t count, float* dout, double* loss,
            void* stream) {
  if (count < 0 || count > (int64_t(1) << 40)) return fail(RRT_ERR_INVALID, "mse: bad count");
  if (count == 0) return RRT_OK;
  if (!out || !target || !dout || !loss) return fail(RRT_ERR_INVALID, "mse: null pointer");
  return launch_mse(out, target, count, dout, loss, static_cast<hipStream_t>(stream));
}

int rrt_adam_step(float* param, void* param_bf16, float* m, float* v, const float* grad,
                  int64_t n, float lr, float beta1, float beta2, float eps, int step,
                  void* stream) {
  if (n < 0 || n > (int64_t(1) << 40)) return fail(RRT_ERR_INVALID, "adam: bad n");
  if (step < 1) return fail(RRT_ERR_INVALID, "adam: step=%d < 1", step);
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return fail(RRT_ERR_INVALID, "adam: bad hyper-parameters");
  if (n == 0) return RRT_OK;
  if (!param || !m || !v || !grad) return fail(RRT_ERR_INVALID, "adam: null pointer");
  return launch_adam(param, param_bf16, m, v, grad, n, lr, beta1, beta2, eps, step,
                     static_cast<hipStream_t>(stream));
}

}  // extern "C"
