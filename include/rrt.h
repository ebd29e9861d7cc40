/*
 * rrt.h -- run-time Haar-domain relighting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of librrt.so.  The operations follow the paper's statement of the
 * problem (Alnasser & Foroosh, "Non-Linear Phase-Shifting of Haar Wavelets
 * for Run-Time All-Frequency Lighting"): lighting and transport are
 * represented by non-standard 2-D Haar coefficients (Sec. III, Sec. V.B);
 * the lighting is rotated into each vertex's local frame directly in the
 * Haar domain (Sec. V.A: the rotated map is g(w) = f(R w); Sec. V.B/V.C:
 * coefficients of every coarser level follow from the finest one by
 * 2x2 averaging and downsampling); outgoing radiance is the inner product of
 * the rotated lighting with the vertex's transfer coefficients (Sec. III,
 * transfer function; Sec. V.C, last algorithm step).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Data pointers are DEVICE pointers owned by the caller.  The library
 *    never frees or retains them.  Host-side descriptor structs are read
 *    during the call only.  Buffers must stay alive until the work queued
 *    on `stream` has completed.
 *  - Every call enqueues asynchronously on `stream` (a hipStream_t passed as
 *    void*; NULL = the null stream) and returns a status: RRT_OK (0) or a
 *    positive rrt_status.  Arguments are validated on the host before any
 *    HIP call is made, so an error return means nothing was enqueued
 *    (except RRT_ERR_DEVICE, reported when a launch itself fails).
 *    rrt_last_error() returns a thread-local message for the last failure.
 *    Nothing aborts and no exception crosses the ABI.
 *  - Device-side data is never trusted for addressing: out-of-range indices
 *    and malformed rotations give unspecified VALUES for the affected
 *    results but never an out-of-bounds access.
 *  - A cube map is [6][n][n] (row-major), n = 2^k with 1 <= n <= 1024
 *    (the rotating calls, phase shift and relight, need n >= 2).  Faces 0..5 are +X,-X,+Y,-Y,+Z,-Z.
 *    Texel (i, j) has U = 2j+1-n, V = 2i+1-n and centre direction
 *      +X ( n,-V,-U)  -X (-n,-V, U)  +Y ( U, n, V)
 *      -Y ( U,-n,-V)  +Z ( U,-V, n)  -Z (-U,-V,-n).
 *  - Coefficients: orthonormal non-standard 2-D Haar of each face, Mallat
 *    quadrant layout (S/H/V/D of a level in the top-left/top-right/
 *    bottom-left/bottom-right quadrants of the current corner;
 *    H = left-right, V = top-bottom, D = mixed, each /2 per 2x2 step).
 *    The flat coefficient index is face*n*n + row*n + col (int32).
 *  - A rotation is a row-major 3x3 float32 matrix R mapping local directions
 *    to the lighting's frame; the rotated lighting is g(w) = L(R w), sampled
 *    at texel centres with the nearest source texel.  For an n x n map R
 *    is quantised to R_q = rint(R * 2^k), k = 22 - log2(n) (entries of R
 *    in [-1, 1]; for other matrices the source texels are unspecified but
 *    always inside the map), and the source texel is found in exact integer
 *    arithmetic (major axis, ties to the lower axis; column
 *    j' = min(n-1, floor(n (sc + |d_a|) / (2 |d_a|))), row likewise), so
 *    results do not depend on floating-point evaluation order.
 */
#ifndef RRT_H
#define RRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 3: rotations quantised at 2^(22 - log2 n) instead of 2^20 (same calls,
   slightly different source texels for general rotations).
   4: transport dtype RRT_S11 (packed 11-bit block-scaled fixed point).
   5: rrt_mlp_decode and rrt_relight_mlp take the weights in the decoder
   layout of rrt_mlp_pack.
   6: the source map is binary32 for RRT_F16 lighting too (its workspace is
   that of RRT_F32 lighting; results closer to the FP64 reference). */
#define RRT_ABI_VERSION 6

typedef enum {
  RRT_OK = 0,
  RRT_ERR_INVALID = 1,      /* bad argument (null pointer, size, alignment) */
  RRT_ERR_UNSUPPORTED = 2,  /* valid but not implemented (dtype/size combination) */
  RRT_ERR_WORKSPACE = 3,    /* workspace missing or smaller than *_workspace() reported */
  RRT_ERR_DEVICE = 4        /* a HIP launch or runtime call failed */
} rrt_status;

typedef enum {
  RRT_F32 = 0,   /* IEEE binary32 */
  RRT_F16 = 1,   /* IEEE binary16 */
  RRT_BF16 = 2,  /* bfloat16 (upper half of binary32) */
  RRT_E4M3 = 3,  /* OCP FP8 E4M3FN (bias 7, max 448, no infinities) with
                    one float32 scale per block of RRT_BLOCK values */
  RRT_S16 = 4,   /* int16 fixed point with one float32 scale per block of
                    RRT_BLOCK values: value = code * scale */
  RRT_S11 = 5    /* 11-bit two's-complement fixed point, codes in
                    [-1023, 1023], one float32 scale per block of RRT_BLOCK
                    values (value = code * scale), packed: a row of nnz
                    values is RRT_S11_WORDS(nnz) uint32 words, value e in
                    bits [11 e, 11 e + 11) of the row's bit stream (bit b in
                    bit b % 32 of word b / 32); bits past the last value are
                    zero.  A block of 64 values fills exactly 22 words, so
                    a row costs 1.4375 bytes per value with its scales. */
} rrt_dtype;

/* Values per scale block of the block-scaled forms (RRT_E4M3, RRT_S16, RRT_S11). */
#define RRT_BLOCK 64
/* uint32 words of one packed RRT_S11 row of nnz values. */
#define RRT_S11_WORDS(nnz) ((11 * (int64_t)(nnz) + 31) / 32)

/* Flags of rrt_relight. */
#define RRT_COMPENSATED 1u  /* Neumaier-compensated accumulation of the dot */
#define RRT_CHAIN_RULE 2u   /* finest level rotated by the chain rule on the
                               source's 2x2 blocks (Sec. V.A-V.B, eq:pde1 to
                               eq:pde3) instead of the exact resampling; the
                               coarser levels follow by the pyramid.  n >= 32
                               and no brdf only (else RRT_ERR_UNSUPPORTED). */

int rrt_abi_version(void);
const char* rrt_status_string(int status);
const char* rrt_last_error(void);

/* ------------------------------------------------------------------------
 * Haar transform of square maps (representation, Sec. III / Sec. V.B):
 * every n x n square is transformed on its own (a cube map is 6 squares,
 * one per face; a longitude-latitude map 2).
 *   pix, coef: [squares][n][n] float32, may not overlap.
 *   squares >= 0 (0 = no-op), 1 <= n <= 1024, n a power of two.
 *   No workspace: for n > 64 the work is split into 64 x 64 tiles plus
 *   one coarse pass, and the tile sums between the two launches are staged
 *   in the output buffer itself.
 * --------------------------------------------------------------------- */
int rrt_haar_forward(const float* pix, float* coef, int n, int64_t squares, void* stream);
int rrt_haar_inverse(const float* coef, float* pix, int n, int64_t squares, void* stream);

/* ------------------------------------------------------------------------
 * Non-linear approximation (Sec. III, Haar-domain methods): keep the k
 * entries of largest magnitude of each row.
 *   x [rows][len] float32; idx [rows][k] int32 and val [rows][k] float32
 *   receive the kept positions in ascending order and their values.
 *   Ties in |x| go to the lower position.  NaN inputs: unspecified choice.
 *   0 <= k <= len, len < 2^31.  Workspace: rrt_topk_workspace() bytes,
 *   256-byte aligned: zero except for at most 8 rows of at least 16384
 *   values with k < len (per-chunk histograms and a candidate list, about
 *   8 len + 1 MiB bytes per row); too small a workspace is
 *   RRT_ERR_WORKSPACE.
 * --------------------------------------------------------------------- */
int rrt_topk_workspace(int64_t rows, int64_t len, int k, size_t* bytes);
int rrt_topk(const float* x, int64_t rows, int64_t len, int k, int32_t* idx, float* val,
             void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Dense Haar-domain rotation (the non-linear phase shift, Sec. V.A-V.C):
 *   coef_out[r] = W S(R_r) W^T coef_in  for r < nrot.
 *   coef_in [6][n][n], rot [nrot][9], coef_out [nrot][6][n][n] float32.
 *   Workspace: rrt_haar_phase_shift_workspace() bytes (256-byte aligned).
 * --------------------------------------------------------------------- */
int rrt_haar_phase_shift_workspace(int n, int nrot, size_t* bytes);
int rrt_haar_phase_shift(const float* coef_in, int n, const float* rot, int nrot,
                         float* coef_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Relighting: radiance[f][v] = sum_k T_v[k] (W S(R_fv) W^T L)[k]
 * (Sec. III transfer-function inner product with the lighting rotated into
 * the vertex frame, Sec. V.A-V.C; rotate, recurse, integrate).
 * --------------------------------------------------------------------- */
typedef struct {
  int n;                 /* face side, 2 <= n <= 1024, power of two */
  int k;                 /* kept lighting coefficients, 1 <= k <= 6 n^2 */
  const int32_t* idx;    /* [k] flat coefficient indices (any order; out-of-range
                            entries ignored; duplicates: one of them wins) */
  const void* val;       /* [k] values, dtype RRT_F32 or RRT_F16 */
  int dtype;             /* rrt_dtype of val (the source map reconstructed
                            from the coefficients is binary32 either way) */
} rrt_light;

typedef struct {
  int64_t nvert;         /* vertices V >= 0 */
  int nnz;               /* coefficients per vertex, 1 <= nnz <= 6 n^2 */
  const int32_t* idx;    /* [V][nnz] flat indices in the vertex's local frame,
                            or NULL for dense rows (then nnz must be 6 n^2 and
                            entry e is coefficient e); out-of-range ignored */
  const void* val;       /* [V][nnz] values of dtype ([V][RRT_S11_WORDS(nnz)]
                            uint32 words for RRT_S11) */
  int dtype;             /* RRT_F32, RRT_BF16, RRT_E4M3, RRT_S16 or RRT_S11 */
  const float* block_scale; /* RRT_E4M3 / RRT_S16 / RRT_S11: [V][ceil(nnz/64)]
                            scales, value = code * scale; otherwise ignored */
  const int32_t* cluster;   /* NULL, or [V] cluster of each vertex: then idx is a
                            per-cluster support table [C][nnz] and vertex v uses
                            row cluster[v] (values stay per vertex);
                            out-of-range clusters contribute nothing */
  int nclusters;            /* C when cluster != NULL */
  const float* brdf;        /* NULL (double product), or the triple product
                               (Sec. III, eq:tripleSum): [M][6 n^2] float32
                               texel-domain BRDF x cosine x solid angle in the
                               local frame (16-byte aligned); the rotated
                               lighting is multiplied by row material[v] texel
                               by texel before the transform, which evaluates
                               sum_ijk C_ijk a_i b_j c_k with a the rotated
                               lighting, b the Haar coefficients of that row
                               and c = the vertex's row (its visibility) */
  const int32_t* material;  /* with brdf: NULL (row 0 for every vertex) or
                               [V] row of each vertex; rows outside [0, M)
                               give radiance 0 */
  int nmaterials;           /* M >= 1 when brdf != NULL */
  const int32_t* order;     /* NULL (vertices in index order) or [V] a
                               permutation of 0..V-1: the order in which the
                               vertices are processed (e.g. rrt_relight_order);
                               results do not depend on it, only the time
                               does; entries outside [0, V) are skipped */
} rrt_transport;

typedef struct {
  int nframes;           /* F >= 1 */
  const float* frame_rot;/* [F][9] object rotations, or NULL (then F must be 1
                            and R_v is used as is) */
  const float* vert_rot; /* [V][9] vertex frames (local -> object) */
} rrt_rotations;
/* R_fv = (R_q(frame f) R_q(vertex v) + 2^(k-1)) >> k, k = 22 - log2(n),
   entry-wise in exact integer arithmetic (flooring shift). */

/* Workspace: the reconstructed source map (6 n^2 float32 values) plus a
   6 n^2 float32 staging buffer (after prepare with RRT_CHAIN_RULE: the
   source's 2x2 block coefficients, float32 (S, H, V, D) per block),
   256-byte aligned.  Only L->n matters for its size. */
int rrt_relight_workspace(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T,
                          unsigned flags, size_t* bytes);
/* radiance: [F][V] float32 (frame-major).  Equivalent to
   rrt_relight_prepare followed by rrt_relight_prepared. */
int rrt_relight(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T,
                float* radiance, unsigned flags, void* ws, size_t ws_bytes, void* stream);

/* rrt_relight without caller memory, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, validation, kernels
   and results as rrt_relight; the workspace is instead a device array of
   RRT_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from the
   first use until the process ends (looked up once per device, with that
   device current).  It uses the current device's array, so `stream` must
   belong to the current device.  The call allocates nothing and never
   calls hipMalloc / hipFree.
     Limit: the relight workspace of rrt_relight_workspace() must fit the
   array: n <= 256 (n = 512 and 1024 return RRT_ERR_UNSUPPORTED before any
   HIP call).
     Every call on a GPU shares that GPU's array: calls that overlap in time
   on one GPU (on different streams, or from different threads without
   ordering) race and give unspecified results; calls ordered on one stream
   are safe.  Nothing depends on what an earlier call left in the array. */
#define RRT_NOALLOC_SCRATCH_BYTES (4u << 20)
int rrt_relight_noalloc(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T,
                        float* radiance, unsigned flags, void* stream);

/* Processing order for rrt_relight: the vertices sorted by the number of
   cube faces their rows touch, most first (a vertex's work grows with it),
   so that the expensive vertices do not start last.  Within a face count
   the order is unspecified.  Reads T->idx (or T->cluster's support rows);
   dense rows (idx NULL) give the index order.  order [V] int32.
   Workspace: rrt_relight_order_workspace() bytes (256-byte aligned). */
int rrt_relight_order_workspace(int64_t nvert, size_t* bytes);
int rrt_relight_order(const rrt_light* L, const rrt_transport* T, int32_t* order, void* ws,
                      size_t ws_bytes, void* stream);

/* The two halves of rrt_relight, for relighting many vertex batches or
   frame sets under one lighting:
   prepare  -- source reconstruction P = W^T L into the workspace (once per
               lighting; Sec. V.B levels read in reverse); with
               RRT_CHAIN_RULE in flags also the 2x2 block coefficients of P
               that the chain rule reads (RRT_COMPENSATED is accepted and
               ignored, so the flags of prepared may be passed as they are);
   prepared -- the per-vertex rotation and inner product reading P from a
               workspace filled by prepare with the same L->n and L->dtype,
               and with RRT_CHAIN_RULE if prepared is given it (the
               workspace is only read, so several calls may share it). */
int rrt_relight_prepare(const rrt_light* L, unsigned flags, void* ws, size_t ws_bytes,
                        void* stream);
int rrt_relight_prepared(const rrt_light* L, const rrt_rotations* R, const rrt_transport* T,
                         float* radiance, unsigned flags, const void* ws, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------------------------
 * Relighting on the longitude-latitude map (Sec. V.A; the elevation rotation
 * plus azimuth shift of its last paragraphs).  The map has H rows (elevation
 * t from +Y) and W = 2H columns (azimuth f), texel (i, j) spans
 * [i, i+1) x [j, j+1) in units of pi/H; it is stored as two H x H squares,
 * square s holding columns s H .. s H + H - 1, each with its own Haar
 * transform, so L->idx and T->idx index [2][H][H] (L->n = H).
 * Vertex v's rotation is R_v = R_y(s_a pi/H) R_x(b) R_y(s_c pi/H) (R_y
 * adds to the azimuth; R_x = [[1,0,0],[0,cos b,-sin b],[0,sin b,cos b]]):
 *   radiance[v] = sum_k T_v[k] (W g_v)[k],  g_v(i, j) = P(source(i, j)),
 * P = W^T L, and source(i, j) the texel of R_x(b) p(i, j + s_c) shifted by
 * s_a columns, p = (sin t sin f, cos t, sin t cos f) at the texel centre.
 * The texel of R_x(b) p is decided in binary32 by one fixed sequence of
 * rounded operations: p from binary32 sines and cosines of the centres,
 * q_y = cb p_y - sb p_z, q_z = sb p_y + cb p_z, rho = sqrt(q_x^2 + q_z^2),
 * row = #{0 < k < H : q_y <= C_k}, c = #{0 < k < H : q_z <= C_k rho} with
 * C_k = binary32 cos(k pi / H), column = c if q_x >= 0 else W - 1 - c.
 *   H: power of two in [4, 512]; transport as rrt_transport without
 *   cluster or brdf; flags: RRT_COMPENSATED only; radiance [V] float32.
 *   Workspace: rrt_relight_latlong_workspace() bytes, 256-byte aligned:
 *   [2 H^2 float32 staging][source map 2 H^2 float32][7 H float32
 *   tables: sin, cos of the row centres (H each), sin, cos of the column
 *   centres (2H each), C_k (H)], each part starting 256-byte aligned.
 * --------------------------------------------------------------------- */
typedef struct {
  const float* elev;     /* [V][2] (cos b, sin b) of R_x(b), binary32 */
  const int32_t* shift;  /* [V][2] (s_a, s_c) in columns, any integers (mod 2H) */
} rrt_latlong_rotations;

int rrt_relight_latlong_workspace(const rrt_light* L, size_t* bytes);
int rrt_relight_latlong(const rrt_light* L, const rrt_latlong_rotations* R,
                        const rrt_transport* T, float* radiance, unsigned flags, void* ws,
                        size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Storage conversion of coefficient values (reduced-precision forms).
 *   src [rows][cols] float32 -> dst [rows][cols] of dtype
 *   ([rows][RRT_S11_WORDS(cols)] uint32 words for RRT_S11):
 *   RRT_F16, RRT_BF16: round to nearest even;
 *   RRT_E4M3, RRT_S16, RRT_S11: per block of RRT_BLOCK values of a row,
 *   with m = max|x| of the block and M = 448 (E4M3), 32767 (S16) or 1023
 *   (S11): scale = m / M (1 if the block is all zero), stored in
 *   block_scale [rows][ceil(cols/64)]; code = round-to-nearest-even of
 *   x * (M / m), saturated to +-M.
 * --------------------------------------------------------------------- */
int rrt_convert(const float* src, int64_t rows, int cols, int dtype, void* dst,
                float* block_scale, void* stream);

/* ------------------------------------------------------------------------
 * Rotation started below the finest level (Sec. V.C, remark after the
 * algorithm: starting `levels` levels coarser divides the rotation work by
 * 4^levels).
 *   out[i] = index at resolution n >> levels of coefficient idx[i] at
 *   resolution n (same face, same Mallat row and column), or -1 when the
 *   coefficient belongs to one of the `levels` finest levels or idx[i] is
 *   outside [0, 6 n^2).  Relighting at n >> levels with the remapped
 *   lighting and transport indices (-1 entries are ignored) rotates the
 *   coarser levels only: the map of 2^levels x 2^levels block sums divided
 *   by 2^levels has exactly those coefficients.
 *   idx, out: [count] int32 device arrays (may be the same array);
 *   n a power of two in [4, 1024], 1 <= levels and n >> levels >= 2.
 * --------------------------------------------------------------------- */
int rrt_coarsen_indices(const int32_t* idx, int64_t count, int n, int levels, int32_t* out,
                        void* stream);

/* ------------------------------------------------------------------------
 * Learned transport decoder (not part of the paper): an MLP maps a vertex's
 * position and normal to its transport values on a per-cluster support.
 *   encode:  gamma(x) = (x, sin(2^k pi x), cos(2^k pi x), k = 0..7) of the 6
 *            inputs (position scaled to [-1,1], unit normal), 102 features
 *            zero-padded to RRT_MLP_IN, stored bfloat16 [B][128]; feature
 *            order: the six inputs, then per band six sines, six cosines.
 *   layers:  z = W a + b; gelu (tanh form) after each of the 4 hidden layers
 *            of width 256; linear output layer of width 256.  Weights are
 *            bfloat16, packed layer after layer, each [out][in] row-major
 *            (RRT_MLP_WEIGHT_COUNT values); biases float32 packed likewise
 *            (RRT_MLP_BIAS_COUNT).  Products accumulate in FP32 on the
 *            matrix cores.
 * --------------------------------------------------------------------- */
#define RRT_MLP_IN 128
#define RRT_MLP_HIDDEN 256
#define RRT_MLP_OUT 256
#define RRT_MLP_WEIGHTS 5
#define RRT_MLP_WEIGHT_COUNT 294912
#define RRT_MLP_BIAS_COUNT 1280

/* pos_nrm [B][6] float32 -> x [B][128] bfloat16. */
int rrt_mlp_encode(const float* pos_nrm, int64_t B, void* x, void* stream);
/* Activation workspace for a batch of B rows (256-byte aligned). */
int rrt_mlp_workspace(int64_t B, size_t* bytes);
/* out [B][256] float32.  Keeps the activations of this batch in ws for a
   following rrt_mlp_backward on the same batch. */
int rrt_mlp_forward(const void* w, const float* bias, const void* x, int64_t B, float* out,
                    void* ws, size_t ws_bytes, void* stream);
/* Decoder weight layout: w_dec receives the RRT_MLP_WEIGHT_COUNT bfloat16
   weights w (row-major per layer, as above) reordered for the matrix-core
   operands of rrt_mlp_decode.  Each layer keeps its offset and size; inside
   it, the operand of rows 32 t .. 32 t + 31 at inputs 16 s .. 16 s + 15 is
   the 512 values at (t * K / 16 + s) * 512 (K = the layer's inputs), value
   8 (m + 32 h) + e holding w[32 t + m][16 s + 8 h + e] (m < 32, h < 2,
   e < 8), so that a wave reads it as one contiguous 1 KiB.  w and w_dec
   are 16-byte aligned device buffers that do not overlap. */
int rrt_mlp_pack(const void* w, void* w_dec, void* stream);
/* Inference of the whole decoder in one kernel, for the transport values of
   B vertices: values[v][j] = out(encode(pos_nrm[v]))[j] * scale[cluster[v]][j]
   (0 for a cluster outside [0, nclusters)).  w_dec: the weights in the
   decoder layout (rrt_mlp_pack), 16-byte aligned; pos_nrm [B][6] float32,
   cluster [B] int32, scale [nclusters][256] float32, values [B][256]
   float32.  No workspace: each 512-thread workgroup keeps the activations
   of 64 vertices in LDS and reads the weights from global memory.  The
   values are bit-identical to rrt_mlp_encode + rrt_mlp_forward (row-major
   weights) followed by the scaling in binary32. */
int rrt_mlp_decode(const void* w_dec, const float* bias, const float* scale, int nclusters,
                   const float* pos_nrm, const int32_t* cluster, int64_t B, float* values,
                   void* stream);
/* Gradients of a scalar whose gradient with respect to out is dout [B][256]:
   dw [RRT_MLP_WEIGHT_COUNT] (overwritten), db [RRT_MLP_BIAS_COUNT]
   (overwritten).  ws must hold the activations of rrt_mlp_forward on the
   same w, x and B. */
int rrt_mlp_backward(const void* w, const void* x, int64_t B, const float* dout, float* dw,
                     float* db, void* ws, size_t ws_bytes, void* stream);
/* Mean squared error: dout = 2 (out - target) / count; *loss (a device
   double) += sum (out - target)^2 / count. */
int rrt_mse(const float* out, const float* target, int64_t count, float* dout, double* loss,
            void* stream);
/* One Adam step on n parameters (FP32 master, moments m and v); also writes
   the bfloat16 copy when param_bf16 is not NULL.  step >= 1. */
int rrt_adam_step(float* param, void* param_bf16, float* m, float* v, const float* grad,
                  int64_t n, float lr, float beta1, float beta2, float eps, int step,
                  void* stream);

/* ------------------------------------------------------------------------
 * Relighting with the learned transport: every vertex's values are decoded
 * by the network on its cluster's support, then relit as by rrt_relight.
 *   values[v][j] = out(encode(pos_nrm[v]))[j] * scale[cluster[v]][j]
 *   (0 for a cluster outside [0, C)), then rrt_relight with the transport
 *   {nvert, nnz = RRT_MLP_OUT, idx = support (per-cluster table),
 *   val = values (RRT_F32), cluster, nclusters = C}.
 *   pos_nrm [V][6] float32, cluster [V] int32; radiance [F][V] float32;
 *   flags as rrt_relight.  The decoded values are those of rrt_mlp_decode
 *   (bit-identical to rrt_mlp_encode + rrt_mlp_forward + the scaling in
 *   binary32); the vertices are relit in the rrt_relight_order order of
 *   their cluster rows (results unchanged).
 *   The vertices are processed in chunks of at most RRT_MLP_CHUNK (equal
 *   sizes): a chunk is decoded (one rrt_mlp_decode launch), ordered and
 *   relit before the next chunk reuses the same space, so the workspace
 *   stops growing at V = RRT_MLP_CHUNK: rrt_relight_mlp_workspace() bytes,
 *   256-byte aligned: the relight workspace, the decoded values of one
 *   chunk (1 KiB per vertex, 64 MiB at most) and the order of one chunk
 *   (5 bytes per vertex): about 65 MiB from V = 65,536 on.
 * --------------------------------------------------------------------- */
#define RRT_MLP_CHUNK 65536
typedef struct {
  const void* w;           /* RRT_MLP_WEIGHT_COUNT bfloat16 weights, decoder layout */
  const float* bias;       /* RRT_MLP_BIAS_COUNT float32 biases */
  const int32_t* support;  /* [C][RRT_MLP_OUT] flat coefficient indices */
  const float* scale;      /* [C][RRT_MLP_OUT] per-slot output scales */
  int nclusters;           /* C >= 1 */
} rrt_mlp;

int rrt_relight_mlp_workspace(const rrt_light* L, const rrt_rotations* R, int64_t nvert,
                              size_t* bytes);
int rrt_relight_mlp(const rrt_light* L, const rrt_rotations* R, const rrt_mlp* M,
                    const float* pos_nrm, const int32_t* cluster, int64_t nvert,
                    float* radiance, unsigned flags, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RRT_H */
