"""Outgoing radiance by rotating the lighting into each vertex's frame and
taking the wavelet-domain inner product with the vertex's transport (FP64).

Test infrastructure only (see the package docstring).

Definition (Sec. II rendering integral without emission; Sec. III: BRDF,
cosine and visibility pre-multiplied into one transfer function turn the
integral into an inner product; Sec. V.C, last algorithm step: the rotated
coefficients enter that product):

    radiance[f][v] = sum_k  T_v[k] * ( W S(R_fv) W^T L )[k]

  L      stored global-frame lighting coefficients (top-K, zero elsewhere)
  T_v    stored transport coefficients of vertex v (top-k, zero elsewhere)
  W      orthonormal per-face Haar transform (oracle.haar)
  S(R)   pixel-domain rotation g(w) = f(R w) (oracle.sphere)
  R_fv   the frame's object rotation composed with the vertex frame

This is the paper's own ground-truth protocol (rotate in the spatial domain,
then transform), evaluated densely over all 6 n^2 coefficients.
"""
import numpy as np

from .haar import haar_forward, haar_inverse
from .select import topk_abs
from .sphere import compose_rotations, quantise_rotation, rotate_pixels


def lighting_coefficients(pixels, k, value_dtype=np.float32):
    """Forward Haar of a [6, n, n] environment and its top-k truncation.
    Returns (idx int32 ascending, values rounded to value_dtype)."""
    coef = haar_forward(np.asarray(pixels, dtype=np.float64)).ravel()
    idx = topk_abs(coef, k)
    return idx.astype(np.int32), coef[idx].astype(value_dtype)


def transport_rows(pixels, nnz, value_dtype=np.float32):
    """Per-vertex forward Haar of pixel-domain transport [B, 6, n, n] and its
    top-nnz truncation -> (idx int32 [B, nnz] ascending, values [B, nnz])."""
    coef = haar_forward(np.asarray(pixels, dtype=np.float64))
    coef = coef.reshape(coef.shape[0], -1)
    idx = np.stack([topk_abs(row, nnz) for row in coef]) if coef.shape[0] else \
        np.zeros((0, nnz), np.int64)
    vals = np.take_along_axis(coef, idx, axis=1)
    return idx.astype(np.int32), vals.astype(value_dtype)


def reconstruct_lighting(idx, val, n):
    """Pixel-domain lighting P = W^T L of the truncated coefficients (FP64)."""
    c = np.zeros(6 * n * n, dtype=np.float64)
    c[np.asarray(idx, np.int64)] = np.asarray(val, dtype=np.float64)
    return haar_inverse(c.reshape(6, n, n))


def frame_vertex_rotation(vert_rot, frame_rot, v, f, n):
    """Quantised R_fv for an n x n map: the vertex frame alone when there is
    no frame rotation, otherwise the fixed-point composition R_obj(f) * F_v."""
    Fv = quantise_rotation(np.asarray(vert_rot)[v], n)
    if frame_rot is None:
        return Fv
    return compose_rotations(quantise_rotation(np.asarray(frame_rot)[f], n), Fv, n)


def phase_shift(coef, R):
    """Dense Haar-domain rotation W S(R) W^T coef of one cube map [6, n, n]."""
    Rq = quantise_rotation(R, np.asarray(coef).shape[-1])
    return haar_forward(rotate_pixels(haar_inverse(coef), Rq))


def relight(light_idx, light_val, n, vert_rot, frame_rot, t_idx, t_val,
            vertices=None, frames=None, return_scale=False):
    """radiance[f][v] (FP64) for the selected frames x vertices.

    light_idx/light_val: stored lighting (values promoted to FP64 as stored).
    vert_rot [V, 3, 3], frame_rot [F, 3, 3] or None.
    t_idx [V, nnz] (None = dense, nnz = 6 n^2), t_val [V, nnz].
    With return_scale, also returns sum_k |T_v[k] ghat[k]| per result: the
    magnitude scale against which rounding errors of a finite-precision
    evaluation of the same sum are measured (its ratio to |radiance| is the
    condition number of the inner product).
    """
    V = np.asarray(vert_rot).shape[0]
    nf = 1 if frame_rot is None else np.asarray(frame_rot).shape[0]
    vertices = np.arange(V) if vertices is None else np.asarray(vertices)
    frames = np.arange(nf) if frames is None else np.asarray(frames)
    P = reconstruct_lighting(light_idx, light_val, n)
    out = np.zeros((len(frames), len(vertices)), dtype=np.float64)
    scale = np.zeros_like(out)
    for a, v in enumerate(vertices):
        T = np.zeros(6 * n * n, dtype=np.float64)
        vals = np.asarray(t_val[v], dtype=np.float64)
        if t_idx is None:
            T[:] = vals
        else:
            T[np.asarray(t_idx[v], np.int64)] = vals
        for b, f in enumerate(frames):
            Rq = frame_vertex_rotation(vert_rot, frame_rot, v, f, n)
            ghat = haar_forward(rotate_pixels(P, Rq)).ravel()
            out[b, a] = np.dot(T, ghat)
            scale[b, a] = np.dot(np.abs(T), np.abs(ghat))
    return (out, scale) if return_scale else out


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))
