"""Chain-rule rotation of the finest level (FP64): the paper's Haar-domain
phase shift, as opposed to the exact resampling of oracle.relight.

Test infrastructure only (see the package docstring).

Sec. V.A-V.B: the H, V and D coefficients of a level are first-order finite
differences of the map, so the rotated map g(w) = f(R w) has its
coefficients given by the chain rule (eq:pde1-eq:pde3) from those of f and
the derivatives of the mapping between the two parameterisations; the
coarser levels follow by the 2x2 recursion.

Discrete reading on the cube map (texel units: texel (i, j) spans
[j, j+1) x [i, i+1) of its face, n x n texels, h = n / 2):

* destination 2x2 block b covers rows 2 bi, 2 bi + 1 and columns 2 bj,
  2 bj + 1; its centre is the point (x, y) = (2 bj + 1, 2 bi + 1) with
  direction d = U mU + V mV + n mN, U = 2x - n, V = 2y - n, where
  (mU, mV, mN) = R (eU, eV, eN) are the rotated axes of the destination face;
* its source block is the block of the source map containing R times that
  direction: the exact nearest-texel map at resolution n / 2 (oracle.sphere);
* the source block's orthonormal coefficients give S_f, the per-texel
  derivatives f_x' = -H_f, f_y' = -V_f and f_x'y' = 2 D_f; the second
  derivatives f_x'x', f_y'y' are not represented at one level and count 0;
* the mapping to source texel coordinates is the gnomonic projection
  x' = h (sc / D + 1), y' = h (tc / D + 1) with (sc, tc, D) the in-face and
  major components of d for the source face; sc, tc, D are linear in (x, y),
  so the first derivatives and the mixed second derivative are analytic:
      s_x  = (sc_x D - sc D_x) / D^2,
      s_xy = 2 sc D_x D_y / D^3 - (sc_x D_y + sc_y D_x) / D^2   (s = sc / D);
* chain rule at the block centre (eq:pde1-eq:pde3 without the vanishing
  second-derivative terms):
      g_x  = f_x' x'_x + f_y' y'_x,     g_y = f_x' x'_y + f_y' y'_y,
      g_xy = f_x'y' (x'_x y'_y + x'_y y'_x) + f_x' x'_xy + f_y' y'_xy;
* the destination block: S_g = S_f, H_g = -g_x, V_g = -g_y, D_g = g_xy / 2;
  its four pixels follow by the inverse 2x2 step, and every coarser level by
  the pyramid.

R is the quantised rotation R_q / 2^k (k = scale_bits(n)), the matrix the exact
map uses.
"""
import numpy as np

from .haar import haar_forward
from .relight import frame_vertex_rotation, reconstruct_lighting
from .sphere import scale_bits, source_index

# Destination face axes: direction = U eU + V eV + n eN (faces +X..-Z).
FACE_AXES = np.array([
    [[0, 0, -1], [0, -1, 0], [1, 0, 0]],
    [[0, 0, 1], [0, -1, 0], [-1, 0, 0]],
    [[1, 0, 0], [0, 0, 1], [0, 1, 0]],
    [[1, 0, 0], [0, 0, -1], [0, -1, 0]],
    [[1, 0, 0], [0, -1, 0], [0, 0, 1]],
    [[-1, 0, 0], [0, -1, 0], [0, 0, -1]],
], dtype=np.float64)                    # [face][eU, eV, eN][xyz]


def source_blocks(P):
    """Orthonormal finest-level (S, H, V, D) of every 2x2 block, [6, n/2, n/2, 4]."""
    a, b = P[:, 0::2, 0::2], P[:, 0::2, 1::2]
    c, d = P[:, 1::2, 0::2], P[:, 1::2, 1::2]
    return np.stack([(a + b + c + d) / 2, (a - b + c - d) / 2,
                     (a + b - c - d) / 2, (a - b - c + d) / 2], axis=-1)


def blocks_to_pixels(B):
    """Inverse 2x2 step: [6, n/2, n/2, 4] (S, H, V, D) -> pixels [6, n, n]."""
    S, H, V, D = B[..., 0], B[..., 1], B[..., 2], B[..., 3]
    F, h, _ = S.shape
    P = np.empty((F, 2 * h, 2 * h))
    P[:, 0::2, 0::2] = (S + H + V + D) / 2
    P[:, 0::2, 1::2] = (S - H + V - D) / 2
    P[:, 1::2, 0::2] = (S + H - V - D) / 2
    P[:, 1::2, 1::2] = (S - H - V + D) / 2
    return P


def gnomonic_jacobian(c, cx, cy, h):
    """Derivatives of the source texel coordinates x' = h (sc / D + 1),
    y' = h (tc / D + 1) along the destination texel axes x and y.

    c = (sc, tc, D): in-face and major components of the direction for the
    source face at the point; cx, cy: their derivatives along x and y, which
    are constant (the direction is linear in the destination coordinates).
    Quotient rule on s = sc / D:
        s_x  = (sc_x D - sc D_x) / D^2,
        s_xy = 2 sc D_x D_y / D^3 - (sc_x D_y + sc_y D_x) / D^2,
    and likewise for t = tc / D.  Returns (x'_x, x'_y, y'_x, y'_y, x'_xy, y'_xy)."""
    sc, tc, D = c
    scx, tcx, Dx = cx
    scy, tcy, Dy = cy
    xx = h * (scx * D - sc * Dx) / D**2
    xy = h * (scy * D - sc * Dy) / D**2
    yx = h * (tcx * D - tc * Dx) / D**2
    yy = h * (tcy * D - tc * Dy) / D**2
    xxy = h * (2 * sc * Dx * Dy / D**3 - (scx * Dy + scy * Dx) / D**2)
    yxy = h * (2 * tc * Dx * Dy / D**3 - (tcx * Dy + tcy * Dx) / D**2)
    return xx, xy, yx, yy, xxy, yxy


def block_jacobian(R, F, sface, U, V, n):
    """gnomonic_jacobian at destination points (U, V) of face F (U = 2x - n,
    V = 2y - n in texel units) for the rotation R (float [3, 3]) and the
    source face `sface` (arrays broadcast together)."""
    mU, mV, mN = (R @ FACE_AXES[F][k] for k in range(3))
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    d = U[..., None] * mU + V[..., None] * mV + n * mN       # [..., 3]
    dx, dy = 2.0 * mU, 2.0 * mV                               # d per texel step in x, y
    sel = FACE_AXES[sface]                                    # source face: rows eU, eV, eN
    c = tuple(np.einsum("...k,...k->...", sel[..., r, :], d) for r in range(3))
    cx = tuple(np.einsum("...k,k->...", sel[..., r, :], dx) for r in range(3))
    cy = tuple(np.einsum("...k,k->...", sel[..., r, :], dy) for r in range(3))
    return gnomonic_jacobian(c, cx, cy, n // 2)


def chain_rotate(P, Rq):
    """Rotated map [6, n, n] with the finest level rotated by the chain rule."""
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[-1]
    h = n // 2
    R = np.asarray(Rq, dtype=np.float64) / float(1 << scale_bits(n))
    src = source_index(Rq, h)                                # [6, h, h] flat at n/2
    Bf = source_blocks(P).reshape(-1, 4)[src]                # [6, h, h, 4]
    sface = src // (h * h)
    bi, bj = np.meshgrid(np.arange(h), np.arange(h), indexing="ij")
    U = (4 * bj + 2 - n).astype(np.float64)
    V = (4 * bi + 2 - n).astype(np.float64)
    out = np.empty((6, h, h, 4))
    for F in range(6):
        xx, xy, yx, yy, xxy, yxy = block_jacobian(R, F, sface[F], U, V, n)
        S, H, Vf, Df = (Bf[F][..., k] for k in range(4))
        fx, fy, fxy = -H, -Vf, 2 * Df
        gx = fx * xx + fy * yx
        gy = fx * xy + fy * yy
        gxy = fxy * (xx * yy + xy * yx) + fx * xxy + fy * yxy
        out[F] = np.stack([S, -gx, -gy, gxy / 2], axis=-1)
    return blocks_to_pixels(out)


def relight_chain(light_idx, light_val, n, vert_rot, frame_rot, t_idx, t_val,
                  vertices=None, frames=None):
    """radiance[f][v] (FP64) with the chain-rule rotation of the finest level
    in place of the exact resampling (otherwise as oracle.relight.relight)."""
    V = np.asarray(vert_rot).shape[0]
    nf = 1 if frame_rot is None else np.asarray(frame_rot).shape[0]
    vertices = np.arange(V) if vertices is None else np.asarray(vertices)
    frames = np.arange(nf) if frames is None else np.asarray(frames)
    P = reconstruct_lighting(light_idx, light_val, n)
    out = np.zeros((len(frames), len(vertices)), dtype=np.float64)
    for a, v in enumerate(vertices):
        T = np.zeros(6 * n * n, dtype=np.float64)
        vals = np.asarray(t_val[v], dtype=np.float64)
        if t_idx is None:
            T[:] = vals
        else:
            T[np.asarray(t_idx[v], np.int64)] = vals
        for b, f in enumerate(frames):
            Rq = frame_vertex_rotation(vert_rot, frame_rot, v, f, n)
            out[b, a] = np.dot(T, haar_forward(chain_rotate(P, Rq)).ravel())
    return out
