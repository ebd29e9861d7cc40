"""Rotation started below the finest level (FP64).

Test infrastructure only (see the package docstring).

The paper notes that the rotation may start at any level coarser than the
finest one, which divides the work by 4^k for k levels skipped (Sec. V.C,
remark after the algorithm).  Exact discrete reading used here:

* dropping the k finest levels of the lighting leaves a map that is constant
  on blocks of B x B texels, B = 2^k;
* the coefficients of the coarser levels are those of the n' x n' map of
  block sums divided by B (n' = n / B, orthonormal Haar), and they sit at
  the same Mallat positions: the top-left n' x n' corner of each face;
* the rotation is carried out at resolution n' with the exact integer map of
  that resolution (oracle.sphere), and only the transport coefficients at
  those positions take part in the inner product.

So the result is `relight` at resolution n' on the remapped lighting and
transport entries; entries at finer positions are dropped.
"""
import numpy as np

from .relight import relight


def coarse_index(idx, n, k):
    """Flat Mallat index at resolution n -> the same coefficient's index at
    n' = n >> k, or -1 for coefficients of the k finest levels."""
    idx = np.asarray(idx, dtype=np.int64)
    nc = n >> k
    face, pos = idx // (n * n), idx % (n * n)
    r, c = pos // n, pos % n
    keep = (idx >= 0) & (idx < 6 * n * n) & (r < nc) & (c < nc)
    return np.where(keep, face * nc * nc + r * nc + c, -1)


def relight_from_level(light_idx, light_val, n, vert_rot, frame_rot, t_idx, t_val, k,
                       vertices=None, frames=None):
    """radiance[f][v] (FP64) with the rotation started k levels below the
    finest one (k = 0 is `relight`)."""
    nc = n >> k
    li = coarse_index(light_idx, n, k)
    lkeep = li >= 0
    vert_rot = np.asarray(vert_rot)
    V = vert_rot.shape[0]
    vertices = np.arange(V) if vertices is None else np.asarray(vertices)
    nf = 1 if frame_rot is None else np.asarray(frame_rot).shape[0]
    frames = np.arange(nf) if frames is None else np.asarray(frames)
    out = np.zeros((len(frames), len(vertices)), dtype=np.float64)
    for a, v in enumerate(vertices):
        if t_idx is None:
            ti = coarse_index(np.arange(6 * n * n), n, k)
        else:
            ti = coarse_index(t_idx[v], n, k)
        keep = ti >= 0
        if not keep.any() or not lkeep.any():
            continue
        tv = np.asarray(t_val[v])[keep]
        out[:, a] = relight(li[lkeep], np.asarray(light_val)[lkeep], nc, vert_rot[v:v + 1],
                            frame_rot, ti[keep][None, :], tv[None, :], frames=frames)[:, 0]
    return out
