"""Rotation of a cube-map signal on the sphere, exact integer geometry.

Test infrastructure only (see the package docstring).

Sec. V.A: a point p of the rotated map takes the value of the original map at
p' = R p (rows R_1, R_2, R_3 of R), i.e. g(w) = f(R w) -- the rotated angles
theta' = acos(R_2 p), phi' = atan(R_1 p / R_3 p) are only a spherical
re-statement of that source point.  The paper notes that the construction
applies to any map with an explicit sphere parameterisation; here the map is
the six-face cube map and the source of each texel is the texel whose pyramid
contains R w (nearest texel at texel centres).

To make the result unique (independent of floating-point evaluation order),
the geometry is exact: R is quantised to integers R_q = rint(R * 2^k) with
k = 22 - log2(n) for an n x n map, texel centres are the integer vectors
below, d = R_q * dir is an exact int64 product, and the source texel follows
from integer comparisons and floor divisions.  With this k every component of
d, and every partial sum of its three terms, is an integer of magnitude below
3 n 2^k = 3 * 2^22 < 2^24 (|R_q| entries <= 2^k, |U|, |V| < n), so the
directions are also exact binary32 numbers; the rotation itself is resolved
to 2^-k (2^-15 at n = 128, far below the texel size 2/n).

Face table (faces 0..5 = +X, -X, +Y, -Y, +Z, -Z; texel (i, j) of an n x n
face has U = 2j+1-n, V = 2i+1-n, the face plane at distance n):
    +X ( n, -V, -U)   -X (-n, -V,  U)   +Y ( U,  n,  V)
    -Y ( U, -n, -V)   +Z ( U, -V,  n)   -Z (-U, -V, -n)
Inverse: the major axis a = argmax |d_k| (ties to the lower k), face
2a + [d_a < 0], in-face coordinates (sc, tc) with
    +X (-z, -y)   -X (z, -y)   +Y (x, z)   -Y (x, -z)   +Z (x, -y)   -Z (-x, -y)
and column j' = min(n-1, floor(n (sc + |d_a|) / (2 |d_a|))), row i' likewise
from tc.
"""
import numpy as np

def scale_bits(n):
    """k = 22 - log2(n): the fixed-point scale of rotations for an n x n map."""
    n = int(n)
    assert n >= 1 and n & (n - 1) == 0, n
    return 22 - (n.bit_length() - 1)


def quantise_rotation(R, n):
    """R_q = rint(R * 2^k), k = scale_bits(n) (round half to even) as int64;
    R is float32/64 of shape [..., 3, 3] (row-major, local -> global)."""
    return np.rint(np.asarray(R, dtype=np.float64) * float(1 << scale_bits(n))).astype(np.int64)


def compose_rotations(Ra_q, Rb_q, n):
    """Fixed-point product (Ra_q Rb_q + 2^(k-1)) >> k, k = scale_bits(n),
    entry-wise, exact int64 with a flooring shift.  Ra is the global object
    rotation of a frame, Rb a vertex's local frame; the result maps local
    directions to the lighting's frame."""
    k = scale_bits(n)
    p = np.matmul(np.asarray(Ra_q, np.int64), np.asarray(Rb_q, np.int64))
    return (p + (1 << (k - 1))) >> k


def texel_centres(n):
    """Integer centre directions of every texel, [6, n, n, 3] int64."""
    idx = np.arange(n, dtype=np.int64)
    i, j = np.meshgrid(idx, idx, indexing="ij")
    U = 2 * j + 1 - n
    V = 2 * i + 1 - n
    N = np.full_like(U, n)
    faces = [
        (N, -V, -U),     # +X
        (-N, -V, U),     # -X
        (U, N, V),       # +Y
        (U, -N, -V),     # -Y
        (U, -V, N),      # +Z
        (-U, -V, -N),    # -Z
    ]
    return np.stack([np.stack(f, axis=-1) for f in faces], axis=0)


def locate(d, n):
    """Source texel (face, i, j) of integer directions d [..., 3] (int64)."""
    d = np.asarray(d, dtype=np.int64)
    ad = np.abs(d)
    a = np.argmax(ad, axis=-1)                       # first maximum: lowest axis
    da = np.take_along_axis(d, a[..., None], axis=-1)[..., 0]
    face = 2 * a + (da < 0)
    D = np.abs(da)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    sc = np.select([face == 0, face == 1, face == 2, face == 3, face == 4, face == 5],
                   [-z, z, x, x, x, -x])
    tc = np.select([face == 0, face == 1, face == 2, face == 3, face == 4, face == 5],
                   [-y, -y, z, -z, -y, -y])
    j = np.minimum(n - 1, (n * (sc + D)) // (2 * D))
    i = np.minimum(n - 1, (n * (tc + D)) // (2 * D))
    return face, i, j


def source_index(Rq, n):
    """Flat source texel (face*n*n + i*n + j) of every local texel, [6, n, n]."""
    d = np.einsum("km,fijm->fijk", np.asarray(Rq, np.int64), texel_centres(n))
    f, i, j = locate(d, n)
    return f * n * n + i * n + j


def rotate_pixels(P, Rq):
    """g[q] = P[source(q)] for a cube map P [6, n, n] (values kept as given)."""
    P = np.asarray(P)
    n = P.shape[-1]
    return P.reshape(-1)[source_index(Rq, n)]
