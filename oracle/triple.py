"""Triple product integral in the per-face Haar basis (FP64).

Test infrastructure only (see the package docstring).

Sec. III (eq:tripleSum): with the lighting a, the BRDF times the cosine b and
the visibility c expanded in one orthonormal basis, the reflected radiance is
sum_ijk C_ijk a_i b_j c_k, where C_ijk integrates the product of three basis
functions.  Discrete reading: the integral over the sphere is the sum over
texels (the texel solid angle is part of b, as it is part of the transport
of the double product) and the basis is the per-face orthonormal Haar basis
of oracle.haar, so

    C_ijk = sum_q Psi_i(q) Psi_j(q) Psi_k(q).

Tripling-coefficient theorem (Sec. III, after eq:tripleSum): C_ijk is
non-zero only when
  (a) all three are the scaling function of one face,
  (b) all three are wavelets of different types on one square, or
  (c) two are the same wavelet and the third is the scaling function of its
      face or a wavelet of a strictly coarser level whose square contains
      the pair's square.
On the unit square the values are 1, 2^l and +-2^l (third function at level
l).  A face here has n x n unit texels, so each basis function is 1/n of its
unit-square counterpart and C_ijk is 1/n of the unit-square value: (a) 1/n;
(b) 1/B for wavelets on a square of side B texels; (c) the value of the third
function on the pair's square: 1/n for the scaling function, +-1/B' for a
coarser wavelet of side B', with the sign of its quadrant (H: left +,
right -; V: top +, bottom -; D: top-left and bottom-right +).

`triple_sum` evaluates sum_ijk C_ijk a_i b_j c_k literally for a sparse c by
enumerating, for each c_k, the pairs (i, j) the theorem leaves; `relight_triple`
applies it per vertex to the exactly rotated lighting (as oracle.relight).
"""
import numpy as np

from .haar import coefficient_block, haar_forward, haar_inverse
from .relight import frame_vertex_rotation, reconstruct_lighting
from .sphere import rotate_pixels

_KINDS = "SHVD"


def basis(idx, n):
    """(face, kind, size, r0, c0) of flat Mallat index idx: the function's
    square has side `size` texels and top-left texel (r0, c0)."""
    face, pos = divmod(int(idx), n * n)
    r, c = divmod(pos, n)
    kind, size, br, bc = coefficient_block(r, c, n)
    return face, kind, size, br * size, bc * size


def _sign_on(kind, size, r0, c0, r, c):
    """Sign of a wavelet (kind, square size at r0, c0) on texel (r, c) of its square."""
    top = (r - r0) < size // 2
    left = (c - c0) < size // 2
    if kind == "H":
        return 1.0 if left else -1.0
    if kind == "V":
        return 1.0 if top else -1.0
    return 1.0 if top == left else -1.0


def tripling_coefficient(i, j, k, n):
    """C_ijk by the tripling-coefficient theorem (texel normalisation)."""
    fs = [basis(x, n) for x in (i, j, k)]
    if len({f[0] for f in fs}) != 1:
        return 0.0
    kinds = [f[1] for f in fs]
    if kinds == ["S", "S", "S"]:                                     # (a)
        return 1.0 / n
    if "S" not in kinds and len(set(kinds)) == 3 and len({f[2:] for f in fs}) == 1:
        return 1.0 / fs[0][2]                                        # (b)
    ids = [int(i), int(j), int(k)]
    for p, q, t in ((0, 1, 2), (0, 2, 1), (1, 2, 0)):                 # (c)
        if ids[p] != ids[q] or ids[t] == ids[p] or fs[p][1] == "S":
            continue
        _, kind, size, r0, c0 = fs[t]
        _, _, ps, pr, pc = fs[p]
        if kind == "S":
            return 1.0 / n
        if size > ps and r0 <= pr < r0 + size and c0 <= pc < c0 + size:
            return _sign_on(kind, size, r0, c0, pr, pc) / size
        return 0.0
    return 0.0


def _face_tables(n):
    """Per Mallat position of one face: kind code (0..3), size, square origin."""
    K = np.zeros((n, n), np.int64)
    Z = np.zeros((n, n), np.int64)
    R0 = np.zeros((n, n), np.int64)
    C0 = np.zeros((n, n), np.int64)
    for r in range(n):
        for c in range(n):
            kind, size, br, bc = coefficient_block(r, c, n)
            K[r, c], Z[r, c], R0[r, c], C0[r, c] = _KINDS.index(kind), size, br * size, bc * size
    return K.ravel(), Z.ravel(), R0.ravel(), C0.ravel()


def _signs(kind, size, r0, c0, R, C):
    """Vectorised _sign_on for texels (R, C) inside the square."""
    top = (R - r0) < size // 2
    left = (C - c0) < size // 2
    if kind == 1:
        return np.where(left, 1.0, -1.0)
    if kind == 2:
        return np.where(top, 1.0, -1.0)
    return np.where(top == left, 1.0, -1.0)


def triple_sum(a, b, c_idx, c_val, n, tables=None):
    """sum_ijk C_ijk a_i b_j c_k for dense a, b [6 n^2] and sparse c (FP64)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    K, Z, R0, C0 = tables if tables is not None else _face_tables(n)
    total = 0.0
    nn = n * n
    for k, ck in zip(np.asarray(c_idx, np.int64), np.asarray(c_val, np.float64)):
        if k < 0 or k >= 6 * nn or ck == 0.0:
            continue
        f, p = divmod(int(k), nn)
        fa, fb = a[f * nn:(f + 1) * nn], b[f * nn:(f + 1) * nn]
        kind, size, r0, c0 = K[p], Z[p], R0[p], C0[p]
        if kind == 0:
            # (a) with (S, S) and (c) with every identical wavelet pair
            total += ck * np.dot(fa, fb) / n
            continue
        s = 0.0
        # (c): the pair (k, k) split over i, j with the face's scaling function
        s += (fa[0] * fb[p] + fa[p] * fb[0]) / n
        # (c): strictly coarser wavelets chi containing k's square, paired with k
        anc = (K > 0) & (Z > size) & (R0 <= r0) & (r0 < R0 + Z) & (C0 <= c0) & (c0 < C0 + Z)
        for x in np.nonzero(anc)[0]:
            sg = _signs(K[x], Z[x], R0[x], C0[x], np.array(r0), np.array(c0)) / Z[x]
            s += (fa[x] * fb[p] + fa[p] * fb[x]) * float(sg)
        # (c): identical finer pairs inside k's square, k the coarser third
        des = (K > 0) & (Z < size) & (R0 >= r0) & (R0 < r0 + size) & (C0 >= c0) & (C0 < c0 + size)
        d = np.nonzero(des)[0]
        if d.size:
            s += np.dot(fa[d] * fb[d], _signs(kind, size, r0, c0, R0[d], C0[d])) / size
        # (b): the two other wavelet types on the same square
        same = np.nonzero((K > 0) & (K != kind) & (Z == size) & (R0 == r0) & (C0 == c0))[0]
        if same.size == 2:
            x, y = same
            s += (fa[x] * fb[y] + fa[y] * fb[x]) / size
        total += ck * s
    return total


def triple_pixels(a, b, c, n):
    """The plain definition: sum over texels of the three reconstructed maps."""
    A = haar_inverse(np.asarray(a, np.float64).reshape(6, n, n))
    B = haar_inverse(np.asarray(b, np.float64).reshape(6, n, n))
    C = haar_inverse(np.asarray(c, np.float64).reshape(6, n, n))
    return float(np.sum(A * B * C))


def magnitude_map(idx, val, n):
    """sum_i |val_i| |Psi_i(q)| per texel [6, n, n]: the magnitude against
    which a finite-precision reconstruction of the map rounds (|Psi_i| is 1/B
    on the square of side B of function i)."""
    c = np.zeros(6 * n * n)
    np.add.at(c, np.asarray(idx, np.int64), np.abs(np.asarray(val, np.float64)))
    c = c.reshape(6, n, n)
    out = np.full((6, n, n), 1.0) * (c[:, :1, :1] / n)
    g = 1                                     # coefficient grid side of the level
    while g < n:
        B = n // g
        lvl = c[:, :g, g:2 * g] + c[:, g:2 * g, :g] + c[:, g:2 * g, g:2 * g]
        out += np.repeat(np.repeat(lvl, B, axis=1), B, axis=2) / B
        g *= 2
    return out


def relight_triple(light_idx, light_val, n, vert_rot, frame_rot, v_idx, v_val, brdf_pix,
                   material=None, vertices=None, frames=None, return_scale=False):
    """radiance[f][v] (FP64) of the triple product: the exactly rotated
    lighting a (oracle.relight), the BRDF-times-cosine b = Haar of
    brdf_pix[material[v]] (pixel-domain, local frame, [M, 6, n, n]) and the
    stored visibility row c = (v_idx[v], v_val[v]).  A material outside
    [0, M) gives 0.  With return_scale, also the magnitude scale
    sum_k |c_k| (1/B_k) sum_{q in square k} |A|(q) |B(q)| of each result,
    |A| the rotated magnitude_map of the lighting: a bound on every term of
    the texel-domain evaluation, the reconstruction of the lighting
    included."""
    brdf_pix = np.asarray(brdf_pix, np.float64).reshape(-1, 6, n, n)
    M = brdf_pix.shape[0]
    V = np.asarray(vert_rot).shape[0]
    nf = 1 if frame_rot is None else np.asarray(frame_rot).shape[0]
    vertices = np.arange(V) if vertices is None else np.asarray(vertices)
    frames = np.arange(nf) if frames is None else np.asarray(frames)
    P = reconstruct_lighting(light_idx, light_val, n)
    Pmag = magnitude_map(light_idx, light_val, n) if return_scale else None
    bcoef = [haar_forward(brdf_pix[m]).ravel() for m in range(M)]
    tables = _face_tables(n)
    K, Z, R0, C0 = tables
    out = np.zeros((len(frames), len(vertices)))
    scale = np.zeros_like(out)
    for ai, v in enumerate(vertices):
        m = 0 if material is None else int(np.asarray(material)[v])
        if m < 0 or m >= M:
            continue
        ci = np.asarray(v_idx[v], np.int64)
        cv = np.asarray(v_val[v], np.float64)
        for bi, f in enumerate(frames):
            Rq = frame_vertex_rotation(vert_rot, frame_rot, v, f, n)
            A = rotate_pixels(P, Rq)
            out[bi, ai] = triple_sum(haar_forward(A).ravel(), bcoef[m], ci, cv, n, tables)
            if return_scale:
                AB = rotate_pixels(Pmag, Rq) * np.abs(brdf_pix[m])
                sat = np.zeros((6, n + 1, n + 1))
                sat[:, 1:, 1:] = AB.cumsum(1).cumsum(2)
                ok = (ci >= 0) & (ci < 6 * n * n)
                f_, p_ = np.divmod(ci[ok], n * n)
                z, r, c = Z[p_], R0[p_], C0[p_]
                box = sat[f_, r + z, c + z] - sat[f_, r, c + z] - sat[f_, r + z, c] + sat[f_, r, c]
                scale[bi, ai] = np.sum(np.abs(cv[ok]) * box / z)
    return (out, scale) if return_scale else out
