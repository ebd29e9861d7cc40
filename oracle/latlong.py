"""Rotation on the longitude-latitude map (FP64 values, binary32 geometry).

Test infrastructure only (see the package docstring).

Sec. V.A derives the rotation on the longitude-latitude map: a direction
p = (sin t sin f, cos t, sin t cos f) (elevation t from +Y, azimuth f), the
rotated map g(p) = f(R p), and the remark that aligning the elevation
rotation with the X axis leaves only R_x plus a shift along the azimuth (last
paragraphs of Sec. V.A and V.C).  Reading used here:

* the map has H rows (t) and W = 2H columns (f), texel (i, j) spans
  [i, i+1) x [j, j+1) in units of pi/H in both angles, and is stored as two
  H x H squares (square s = columns s H .. s H + H - 1), each with its own
  2-D Haar transform (as a cube face);
* a vertex rotation is R = R_y(s_a d) R_x(b) R_y(s_c d), d = pi/H, with
  integer azimuth shifts s_a, s_c: the two azimuth rotations are exact
  cyclic shifts of whole columns; R_x(b) is given by (cos b, sin b) in
  binary32, R_x = [[1,0,0],[0,cos b,-sin b],[0,sin b,cos b]];
  R_y(a) maps azimuth f to f + a;
* destination texel (i, j) takes the source texel of R p(i, j + s_c) shifted
  by s_a columns, where the texel of a direction q is decided in binary32 by
  one fixed sequence of rounded operations (the kernel's precision; every
  operation below is a separate IEEE binary32 operation, no fused
  multiply-add):
      p = (S_i * s_j, c_i, S_i * k_j)     S_i, c_i: sin, cos of row centre i;
                                          s_j, k_j: sin, cos of column centre j
      q_y = cb * p_y - sb * p_z,  q_z = sb * p_y + cb * p_z,  q_x = p_x
      rho = sqrt(q_x * q_x + q_z * q_z)
      row i' = #{k in 1..H-1 : q_y <= C_k}          (C_k = cos(k pi / H))
      c      = #{k in 1..H-1 : q_z <= C_k * rho}
      column j' = c if q_x >= 0 else W - 1 - c, then (j' + s_a) mod W;
  q is not normalised (|q| = 1 within a few roundings), which moves a
  boundary by about 1e-7 rad.  The tables are the binary32 roundings of the
  exact sines and cosines (`grid`).
"""
import numpy as np

from .haar import haar_forward, haar_inverse


def grid(H):
    """Binary32 tables of the map: (sin, cos) of the H row centres, (sin, cos)
    of the 2H column centres and C_k = cos(k pi / H), k = 0..H-1 (C_0 = 1 is
    not used)."""
    t = (np.arange(H) + 0.5) * np.pi / H
    f = (np.arange(2 * H) + 0.5) * np.pi / H
    C = np.cos(np.arange(H) * np.pi / H)
    f32 = np.float32
    return (np.sin(t).astype(f32), np.cos(t).astype(f32), np.sin(f).astype(f32),
            np.cos(f).astype(f32), C.astype(f32))


def source_index(H, cb, sb, s_a, s_c):
    """Flat source index [2, H, H] (square-major) of every destination texel."""
    W = 2 * H
    St, ct, sf, kf, C = grid(H)
    cb, sb = np.float32(cb), np.float32(sb)
    i = np.arange(H)[:, None]
    j = np.arange(W)[None, :]
    jc = (j + int(s_c)) % W
    with np.errstate(all="ignore"):
        px = St[i] * sf[jc]
        py = np.broadcast_to(ct[i], px.shape)
        pz = St[i] * kf[jc]
        qy = cb * py - sb * pz
        qz = sb * py + cb * pz
        qx = px
        rho = np.sqrt(qx * qx + qz * qz)
        Ck = C[1:].reshape(-1, 1, 1)
        row = np.sum(qy[None] <= Ck, axis=0)
        c = np.sum(qz[None] <= Ck * rho[None], axis=0)
    col = np.where(qx >= 0, c, W - 1 - c)
    col = (col + int(s_a)) % W
    src = (col // H) * H * H + row * H + (col % H)          # [H, W] destination layout
    return np.stack([src[:, :H], src[:, H:]])                # -> [2, H, H]


def rotate(P, cb, sb, s_a, s_c):
    """Rotated map g = P[source] of a [2, H, H] lat-long map."""
    P = np.asarray(P)
    H = P.shape[-1]
    return P.reshape(-1)[source_index(H, cb, sb, s_a, s_c)]


def relight_latlong(light_idx, light_val, H, elev, shift, t_idx, t_val, vertices=None,
                    return_scale=False):
    """radiance[1][v] (FP64): the lat-long counterpart of oracle.relight.relight.

    elev [V, 2] binary32 (cos b, sin b), shift [V, 2] int (s_a, s_c);
    t_idx [V, nnz] flat indices over [2, H, H] (None = dense), t_val [V, nnz]."""
    N = 2 * H * H
    c = np.zeros(N)
    c[np.asarray(light_idx, np.int64)] = np.asarray(light_val, np.float64)
    P = haar_inverse(c.reshape(2, H, H))
    elev = np.asarray(elev, np.float32)
    shift = np.asarray(shift, np.int64)
    V = elev.shape[0]
    vertices = np.arange(V) if vertices is None else np.asarray(vertices)
    out = np.zeros((1, len(vertices)))
    scale = np.zeros_like(out)
    for a, v in enumerate(vertices):
        T = np.zeros(N)
        vals = np.asarray(t_val[v], np.float64)
        if t_idx is None:
            T[:] = vals
        else:
            ti = np.asarray(t_idx[v], np.int64)
            ok = (ti >= 0) & (ti < N)
            T[ti[ok]] = vals[ok]
        ghat = haar_forward(rotate(P, elev[v, 0], elev[v, 1], shift[v, 0], shift[v, 1])).ravel()
        out[0, a] = np.dot(T, ghat)
        scale[0, a] = np.dot(np.abs(T), np.abs(ghat))
    return (out, scale) if return_scale else out
