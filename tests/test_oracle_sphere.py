"""Pins of the checker's rotation geometry (no GPU).

* hand-derived source texels (tests/golden/index_map_n2.txt);
* the integer face table against the independently written float texel
  directions of the scene generator;
* identity rotation -> identity map; the 24 rotations of the cube group ->
  bijections whose Haar action is a signed permutation;
* brute force: for random and boundary-heavy rotations, every source texel
  is the one found by enumerating all texels whose pyramid contains R w
  (integer inequalities, no division), with the stated tie rules;
* fixed-point quantisation and composition exact inside the cube group;
* int32 headroom of R_q * dir up to n = 1024.
"""
import itertools
import os

import numpy as np
import pytest

from oracle.haar import haar_forward, haar_inverse
from oracle.sphere import (compose_rotations, locate, quantise_rotation, rotate_pixels,
                           scale_bits, source_index, texel_centres)
from scenes.scene import random_rotations, texel_directions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cube_group():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            M = np.zeros((3, 3))
            for r in range(3):
                M[r, perm[r]] = signs[r]
            if np.linalg.det(M) > 0:
                mats.append(M)
    assert len(mats) == 24
    return mats


def test_golden_index_map():
    with open(os.path.join(GOLDEN, "index_map_n2.txt")) as fh:
        lines = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    R = np.array([float(t) for t in lines[0][1:]]).reshape(3, 3)
    src = source_index(quantise_rotation(R, 2), 2)
    for row in lines[1:]:
        f, i, j, sf, si, sj = map(int, row)
        assert src[f, i, j] == sf * 4 + si * 2 + sj


@pytest.mark.parametrize("n", [2, 8, 32])
def test_face_table_matches_scene_directions(n):
    c = texel_centres(n).astype(np.float64)
    c /= np.linalg.norm(c, axis=-1, keepdims=True)
    np.testing.assert_allclose(c, texel_directions(n), atol=1e-15)


def test_face_centres_and_adjacency():
    n = 4
    c = texel_centres(n)
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    for f in range(6):
        np.testing.assert_array_equal(np.sign(c[f].sum(axis=(0, 1))), axes[f])
    # every texel edge is shared by exactly two texels: the 4*6*n^2 corner
    # rays, counted with multiplicity, cover each cube-grid edge twice
    edges = {}
    for f in range(6):
        for i in range(n):
            for j in range(n):
                d = c[f, i, j]
                a = int(np.argmax(np.abs(d)))
                e = [k for k in range(3) if k != a]
                corners = []
                for du, dv in [(-1, -1), (-1, 1), (1, 1), (1, -1)]:
                    p = d.copy()
                    p[e[0]] += du
                    p[e[1]] += dv
                    corners.append(tuple(p))
                for k in range(4):
                    key = tuple(sorted([corners[k], corners[(k + 1) % 4]]))
                    edges[key] = edges.get(key, 0) + 1
    assert set(edges.values()) == {2}


@pytest.mark.parametrize("n", [1, 2, 8, 64])
def test_identity_rotation_is_identity(n):
    src = source_index(quantise_rotation(np.eye(3), n), n)
    np.testing.assert_array_equal(src.ravel(), np.arange(6 * n * n))


@pytest.mark.parametrize("n", [2, 4, 16])
def test_cube_group_bijection_and_signed_permutation(n):
    for M in cube_group():
        src = source_index(quantise_rotation(M, n), n).ravel()
        assert np.array_equal(np.sort(src), np.arange(6 * n * n))
    if n <= 4:
        for M in cube_group():
            Rq = quantise_rotation(M, n)
            cols = []
            for k in range(6 * n * n):
                e = np.zeros(6 * n * n)
                e[k] = 1.0
                p = haar_inverse(e.reshape(6, n, n))
                cols.append(haar_forward(rotate_pixels(p, Rq)).ravel())
            A = np.stack(cols, 1)
            np.testing.assert_allclose(np.abs(A).sum(0), 1.0, atol=1e-12)
            np.testing.assert_allclose(np.abs(A).sum(1), 1.0, atol=1e-12)
            assert np.all(np.isclose(A, 0) | np.isclose(np.abs(A), 1))


def test_quarter_turn_haar_action_n2():
    # quarter turn about +Y: the +Y face image turns by 90 degrees and its
    # coefficients map (S, H, V, D) -> (S, -V, H, -D) (hand derivation:
    # g = [[c, a], [d, b]] for f = [[a, b], [c, d]]).
    R = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], float)
    rng = np.random.default_rng(3)
    f = rng.normal(size=(6, 2, 2))
    g = haar_forward(rotate_pixels(f, quantise_rotation(R, 2)))
    F = haar_forward(f)
    S, H, V, D = F[2, 0, 0], F[2, 0, 1], F[2, 1, 0], F[2, 1, 1]
    np.testing.assert_allclose([g[2, 0, 0], g[2, 0, 1], g[2, 1, 0], g[2, 1, 1]], [S, -V, H, -D],
                               atol=1e-14)


def _face_frames(n):
    """(e_U, e_V, e_N) of every face derived from the forward table."""
    c = texel_centres(n)
    eU = (c[:, 0, 1] - c[:, 0, 0]) // 2
    eV = (c[:, 1, 0] - c[:, 0, 0]) // 2
    U0, V0 = 1 - n, 1 - n
    eN = (c[:, 0, 0] - U0 * eU - V0 * eV) // n
    return eU, eV, eN


def _brute_force_source(d, n, frames):
    eU, eV, eN = frames
    cands = []
    for f in range(6):
        u, v, w = int(d @ eU[f]), int(d @ eV[f]), int(d @ eN[f])
        if w > 0 and abs(u) <= w and abs(v) <= w:
            cands.append((f, u, v, w))
    best = min(cands, key=lambda t: t[0] // 2)          # tie between faces: lowest axis
    f, u, v, w = best
    js = [j for j in range(n) if (2 * j - n) * w <= n * u <= (2 * j + 2 - n) * w]
    is_ = [i for i in range(n) if (2 * i - n) * w <= n * v <= (2 * i + 2 - n) * w]
    return f, max(is_), max(js)                          # in-face ties: higher index


def _boundary_rotations():
    out = []
    for ax in range(3):
        for ang in (np.pi / 4, np.pi / 8, np.pi / 3):
            c, s = np.cos(ang), np.sin(ang)
            M = np.eye(3)
            o = [k for k in range(3) if k != ax]
            M[o[0], o[0]] = c
            M[o[0], o[1]] = -s
            M[o[1], o[0]] = s
            M[o[1], o[1]] = c
            out.append(M)
    return out


@pytest.mark.parametrize("n", [2, 4, 8])
def test_index_map_brute_force(n):
    frames = _face_frames(n)
    rots = list(random_rotations(99, 6)) + _boundary_rotations() + cube_group()[:4]
    c = texel_centres(n)
    for R in rots:
        Rq = quantise_rotation(R, n)
        d = np.einsum("km,fijm->fijk", Rq, c)
        f, i, j = locate(d, n)
        for idx in np.ndindex(6, n, n):
            assert (f[idx], i[idx], j[idx]) == _brute_force_source(d[idx], n, frames), (R, idx)


@pytest.mark.parametrize("n", [1, 2, 128, 1024])
def test_quantise_and_compose(n):
    k = scale_bits(n)
    assert k == 22 - int(np.log2(n))
    Rq = quantise_rotation(np.eye(3), n)
    np.testing.assert_array_equal(Rq, np.eye(3, dtype=np.int64) << k)
    G = cube_group()
    for A, B in itertools.product(G[:8], G):
        np.testing.assert_array_equal(
            compose_rotations(quantise_rotation(A, n), quantise_rotation(B, n), n),
            quantise_rotation(A @ B, n))
    R = random_rotations(5, 16)
    for r in R:
        np.testing.assert_array_equal(
            compose_rotations(quantise_rotation(np.eye(3), n), quantise_rotation(r, n), n),
            quantise_rotation(r, n))
    # half-to-even rounding of an exact tie
    assert quantise_rotation(np.full((3, 3), 2.5 / (1 << k)), n)[0, 0] == 2


@pytest.mark.parametrize("n", [1, 2, 128, 1024])
def test_directions_are_exact_binary32_integers(n):
    """Every term, partial sum and total of R_q (U eU + V eV + n eN) stays
    below 2^24 in magnitude, so binary32 holds it exactly: the worst case
    over random rotations and the bound 3 n 2^k = 3 * 2^22."""
    k = scale_bits(n)
    assert 3 * n * (1 << k) == 3 << 22 and (3 << 22) < (1 << 24)
    R = random_rotations(7, 2000).astype(np.float64)
    Rq = quantise_rotation(R, n)
    assert np.abs(Rq).max() <= (1 << k)
    corner = np.array([n, n - 1, n - 1]) if n > 1 else np.array([1, 0, 0])
    worst = np.abs(Rq).astype(np.int64) @ corner
    assert worst.max() < (1 << 24)
    # the texel directions themselves round-trip through binary32
    m = min(n, 16)
    d = np.einsum("rkm,fijm->rfijk", Rq[:50], texel_centres(m) * (n // m))
    assert np.array_equal(d.astype(np.float32).astype(np.int64), d)


@pytest.mark.parametrize("n", [4, 16])
def test_cube_group_equivariance(n):
    """Pre-rotating the map by a cube rotation C equals composing C into the
    vertex rotation (exact: C maps texel pyramids onto texel pyramids)."""
    rng = np.random.default_rng(11)
    P = rng.normal(size=(6, n, n))
    for C in cube_group():
        Cq = quantise_rotation(C, n)
        Pc = rotate_pixels(P, Cq)                       # f'(w) = f(C w)
        for R in random_rotations(13, 3):
            Rq = quantise_rotation(R, n)
            a = rotate_pixels(Pc, Rq)                   # f'(R w) = f(C R w)
            b = rotate_pixels(P, compose_rotations(Cq, Rq, n))
            np.testing.assert_array_equal(a, b)
