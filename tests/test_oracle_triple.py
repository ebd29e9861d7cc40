"""Pins of the triple product (oracle/triple.py) against facts fixed
independently of its case analysis: every tripling coefficient of the theorem
equals the brute-force sum of the product of the three basis functions
(taken from the pinned inverse transform), the non-zero values are the
paper's 1, 2^l, +-2^l up to the texel normalisation 1/n, the literal triple
sum equals the texel-domain integral of the three reconstructed maps, a
constant BRDF reduces it to the double product, and the untruncated BRDF and
visibility give the double product with their texel-wise product."""
import itertools

import numpy as np
import pytest

from oracle.haar import haar_forward, haar_inverse
from oracle.relight import relight
from oracle.triple import (magnitude_map, relight_triple, triple_pixels, triple_sum,
                           tripling_coefficient)

pytestmark = pytest.mark.filterwarnings("ignore")


def _basis_matrix(n):
    """Row i = basis function i on the 6 n^2 texels (inverse transform of e_i)."""
    N = 6 * n * n
    return np.stack([haar_inverse(np.eye(N)[i].reshape(6, n, n)).ravel() for i in range(N)])


def test_tripling_coefficients_brute_force_n2():
    n = 2
    Bm = _basis_matrix(n)
    C = np.einsum("iq,jq,kq->ijk", Bm, Bm, Bm)
    N = 6 * n * n
    got = np.array([[[tripling_coefficient(i, j, k, n) for k in range(N)] for j in range(N)]
                    for i in range(N)])
    np.testing.assert_allclose(got, C, atol=1e-14)


@pytest.mark.parametrize("n", [4, 8])
def test_tripling_coefficients_brute_force_one_face(n):
    """All triples of face 2 at n = 4; 20,000 random same-face triples plus
    1,000 cross-face ones at n = 8."""
    Bm = _basis_matrix(n)
    nn = n * n
    rng = np.random.default_rng(n)
    if n == 4:
        trip = list(itertools.product(range(2 * nn, 3 * nn), repeat=3))
    else:
        f = rng.integers(0, 6, size=20000)
        trip = list(zip(*(f * nn + rng.integers(0, nn, size=20000) for _ in range(3))))
        # bias towards the structured cases: repeated indices and shared squares
        trip += [(i, i, k) for i, k in zip(rng.integers(0, nn, 3000), rng.integers(0, nn, 3000))]
        trip += [(i, k, i) for i, k in zip(rng.integers(0, nn, 3000), rng.integers(0, nn, 3000))]
        trip += list(zip(*(rng.integers(0, 6 * nn, size=1000) for _ in range(3))))
    for i, j, k in trip:
        want = float(np.sum(Bm[i] * Bm[j] * Bm[k]))
        assert abs(tripling_coefficient(i, j, k, n) - want) < 1e-14, (i, j, k, want)


def test_nonzero_values_are_the_papers_up_to_1_over_n():
    """n C_ijk lies in {1} (all scaling), {2^l} (three types on one square)
    or {+-2^l} (identical pair), l the level of the (third) function with
    l = 0 for the scaling function and the face-sized wavelets.  At n = 8
    the levels are 0, 1, 2; a coarser third wavelet is at level 0 or 1, so
    the negative values are -1 and -2."""
    n = 8
    nn = n * n
    seen = set()
    for i, j, k in itertools.product(range(nn), repeat=3):
        c = tripling_coefficient(i, j, k, n) * n
        if c == 0.0:
            continue
        l = np.log2(abs(c))
        assert abs(l - round(l)) < 1e-12 and 0 <= round(l) <= 2, (i, j, k, c)
        seen.add(round(c, 9))
    assert seen == {1.0, 2.0, 4.0, -1.0, -2.0}


@pytest.mark.parametrize("n,nnz", [(2, 10), (4, 40), (8, 120), (16, 300)])
def test_triple_sum_is_the_texel_integral(n, nnz):
    rng = np.random.default_rng(10 + n)
    N = 6 * n * n
    a = rng.normal(size=N)
    b = rng.normal(size=N)
    ci = np.sort(rng.choice(N, nnz, replace=False))
    cv = rng.normal(size=nnz)
    c = np.zeros(N)
    c[ci] = cv
    got = triple_sum(a, b, ci, cv, n)
    want = triple_pixels(a, b, c, n)
    assert abs(got - want) <= 1e-11 * (1 + np.abs(a).sum() * np.abs(b).max() * np.abs(cv).sum())


def _scene(n, V, nnz, seed):
    rng = np.random.default_rng(seed)
    N = 6 * n * n
    li = np.sort(rng.choice(N, N // 3, replace=False)).astype(np.int32)
    lv = rng.normal(size=li.size)
    ti = np.stack([np.sort(rng.choice(N, nnz, replace=False)) for _ in range(V)]).astype(np.int32)
    tv = rng.normal(size=(V, nnz))
    from scenes.scene import random_rotations
    R = np.stack(list(random_rotations(seed, V))).astype(np.float32)
    return li, lv, R, ti, tv


def test_constant_brdf_is_the_double_product():
    n = 8
    li, lv, R, ti, tv = _scene(n, 4, 60, 21)
    got = relight_triple(li, lv, n, R, None, ti, tv, np.ones((1, 6, n, n)))
    want = relight(li, lv, n, R, None, ti, tv)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11)


def test_untruncated_factors_give_the_premultiplied_transport():
    """b = Phong lobe x cosine x solid angle, c = visibility, both complete:
    the triple product equals the double product with their texel product
    (the premultiplied transport)."""
    from scenes.scene import phong_lobe, texel_directions, texel_solid_angles, visibility_np
    n = 8
    li, lv, R, _, _ = _scene(n, 3, 10, 22)
    lobe = phong_lobe([7.0, 30.0], texel_directions(n)[..., 1], texel_solid_angles(n))  # [2, 6, n, n]
    vis = visibility_np(5, np.arange(3), n).astype(np.float64)
    mat = np.array([1, 0, 1])
    N = 6 * n * n
    vi = np.tile(np.arange(N, dtype=np.int32), (3, 1))
    vv = haar_forward(vis).reshape(3, N)
    got = relight_triple(li, lv, n, R, None, vi, vv, lobe, mat)
    T = haar_forward(lobe[mat] * vis).reshape(3, N)
    want = relight(li, lv, n, R, None, None, T)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def test_invalid_material_gives_zero_and_scale_bounds_terms():
    n = 4
    li, lv, R, ti, tv = _scene(n, 3, 20, 23)
    brdf = np.random.default_rng(1).uniform(0.0, 1.0, size=(2, 6, n, n))
    out, scale = relight_triple(li, lv, n, R, None, ti, tv, brdf, np.array([0, 2, -1]),
                                return_scale=True)
    assert out[0, 1] == 0.0 and out[0, 2] == 0.0 and abs(out[0, 0]) > 0
    assert abs(out[0, 0]) <= scale[0, 0]


def test_magnitude_map_is_the_absolute_basis_sum():
    """magnitude_map = sum_i |v_i| |Psi_i| with the basis functions taken from
    the pinned inverse transform."""
    n = 4
    Bm = _basis_matrix(n)
    rng = np.random.default_rng(4)
    idx = rng.choice(6 * n * n, 50, replace=False)
    val = rng.normal(size=50)
    want = (np.abs(val)[:, None] * np.abs(Bm[idx])).sum(0).reshape(6, n, n)
    np.testing.assert_allclose(magnitude_map(idx, val, n), want, rtol=1e-13, atol=1e-13)
