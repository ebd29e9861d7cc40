"""Pins of the checker's relighting, selection and of the scene generators
(no GPU).

* constant lighting: radiance = n c sum_F T[DC_F] for every rotation
  (closed form; the rotated constant map is the same constant);
* Parseval: the wavelet-domain inner product equals the pixel-domain sum of
  (W^T T)(q) g(q) with g gathered texel by texel in a plain loop;
* identity rotation: radiance = <T, L> with no rotation at all;
* a delta light at one texel reaches exactly the local texels that pull
  from it;
* the selection rule on hand-made ties; the dense phase shift is orthogonal
  (rotations of the cube group) and preserves a constant map;
* generators: total solid angle 4 pi, Phong normalisation -> 1, the
  occlusion rate, numpy/torch visibility agree bit for bit, Philox known
  answers.
"""
import numpy as np
import pytest

from oracle.haar import haar_forward, haar_inverse
from oracle.relight import (lighting_coefficients, phase_shift, reconstruct_lighting,
                            relight, transport_rows)
from oracle.select import topk_abs, topk_rows
from oracle.sphere import quantise_rotation, source_index
from scenes.philox import philox4x32_np, philox4x32_torch
from scenes.scene import (WORKLOADS, Workload, lighting_pixels, phong_lobe, random_rotations,
                          texel_directions, texel_solid_angles, transport_pixels,
                          transport_pixels_torch, visibility_np)


def _small_scene(n=8, V=5, nnz=20, seed=0):
    rng = np.random.default_rng(seed)
    L = rng.lognormal(size=(6, n, n)).astype(np.float32)
    li, lv = lighting_coefficients(L, 6 * n * n)
    T = rng.normal(size=(V, 6, n, n))
    ti, tv = transport_rows(T, nnz)
    R = random_rotations(seed + 1, V)
    return L, li, lv, ti, tv, R


@pytest.mark.parametrize("n", [4, 16])
def test_constant_lighting_closed_form(n):
    c = 1.75
    L = np.full((6, n, n), c, dtype=np.float32)
    li, lv = lighting_coefficients(L, 6)             # exactly the six DCs
    assert sorted(li.tolist()) == [f * n * n for f in range(6)]
    rng = np.random.default_rng(2)
    T = rng.normal(size=(4, 6, n, n))
    ti, tv = transport_rows(T, 6 * n * n // 2)
    R = random_rotations(4, 4)
    out = relight(li, lv, n, R, None, ti, tv)
    for v in range(4):
        full = np.zeros(6 * n * n)
        full[ti[v]] = tv[v]
        expect = n * c * sum(full[f * n * n] for f in range(6))
        assert abs(out[0, v] - expect) <= 1e-12 * max(1.0, abs(expect))


def test_parseval_pixel_domain_loop():
    n = 4
    _, li, lv, ti, tv, R = _small_scene(n=n, V=3, nnz=30)
    out = relight(li, lv, n, R, None, ti, tv)
    P = reconstruct_lighting(li, lv, n)
    for v in range(3):
        T = np.zeros(6 * n * n)
        T[ti[v]] = tv[v]
        t_pix = haar_inverse(T.reshape(6, n, n))
        src = source_index(quantise_rotation(R[v], n), n)
        acc = 0.0
        for f in range(6):
            for i in range(n):
                for j in range(n):
                    s = src[f, i, j]
                    acc += t_pix[f, i, j] * P[s // (n * n), (s // n) % n, s % n]
        assert abs(out[0, v] - acc) < 1e-11 * max(1.0, abs(acc))


def test_identity_rotation_plain_inner_product():
    n = 8
    _, li, lv, ti, tv, _ = _small_scene(n=n, V=4, nnz=40)
    R = np.tile(np.eye(3, dtype=np.float32), (4, 1, 1))
    out = relight(li, lv, n, R, None, ti, tv)
    Lc = np.zeros(6 * n * n)
    Lc[li] = lv
    for v in range(4):
        assert abs(out[0, v] - np.dot(tv[v].astype(np.float64), Lc[ti[v]])) < 1e-12


def test_delta_light():
    n = 8
    p = 2 * n * n + 3 * n + 5                           # one texel of +Y
    L = np.zeros((6, n, n), np.float32)
    L.reshape(-1)[p] = 4.0
    li, lv = lighting_coefficients(L, 6 * n * n)
    R = random_rotations(21, 3)
    rng = np.random.default_rng(5)
    T = rng.normal(size=(3, 6, n, n))
    ti, tv = transport_rows(T, 6 * n * n)
    out = relight(li, lv, n, R, None, ti, tv)
    for v in range(3):
        src = source_index(quantise_rotation(R[v], n), n).ravel()
        tp = haar_inverse(np.asarray(tv[v], np.float64)[np.argsort(ti[v])].reshape(6, n, n)).ravel()
        expect = 4.0 * tp[src == p].sum()
        assert abs(out[0, v] - expect) < 1e-11


def test_phase_shift_orthogonal_and_constant():
    n = 4
    rng = np.random.default_rng(8)
    c = rng.normal(size=(6, n, n))
    M = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], float)
    out = phase_shift(c, M)
    assert abs(np.sum(out ** 2) - np.sum(c ** 2)) < 1e-10
    const = haar_forward(np.full((6, n, n), 2.0))
    for R in random_rotations(31, 4):
        np.testing.assert_allclose(phase_shift(const, R), const, atol=1e-12)


def test_topk_ties_and_order():
    x = np.array([1.0, -3.0, 3.0, 0.5, -3.0, 2.0])
    assert topk_abs(x, 2).tolist() == [1, 2]           # |3| ties -> lower indices
    assert topk_abs(x, 3).tolist() == [1, 2, 4]
    assert topk_abs(x, 4).tolist() == [1, 2, 4, 5]
    assert topk_abs(x, 0).tolist() == []
    assert topk_abs(x, 6).tolist() == list(range(6))
    rng = np.random.default_rng(1)
    for _ in range(20):
        y = rng.integers(-4, 5, size=37).astype(float)
        k = int(rng.integers(0, 38))
        brute = sorted(sorted(range(37), key=lambda i: (-abs(y[i]), i))[:k])
        assert topk_abs(y, k).tolist() == brute
    idx, vals = topk_rows(np.array([[0.0, 2.0, -5.0], [1.0, 1.0, 1.0]]), 2)
    assert idx.tolist() == [[1, 2], [0, 1]] and vals.tolist() == [[2.0, -5.0], [1.0, 1.0]]


# --- generators -------------------------------------------------------------
def test_solid_angles_sum_to_sphere():
    for n in (1, 4, 32, 128):
        assert abs(6 * texel_solid_angles(n).sum() - 4 * np.pi) < 1e-12


def test_phong_normalisation_converges():
    # (n+2)/(2 pi) int_H cos^(n+1) dw = 1; the texel sum converges as n grows
    errs = []
    for n in (16, 64, 256):
        cos_y = texel_directions(n)[..., 1]
        lobe = phong_lobe([10.0], cos_y, texel_solid_angles(n))
        errs.append(abs(lobe.sum() - 1.0))
    assert errs[-1] < 2e-3 and errs[0] > errs[1] > errs[2]


def test_visibility_rate_and_backends():
    import torch
    w = Workload(9, "t", 16, 6, 4, 1, 6, 1.0, 5.0, "random")
    vis = visibility_np(9, np.arange(200), 16, 0.3)
    assert abs(1.0 - vis.mean() - 0.3) < 0.005
    exps = np.array([1.5, 7.0, 60.0])
    a = transport_pixels(w, exps, [3, 4, 5])
    b = transport_pixels_torch(w, exps, [3, 4, 5], "cpu").numpy()
    assert np.array_equal(a > 0, b > 0)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=0)
    c0 = torch.tensor([0, 0xFFFFFFFF], dtype=torch.int64)
    out_t = philox4x32_torch(c0, c0, c0, c0, 0, 0)
    out_n = philox4x32_np(np.array([0, 0xFFFFFFFF]), np.array([0, 0xFFFFFFFF]),
                          np.array([0, 0xFFFFFFFF]), np.array([0, 0xFFFFFFFF]), 0, 0)
    for x, y in zip(out_t, out_n):
        assert x.tolist() == y.tolist()


def test_philox_known_answers():
    # published known-answer vectors of Philox4x32-10
    out = philox4x32_np(0, 0, 0, 0, 0, 0)
    assert [int(v) for v in out] == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    m = 0xFFFFFFFF
    out = philox4x32_np(m, m, m, m, m, m)
    assert [int(v) for v in out] == [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    out = philox4x32_np(0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822, 0x299f31d0)
    assert [int(v) for v in out] == [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_lighting_generator():
    L = lighting_pixels(2, 32)
    assert L.shape == (6, 32, 32) and L.dtype == np.float32
    assert (L > 900).sum() >= 1 and (L > 900).sum() <= 4
    assert 0.9 < np.median(L) < 1.1                          # log-normal(0,1) median 1


def test_transport_rows_csr_form():
    w = WORKLOADS[2]
    wl = Workload(2, "t", 16, 64, 8, 1, 32, 1.0, 200.0, "random")
    T = transport_pixels(wl, np.array([2.0, 150.0]), [0, 1])
    idx, val = transport_rows(T, 32)
    assert idx.dtype == np.int32 and val.dtype == np.float32
    assert np.all(np.diff(idx, axis=1) > 0)
    assert w.nnz == 256
