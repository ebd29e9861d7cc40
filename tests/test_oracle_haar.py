"""Pins of the checker's Haar transform against things the paper and plain
mathematics fix (no GPU).

* a hand-computed 4x4 example (tests/golden/haar_4x4.txt);
* one 2x2 step is the 4-point Hadamard matrix / 2;
* orthonormality by brute force, Parseval, perfect reconstruction;
* a constant face has only the DC coefficient N*c;
* the paper's direct coarse-level formula (Sec. V.B: triangle kernel h_t on
  row/column finite differences, box kernel h_s, downsampling by 2^(l+2))
  reproduces every H, V and D coefficient of every level;
* the recursive evaluation of Sec. V.C (repeated convolution with the
  3-tap h_t upsampled by 2^l) regenerates the level kernels.
"""
import os

import numpy as np
import pytest

from oracle.haar import coefficient_block, haar_forward, haar_inverse

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden_haar():
    rows = {"input": [], "output": []}
    cur = None
    with open(os.path.join(GOLDEN, "haar_4x4.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line in rows:
                cur = line
                continue
            rows[cur].append([float(t) for t in line.split()])
    return np.array(rows["input"]), np.array(rows["output"])


def test_golden_4x4():
    x, y = _read_golden_haar()
    np.testing.assert_array_equal(haar_forward(x), y)
    np.testing.assert_array_equal(haar_inverse(y), x)


def test_single_step_is_hadamard():
    # coefficients (S, H, V, D) of [[a, b], [c, d]] = (1/2) Hadamard_4 (a, b, c, d)
    had = 0.5 * np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], float)
    for k in range(4):
        e = np.zeros(4)
        e[k] = 1.0
        out = haar_forward(e.reshape(2, 2))
        got = np.array([out[0, 0], out[0, 1], out[1, 0], out[1, 1]])
        np.testing.assert_array_equal(got, had[:, k])


@pytest.mark.parametrize("n", [2, 4, 8])
def test_orthonormal_brute_force(n):
    W = np.stack([haar_forward(np.eye(n * n)[k].reshape(n, n)).ravel() for k in range(n * n)], 1)
    np.testing.assert_allclose(W @ W.T, np.eye(n * n), atol=1e-15)
    Wi = np.stack([haar_inverse(np.eye(n * n)[k].reshape(n, n)).ravel() for k in range(n * n)], 1)
    np.testing.assert_allclose(Wi, W.T, atol=1e-15)


def test_parseval_and_reconstruction():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(6, 32, 32))
    c = haar_forward(x)
    assert abs(np.sum(c * c) - np.sum(x * x)) < 1e-9 * np.sum(x * x)
    np.testing.assert_allclose(haar_inverse(c), x, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 8, 64])
def test_constant_face_has_only_dc(n):
    c = haar_forward(np.full((n, n), 3.25))
    expect = np.zeros((n, n))
    expect[0, 0] = n * 3.25
    np.testing.assert_allclose(c, expect, atol=1e-12)


def test_coefficient_block_layout():
    n = 8
    assert coefficient_block(0, 0, n) == ("S", 8, 0, 0)
    assert coefficient_block(0, 1, n) == ("H", 8, 0, 0)
    assert coefficient_block(1, 0, n) == ("V", 8, 0, 0)
    assert coefficient_block(1, 1, n) == ("D", 8, 0, 0)
    assert coefficient_block(2, 7, n) == ("H", 2, 2, 3)
    assert coefficient_block(5, 2, n) == ("V", 2, 1, 2)
    assert coefficient_block(6, 6, n) == ("D", 2, 2, 2)
    assert coefficient_block(3, 1, n) == ("V", 4, 1, 1)


# --- the paper's direct coarse-level formula -------------------------------
def _tri(l):
    """h_t of level j-l: 2^(l+1) - |t| for |t| <= 2^(l+1) - 1."""
    r = (1 << (l + 1)) - 1
    t = np.arange(-r, r + 1)
    return (1 << (l + 1)) - np.abs(t)


def _paper_coefficients(g, kind, l):
    """Coefficients of block side B = 2^(l+2) from the finest-level finite
    differences of g, per the paper's kernel formula (with the box kernel
    read as having 2^(l+2) taps and the triangle centred on the block's last
    top/left row/column)."""
    n = g.shape[0]
    B = 1 << (l + 2)
    tri = _tri(l)
    r = len(tri) // 2
    pad = np.zeros((n + 2, n + 2))
    pad[:n, :n] = g
    gr = pad[:n + 1, :n + 1] - pad[1:n + 2, :n + 1]             # g(r,c) - g(r+1,c)
    gc = pad[:n + 1, :n + 1] - pad[:n + 1, 1:n + 2]             # g(r,c) - g(r,c+1)
    grc = pad[:n + 1, :n + 1] - pad[1:, :n + 1] - pad[:n + 1, 1:] + pad[1:, 1:]
    out = np.zeros((n // B, n // B))
    for br in range(n // B):
        for bc in range(n // B):
            r0, c0 = br * B, bc * B
            tc_r, tc_c = r0 + B // 2 - 1, c0 + B // 2 - 1         # triangle centres
            acc = 0.0
            if kind == "V":      # triangle along rows on g_theta, box along columns
                for c in range(c0, c0 + B):
                    for k, t in enumerate(range(tc_r - r, tc_r + r + 1)):
                        acc += tri[k] * gr[t, c]
            elif kind == "H":    # roles interchanged
                for rr in range(r0, r0 + B):
                    for k, t in enumerate(range(tc_c - r, tc_c + r + 1)):
                        acc += tri[k] * gc[rr, t]
            else:                # cross-derivative, triangle in both directions
                for ka, ta in enumerate(range(tc_r - r, tc_r + r + 1)):
                    for kb, tb in enumerate(range(tc_c - r, tc_c + r + 1)):
                        acc += tri[ka] * tri[kb] * grc[ta, tb]
            out[br, bc] = acc / B
    return out


@pytest.mark.parametrize("kind", ["H", "V", "D"])
def test_paper_direct_formula_matches_pyramid(kind):
    n = 16
    g = np.random.default_rng(1).normal(size=(n, n))
    c = haar_forward(g)
    for l in range(-1, 3):                   # block sides 2, 4, 8, 16
        B = 1 << (l + 2)
        q = n // B
        expect = {"H": c[:q, q:2 * q], "V": c[q:2 * q, :q], "D": c[q:2 * q, q:2 * q]}[kind]
        got = _paper_coefficients(g, kind, l)
        np.testing.assert_allclose(got, expect, atol=1e-12, err_msg=f"{kind} l={l}")


def test_recursive_kernel_factorisation():
    # h_{t, j-l} = h_{t, j-l+1} * (h_{t, j} upsampled by 2^l): the repeated
    # convolution of Sec. V.C regenerates every level's triangle.
    base = _tri(0)                             # [1, 2, 1]
    cur = base.copy()
    for l in range(1, 5):
        up = np.zeros(2 * (1 << l) + 1)
        up[::1 << l] = base
        cur = np.convolve(cur, up)
        np.testing.assert_array_equal(cur, _tri(l))
    # The printed single-step form h_{t,j} * h^l_{t,j} matches only for l = 1.
    up2 = np.zeros(2 * 4 + 1)
    up2[::4] = base
    assert not np.array_equal(np.convolve(base, up2), _tri(2))
