"""Pins of the longitude-latitude rotation (oracle/latlong.py) against facts
fixed independently of its binary32 decision sequence: its tables are the
binary32 roundings of the exact sines and cosines (checked with Python's
math module), the identity is the identity, azimuth shifts are cyclic column
shifts, the half turn about X has a closed form, the map agrees with FP64
spherical geometry (arccos / arctan2 of R p for R = R_y R_x R_y) on every
texel not within 1e-5 rad of a cell boundary, and the relit result has the
constant-lighting closed form and the identity-rotation inner product."""
import math

import numpy as np
import pytest

from oracle.haar import haar_forward
from oracle.latlong import grid, relight_latlong, rotate, source_index

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.mark.parametrize("H", [4, 8, 128, 512])
def test_grid_is_rounded_exact_trig(H):
    St, ct, sf, kf, C = grid(H)
    for i in range(H):
        t = (i + 0.5) * math.pi / H
        assert St[i] == np.float32(math.sin(t)) and ct[i] == np.float32(math.cos(t))
        assert C[i] == np.float32(math.cos(i * math.pi / H))
    for j in range(2 * H):
        f = (j + 0.5) * math.pi / H
        assert sf[j] == np.float32(math.sin(f)) and kf[j] == np.float32(math.cos(f))
    assert np.all(np.diff(C) < 0)                   # strictly decreasing: counts = searches


def _dest_layout(src, H):
    """[2, H, H] -> [H, 2H] destination rows/columns."""
    return np.concatenate([src[0], src[1]], axis=1)


def _flat(row, col, H):
    return (col // H) * H * H + row * H + (col % H)


@pytest.mark.parametrize("H", [4, 16, 64])
def test_identity_and_shifts(H):
    W = 2 * H
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    assert np.array_equal(_dest_layout(source_index(H, 1.0, 0.0, 0, 0), H), _flat(i, j, H))
    for sa, sc in [(1, 0), (0, 5), (3, W - 1), (W + 2, -7)]:
        got = _dest_layout(source_index(H, 1.0, 0.0, sa, sc), H)
        assert np.array_equal(got, _flat(i, (j + sa + sc) % W, H)), (sa, sc)


@pytest.mark.parametrize("H", [4, 32, 128])
def test_half_turn_about_x(H):
    """R_x(pi): (x, y, z) -> (x, -y, -z), so elevation t -> pi - t and
    azimuth f -> pi - f: row H-1-i, column (H-1-j) mod 2H."""
    W = 2 * H
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    got = _dest_layout(source_index(H, -1.0, 0.0, 0, 0), H)
    assert np.array_equal(got, _flat(H - 1 - i, (H - 1 - j) % W, H))


def _ry(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


@pytest.mark.parametrize("H,seed", [(16, 1), (64, 2), (128, 3), (256, 4)])
def test_agrees_with_fp64_geometry_away_from_boundaries(H, seed):
    W = 2 * H
    d = np.pi / H
    rng = np.random.default_rng(seed)
    t, f = (np.arange(H) + 0.5) * d, (np.arange(W) + 0.5) * d
    T, F = np.meshgrid(t, f, indexing="ij")
    p = np.stack([np.sin(T) * np.sin(F), np.cos(T), np.sin(T) * np.cos(F)], axis=-1)
    checked = 0
    for _ in range(4):
        b = math.acos(rng.uniform(-1, 1))
        cb, sb = np.float32(math.cos(b)), np.float32(math.sin(b))
        sa, sc = (int(x) for x in rng.integers(0, W, 2))
        bb = math.atan2(float(sb), float(cb))
        Rx = np.array([[1, 0, 0], [0, math.cos(bb), -math.sin(bb)], [0, math.sin(bb), math.cos(bb)]])
        R = _ry(sa * d) @ Rx @ _ry(sc * d)
        q = p @ R.T
        q /= np.linalg.norm(q, axis=-1, keepdims=True)
        tq = np.arccos(np.clip(q[..., 1], -1, 1))
        fq = np.arctan2(q[..., 0], q[..., 2]) % (2 * np.pi)
        row = np.floor(tq / d).astype(np.int64)
        col = np.floor(fq / d).astype(np.int64) % W
        mt = np.minimum(tq / d - row, row + 1 - tq / d) * d
        mf = np.minimum(fq / d - np.floor(fq / d), np.floor(fq / d) + 1 - fq / d) * d * np.sin(tq)
        safe = (mt > 1e-5) & (mf > 1e-5)
        got = _dest_layout(source_index(H, cb, sb, sa, sc), H)
        want = _flat(np.minimum(row, H - 1), col, H)
        assert np.array_equal(got[safe], want[safe])
        assert safe.mean() > 0.99
        checked += int(safe.sum())
    assert checked > 0


def test_haar_per_square_and_constant_lighting():
    """A constant map c has one coefficient per square, H c; rotation keeps it
    constant, so radiance = H c (T[DC_0] + T[DC_1])."""
    H, c = 16, 2.5
    N = 2 * H * H
    li = np.arange(N, dtype=np.int32)
    lv = haar_forward(np.full((2, H, H), c)).ravel()
    assert np.allclose(lv[[0, H * H]], H * c) and np.allclose(np.delete(lv, [0, H * H]), 0)
    rng = np.random.default_rng(7)
    ti = np.stack([np.sort(rng.choice(N, 40, replace=False)) for _ in range(3)])
    ti[:, 0] = 0
    ti = np.sort(ti, axis=1).astype(np.int32)
    tv = rng.normal(size=(3, 40))
    elev = np.array([[0.3, 0.953939], [-0.8, 0.6], [1.0, 0.0]], np.float32)
    shift = np.array([[3, 9], [0, 31], [5, 5]])
    got = relight_latlong(li, lv, H, elev, shift, ti, tv)
    for v in range(3):
        want = H * c * (tv[v][ti[v] == 0].sum() + tv[v][ti[v] == H * H].sum())
        assert abs(got[0, v] - want) <= 1e-10 * (1 + abs(want))


def test_identity_rotation_is_a_plain_inner_product():
    H = 8
    N = 2 * H * H
    rng = np.random.default_rng(8)
    li = np.sort(rng.choice(N, 60, replace=False)).astype(np.int32)
    lv = rng.normal(size=60)
    ti = np.stack([np.sort(rng.choice(N, 30, replace=False)) for _ in range(2)]).astype(np.int32)
    tv = rng.normal(size=(2, 30))
    got = relight_latlong(li, lv, H, np.array([[1.0, 0.0]] * 2, np.float32), np.zeros((2, 2)),
                          ti, tv)
    L = np.zeros(N)
    L[li] = lv
    for v in range(2):
        assert abs(got[0, v] - np.dot(L[ti[v]], tv[v])) <= 1e-12


def test_rotate_is_a_gather():
    H = 8
    P = np.arange(2 * H * H, dtype=np.float64).reshape(2, H, H)
    g = rotate(P, np.float32(0.6), np.float32(0.8), 3, 4)
    assert np.array_equal(g, source_index(H, 0.6, 0.8, 3, 4).astype(np.float64))
