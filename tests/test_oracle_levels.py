"""Pins of the coarse-level start (oracle/levels.py) against facts fixed by
the orthonormal Haar pyramid and the cube group, independent of the code
under test: the index remap is a bijection of the coarse corner, the coarse
corner of the pyramid equals the pyramid of the block-sum map, k = 0 is the
full method, the identity rotation reduces to a plain inner product, a
cube-group rotation commutes with the coarsening, constant lighting has its
closed form."""
import numpy as np
import pytest

from oracle.haar import haar_forward
from oracle.levels import coarse_index, relight_from_level
from oracle.relight import relight

pytestmark = pytest.mark.filterwarnings("ignore")


def _block_sum_over_B(P, B):
    F, n, _ = P.shape
    return P.reshape(F, n // B, B, n // B, B).sum(axis=(2, 4)) / B


def test_coarse_index_bijection_and_hand_values():
    n, k = 8, 1
    ci = coarse_index(np.arange(6 * n * n), n, k)
    kept = ci[ci >= 0]
    assert np.array_equal(np.sort(kept), np.arange(6 * 4 * 4))
    assert (ci < 0).sum() == 6 * (64 - 16)
    # face 2, row 1, column 3 -> 2*16 + 1*4 + 3; face 0, row 4 -> finer level
    assert coarse_index([2 * 64 + 1 * 8 + 3], n, k)[0] == 39
    assert coarse_index([0 * 64 + 4 * 8 + 0], n, k)[0] == -1
    assert coarse_index([-5, 6 * 64], n, k).tolist() == [-1, -1]


@pytest.mark.parametrize("n,k", [(8, 1), (16, 2), (32, 3)])
def test_coarse_corner_is_pyramid_of_block_sums(n, k):
    rng = np.random.default_rng(n + k)
    P = rng.normal(size=(6, n, n))
    B = 1 << k
    nc = n // B
    full = haar_forward(P)
    coarse = haar_forward(_block_sum_over_B(P, B))
    np.testing.assert_allclose(full[:, :nc, :nc], coarse, rtol=1e-12, atol=1e-12)


def _scene(n, V, nnz, seed):
    rng = np.random.default_rng(seed)
    K = 6 * n * n // 3
    li = np.sort(rng.choice(6 * n * n, K, replace=False)).astype(np.int32)
    lv = rng.normal(size=K)
    ti = np.stack([np.sort(rng.choice(6 * n * n, nnz, replace=False)) for _ in range(V)]).astype(np.int32)
    tv = rng.normal(size=(V, nnz))
    return li, lv, ti, tv


def test_level_zero_is_the_full_method():
    n = 8
    li, lv, ti, tv = _scene(n, 3, 40, 1)
    rng = np.random.default_rng(2)
    q = rng.normal(size=(3, 4))
    from scenes.scene import quaternion_rotations
    R = quaternion_rotations(q).astype(np.float32)
    np.testing.assert_array_equal(relight_from_level(li, lv, n, R, None, ti, tv, 0),
                                  relight(li, lv, n, R, None, ti, tv))


@pytest.mark.parametrize("k", [1, 2])
def test_identity_rotation_is_a_plain_inner_product(k):
    n = 16
    li, lv, ti, tv = _scene(n, 4, 200, 3)
    R = np.tile(np.eye(3, dtype=np.float32), (4, 1, 1))
    got = relight_from_level(li, lv, n, R, None, ti, tv, k)
    L = np.zeros(6 * n * n)
    L[li] = lv
    for v in range(4):
        keep = coarse_index(ti[v], n, k) >= 0
        want = np.dot(L[ti[v][keep]], tv[v][keep])
        assert abs(got[0, v] - want) <= 1e-12 * (1 + abs(want))


@pytest.mark.parametrize("k", [1, 2])
def test_cube_rotation_commutes_with_coarsening(k):
    """A quarter turn maps blocks onto blocks: rotating at n' equals the
    full-resolution result restricted to the coarse coefficients."""
    n = 16
    li, lv, ti, tv = _scene(n, 3, 300, 4)
    rots = np.array([[[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
                     [[1, 0, 0], [0, 0, -1], [0, 1, 0]],
                     [[0, -1, 0], [1, 0, 0], [0, 0, 1]]], dtype=np.float32)
    got = relight_from_level(li, lv, n, rots, None, ti, tv, k)
    for v in range(3):
        keep = coarse_index(ti[v], n, k) >= 0
        want = relight(li, lv, n, rots[v:v + 1], None, ti[v:v + 1, keep], tv[v:v + 1, keep])
        assert abs(got[0, v] - want[0, 0]) <= 1e-11 * (1 + abs(want[0, 0]))


def test_constant_lighting_closed_form():
    n, k, c = 16, 2, 1.75
    li = np.arange(6 * n * n, dtype=np.int32)
    lv = haar_forward(np.full((6, n, n), c)).ravel()
    rng = np.random.default_rng(5)
    ti = np.stack([np.sort(rng.choice(6 * n * n, 100, replace=False)) for _ in range(2)])
    ti[:, 0] = 0                      # face 0 scaling coefficient always present
    ti = np.sort(ti, axis=1).astype(np.int32)
    tv = rng.normal(size=(2, 100))
    from scenes.scene import quaternion_rotations
    R = quaternion_rotations(rng.normal(size=(2, 4))).astype(np.float32)
    got = relight_from_level(li, lv, n, R, None, ti, tv, k)
    for v in range(2):
        dc = [f * n * n for f in range(6)]
        want = sum(n * c * tv[v][ti[v] == d].sum() for d in dc)
        assert abs(got[0, v] - want) <= 1e-10 * (1 + abs(want))


def test_coarse_start_error_on_benchmark_scene():
    """Measurement, not a pin: relative L2 error of starting the rotation 1,
    2, 3 levels below the finest one on 40 vertices of the benchmark scene
    (6 x 128^2, top-1024 lighting, CSR-256 Phong transport, random frames)
    against the exact method.  Only a loose sanity bound is asserted: the
    error need not grow monotonically with the skipped levels."""
    from cases import build_case
    from oracle.relight import rel_l2
    from scenes.scene import WORKLOADS
    w = WORKLOADS[2]
    case = build_case(w, np.arange(0, 50000, 1250))
    exact = relight(case["light_idx"], case["light_val"], w.n, case["vert_rot"], None,
                    case["t_idx"], case["t_val"])
    errs = []
    for k in (1, 2, 3):
        approx = relight_from_level(case["light_idx"], case["light_val"], w.n, case["vert_rot"],
                                    None, case["t_idx"], case["t_val"], k)
        errs.append(rel_l2(approx[0], exact[0]))
    print("coarse-level start rel-L2 (k = 1, 2, 3):", ["%.3e" % e for e in errs])
    assert all(0.0 < e < 0.5 for e in errs)


def test_transport_budget_error_on_benchmark_scene():
    """Measurement, not a pin: relative L2 error of keeping only the m
    largest transport coefficients per vertex (m = 4, 16, 64, 256; the
    coefficient budgets of Sec. VI) on 40 vertices of the benchmark scene
    against the untruncated transport (all 6 n^2 coefficients), both with the
    exact rotation.  The error must shrink as the budget grows."""
    import dataclasses

    from cases import build_case, stored_transport
    from oracle.relight import rel_l2
    from scenes.scene import WORKLOADS
    w = WORKLOADS[2]
    vids = np.arange(0, 50000, 1250)
    case = build_case(w, vids)
    wd = dataclasses.replace(w, nnz=6 * w.n * w.n)
    _, dense = stored_transport(wd, vids)
    full = relight(case["light_idx"], case["light_val"], w.n, case["vert_rot"], None, None, dense)
    errs = []
    for m in (4, 16, 64, 256):
        ti, tv = stored_transport(dataclasses.replace(w, nnz=m), vids)
        got = relight(case["light_idx"], case["light_val"], w.n, case["vert_rot"], None, ti, tv)
        errs.append(rel_l2(got[0], full[0]))
    print("\ntransport budget rel-L2 (m = 4, 16, 64, 256):", ["%.3e" % e for e in errs])
    assert all(a > b for a, b in zip(errs, errs[1:]))
