"""Pins of the chain-rule rotation (oracle/chain.py) against facts fixed
independently of it: its face table reproduces the texel directions of the
exact geometry, its 2x2 step is the finest level of the Haar pyramid, the
identity rotation leaves the map unchanged, every rotation of the cube
group (where the mapping is a signed axis permutation and the chain rule is
exact) gives the exact resampling, and on a smooth map the result converges
to the exact resampling at first order in the texel size."""
import itertools

import numpy as np
import pytest

from oracle.chain import FACE_AXES, blocks_to_pixels, chain_rotate, relight_chain, source_blocks
from oracle.haar import haar_forward
from oracle.relight import relight
from oracle.sphere import quantise_rotation, rotate_pixels, texel_centres


def _cube_group():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            M = np.zeros((3, 3))
            for r in range(3):
                M[r, perm[r]] = signs[r]
            if np.linalg.det(M) > 0:
                mats.append(M)
    return mats


def test_face_axes_reproduce_texel_directions():
    n = 8
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    U, V = 2 * j + 1 - n, 2 * i + 1 - n
    tc = texel_centres(n)
    for F in range(6):
        d = U[..., None] * FACE_AXES[F][0] + V[..., None] * FACE_AXES[F][1] + n * FACE_AXES[F][2]
        assert np.array_equal(d, tc[F])


def test_block_step_is_the_finest_pyramid_level():
    n = 8
    P = np.random.default_rng(0).normal(size=(6, n, n))
    B = source_blocks(P)
    W = haar_forward(P)
    h = n // 2
    # the finest level of the Mallat layout: H, V, D quadrants of the full face
    np.testing.assert_allclose(B[..., 1], W[:, :h, h:], atol=1e-12)
    np.testing.assert_allclose(B[..., 2], W[:, h:, :h], atol=1e-12)
    np.testing.assert_allclose(B[..., 3], W[:, h:, h:], atol=1e-12)
    np.testing.assert_allclose(blocks_to_pixels(B), P, atol=1e-12)


def test_identity_rotation_keeps_the_map():
    P = np.random.default_rng(1).normal(size=(6, 16, 16))
    np.testing.assert_allclose(chain_rotate(P, quantise_rotation(np.eye(3), 16)), P, atol=1e-12)


def test_cube_group_gives_the_exact_resampling():
    P = np.random.default_rng(2).normal(size=(6, 8, 8))
    mats = _cube_group()
    assert len(mats) == 24
    for M in mats:
        Rq = quantise_rotation(M, 8)
        np.testing.assert_allclose(chain_rotate(P, Rq), rotate_pixels(P, Rq), atol=1e-12)


def test_first_order_convergence_on_a_smooth_map():
    from scenes.scene import quaternion_rotations
    a = np.array([0.3, -0.5, 0.8])
    b = np.array([0.2, 0.7, -0.1])
    R = quaternion_rotations(np.array([0.9, 0.2, -0.3, 0.25]))
    errs = []
    for n in (16, 32, 64):
        Rq = quantise_rotation(R, n)
        w = texel_centres(n).astype(np.float64)
        w /= np.linalg.norm(w, axis=-1, keepdims=True)
        f = (w @ a) ** 2 + np.sin(3 * (w @ b))
        ex = rotate_pixels(f, Rq)
        errs.append(np.linalg.norm(chain_rotate(f, Rq) - ex) / np.linalg.norm(ex))
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs


def test_relight_chain_equals_relight_for_cube_rotations():
    rng = np.random.default_rng(3)
    n = 8
    li = np.arange(6 * n * n, dtype=np.int32)
    lv = rng.normal(size=6 * n * n)
    ti = np.stack([np.sort(rng.choice(6 * n * n, 50, replace=False)) for _ in range(3)]).astype(np.int32)
    tv = rng.normal(size=(3, 50))
    R = np.stack(_cube_group()[5:8]).astype(np.float32)
    np.testing.assert_allclose(relight_chain(li, lv, n, R, None, ti, tv),
                               relight(li, lv, n, R, None, ti, tv), rtol=1e-12, atol=1e-12)


def _psnr(got, ref):
    """10 log10(max(ref)^2 / MSE) over the compared quantity."""
    return 10.0 * np.log10(np.max(ref) ** 2 / np.mean((got - ref) ** 2))


def test_chain_rule_error_on_benchmark_scene():
    """Measurement, not a pin: error of the chain-rule rotation against the
    exact method on 40 vertices of the benchmark scene (6 x 128^2, top-1024
    lighting, CSR-256 Phong transport): relative L2 and PSNR of the radiance,
    and PSNR of the rotated map itself for that lighting and for a smooth
    one (a quadratic in the direction).  The first-order rule drops the
    second derivatives, which the benchmark's HDR lighting (iid texels plus
    point lights) has in abundance, so only loose sanity bounds are
    asserted."""
    from cases import build_case
    from oracle.relight import rel_l2, reconstruct_lighting
    from scenes.scene import WORKLOADS, random_rotations, texel_directions
    w = WORKLOADS[2]
    case = build_case(w, np.arange(0, 50000, 1250))
    exact = relight(case["light_idx"], case["light_val"], w.n, case["vert_rot"], None,
                    case["t_idx"], case["t_val"])
    approx = relight_chain(case["light_idx"], case["light_val"], w.n, case["vert_rot"], None,
                           case["t_idx"], case["t_val"])
    e = rel_l2(approx[0], exact[0])
    print("\nchain rule, benchmark scene radiance: rel-L2 %.3e, PSNR %.1f dB"
          % (e, _psnr(approx[0], exact[0])))
    assert 0.0 < e < 0.5
    P = reconstruct_lighting(case["light_idx"], case["light_val"], w.n)
    d = texel_directions(w.n)
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    smooth = 1.0 + d[..., 0] + 0.5 * d[..., 1] * d[..., 2] + 0.25 * d[..., 2] ** 2
    for name, M in (("benchmark lighting", P), ("smooth map", smooth)):
        ps, es = [], []
        for R in random_rotations(7, 3):
            Rq = quantise_rotation(np.asarray(R, np.float32), w.n)
            a, b = chain_rotate(M, Rq), rotate_pixels(M, Rq)
            ps.append(_psnr(a, b))
            es.append(np.linalg.norm(a - b) / np.linalg.norm(b))
        print("chain rule, rotated %s: PSNR %.1f dB, rel-L2 %.3e (mean of 3 rotations)"
              % (name, np.mean(ps), np.mean(es)))
    assert np.mean(es) < 2e-2          # the smooth map: first-order accurate
