"""Pins of the chain-rule rotation (oracle/chain.py) against facts fixed
independently of it: its face table reproduces the texel directions of the
exact geometry, its 2x2 step is the finest level of the Haar pyramid, the
identity rotation leaves the map unchanged, every rotation of the cube
group (where the mapping is a signed axis permutation and the chain rule is
exact) gives the exact resampling, and on a smooth map the result converges
to the exact resampling at first order in the texel size.  The analytic
Jacobian of the gnomonic map (the first derivatives and the mixed second
derivatives that carry D_x and D_y, which vanish under the cube group) is
pinned against central differences of an independently written projection
and, to second order, by a source map affine in source-face coordinates,
where the chain rule is exact for the continuous derivatives; mistakes
planted in the oracle's Jacobian fail both pins."""
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


# ---------------------------------------------------------------------------
# The analytic Jacobian of the gnomonic map (eq:pde1-eq:pde3 need x'_x, x'_y,
# y'_x, y'_y and the mixed x'_xy, y'_xy), pinned against numerical
# differentiation of the projection written out independently below.
# ---------------------------------------------------------------------------
def _dest_direction(F, x, y, n):
    """Direction of the continuous destination point (x, y) of face F (texel
    (i, j) spans [j, j+1) x [i, i+1)): the face table of the exact geometry
    with U = 2x - n, V = 2y - n."""
    U, V = 2.0 * x - n, 2.0 * y - n
    N = float(n)
    return np.array([(N, -V, -U), (-N, -V, U), (U, N, V),
                     (U, -N, -V), (U, -V, N), (-U, -V, -N)][F], dtype=np.float64)


def _source_coords(sface, w, n):
    """Continuous texel coordinates (x', y') of direction w projected on the
    plane of face `sface`: in-face components (sc, tc) over the major one,
    mapped from [-1, 1] to [0, n)."""
    x, y, z = w
    sc, tc, ma = [(-z, -y, x), (z, -y, -x), (x, z, y),
                  (x, -z, -y), (x, -y, z), (-x, -y, -z)][sface]
    return 0.5 * n * (sc / ma + 1.0), 0.5 * n * (tc / ma + 1.0)


def test_projection_tables_match_the_exact_geometry():
    n = 8
    tc = texel_centres(n)
    for F in range(6):
        for i in range(n):
            for j in range(n):
                d = _dest_direction(F, j + 0.5, i + 0.5, n)
                assert np.array_equal(d, tc[F, i, j])
                xs, ys = _source_coords(F, d, n)
                assert (xs, ys) == (j + 0.5, i + 0.5)


def _numeric_jacobian(R, F, sface, x, y, n, e1=1e-3, e2=3e-3):
    """Central differences of x'(x, y), y'(x, y) = projection on `sface` of
    R times the destination direction: first derivatives with step e1, the
    mixed second derivative with step e2 (both O(e^2) accurate)."""
    def xy(a, b):
        return np.array(_source_coords(sface, R @ _dest_direction(F, a, b, n), n))
    dxv = (xy(x + e1, y) - xy(x - e1, y)) / (2 * e1)
    dyv = (xy(x, y + e1) - xy(x, y - e1)) / (2 * e1)
    dxy = (xy(x + e2, y + e2) - xy(x + e2, y - e2) - xy(x - e2, y + e2)
           + xy(x - e2, y - e2)) / (4 * e2 * e2)
    return dxv[0], dyv[0], dxv[1], dyv[1], dxy[0], dxy[1]


def _general_rotations(count, seed):
    from scenes.scene import quaternion_rotations
    g = np.random.default_rng(seed)
    return [quaternion_rotations(q / np.linalg.norm(q)) for q in g.normal(size=(count, 4))]


def _jacobian_mismatch(n=32, rotations=4, seed=11):
    """Largest relative mismatch between chain.block_jacobian and the
    numerical derivatives at destination block centres of every face, for
    general rotations (D_x, D_y != 0) and the source face the exact map picks."""
    import oracle.chain as chain
    from oracle.sphere import quantise_rotation, source_index, scale_bits
    h = n // 2
    worst = 0.0
    g = np.random.default_rng(seed + 1)
    for R in _general_rotations(rotations, seed):
        Rq = quantise_rotation(np.asarray(R, np.float32), n)
        Rf = Rq.astype(np.float64) / float(1 << scale_bits(n))
        sface = source_index(Rq, h) // (h * h)
        for F in range(6):
            for bi, bj in g.integers(0, h, size=(6, 2)):
                x, y = 2.0 * bj + 1.0, 2.0 * bi + 1.0
                got = chain.block_jacobian(Rf, F, sface[F, bi, bj], 2 * x - n, 2 * y - n, n)
                ref = _numeric_jacobian(Rf, F, sface[F, bi, bj], x, y, n)
                scale = max(abs(r) for r in ref[:4])        # O(1) first derivatives
                for a, b, s in zip(got, ref, [scale] * 4 + [scale / n] * 2):
                    worst = max(worst, abs(float(a) - b) / s)
    return worst


def test_gnomonic_jacobian_matches_central_differences():
    assert _jacobian_mismatch() < 1e-6    # measured 1.9e-7


def _affine_mismatch(n=32, seed=5):
    """Second-order pin.  The source map is affine in continuous source
    coordinates, f = a + b x' + c y' sampled at texel centres, so every source
    block has H = -b, V = -c, D = 0.  The rotated map sampled continuously,
    g(x, y) = f(x'(x, y), y'(x, y)), has the exact derivatives
    g_x = b x'_x + c y'_x and g_xy = b x'_xy + c y'_xy, which is what the chain
    rule yields; the destination block's H, V, D are then the central
    differences of g over its four texel centres, equal to -g_x, -g_y, g_xy / 2
    at the block centre to O(1/n^2).  Small rotations keep the compared blocks
    (the centre region of every face) inside one source face.
    Returns the largest mismatch relative to the coefficients' scale."""
    from oracle.chain import chain_rotate, source_blocks
    from oracle.sphere import quantise_rotation, source_index, scale_bits
    from scenes.scene import quaternion_rotations
    a, b, c = 0.7, 0.013, -0.021
    worst = 0.0
    for axis in ([0.3, 0.8, -0.5], [-0.6, 0.2, 0.77], [0.1, -0.4, -0.9]):
        ax = np.asarray(axis) / np.linalg.norm(axis)
        ang = 0.17
        R = quaternion_rotations(np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * ax]))
        Rq = quantise_rotation(np.asarray(R, np.float32), n)
        Rf = Rq.astype(np.float64) / float(1 << scale_bits(n))
        h = n // 2
        sface = source_index(Rq, h) // (h * h)
        jj, ii = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
        P = np.broadcast_to(a + b * jj + c * ii, (6, n, n))
        got = source_blocks(chain_rotate(P, Rq))             # [6, h, h, (S, H, V, D)]
        for F in range(6):
            for bi in range(h // 2 - 3, h // 2 + 3):
                for bj in range(h // 2 - 3, h // 2 + 3):
                    sf = sface[F, bi, bj]

                    def g(x, y):
                        xs, ys = _source_coords(sf, Rf @ _dest_direction(F, x, y, n), n)
                        return a + b * xs + c * ys
                    x0, y0 = 2 * bj + 0.5, 2 * bi + 0.5
                    pa, pb = g(x0, y0), g(x0 + 1, y0)
                    pc, pd = g(x0, y0 + 1), g(x0 + 1, y0 + 1)
                    exact = np.array([(pa - pb + pc - pd) / 2, (pa + pb - pc - pd) / 2,
                                      (pa - pb - pc + pd) / 2])
                    err = np.abs(got[F, bi, bj, 1:] - exact)
                    # H, V against |b| + |c|; D (a second difference) against that over n
                    worst = max(worst, err[0] / (abs(b) + abs(c)), err[1] / (abs(b) + abs(c)),
                                err[2] * n / (abs(b) + abs(c)))
    return worst


def test_affine_map_matches_exact_differences_to_second_order():
    assert _affine_mismatch() < 1e-3      # measured 3.8e-5


_MUTATIONS = [
    ("x'_x: sign of the sc D_x term", "(scx * D - sc * Dx)", "(scx * D + sc * Dx)"),
    ("x'_y: sign of the sc D_y term", "(scy * D - sc * Dy)", "(scy * D + sc * Dy)"),
    ("y'_x: sign of the tc D_x term", "(tcx * D - tc * Dx)", "(tcx * D + tc * Dx)"),
    ("y'_y: sign of the tc D_y term", "(tcy * D - tc * Dy)", "(tcy * D + tc * Dy)"),
    ("x'_xy: sign of 2 sc D_x D_y / D^3", "(2 * sc * Dx * Dy / D**3 -", "(-2 * sc * Dx * Dy / D**3 -"),
    ("y'_xy: sign of 2 tc D_x D_y / D^3", "(2 * tc * Dx * Dy / D**3 -", "(-2 * tc * Dx * Dy / D**3 -"),
    ("x'_xy: sign of sc_y D_x", "(scx * Dy + scy * Dx)", "(scx * Dy - scy * Dx)"),
    ("y'_xy: sign of tc_x D_y", "(tcx * Dy + tcy * Dx)", "(-tcx * Dy + tcy * Dx)"),
    ("x'_xy dropped", "return xx, xy, yx, yy, xxy, yxy", "return xx, xy, yx, yy, 0 * xxy, yxy"),
    ("y'_xy dropped", "return xx, xy, yx, yy, xxy, yxy", "return xx, xy, yx, yy, xxy, 0 * yxy"),
]


@pytest.mark.parametrize("name,old,new", _MUTATIONS, ids=[m[0] for m in _MUTATIONS])
def test_pins_catch_planted_mistakes(monkeypatch, name, old, new):
    """Each mistake planted in the oracle's Jacobian (a flipped sign of a
    term carrying D_x or D_y, a dropped mixed derivative) fails both pins."""
    import inspect
    import textwrap

    import oracle.chain as chain
    src = textwrap.dedent(inspect.getsource(chain.gnomonic_jacobian))
    assert old in src, name
    scope = {}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), vars(chain).copy(), scope)
    monkeypatch.setattr(chain, "gnomonic_jacobian", scope["gnomonic_jacobian"])
    assert _jacobian_mismatch() > 1e-2, name  # measured 1.5 .. 3.8
    assert _affine_mismatch() > 5e-3, name   # measured 1.1e-2 .. 1.1e-1
