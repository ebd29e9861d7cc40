"""GPU parity of the HIP path (through the C ABI) against the FP64 checker.

Tolerances of the FP32 path:
  * workload-shaped cases (the paper-style scenes: n >= 32, Phong transport,
    HDR lighting): rel-L2 per frame <= 1e-5 against the FP64 checker on the
    same stored inputs;
  * every element (all cases): |got - ref| <= 1e-5 |ref| + 2e-7 s, where
    s = sum_k |T_k ghat_k| is the checker's magnitude scale of the inner
    product.  2e-7 is about 3.4 binary32 unit roundoffs: the FP32 pipeline
    (reconstruction, gather, 2x2 levels, products, tree sum) perturbs each
    term by a few roundoffs, so ill-conditioned tiny cases (cancelling terms,
    s >> |ref|) are judged against s instead of |ref|.
Integer work (selection indices, storage codes) is compared bit for bit.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def rrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_07272_amd as m
    return m


def dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def check_frames(got, ref_scale, tol=TOL_F32, rel_l2=True):
    """ref_scale = (reference [F, V], magnitude scale [F, V])."""
    from cases import frame_errors
    ref, scale = ref_scale
    got = np.asarray(got, np.float64)
    bound = 1e-5 * np.abs(ref) + 2e-7 * scale
    worst = np.max(np.abs(got - ref) - bound) if ref.size else -1.0
    assert worst <= 0.0, (np.abs(got - ref) / np.maximum(bound, 1e-300)).max()
    errs = frame_errors(got, ref) if ref.size else [0.0]
    if rel_l2:
        assert max(errs) <= tol, errs
    return max(errs)


# ---------------------------------------------------------------- Haar (a1, a3)
def _forward_magnitude(x):
    """|W| |x|: at every coefficient of a block of side B (its S, H, V and D
    alike) the block's sum of |x| divided by B, in the Mallat layout."""
    x = np.abs(np.asarray(x, np.float64))
    out = np.empty_like(x)
    cur, n = x, x.shape[-1]
    while n > 1:
        h = n // 2
        s = (cur[..., 0::2, 0::2] + cur[..., 0::2, 1::2] + cur[..., 1::2, 0::2] + cur[..., 1::2, 1::2]) / 2
        out[..., :h, h:n] = s
        out[..., h:n, :h] = s
        out[..., h:n, h:n] = s
        cur, n = s, h
    out[..., :1, :1] = cur
    return out


def _inverse_magnitude(c):
    """|W^T| |c|: every pixel's sum over its ancestors' |coefficient| / B."""
    c = np.abs(np.asarray(c, np.float64))
    N = c.shape[-1]
    cur, n = c[..., :1, :1], 1
    while n < N:
        S, H, V, D = cur, c[..., :n, n:2 * n], c[..., n:2 * n, :n], c[..., n:2 * n, n:2 * n]
        t = (S + H + V + D) / 2
        nxt = np.empty(c.shape[:-2] + (2 * n, 2 * n))
        for dr in (0, 1):
            for dc in (0, 1):
                nxt[..., dr::2, dc::2] = t
        cur, n = nxt, 2 * n
    return cur


@pytest.mark.parametrize("n,count", [(1, 2), (2, 3), (8, 1), (32, 2), (64, 3), (128, 1), (256, 2),
                                     (512, 1), (1024, 1)])
def test_haar_forward_inverse(rrt, n, count):
    """Element by element: each output of the FP32 transform passes through
    at most 2 log2(n) + 2 binary32 roundings of partial sums whose size is
    bounded by the magnitude transform (|W| |x| forward, |W^T| |c|
    inverse), so |got - ref| <= 2^-23 (2 log2 n + 2) |W| |x|."""
    from oracle.haar import haar_forward, haar_inverse
    rng = np.random.default_rng(n + count)
    x = rng.normal(size=(count, 6, n, n)).astype(np.float32)
    depth = 2 * int(np.log2(n)) + 2
    got = rrt.haar_forward(dev(x)).cpu().numpy()
    ref = haar_forward(x.astype(np.float64))
    bound = 2.0 ** -23 * depth * _forward_magnitude(x)
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))
    assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)
    back = rrt.haar_inverse(dev(got)).cpu().numpy()
    ref_back = haar_inverse(got.astype(np.float64))
    bound = 2.0 ** -23 * depth * _inverse_magnitude(got)
    assert np.all(np.abs(back - ref_back) <= bound), float(np.max(np.abs(back - ref_back) / bound))
    assert np.linalg.norm(back - ref_back) <= 1e-6 * np.linalg.norm(ref_back)


# ---------------------------------------------------------------- selection (a2)
@pytest.mark.parametrize("rows,length,k", [(1, 1, 1), (3, 5, 2), (2, 1000, 7), (4, 1025, 1025),
                                           (1, 98304, 1024), (5, 6144, 256), (2, 3000, 0),
                                           (2, 20000, 1), (3, 16384, 16383), (1, 300001, 5000),
                                           (8, 24576, 2048), (9, 16384, 100)])
def test_topk_exact(rrt, rows, length, k):
    from oracle.select import topk_abs
    rng = np.random.default_rng(rows * 7 + length)
    x = rng.normal(size=(rows, length)).astype(np.float32)
    x[:, ::3] = np.round(x[:, ::3] * 2)          # many exact ties, signed zeros
    if length > 10:
        x[0, 5] = -0.0
    idx, val = rrt.topk(dev(x), k)
    idx, val = idx.cpu().numpy(), val.cpu().numpy()
    for r in range(rows):
        want = topk_abs(x[r], k)
        assert idx[r].tolist() == want.tolist()
        assert np.array_equal(val[r].view(np.uint32), x[r][want].view(np.uint32))


@pytest.mark.parametrize("case", ["constant", "few_levels"])
def test_topk_long_row_ties(rrt, case):
    """Long rows (the chunked selection) whose threshold falls inside a run of
    equal magnitudes: the kept equal keys are the lowest positions."""
    from oracle.select import topk_abs
    rng = np.random.default_rng(11)
    length, k = 40000, 3000
    if case == "constant":
        x = np.where(rng.random(length) < 0.5, -1.5, 1.5).astype(np.float32)
    else:
        x = rng.choice(np.array([0.25, -0.5, 1.0, -2.0], np.float32), size=length)
    x = x.reshape(1, -1)
    idx, val = rrt.topk(dev(x), k)
    want = topk_abs(x[0], k)
    assert idx.cpu().numpy()[0].tolist() == want.tolist()
    assert np.array_equal(val.cpu().numpy()[0].view(np.uint32), x[0][want].view(np.uint32))


# ---------------------------------------------------------------- storage forms (a7)
def test_convert_bf16_f16(rrt):
    rng = np.random.default_rng(3)
    x = (rng.normal(size=(37, 300)) * np.exp(rng.normal(size=(37, 300)) * 4)).astype(np.float32)
    t = dev(x)
    assert torch.equal(rrt.convert(t, "bf16").view(torch.int16), t.to(torch.bfloat16).view(torch.int16))
    assert torch.equal(rrt.convert(t, "f16").view(torch.int16), t.to(torch.float16).view(torch.int16))


def test_convert_e4m3(rrt):
    rng = np.random.default_rng(4)
    cols = 300                                    # ragged last block
    x = (rng.normal(size=(9, cols)) * np.exp(rng.normal(size=(9, cols)) * 3)).astype(np.float32)
    x[2, :64] = 0.0                               # all-zero block -> scale 1
    codes, scale = rrt.convert(dev(x), "e4m3")
    codes, scale = codes.cpu(), scale.cpu().numpy()
    nblk = (cols + 63) // 64
    for r in range(9):
        for b in range(nblk):
            blk = x[r, b * 64:(b + 1) * 64]
            amax = np.float32(np.max(np.abs(blk)))
            inv = np.float32(448.0) / amax if amax > 0 else np.float32(1.0)
            sc = amax / np.float32(448.0) if amax > 0 else np.float32(1.0)
            assert scale[r, b] == sc
            want = torch.from_numpy((blk * inv).astype(np.float32)).to(torch.float8_e4m3fn)
            assert torch.equal(codes[r, b * 64:(b + 1) * 64], want.view(torch.uint8)), (r, b)


def test_convert_s16(rrt):
    rng = np.random.default_rng(5)
    cols = 200
    x = (rng.normal(size=(7, cols)) * np.exp(rng.normal(size=(7, cols)) * 3)).astype(np.float32)
    x[1, 64:128] = 0.0
    codes, scale = rrt.convert(dev(x), "s16")
    codes, scale = codes.cpu().numpy(), scale.cpu().numpy()
    for r in range(7):
        for b in range((cols + 63) // 64):
            blk = x[r, b * 64:(b + 1) * 64]
            amax = np.float32(np.max(np.abs(blk)))
            inv = np.float32(32767.0) / amax if amax > 0 else np.float32(1.0)
            sc = amax / np.float32(32767.0) if amax > 0 else np.float32(1.0)
            assert scale[r, b] == sc
            want = np.clip(np.rint(blk * inv), -32767, 32767).astype(np.int16)
            assert np.array_equal(codes[r, b * 64:(b + 1) * 64], want), (r, b)


def _s11_pack(codes):
    """Reference packing of RRT_S11 (include/rrt.h): code e of a row in bits
    [11 e, 11 e + 11) of the row's little-endian uint32 word stream, zero
    bits after the last code."""
    rows, cols = codes.shape
    words = (11 * cols + 31) // 32
    out = np.zeros((rows, words), np.uint32)
    for r in range(rows):
        stream = 0
        for e in range(cols):
            stream |= (int(codes[r, e]) & 0x7ff) << (11 * e)
        for k in range(words):
            out[r, k] = (stream >> (32 * k)) & 0xffffffff
    return out


@pytest.mark.parametrize("cols", [1, 63, 64, 200, 256, 600])
def test_convert_s11(rrt, cols):
    """Packed 11-bit codes bit for bit against the definition: per 64-value
    block code = RNE(x 1023 / max|x|) within [-1023, 1023], scale =
    max|x| / 1023 (1 for an all-zero block), ragged last blocks."""
    rng = np.random.default_rng(6 + cols)
    x = (rng.normal(size=(7, cols)) * np.exp(rng.normal(size=(7, cols)) * 3)).astype(np.float32)
    x[1, :min(cols, 64)] = 0.0
    codes, scale = rrt.convert(dev(x), "s11")
    assert tuple(codes.shape) == (7, rrt.s11_words(cols))
    codes, scale = codes.cpu().numpy().view(np.uint32), scale.cpu().numpy()
    want = np.zeros((7, cols), np.int64)
    for r in range(7):
        for b in range((cols + 63) // 64):
            blk = x[r, b * 64:(b + 1) * 64]
            amax = np.float32(np.max(np.abs(blk)))
            inv = np.float32(1023.0) / amax if amax > 0 else np.float32(1.0)
            sc = amax / np.float32(1023.0) if amax > 0 else np.float32(1.0)
            assert scale[r, b] == sc
            want[r, b * 64:(b + 1) * 64] = np.clip(np.rint(blk * inv), -1023, 1023)
    assert np.array_equal(codes, _s11_pack(want))


@pytest.mark.parametrize("form", ["e4m3", "s16", "s11"])
@pytest.mark.parametrize("nnz", [100, 256, 600])
def test_relight_block_scaled_forms(rrt, form, nnz):
    """The kernel's decoding of each block-scaled form (E4M3 through the
    hardware FP8 conversion, packed S11, S16) against the checker fed the
    decoded stored values: FP32 bar.  nnz = 600 also decodes the entries
    past the LDS list from global memory in every block."""
    from cases import build_case, decode_storage, reference, workload
    w = workload(410 + nnz, 64, 1024, 23, nnz, nframes=2)
    case = build_case(w)
    codes, scale = rrt.convert(dev(case["t_val"]), form)
    dec = decode_storage(form, codes, scale, nnz)
    out = rrt.relight(64, dev(case["light_idx"]), dev(case["light_val"]), dev(case["vert_rot"]),
                      dev(case["t_idx"]), codes, block_scale=scale,
                      frame_rot=dev(case["frame_rot"]))
    torch.cuda.synchronize()
    check_frames(out.cpu().numpy(), reference(dict(case, t_val=dec), return_scale=True))


# ---------------------------------------------------------------- dense phase shift (a4+a5)
@pytest.mark.parametrize("n", [2, 4, 8, 32, 256])
def test_phase_shift(rrt, n):
    from oracle.relight import phase_shift
    from scenes.scene import random_rotations
    rng = np.random.default_rng(n)
    coef = rng.normal(size=(6, n, n)).astype(np.float32)
    rots = list(random_rotations(50 + n, 3))
    rots.append(np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], np.float32))
    c, s = np.cos(np.pi / 4), np.sin(np.pi / 4)
    rots.append(np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], np.float32))
    R = np.stack(rots).astype(np.float32)
    got = rrt.haar_phase_shift(dev(coef), dev(R)).cpu().numpy()
    for r in range(len(R)):
        ref = phase_shift(coef.astype(np.float64), R[r])
        assert np.linalg.norm(got[r] - ref) <= 2e-6 * np.linalg.norm(ref), r


@pytest.mark.parametrize("n", [8, 32, 128])
def test_phase_shift_index_map_exact(rrt, n):
    """Rotating a texel-ID map (P[q] = q) through the public phase shift and
    transforming back gives the source index of every texel: compared bit
    for bit with the checker's integer map, for random, boundary-heavy
    (45-degree, 22.5-degree) and cube-group rotations."""
    from oracle.haar import haar_forward, haar_inverse
    from oracle.sphere import quantise_rotation, source_index
    from scenes.scene import random_rotations
    ids = np.arange(6 * n * n, dtype=np.float64).reshape(6, n, n)
    coef = haar_forward(ids).astype(np.float32)
    rots = list(random_rotations(70 + n, 6))
    for ang in (np.pi / 4, np.pi / 8):
        c, s_ = np.cos(ang), np.sin(ang)
        rots += [np.array([[1, 0, 0], [0, c, -s_], [0, s_, c]]), np.array([[c, 0, s_], [0, 1, 0], [-s_, 0, c]])]
    rots.append(np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]))
    R = np.stack(rots).astype(np.float32)
    out = rrt.haar_phase_shift(dev(coef), dev(R)).cpu().numpy().astype(np.float64)
    for r in range(len(R)):
        got = np.rint(haar_inverse(out[r])).astype(np.int64)
        want = source_index(quantise_rotation(R[r], n), n)
        assert np.array_equal(got, want), (r, int((got != want).sum()))


# ---------------------------------------------------------------- relight (a3-a6)
def run_relight(rrt, case, **kw):
    out = rrt.relight(case["n"], dev(case["light_idx"]), dev(case["light_val"]),
                      dev(case["vert_rot"]), None if case["t_idx"] is None else dev(case["t_idx"]),
                      dev(case["t_val"]),
                      frame_rot=None if case["frame_rot"] is None else dev(case["frame_rot"]), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("compensated", [False, True])
def test_relight_dense_n32(rrt, compensated):
    """Dense transport and dense lighting at n = 32, 67 vertices (ragged)."""
    from cases import build_case, reference, workload
    w = workload(101, 32, 6 * 32 * 32, 67, 6 * 32 * 32, exp_lo=1.0, exp_hi=64.0,
                 vertex_frames="normals")
    case = build_case(w)
    got = run_relight(rrt, case, compensated=compensated)
    check_frames(got, reference(case, return_scale=True))


@pytest.mark.parametrize("n,k,nnz,V", [(2, 24, 24, 5), (4, 40, 17, 9), (8, 100, 64, 33),
                                       (16, 300, 128, 20), (64, 1024, 256, 21),
                                       (128, 1024, 256, 41)])
def test_relight_sparse(rrt, n, k, nnz, V):
    from cases import build_case, reference, workload
    w = workload(200 + n, n, k, V, nnz, exp_lo=1.0, exp_hi=200.0)
    case = build_case(w)
    check_frames(run_relight(rrt, case), reference(case, return_scale=True), rel_l2=n >= 32)


@pytest.mark.parametrize("n", [32, 64, 128])
def test_relight_gather_exact(rrt, n):
    """Source-index exactness inside relight (both gather paths): the
    lighting is a texel-ID map (P[q] = q) and vertex row r holds a single
    finest-level H, V or D coefficient, so each radiance is (+-a +-b +-c +-d)/2
    of four gathered source indices.  A wrong index moves a result by at
    least 1/2; reconstruction rounding stays below 0.05.  Random,
    boundary-heavy (22.5 / 45 degree) and cube-group rotations."""
    from oracle.haar import haar_forward
    from oracle.sphere import quantise_rotation, rotate_pixels
    from scenes.scene import random_rotations
    ids = np.arange(6 * n * n, dtype=np.float64).reshape(6, n, n)
    light = haar_forward(ids).ravel().astype(np.float32)
    light_idx = np.arange(6 * n * n, dtype=np.int32)
    h = n // 2
    rr, cc = np.meshgrid(np.arange(h), np.arange(h), indexing="ij")
    pos = []
    for f in range(6):
        for (dr, dc) in [(0, h), (h, 0), (h, h)]:        # H, V, D quadrants of level 1
            pos.append(f * n * n + (rr + dr) * n + (cc + dc))
    rows = np.concatenate([p_.ravel() for p_ in pos]).astype(np.int32)
    V = rows.size
    rots = list(random_rotations(500 + n, 3))
    for ang in (np.pi / 4, np.pi / 8):
        c_, s_ = np.cos(ang), np.sin(ang)
        rots.append(np.array([[c_, -s_, 0], [s_, c_, 0], [0, 0, 1]]))
    rots.append(np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]]))
    for R in rots:
        R = np.asarray(R, np.float32)
        out = rrt.relight(n, dev(light_idx), dev(light), dev(np.tile(R, (V, 1, 1))),
                          dev(rows.reshape(V, 1)), dev(np.ones((V, 1), np.float32)))
        got = out.cpu().numpy()[0]
        want = haar_forward(rotate_pixels(ids, quantise_rotation(R, n))).ravel()[rows]
        err = np.abs(got - want)
        assert err.max() < 0.05, (R, int((err >= 0.05).sum()), float(err.max()))


@pytest.mark.parametrize("n,V", [(512, 3), (1024, 2)])
def test_relight_large_faces(rrt, n, V):
    """n = 512 and 1024: many regions per face and the FP64 levels above them."""
    from cases import build_case, reference, workload
    w = workload(310 + n, n, 4096, V, 256, exp_lo=1.0, exp_hi=4.0)
    case = build_case(w)
    check_frames(run_relight(rrt, case), reference(case, return_scale=True))


def test_relight_frames_composition(rrt):
    """Frame rotations composed with vertex frames (fixed-point rule)."""
    from cases import build_case, reference, workload
    w = workload(301, 32, 512, 13, 256, nframes=5)
    case = build_case(w)
    check_frames(run_relight(rrt, case), reference(case, return_scale=True))


def test_relight_n256_regions(rrt):
    """n = 256: 8 x 8 blocks of 32 x 32 per face, the FP64 levels above them, and
    the source map written by 64 x 64 inverse-Haar tiles plus their coarse pass."""
    from cases import build_case, reference, workload
    w = workload(302, 256, 2048, 6, 256, exp_lo=1.0, exp_hi=8.0)   # low exponents: 5 faces
    case = build_case(w)
    assert len(np.unique(case["t_idx"] // (256 * 256))) > 1
    check_frames(run_relight(rrt, case), reference(case, return_scale=True))


def test_relight_edge_cases(rrt):
    from cases import build_case, reference, workload
    w = workload(303, 16, 64, 4, 32)
    case = build_case(w)
    # empty vertex set: nothing to do, no error
    empty = dict(case, vert_rot=case["vert_rot"][:0], t_idx=case["t_idx"][:0], t_val=case["t_val"][:0])
    assert run_relight(rrt, empty).shape == (1, 0)
    # single coefficient, single light coefficient
    one = dict(case, light_idx=case["light_idx"][:1], light_val=case["light_val"][:1],
               t_idx=case["t_idx"][:, :1].copy(), t_val=case["t_val"][:, :1].copy())
    check_frames(run_relight(rrt, one), reference(one, return_scale=True), rel_l2=False)
    # out-of-range transport indices are ignored
    bad = dict(case, t_idx=case["t_idx"].copy())
    bad["t_idx"][:, 3] = -5
    bad["t_idx"][:, 7] = 6 * 16 * 16 + 2
    ok = dict(case, t_val=case["t_val"].copy())
    ok["t_val"][:, [3, 7]] = 0.0
    check_frames(run_relight(rrt, bad), reference(ok, return_scale=True), rel_l2=False)


def test_relight_identity_and_constant(rrt):
    """Closed forms: identity rotation = plain inner product; constant
    lighting c -> n c sum_F T[DC_F]."""
    from cases import build_case, workload
    n = 32
    w = workload(304, n, 6, 8, 200)
    case = build_case(w)
    L = np.zeros(6 * n * n)
    L[case["light_idx"]] = case["light_val"]
    const = dict(case, light_idx=np.arange(6, dtype=np.int32) * n * n,
                 light_val=np.full(6, n * 2.0, np.float32))
    got = run_relight(rrt, const)[0]
    for v in range(8):
        full = np.zeros(6 * n * n)
        full[case["t_idx"][v]] = case["t_val"][v]
        assert abs(got[v] - 2.0 * n * sum(full[f * n * n] for f in range(6))) <= 1e-5 * abs(got[v])
    ident = dict(case, vert_rot=np.tile(np.eye(3, dtype=np.float32), (8, 1, 1)))
    got = run_relight(rrt, ident)[0]
    for v in range(8):
        ref = np.dot(case["t_val"][v].astype(np.float64), L[case["t_idx"][v]])
        assert abs(got[v] - ref) <= 1e-5 * abs(ref)


def test_relight_workspace_reuse_and_determinism(rrt):
    from cases import build_case, workload
    w = workload(305, 64, 512, 30, 256)
    case = build_case(w)
    a = run_relight(rrt, case)
    b = run_relight(rrt, case)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- coarse-level start (f3)
@pytest.mark.parametrize("n,levels", [(4, 1), (16, 1), (64, 2), (128, 3), (1024, 9)])
def test_coarsen_indices_exact(rrt, n, levels):
    from oracle.levels import coarse_index
    rng = np.random.default_rng(n + levels)
    idx = rng.integers(-3, 6 * n * n + 3, size=20000).astype(np.int32)
    got = rrt.coarsen_indices(dev(idx), n, levels).cpu().numpy()
    assert np.array_equal(got, coarse_index(idx, n, levels))


@pytest.mark.parametrize("n,levels,frames", [(64, 1, 1), (64, 2, 3), (128, 3, 1)])
def test_relight_from_coarser_level(rrt, n, levels, frames):
    """Relighting at n >> levels with remapped lighting and transport entries
    against the checker's coarse-level start on the same stored inputs."""
    from cases import build_case, frame_errors, workload
    from oracle.levels import relight_from_level
    w = workload(40 + n + levels, n, 1024, 40, 256, nframes=frames)
    case = build_case(w)
    ref = relight_from_level(case["light_idx"], case["light_val"], n, case["vert_rot"],
                             case["frame_rot"], case["t_idx"], case["t_val"], levels)
    nc = n >> levels
    li = rrt.coarsen_indices(dev(case["light_idx"]), n, levels)
    ti = rrt.coarsen_indices(dev(case["t_idx"]), n, levels)
    out = rrt.relight(nc, li, dev(case["light_val"]), dev(case["vert_rot"]), ti,
                      dev(case["t_val"]),
                      frame_rot=None if case["frame_rot"] is None else dev(case["frame_rot"]))
    assert max(frame_errors(out.cpu().numpy(), ref)) <= 1e-5



# ---------------------------------------------------------------- chain rule (f1)
from cases import chain_reference  # noqa: E402  (the checker's chain rule with its scale)


@pytest.mark.parametrize("n,nframes,compensated", [(32, 1, False), (64, 3, True), (128, 1, False)])
def test_relight_chain_rule(rrt, n, nframes, compensated):
    """Chain-rule rotation of the finest level against the checker's
    chain_rotate on the same stored inputs (workload-shaped scenes)."""
    from cases import build_case, workload
    w = workload(600 + n, n, 1024, 37, 256, nframes=nframes)
    case = build_case(w)
    got = run_relight(rrt, case, compensated=compensated, chain_rule=True)
    check_frames(got, chain_reference(case))


def test_relight_chain_rule_prepared_and_cube_rotations(rrt):
    """prepare + prepared with the chain rule equals the one-call form bit for
    bit; under cube-group rotations (where the mapping is a permutation of
    whole blocks) the chain rule equals the exact method."""
    from cases import build_case, reference, workload
    from oracle.chain import FACE_AXES
    n = 64
    w = workload(640, n, 1024, 24, 256)
    case = build_case(w)
    # 24 cube-group rotations: signed permutation matrices of determinant 1
    rots = []
    import itertools
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            M = np.zeros((3, 3))
            for r in range(3):
                M[r, perm[r]] = signs[r]
            if np.linalg.det(M) > 0:
                rots.append(M)
    assert len(rots) == 24 and FACE_AXES.shape == (6, 3, 3)
    case = dict(case, vert_rot=np.stack(rots).astype(np.float32))
    one = run_relight(rrt, case, chain_rule=True)
    check_frames(one, reference(case, return_scale=True))
    prep = rrt.prepare_lighting(n, dev(case["light_idx"]), dev(case["light_val"]), chain_rule=True)
    two = rrt.relight_prepared(prep, dev(case["vert_rot"]), dev(case["t_idx"]), dev(case["t_val"]))
    torch.cuda.synchronize()
    assert np.array_equal(one, two.cpu().numpy())


# ---------------------------------------------------------------- triple product (f2)
def run_triple(rrt, case, **kw):
    out = rrt.relight(case["n"], dev(case["light_idx"]), dev(case["light_val"]),
                      dev(case["vert_rot"]), dev(case["t_idx"]), dev(case["t_val"]),
                      frame_rot=None if case["frame_rot"] is None else dev(case["frame_rot"]),
                      brdf=dev(case["brdf"]), material=dev(case["material"]), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,V,nnz,M,frames", [(2, 7, 24, 2, 1), (4, 9, 40, 2, 1),
                                              (16, 21, 128, 3, 1), (32, 37, 256, 4, 2),
                                              (64, 23, 256, 8, 1), (128, 17, 256, 8, 1)])
def test_relight_triple_product(rrt, n, V, nnz, M, frames):
    """BRDF and visibility kept separate: the device's texel-domain product
    against the checker's literal tripling-coefficient sum on the same stored
    inputs (materials, visibility rows, lighting)."""
    from cases import triple_case, workload
    from oracle.triple import relight_triple
    w = workload(700 + n, n, min(1024, 6 * n * n), V, nnz, nframes=frames)
    case = triple_case(w, M)
    ref = relight_triple(case["light_idx"], case["light_val"], n, case["vert_rot"],
                         case["frame_rot"], case["t_idx"], case["t_val"], case["brdf"],
                         case["material"], return_scale=True)
    check_frames(run_triple(rrt, case, compensated=(n == 32)), ref, rel_l2=n >= 32)


def test_relight_triple_edge_cases(rrt):
    """Materials outside [0, M) give exactly 0; a BRDF of ones gives the
    double product bit for bit; no material table means row 0; the chain
    rule refuses a BRDF."""
    from cases import triple_case, workload
    n = 32
    case = triple_case(workload(760, n, 1024, 12, 256), 3)
    mat = case["material"].copy()
    mat[[1, 5, 9]] = [-1, 3, 1 << 30]
    got = run_triple(rrt, dict(case, material=mat))
    assert np.all(got[0, [1, 5, 9]] == 0.0) and np.all(got[0, [0, 2, 3]] != 0.0)
    ones = dict(case, brdf=np.ones((2, 6, n, n), np.float32), material=np.zeros(12, np.int32))
    plain = run_relight(rrt, dict(case, t_idx=case["t_idx"], t_val=case["t_val"]))
    assert np.array_equal(run_triple(rrt, ones), plain)
    r0 = rrt.relight(n, dev(case["light_idx"]), dev(case["light_val"]), dev(case["vert_rot"]),
                     dev(case["t_idx"]), dev(case["t_val"]), brdf=dev(case["brdf"]))
    both = run_triple(rrt, dict(case, material=np.zeros(12, np.int32)))
    assert np.array_equal(r0.cpu().numpy(), both)
    with pytest.raises(RuntimeError):
        rrt.relight(n, dev(case["light_idx"]), dev(case["light_val"]), dev(case["vert_rot"]),
                    dev(case["t_idx"]), dev(case["t_val"]), brdf=dev(case["brdf"]),
                    material=dev(case["material"]), chain_rule=True)


# ---------------------------------------------------------------- lat-long map (f4)
def _ll_workload(cfg, H, k, V, nnz):
    from scenes.latlong import LatLongWorkload
    return LatLongWorkload(cfg, f"test{cfg}", H, k, V, nnz, 1.0, 200.0)


def run_latlong(rrt, case, **kw):
    out = rrt.relight_latlong(case["H"], dev(case["light_idx"]), dev(case["light_val"]),
                              dev(case["elev"]), dev(case["shift"]), dev(case["t_idx"]),
                              dev(case["t_val"]), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()[None, :]


@pytest.mark.parametrize("H", [4, 16, 128, 512])
def test_latlong_grid_tables_exact(rrt, H):
    """The device's binary32 tables equal the checker's bit for bit."""
    from oracle.latlong import grid
    case = dict(H=H, light_idx=np.array([0], np.int32), light_val=np.array([1.0], np.float32),
                elev=np.array([[1.0, 0.0]], np.float32), shift=np.zeros((1, 2), np.int32),
                t_idx=np.array([[0]], np.int32), t_val=np.array([[1.0]], np.float32))
    cells = 2 * H * H
    off = 2 * (((cells * 4) + 255) // 256 * 256)
    ws = torch.zeros(off + (7 * H * 4 + 255) // 256 * 256, dtype=torch.uint8, device="cuda")
    rrt.relight_latlong(H, dev(case["light_idx"]), dev(case["light_val"]), dev(case["elev"]),
                        dev(case["shift"]), dev(case["t_idx"]), dev(case["t_val"]), workspace=ws)
    torch.cuda.synchronize()
    got = ws[off:off + 7 * H * 4].cpu().view(torch.float32).numpy()
    want = np.concatenate(grid(H))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("H,V,nnz,k,comp", [(4, 9, 20, 32, False), (8, 17, 64, 128, False),
                                            (16, 23, 128, 256, True), (32, 31, 256, 1024, False),
                                            (64, 29, 256, 1024, False), (128, 19, 256, 1024, True),
                                            (256, 7, 256, 2048, False), (512, 3, 256, 2048, False)])
def test_relight_latlong(rrt, H, V, nnz, k, comp):
    """Lat-long relighting against the checker's binary32 rule + FP64 levels
    and dot on the same stored inputs."""
    from cases import latlong_case
    from oracle.latlong import relight_latlong
    case = latlong_case(_ll_workload(900 + H, H, k, V, nnz))
    ref = relight_latlong(case["light_idx"], case["light_val"], H, case["elev"], case["shift"],
                          case["t_idx"], case["t_val"], return_scale=True)
    check_frames(run_latlong(rrt, case, compensated=comp), ref, rel_l2=H >= 32)


@pytest.mark.parametrize("H", [16, 64, 128])
def test_relight_latlong_gather_exact(rrt, H):
    """Source-index exactness of the lat-long rule: a texel-ID lighting and
    rows holding one finest-level H, V or D coefficient each, so a radiance
    is (+-a +-b +-c +-d)/2 of four gathered source indices; random and
    boundary-heavy elevations (b = 0, pi/2, pi, pi/4) with shifts."""
    from oracle.haar import haar_forward
    from oracle.latlong import rotate
    ids = np.arange(2 * H * H, dtype=np.float64).reshape(2, H, H)
    light = haar_forward(ids).ravel().astype(np.float32)
    light_idx = np.arange(2 * H * H, dtype=np.int32)
    h = H // 2
    rr, cc = np.meshgrid(np.arange(h), np.arange(h), indexing="ij")
    pos = [f * H * H + (rr + dr) * H + (cc + dc) for f in range(2) for dr, dc in [(0, h), (h, 0), (h, h)]]
    rows = np.concatenate([p_.ravel() for p_ in pos]).astype(np.int32)
    V = rows.size
    rng = np.random.default_rng(H)
    elevs = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (np.cos(np.pi / 4), np.sin(np.pi / 4))]
    elevs += [(np.cos(b), np.sin(b)) for b in np.arccos(rng.uniform(-1, 1, 3))]
    for cb, sb in elevs:
        e = np.array([cb, sb], np.float32)
        sh = rng.integers(-3 * H, 3 * H, 2).astype(np.int32)
        out = rrt.relight_latlong(H, dev(light_idx), dev(light), dev(np.tile(e, (V, 1))),
                                  dev(np.tile(sh, (V, 1))), dev(rows.reshape(V, 1)),
                                  dev(np.ones((V, 1), np.float32)))
        got = out.cpu().numpy()
        want = haar_forward(rotate(ids, e[0], e[1], sh[0], sh[1])).ravel()[rows]
        err = np.abs(got - want)
        assert err.max() < 0.05, (e, sh, int((err >= 0.05).sum()), float(err.max()))


def test_relight_latlong_scene_ties_exact(rrt):
    """Source-index exactness on the 128 x 256 scene's own rotations (its
    first 64 vertices, one call): about one in six has texels whose azimuth
    decision is an exact binary32 tie, q_z equal to the rounded C_k rho, which
    only a correctly rounded rho decides as the rule does.  Rows and lighting
    as in the texel-ID test above."""
    from oracle.haar import haar_forward
    from oracle.latlong import grid, rotate
    from scenes.latlong import LATLONG_WORKLOADS, rotations
    w = next(x for x in LATLONG_WORKLOADS.values() if x.H == 128)
    H, W, nrot = w.H, 2 * w.H, 64
    elev, shift = rotations(w)
    elev, shift = elev[:nrot], shift[:nrot]
    # the premise: some of these rotations hold exact ties
    St, ct, sf, kf, C = grid(H)
    i, j = np.arange(H)[:, None], np.arange(W)[None, :]
    px, py, pz = St[i] * sf[j], ct[i] * np.ones_like(sf[j]), St[i] * kf[j]
    tied = 0
    for cb, sb in elev:
        qz = sb * py + cb * pz
        rho = np.sqrt(px * px + qz * qz)
        tied += bool(np.any(qz[None] == C[1:, None, None] * rho[None]))
    assert tied >= 4, tied
    ids = np.arange(2 * H * H, dtype=np.float64).reshape(2, H, H)
    light = haar_forward(ids).ravel().astype(np.float32)
    h = H // 2
    rr, cc = np.meshgrid(np.arange(h), np.arange(h), indexing="ij")
    pos = [f * H * H + (rr + dr) * H + (cc + dc) for f in range(2) for dr, dc in [(0, h), (h, 0), (h, h)]]
    rows = np.concatenate([p_.ravel() for p_ in pos]).astype(np.int32)
    R = rows.size
    out = rrt.relight_latlong(H, dev(np.arange(2 * H * H, dtype=np.int32)), dev(light),
                              dev(np.repeat(elev, R, axis=0)), dev(np.repeat(shift, R, axis=0)),
                              dev(np.tile(rows, nrot).reshape(-1, 1)),
                              dev(np.ones((nrot * R, 1), np.float32)))
    got = out.cpu().numpy().reshape(nrot, R)
    for v in range(nrot):
        want = haar_forward(rotate(ids, elev[v, 0], elev[v, 1], shift[v, 0], shift[v, 1])).ravel()[rows]
        err = np.abs(got[v] - want)
        assert err.max() < 0.05, (v, elev[v], shift[v], int((err >= 0.05).sum()))


def test_relight_latlong_edge_cases(rrt):
    """Empty vertex set; shifts reduced mod 2H; binary16 lighting; out-of-range
    transport entries ignored."""
    from cases import latlong_case
    from oracle.latlong import relight_latlong
    H = 32
    case = latlong_case(_ll_workload(950, H, 512, 12, 128))
    empty = dict(case, elev=case["elev"][:0], shift=case["shift"][:0], t_idx=case["t_idx"][:0],
                 t_val=case["t_val"][:0])
    assert run_latlong(rrt, empty).shape == (1, 0)
    base = run_latlong(rrt, case)
    wrapped = run_latlong(rrt, dict(case, shift=case["shift"] + np.array([[4 * H, -6 * H]], np.int32)))
    assert np.array_equal(base, wrapped)
    bad = dict(case, t_idx=case["t_idx"].copy())
    bad["t_idx"][:, 5] = 2 * H * H + 3
    bad["t_idx"][:, 7] = -1
    ref = relight_latlong(bad["light_idx"], bad["light_val"], H, bad["elev"], bad["shift"],
                          bad["t_idx"], bad["t_val"], return_scale=True)
    check_frames(run_latlong(rrt, bad), ref)
    half = run_latlong(rrt, dict(case, light_val=case["light_val"].astype(np.float16)),
                       compensated=True)
    from cases import frame_errors
    ref16 = relight_latlong(case["light_idx"], case["light_val"].astype(np.float16), H, case["elev"],
                            case["shift"], case["t_idx"], case["t_val"])
    assert max(frame_errors(half, ref16)) <= 2e-3


# ---------------------------------------------------------------- rows x storage forms
def _decoded(rrt, vals, form):
    """Device storage conversion of [V, nnz] values and the float32 values the
    kernel decodes from it (code x scale in binary32), for the checker."""
    t = dev(vals)
    if form == "bf16":
        codes = rrt.convert(t, "bf16")
        return codes, None, codes.float().cpu().numpy()
    codes, scale = rrt.convert(t, form)
    sc = np.repeat(scale.cpu().numpy(), 64, axis=1)[:, :vals.shape[1]]
    assert form == "s16"
    return codes, scale, codes.cpu().numpy().astype(np.float32) * sc


def test_chain_rule_with_f16_lighting(rrt):
    """Chain rule with a binary16 lighting (source map and block coefficients
    from binary16 texels) and compensated accumulation, against the checker
    fed the same binary16 lighting values: the only extra error is the
    binary16 rounding of the reconstructed map."""
    from cases import build_case, frame_errors, workload
    w = workload(620, 64, 1024, 29, 256)
    case = build_case(w)
    case16 = dict(case, light_val=case["light_val"].astype(np.float16))
    got = rrt.relight(64, dev(case16["light_idx"]), dev(case16["light_val"]), dev(case16["vert_rot"]),
                      dev(case16["t_idx"]), dev(case16["t_val"]), compensated=True,
                      chain_rule=True).cpu().numpy()
    ref, _ = chain_reference(case16)
    assert max(frame_errors(got, ref)) <= 2e-3


def test_triple_product_with_bf16_visibility(rrt):
    """Triple product with the visibility rows stored in BF16: against the
    checker on the decoded BF16 values at the FP32 tolerance."""
    from cases import triple_case, workload
    from oracle.triple import relight_triple
    n = 32
    case = triple_case(workload(780, n, 1024, 19, 256), 3)
    codes, _, decoded = _decoded(rrt, case["t_val"], "bf16")
    out = rrt.relight(n, dev(case["light_idx"]), dev(case["light_val"]), dev(case["vert_rot"]),
                      dev(case["t_idx"]), codes, brdf=dev(case["brdf"]),
                      material=dev(case["material"])).cpu().numpy()
    ref = relight_triple(case["light_idx"], case["light_val"], n, case["vert_rot"], None,
                         case["t_idx"], decoded, case["brdf"], case["material"], return_scale=True)
    check_frames(out, ref)


def test_latlong_with_s16_transport(rrt):
    """Lat-long relight with S16 block-scaled transport rows: against the
    checker on the decoded values at the FP32 tolerance."""
    from cases import latlong_case
    from oracle.latlong import relight_latlong
    H = 64
    case = latlong_case(_ll_workload(960, H, 1024, 21, 256))
    codes, scale, decoded = _decoded(rrt, case["t_val"], "s16")
    out = rrt.relight_latlong(H, dev(case["light_idx"]), dev(case["light_val"]), dev(case["elev"]),
                              dev(case["shift"]), dev(case["t_idx"]), codes, block_scale=scale,
                              compensated=True).cpu().numpy()[None, :]
    ref = relight_latlong(case["light_idx"], case["light_val"], H, case["elev"], case["shift"],
                          case["t_idx"], decoded, return_scale=True)
    check_frames(out, ref)


# ---------------------------------------------------------------- processing order
def test_relight_order_heavy_first_and_results_unchanged(rrt):
    """rrt_relight_order is a permutation sorting the vertices by the faces
    their rows touch, most first; relighting in that order, in reverse or
    in a random order gives the index-order result bit for bit; entries
    outside [0, V) are skipped (those vertices keep what out held)."""
    from cases import build_case, workload
    w = workload(980, 32, 1024, 257, 256, exp_lo=1.0, exp_hi=30.0)
    case = build_case(w)
    order = rrt.relight_order(32, dev(case["t_idx"])).cpu().numpy()
    V = case["t_idx"].shape[0]
    assert np.array_equal(np.sort(order), np.arange(V))
    faces = np.array([len(np.unique(r[(r >= 0) & (r < 6 * 32 * 32)] // (32 * 32)))
                      for r in case["t_idx"]])
    assert np.all(np.diff(faces[order]) <= 0) and faces.max() > faces.min()
    base = run_relight(rrt, case)
    rng = np.random.default_rng(3)
    for o in (order, order[::-1].copy(), rng.permutation(V).astype(np.int32)):
        assert np.array_equal(run_relight(rrt, case, order=dev(o.astype(np.int32))), base)
    partial = order.copy()
    partial[[0, 5]] = [-1, V]
    out = torch.full((1, V), float("nan"), device="cuda")
    got = run_relight(rrt, case, order=dev(partial), out=out)
    skipped = order[[0, 5]]
    keep = np.setdiff1d(np.arange(V), skipped)
    assert np.all(np.isnan(got[0, skipped])) and np.array_equal(got[0, keep], base[0, keep])
    # dense rows: every vertex alike, the index order
    dense = rrt.relight_order(4, None, nvert=7)
    assert np.array_equal(dense.cpu().numpy(), np.arange(7))
    # cluster support rows: the order follows each vertex's cluster row
    cl = np.array([1, 0, 1, 2, 0], np.int32)
    sup = case["t_idx"][[int(np.argmax(faces)), int(np.argmin(faces)), 7]]
    co = rrt.relight_order(32, dev(sup), cluster=dev(cl)).cpu().numpy()
    fs = np.array([faces[int(np.argmax(faces))], faces[int(np.argmin(faces))], faces[7]])[cl]
    assert np.array_equal(np.sort(co), np.arange(5)) and np.all(np.diff(fs[co]) <= 0)
