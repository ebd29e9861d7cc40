"""The C ABI on the host (no GPU needed): librrt.so loads, exports every
symbol include/rrt.h declares, and rejects bad arguments before any HIP call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "rrt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rrt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def rrt():
    import paper_1705_07272_amd as m
    return m


def test_exports_every_declared_symbol(rrt):
    syms = _declared_symbols()
    assert len(syms) >= 12
    raw = ctypes.CDLL(rrt._abi.LIB_PATH)
    for s in syms:
        assert hasattr(raw, s), s
    assert set(syms) == set(rrt._abi.SIGNATURES), "binding and header disagree"


def test_version_and_strings(rrt):
    lib = rrt.lib
    assert lib.rrt_abi_version() == 6
    assert lib.rrt_status_string(0) == b"ok"
    assert lib.rrt_status_string(3) == b"workspace too small"
    assert lib.rrt_status_string(99) == b"unknown status"


def _p(x):
    return ctypes.c_void_p(x)


def test_haar_validation(rrt):
    lib = rrt.lib
    E = rrt._abi
    assert lib.rrt_haar_forward(_p(8), _p(16), 3, 1, None) == E.RRT_ERR_INVALID
    assert b"power of two" in lib.rrt_last_error()
    assert lib.rrt_haar_forward(_p(8), _p(16), 2048, 1, None) == E.RRT_ERR_INVALID
    assert lib.rrt_haar_forward(_p(8), _p(16), 8, -1, None) == E.RRT_ERR_INVALID
    assert lib.rrt_haar_forward(_p(0), _p(16), 8, 1, None) == E.RRT_ERR_INVALID
    assert lib.rrt_haar_forward(_p(16), _p(16), 8, 1, None) == E.RRT_ERR_INVALID
    assert lib.rrt_haar_forward(_p(0), _p(0), 8, 0, None) == E.RRT_OK          # empty: no-op
    assert lib.rrt_haar_inverse(_p(8), _p(16), 0, 1, None) == E.RRT_ERR_INVALID


def test_topk_validation(rrt):
    lib = rrt.lib
    E = rrt._abi
    nb = ctypes.c_size_t(7)
    assert lib.rrt_topk_workspace(1, 10, 3, ctypes.byref(nb)) == E.RRT_OK and nb.value == 0
    assert lib.rrt_topk_workspace(1, 10, 11, ctypes.byref(nb)) == E.RRT_ERR_INVALID
    assert lib.rrt_topk(_p(8), 1, 10, 11, _p(8), _p(8), None, 0, None) == E.RRT_ERR_INVALID
    assert lib.rrt_topk(_p(0), 1, 10, 3, _p(8), _p(8), None, 0, None) == E.RRT_ERR_INVALID
    assert lib.rrt_topk(_p(0), 0, 10, 3, _p(0), _p(0), None, 0, None) == E.RRT_OK
    assert lib.rrt_topk(_p(0), 4, 10, 0, _p(0), _p(0), None, 0, None) == E.RRT_OK
    # a few long rows take the chunked selection, which needs a workspace
    assert lib.rrt_topk_workspace(1, 98304, 1024, ctypes.byref(nb)) == E.RRT_OK
    need = nb.value
    assert need >= 2 * 4 * 98304
    assert lib.rrt_topk_workspace(9, 98304, 1024, ctypes.byref(nb)) == E.RRT_OK and nb.value == 0
    assert lib.rrt_topk_workspace(1, 98304, 98304, ctypes.byref(nb)) == E.RRT_OK and nb.value == 0
    assert lib.rrt_topk(_p(256), 1, 98304, 1024, _p(256), _p(256), None, 0, None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_topk(_p(256), 1, 98304, 1024, _p(256), _p(256), _p(256), need - 1,
                        None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_topk(_p(256), 1, 98304, 1024, _p(256), _p(256), _p(260), need,
                        None) == E.RRT_ERR_INVALID


def test_phase_shift_validation(rrt):
    lib = rrt.lib
    E = rrt._abi
    nb = ctypes.c_size_t(0)
    assert lib.rrt_haar_phase_shift_workspace(8, 3, ctypes.byref(nb)) == E.RRT_OK
    assert nb.value >= 4 * 6 * 64 * 4
    assert lib.rrt_haar_phase_shift_workspace(1, 3, ctypes.byref(nb)) == E.RRT_ERR_INVALID
    assert lib.rrt_haar_phase_shift(_p(8), 8, _p(8), 3, _p(8), _p(256), 16, None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_haar_phase_shift(_p(8), 8, _p(8), 3, _p(8), _p(0), 1 << 20, None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_haar_phase_shift(_p(8), 8, _p(8), 3, _p(8), _p(257), 1 << 20, None) == E.RRT_ERR_INVALID
    assert lib.rrt_haar_phase_shift(_p(8), 8, _p(8), 70000, _p(8), _p(256), 1 << 30, None) == E.RRT_ERR_INVALID


def _desc(rrt, n=8, k=10, nframes=1, frame_rot=0, nvert=5, nnz=16, tidx=8, tval=8,
          tdtype=0, ldtype=0, scale=0):
    E = rrt._abi
    L = E.Light(n, k, 8, 8, ldtype)
    R = E.Rotations(nframes, frame_rot, 8)
    T = E.Transport(nvert, nnz, tidx, tval, tdtype, scale)
    return L, R, T


def _relight_ws(rrt, L, R, T, flags=0):
    nb = ctypes.c_size_t(0)
    st = rrt.lib.rrt_relight_workspace(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), flags,
                                       ctypes.byref(nb))
    return st, nb.value


def test_relight_validation(rrt):
    E = rrt._abi
    st, nb = _relight_ws(rrt, *_desc(rrt))
    assert st == E.RRT_OK and nb == 256 * ((6 * 64 * 4 + 255) // 256) * 2
    st16, nb16 = _relight_ws(rrt, *_desc(rrt, ldtype=E.RRT_F16))
    assert st16 == E.RRT_OK and nb16 == nb          # binary32 source map for either lighting
    cases = [
        (dict(n=3), E.RRT_ERR_INVALID),
        (dict(n=1), E.RRT_ERR_INVALID),
        (dict(k=0), E.RRT_ERR_INVALID),
        (dict(k=6 * 64 + 1), E.RRT_ERR_INVALID),
        (dict(nframes=0), E.RRT_ERR_INVALID),
        (dict(nframes=2), E.RRT_ERR_INVALID),                  # no frame rotations
        (dict(nnz=0), E.RRT_ERR_INVALID),
        (dict(tidx=0, nnz=16), E.RRT_ERR_INVALID),             # dense needs nnz = 6 n^2
        (dict(tdtype=E.RRT_F16), E.RRT_ERR_UNSUPPORTED),
        (dict(ldtype=E.RRT_BF16), E.RRT_ERR_UNSUPPORTED),
        (dict(tdtype=E.RRT_E4M3), E.RRT_ERR_INVALID),          # needs block scales
        (dict(tdtype=E.RRT_S16), E.RRT_ERR_INVALID),
        (dict(tdtype=E.RRT_S11), E.RRT_ERR_INVALID),
        (dict(tdtype=7), E.RRT_ERR_UNSUPPORTED),
        (dict(nvert=-1), E.RRT_ERR_INVALID),
        (dict(tval=0), E.RRT_ERR_INVALID),
    ]
    for kw, want in cases:
        st, _ = _relight_ws(rrt, *_desc(rrt, **kw))
        assert st == want, (kw, st, rrt.lib.rrt_last_error())
    assert _relight_ws(rrt, *_desc(rrt, tidx=0, nnz=6 * 64))[0] == E.RRT_OK
    assert _relight_ws(rrt, *_desc(rrt, tdtype=E.RRT_E4M3, scale=8))[0] == E.RRT_OK
    assert _relight_ws(rrt, *_desc(rrt, tdtype=E.RRT_S16, scale=8))[0] == E.RRT_OK
    assert _relight_ws(rrt, *_desc(rrt, tdtype=E.RRT_S11, scale=8))[0] == E.RRT_OK
    L, R, T = _desc(rrt)
    lib = rrt.lib
    assert lib.rrt_relight(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8), 0, _p(256),
                           16, None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_relight(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8), 4, _p(256),
                           1 << 20, None) == E.RRT_ERR_INVALID                 # unknown flag
    assert lib.rrt_relight(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(0), 0, _p(256),
                           1 << 20, None) == E.RRT_ERR_INVALID                 # null radiance
    assert lib.rrt_relight(None, ctypes.byref(R), ctypes.byref(T), _p(8), 0, _p(256), 1 << 20,
                           None) == E.RRT_ERR_INVALID
    # chain rule: n >= 32 only, checked before anything is enqueued
    assert lib.rrt_relight(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8),
                           E.RRT_CHAIN_RULE, _p(256), 1 << 20, None) == E.RRT_ERR_UNSUPPORTED
    assert lib.rrt_relight_prepare(ctypes.byref(L), E.RRT_CHAIN_RULE, _p(256), 1 << 20,
                                   None) == E.RRT_ERR_UNSUPPORTED
    assert lib.rrt_relight_prepare(ctypes.byref(L), 8, _p(256), 1 << 20,
                                   None) == E.RRT_ERR_INVALID
    assert lib.rrt_relight_prepared(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8),
                                    E.RRT_CHAIN_RULE | E.RRT_COMPENSATED, _p(256), 1 << 20,
                                    None) == E.RRT_ERR_UNSUPPORTED


def test_relight_noalloc_validation(rrt):
    """Every rejection of the no-allocation relight happens before its first
    HIP call (no GPU here): the relight's own checks, then the scratch limit
    (n <= 256: the n = 512 workspace is 12 MiB against 4 MiB)."""
    E = rrt._abi
    lib = rrt.lib

    def call(L, R, T, out=8, flags=0):
        return lib.rrt_relight_noalloc(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T),
                                       _p(out), flags, None)

    assert E.RRT_NOALLOC_SCRATCH_BYTES == 4 << 20
    for n in (512, 1024):
        assert call(*_desc(rrt, n=n)) == E.RRT_ERR_UNSUPPORTED
        assert b"scratch" in lib.rrt_last_error()
    assert _relight_ws(rrt, *_desc(rrt, n=256))[1] <= E.RRT_NOALLOC_SCRATCH_BYTES
    assert _relight_ws(rrt, *_desc(rrt, n=512, ldtype=E.RRT_F16))[1] > E.RRT_NOALLOC_SCRATCH_BYTES
    assert call(*_desc(rrt, n=3)) == E.RRT_ERR_INVALID
    assert call(*_desc(rrt, nframes=2)) == E.RRT_ERR_INVALID
    assert call(*_desc(rrt), out=0) == E.RRT_ERR_INVALID                   # null radiance
    assert call(*_desc(rrt), flags=4) == E.RRT_ERR_INVALID                 # unknown flag
    assert call(*_desc(rrt), flags=E.RRT_CHAIN_RULE) == E.RRT_ERR_UNSUPPORTED   # n < 32
    L, R, T = _desc(rrt)
    assert lib.rrt_relight_noalloc(None, ctypes.byref(R), ctypes.byref(T), _p(8), 0,
                                   None) == E.RRT_ERR_INVALID


def test_convert_validation(rrt):
    lib = rrt.lib
    E = rrt._abi
    assert lib.rrt_convert(_p(8), 2, 3, E.RRT_F32, _p(8), None, None) == E.RRT_ERR_UNSUPPORTED
    assert lib.rrt_convert(_p(8), 2, 3, E.RRT_E4M3, _p(8), None, None) == E.RRT_ERR_INVALID
    assert lib.rrt_convert(_p(8), 2, 3, E.RRT_S16, _p(8), None, None) == E.RRT_ERR_INVALID
    assert lib.rrt_convert(_p(8), 2, 3, E.RRT_S11, _p(8), None, None) == E.RRT_ERR_INVALID
    assert lib.rrt_convert(_p(0), 2, 3, E.RRT_BF16, _p(8), None, None) == E.RRT_ERR_INVALID
    assert lib.rrt_convert(_p(0), 0, 3, E.RRT_BF16, _p(0), None, None) == E.RRT_OK


def test_cluster_transport_validation(rrt):
    E = rrt._abi
    L, R, T = _desc(rrt)
    T.cluster = 8
    T.nclusters = 0
    assert _relight_ws(rrt, L, R, T)[0] == E.RRT_ERR_INVALID
    T.nclusters = 4
    assert _relight_ws(rrt, L, R, T)[0] == E.RRT_OK
    T.idx = 0
    assert _relight_ws(rrt, L, R, T)[0] == E.RRT_ERR_INVALID


def test_mlp_validation(rrt):
    lib = rrt.lib
    E = rrt._abi
    nb = ctypes.c_size_t(0)
    assert lib.rrt_mlp_workspace(4096, ctypes.byref(nb)) == E.RRT_OK and nb.value > 4096 * 256 * 20
    assert lib.rrt_mlp_workspace(-1, ctypes.byref(nb)) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_encode(_p(0), 10, _p(8), None) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_encode(_p(0), 0, _p(0), None) == E.RRT_OK
    assert lib.rrt_mlp_forward(_p(8), _p(8), _p(8), 64, _p(8), _p(256), 16, None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_mlp_forward(_p(0), _p(8), _p(8), 64, _p(8), _p(256), 1 << 30, None) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_backward(_p(8), _p(8), 0, _p(8), _p(8), _p(8), _p(256), 1 << 30, None) == E.RRT_ERR_INVALID
    assert lib.rrt_mse(_p(0), _p(8), 10, _p(8), _p(8), None) == E.RRT_ERR_INVALID
    # whole-decoder inference: no workspace, clusters >= 1, every pointer
    dec = lambda w=16, C=4, pos=8, clu=8, B=10, out=8: lib.rrt_mlp_decode(  # noqa: E731
        _p(w), _p(8), _p(8), C, _p(pos), _p(clu), B, _p(out), None)
    assert dec(C=0) == E.RRT_ERR_INVALID
    assert dec(w=0) == E.RRT_ERR_INVALID
    assert dec(w=24) == E.RRT_ERR_INVALID        # decoder weights 16-byte aligned
    assert dec(clu=0) == E.RRT_ERR_INVALID
    assert dec(out=0) == E.RRT_ERR_INVALID
    assert dec(B=-1) == E.RRT_ERR_INVALID
    assert dec(B=0, w=0, pos=0, clu=0, out=0) == E.RRT_OK
    # decoder layout: both buffers, 16-byte aligned, not overlapping
    n = 2 * E.RRT_MLP_WEIGHT_COUNT
    assert lib.rrt_mlp_pack(_p(0), _p(1 << 24), None) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_pack(_p(1 << 24), _p(0), None) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_pack(_p(1 << 24), _p((1 << 24) + n - 16), None) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_pack(_p((1 << 24) + n - 16), _p(1 << 24), None) == E.RRT_ERR_INVALID
    assert lib.rrt_mlp_pack(_p(1 << 24), _p((1 << 26) + 8), None) == E.RRT_ERR_INVALID
    f = ctypes.c_float
    assert lib.rrt_adam_step(_p(8), None, _p(8), _p(8), _p(8), 10, f(1e-3), f(0.9), f(0.999), f(1e-8), 0, None) == E.RRT_ERR_INVALID
    assert lib.rrt_adam_step(_p(8), None, _p(8), _p(8), _p(8), 10, f(1e-3), f(1.0), f(0.999), f(1e-8), 1, None) == E.RRT_ERR_INVALID
    assert lib.rrt_adam_step(_p(0), None, _p(0), _p(0), _p(0), 0, f(1e-3), f(0.9), f(0.999), f(1e-8), 1, None) == E.RRT_OK


def test_coarsen_validation(rrt):
    lib, E = rrt.lib, rrt._abi
    assert lib.rrt_coarsen_indices(_p(8), 10, 2, 1, _p(8), None) == E.RRT_ERR_INVALID    # n < 4
    assert lib.rrt_coarsen_indices(_p(8), 10, 12, 1, _p(8), None) == E.RRT_ERR_INVALID   # not 2^k
    assert lib.rrt_coarsen_indices(_p(8), 10, 16, 0, _p(8), None) == E.RRT_ERR_INVALID   # levels 0
    assert lib.rrt_coarsen_indices(_p(8), 10, 16, 4, _p(8), None) == E.RRT_ERR_INVALID   # n' = 1
    assert lib.rrt_coarsen_indices(_p(0), 10, 16, 2, _p(8), None) == E.RRT_ERR_INVALID   # null
    assert lib.rrt_coarsen_indices(_p(0), 0, 16, 3, _p(0), None) == E.RRT_OK             # empty



def test_triple_product_validation(rrt):
    """A BRDF table needs nmaterials >= 1 and 16-byte alignment; the chain
    rule refuses it.  Checked before anything is enqueued."""
    E = rrt._abi
    lib = rrt.lib

    def desc(n=32, brdf=256, nmat=2):
        L = E.Light(n, 10, 8, 8, 0)
        R = E.Rotations(1, 0, 8)
        T = E.Transport(5, 16, 8, 8, 0, 0, 0, 0, brdf, 0, nmat)
        return L, R, T

    assert _relight_ws(rrt, *desc())[0] == E.RRT_OK
    assert _relight_ws(rrt, *desc(nmat=0))[0] == E.RRT_ERR_INVALID
    assert _relight_ws(rrt, *desc(brdf=264))[0] == E.RRT_ERR_INVALID
    assert _relight_ws(rrt, *desc(brdf=0, nmat=0))[0] == E.RRT_OK
    L, R, T = desc()
    assert lib.rrt_relight(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8),
                           E.RRT_CHAIN_RULE, _p(256), 1 << 30, None) == E.RRT_ERR_UNSUPPORTED
    assert lib.rrt_relight_prepared(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8),
                                    E.RRT_CHAIN_RULE, _p(256), 1 << 30,
                                    None) == E.RRT_ERR_UNSUPPORTED


def test_latlong_validation(rrt):
    """Lat-long relight: H a power of two in [4, 512], sizes over 2 H^2,
    no cluster or brdf, flags RRT_COMPENSATED only, workspace checked."""
    E = rrt._abi
    lib = rrt.lib

    def call(H=16, k=10, nnz=16, nvert=5, cluster=0, brdf=0, flags=0, ws=256, wsb=1 << 20,
             elev=8, shift=8):
        L = E.Light(H, k, 8, 8, 0)
        R = E.LatLongRotations(elev, shift)
        T = E.Transport(nvert, nnz, 8, 8, 0, 0, cluster, 1 if cluster else 0, brdf, 0,
                        1 if brdf else 0)
        return lib.rrt_relight_latlong(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), _p(8),
                                       flags, _p(ws), wsb, None)

    nb = ctypes.c_size_t(0)
    L = E.Light(16, 10, 8, 8, 0)
    assert lib.rrt_relight_latlong_workspace(ctypes.byref(L), ctypes.byref(nb)) == E.RRT_OK
    cells = 2 * 16 * 16
    assert nb.value == 2 * ((cells * 4 + 255) // 256 * 256) + 512
    assert call(H=2) == E.RRT_ERR_INVALID
    assert call(H=12) == E.RRT_ERR_INVALID
    assert call(H=1024) == E.RRT_ERR_INVALID
    assert call(k=cells + 1) == E.RRT_ERR_INVALID
    assert call(nnz=cells + 1) == E.RRT_ERR_INVALID
    assert call(cluster=8) == E.RRT_ERR_UNSUPPORTED
    assert call(brdf=256) == E.RRT_ERR_UNSUPPORTED
    assert call(flags=E.RRT_CHAIN_RULE) == E.RRT_ERR_INVALID
    assert call(wsb=64) == E.RRT_ERR_WORKSPACE
    assert call(elev=0) == E.RRT_ERR_INVALID


def test_relight_mlp_validation(rrt):
    """The learned relight checks the decoder, sizes, flags and workspace
    before anything is enqueued."""
    E = rrt._abi
    lib = rrt.lib
    L = E.Light(16, 10, 8, 8, 0)
    R = E.Rotations(1, 0, 8)
    nb = ctypes.c_size_t(0)
    assert lib.rrt_relight_mlp_workspace(ctypes.byref(L), ctypes.byref(R), 100,
                                         ctypes.byref(nb)) == E.RRT_OK
    assert nb.value > 100 * 256 * 4
    assert lib.rrt_relight_mlp_workspace(ctypes.byref(L), ctypes.byref(R), -1,
                                         ctypes.byref(nb)) == E.RRT_ERR_INVALID

    def ws(nvert):
        assert lib.rrt_relight_mlp_workspace(ctypes.byref(L), ctypes.byref(R), nvert,
                                             ctypes.byref(nb)) == E.RRT_OK
        return nb.value
    # the decoded values live one chunk at a time (equal chunks of at most
    # 65,536 vertices): the workspace never exceeds that of one full chunk
    top = ws(65536)
    assert top < 96 << 20
    assert top - ws(65535) >= 1024
    for nvert in (65537, 100_000, 1_000_000, 2_000_000_000):
        assert ws(nvert) <= top

    def call(M, nvert=100, flags=0, wsb=1 << 30, pos=8, clu=8, L=L):
        return lib.rrt_relight_mlp(ctypes.byref(L), ctypes.byref(R),
                                   None if M is None else ctypes.byref(M), _p(pos), _p(clu), nvert,
                                   _p(8), flags, _p(256), wsb, None)

    good = E.Mlp(16, 8, 8, 8, 4)
    assert call(None) == E.RRT_ERR_INVALID
    assert call(E.Mlp(8, 8, 8, 8, 4)) == E.RRT_ERR_INVALID      # weights 16-byte aligned
    assert call(E.Mlp(8, 8, 8, 8, 0)) == E.RRT_ERR_INVALID
    assert call(E.Mlp(0, 8, 8, 8, 4)) == E.RRT_ERR_INVALID
    assert call(good, pos=0) == E.RRT_ERR_INVALID
    assert call(good, flags=8) == E.RRT_ERR_INVALID
    assert call(good, wsb=1024) == E.RRT_ERR_WORKSPACE
    assert call(good, L=E.Light(4, 10, 8, 8, 0)) == E.RRT_ERR_INVALID   # 96 < 256 coefficients


def test_relight_order_validation(rrt):
    E = rrt._abi
    lib = rrt.lib
    nb = ctypes.c_size_t(0)
    assert lib.rrt_relight_order_workspace(1000, ctypes.byref(nb)) == E.RRT_OK and nb.value >= 1000
    assert lib.rrt_relight_order_workspace(-1, ctypes.byref(nb)) == E.RRT_ERR_INVALID
    L = E.Light(16, 1, 8, 8, 0)
    T = E.Transport(100, 16, 8, 8, 0, 0, 0, 0, 0, 0, 0, 0)
    assert lib.rrt_relight_order(ctypes.byref(L), ctypes.byref(T), _p(0), _p(256), 1 << 20,
                                 None) == E.RRT_ERR_INVALID                  # null order
    assert lib.rrt_relight_order(ctypes.byref(L), ctypes.byref(T), _p(8), _p(256), 16,
                                 None) == E.RRT_ERR_WORKSPACE
    assert lib.rrt_relight_order(ctypes.byref(E.Light(12, 1, 8, 8, 0)), ctypes.byref(T), _p(8),
                                 _p(256), 1 << 20, None) == E.RRT_ERR_INVALID
    empty = E.Transport(0, 16, 8, 8, 0, 0, 0, 0, 0, 0, 0, 0)
    assert lib.rrt_relight_order(ctypes.byref(L), ctypes.byref(empty), _p(0), _p(0), 0,
                                 None) == E.RRT_OK
