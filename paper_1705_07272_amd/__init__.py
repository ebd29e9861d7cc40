"""Run-time Haar-domain relighting on MI355X (gfx950).

Thin torch-facing binding of librrt.so: every function checks and marshals
its tensor arguments and calls the C ABI of include/rrt.h; all arithmetic
runs in the library's HIP kernels.  torch provides device memory and the
current stream only.

Every function checks the shapes of its tensors against the sizes it passes
to the library (vertex count, row length, block count, frame count, ...)
before it checks devices or calls into the library, and raises ValueError on
a mismatch: the kernels index their buffers by those sizes, so a tensor of
the wrong shape would otherwise be read or written out of bounds.
"""
import ctypes

import torch

from . import _abi
from ._abi import (RRT_BF16, RRT_BLOCK, RRT_CHAIN_RULE, RRT_COMPENSATED, RRT_E4M3, RRT_F16, RRT_F32,  # noqa: F401
                   RRT_S11, RRT_S16, LatLongRotations, Light, Mlp, RrtError, Rotations, Transport, check,
                   lib)

__all__ = ["haar_forward", "haar_inverse", "topk", "coarsen_indices", "haar_phase_shift", "relight",
           "relight_noalloc",
           "relight_latlong", "relight_mlp", "relight_order", "mlp_encode", "mlp_pack", "mlp_decode",
           "mlp_forward", "mlp_backward", "mlp_workspace", "mse", "adam_step",
           "relight_workspace_bytes", "PreparedLighting", "prepare_lighting", "convert",
           "project_rows", "RrtError", "lib"]

_DTYPES = {torch.float32: RRT_F32, torch.float16: RRT_F16, torch.bfloat16: RRT_BF16,
           torch.uint8: RRT_E4M3, torch.int16: RRT_S16, torch.int32: RRT_S11}
# dtypes of stored transport values (int32: packed 11-bit words)
_TRANSPORT_DTYPES = (torch.float32, torch.bfloat16, torch.uint8, torch.int16, torch.int32)


def s11_words(nnz):
    """int32 words of one packed 11-bit row of nnz values (RRT_S11_WORDS)."""
    return (11 * nnz + 31) // 32


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, name, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _numel(t, name, count):
    """t (a tensor, or None) holds exactly `count` elements."""
    if t is not None and t.numel() != count:
        raise ValueError(f"{name} has shape {tuple(t.shape)} ({t.numel()} elements), "
                         f"expected {count} elements")


def _rows(t, name, rows, cols):
    """t is [rows, cols] (a 1-D tensor stands for one row)."""
    if t is None:
        return
    shape = tuple(t.shape)
    ok = (t.dim() == 2 and shape == (rows, cols)) or (t.dim() == 1 and rows == 1 and shape == (cols,))
    if not ok:
        raise ValueError(f"{name} has shape {shape}, expected ({rows}, {cols})")


def _rotations(t, name):
    """[count, 3, 3] or [count, 9] rotations -> count."""
    if t.dim() == 0 or t.numel() != 9 * t.shape[0]:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (count, 3, 3)")
    return t.shape[0]


def _nblk(nnz):
    return (nnz + RRT_BLOCK - 1) // RRT_BLOCK


def _transport_shapes(nvert, t_idx, t_val, block_scale, cluster=None, brdf=None, material=None,
                      order=None, n=None, squares=6):
    """Shapes of a transport given as tensors; returns nnz."""
    if t_val.dim() not in (1, 2):
        raise ValueError(f"transport_val has shape {tuple(t_val.shape)}, expected (V, nnz)")
    if t_val.dtype == torch.int32:
        # packed 11-bit rows: nnz comes from the index rows (or the dense map)
        if t_idx is not None:
            if t_idx.dim() not in (1, 2):
                raise ValueError(f"transport_idx has shape {tuple(t_idx.shape)}, expected (V, nnz)")
            nnz = t_idx.shape[-1]
        elif n is not None:
            nnz = squares * n * n
        else:
            raise ValueError("packed 11-bit transport needs index rows or the map size")
        _rows(t_val, "transport_val", nvert, s11_words(nnz))
    else:
        nnz = t_val.shape[-1] if t_val.dim() > 1 else t_val.numel()
        _rows(t_val, "transport_val", nvert, nnz)
    if cluster is not None:
        _numel(cluster, "cluster", nvert)
        if t_idx is None or t_idx.dim() != 2 or t_idx.shape[1] != nnz:
            raise ValueError("with cluster, transport_idx must be a support table (C, nnz) "
                             f"with nnz = {nnz}")
    elif t_idx is not None:
        _rows(t_idx, "transport_idx", nvert, nnz)
    if t_val.dtype in (torch.uint8, torch.int16, torch.int32):
        if block_scale is None:
            raise ValueError("block-scaled transport (uint8 / int16 / packed int32 codes) needs "
                             "block_scale")
        _rows(block_scale, "block_scale", nvert, _nblk(nnz))
    if brdf is not None:
        if n is None or brdf.dim() == 0 or brdf.numel() != brdf.shape[0] * squares * n * n:
            raise ValueError(f"brdf has shape {tuple(brdf.shape)}, expected (M, {squares}, n, n)")
        _numel(material, "material", nvert)
    _numel(order, "order", nvert)
    return nnz


def _light_shapes(light_idx, light_val):
    if light_idx.dim() != 1 or tuple(light_val.shape) != tuple(light_idx.shape):
        raise ValueError(f"light_idx {tuple(light_idx.shape)} and light_val "
                         f"{tuple(light_val.shape)} must be the same 1-D shape")


def _ptr_or_null(t, name, dtype=None):
    return ctypes.c_void_p(0) if t is None else _dev(t, name, dtype)


def _workspace(nbytes, device):
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


def _square(t, name):
    """[..., n, n] -> n."""
    if t.dim() < 2 or t.shape[-1] != t.shape[-2]:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (..., n, n)")
    return t.shape[-1]


def haar_forward(pix, out=None):
    """Haar transform of every n x n square of [..., n, n] float32 (cube maps
    [..., 6, n, n], lat-long maps [..., 2, H, H])."""
    n = _square(pix, "pix")
    count = pix.numel() // (n * n) if pix.numel() else 0
    _numel(out, "out", pix.numel())
    out = torch.empty_like(pix) if out is None else out
    check(lib.rrt_haar_forward(_dev(pix, "pix", torch.float32), _dev(out, "out", torch.float32),
                               n, count, _stream()))
    return out


def haar_inverse(coef, out=None):
    n = _square(coef, "coef")
    count = coef.numel() // (n * n) if coef.numel() else 0
    _numel(out, "out", coef.numel())
    out = torch.empty_like(coef) if out is None else out
    check(lib.rrt_haar_inverse(_dev(coef, "coef", torch.float32), _dev(out, "out", torch.float32),
                               n, count, _stream()))
    return out


def topk(x, k, out=None, workspace=None):
    """Row-wise k largest |x| -> (idx int32 ascending, values) for x [rows, len].
    out: optional (idx, val) tensors to fill; workspace: optional device
    buffer of at least rrt_topk_workspace() bytes."""
    if x.dim() != 2:
        raise ValueError(f"x has shape {tuple(x.shape)}, expected (rows, len)")
    rows, length = x.shape
    if not 0 <= k <= length:
        raise ValueError(f"k={k} not in [0, {length}]")
    if out is None:
        idx = torch.empty((rows, k), dtype=torch.int32, device=x.device)
        val = torch.empty((rows, k), dtype=torch.float32, device=x.device)
    else:
        idx, val = out
        _numel(idx, "idx", rows * k)
        _numel(val, "val", rows * k)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_topk_workspace(rows, length, k, ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, x.device) if workspace is None else workspace
    if ws.dtype != torch.uint8:
        raise TypeError("workspace must be a uint8 tensor")
    check(lib.rrt_topk(_dev(x, "x", torch.float32), rows, length, k, _dev(idx, "idx", torch.int32),
                       _dev(val, "val", torch.float32), _dev(ws, "ws"), ws.numel(), _stream()))
    return idx, val


def topk_workspace_bytes(rows, length, k):
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_topk_workspace(rows, length, k, ctypes.byref(nbytes)))
    return nbytes.value


def coarsen_indices(idx, n, levels):
    """Flat coefficient indices at resolution n -> the same coefficients'
    indices at n >> levels, -1 for the `levels` finest levels."""
    out = torch.empty_like(idx)
    check(lib.rrt_coarsen_indices(_dev(idx, "idx", torch.int32), idx.numel(), n, levels,
                                  _dev(out, "out"), _stream()))
    return out


def haar_phase_shift(coef, rot):
    """Dense Haar-domain rotation of one cube map [6, n, n] by rot [r, 3, 3]."""
    n = _square(coef, "coef")
    if tuple(coef.shape) != (6, n, n):
        raise ValueError(f"coef has shape {tuple(coef.shape)}, expected (6, n, n)")
    nrot = _rotations(rot, "rot")
    out = torch.empty((nrot, 6, n, n), dtype=torch.float32, device=coef.device)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_haar_phase_shift_workspace(n, nrot, ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, coef.device)
    check(lib.rrt_haar_phase_shift(_dev(coef, "coef", torch.float32), n,
                                   _dev(rot, "rot", torch.float32), nrot,
                                   _dev(out, "out"), _dev(ws, "ws"), nbytes.value, _stream()))
    return out


def _descriptors(n, light_idx, light_val, vert_rot, t_idx, t_val, frame_rot, block_scale,
                 cluster=None, brdf=None, material=None, order=None, out=None):
    _light_shapes(light_idx, light_val)
    nvert = _rotations(vert_rot, "vert_rot")
    nframes = 1 if frame_rot is None else _rotations(frame_rot, "frame_rot")
    _numel(out, "out", nframes * nvert)
    nnz = _transport_shapes(nvert, t_idx, t_val, block_scale, cluster, brdf, material, order, n)
    L = Light(n, light_idx.numel(), _dev(light_idx, "light_idx", torch.int32).value,
              _dev(light_val, "light_val", (torch.float32, torch.float16)).value,
              _DTYPES[light_val.dtype])
    nframes = 1 if frame_rot is None else frame_rot.shape[0]
    R = Rotations(nframes, _ptr_or_null(frame_rot, "frame_rot", torch.float32).value,
                  _dev(vert_rot, "vert_rot", torch.float32).value)
    nvert = vert_rot.shape[0]
    T = Transport(nvert, nnz, _ptr_or_null(t_idx, "transport_idx", torch.int32).value,
                  _dev(t_val, "transport_val", _TRANSPORT_DTYPES).value,
                  _DTYPES[t_val.dtype],
                  _ptr_or_null(block_scale, "block_scale", torch.float32).value,
                  _ptr_or_null(cluster, "cluster", torch.int32).value,
                  0 if cluster is None else t_idx.shape[0],
                  _ptr_or_null(brdf, "brdf", torch.float32).value,
                  _ptr_or_null(material, "material", torch.int32).value,
                  0 if brdf is None else brdf.shape[0],
                  _ptr_or_null(order, "order", torch.int32).value)
    return L, R, T


def _flags(compensated, chain_rule):
    return (RRT_COMPENSATED if compensated else 0) | (RRT_CHAIN_RULE if chain_rule else 0)


def relight_workspace_bytes(n, light_idx, light_val, vert_rot, t_idx, t_val, frame_rot=None,
                            block_scale=None, compensated=False, chain_rule=False):
    L, R, T = _descriptors(n, light_idx, light_val, vert_rot, t_idx, t_val, frame_rot, block_scale)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_workspace(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T),
                                    _flags(compensated, chain_rule), ctypes.byref(nbytes)))
    return nbytes.value


def relight(n, light_idx, light_val, vert_rot, t_idx, t_val, frame_rot=None, block_scale=None,
            compensated=False, out=None, workspace=None, cluster=None, chain_rule=False,
            brdf=None, material=None, order=None):
    """radiance [F, V] float32.

    light_idx [k] int32, light_val [k] float32|float16; vert_rot [V, 3, 3]
    float32; t_idx [V, nnz] int32 or None (dense rows); t_val [V, nnz]
    float32|bfloat16|uint8 (E4M3 codes)|int16 (fixed-point codes), the
    block-scaled forms with block_scale [V, ceil(nnz/64)];
    frame_rot [F, 3, 3] float32 or None.  With cluster [V] int32, t_idx is a
    per-cluster support table [C, nnz] and vertex v uses row cluster[v].
    chain_rule: rotate the finest level by the chain rule (n >= 32).
    brdf [M, 6, n, n] float32 (texel-domain BRDF x cosine x solid angle in the
    local frame) with material [V] int32 or None: the triple product, t_* then
    hold the visibility rows.
    order [V] int32: processing order of the vertices (relight_order), or None.
    """
    L, R, T = _descriptors(n, light_idx, light_val, vert_rot, t_idx, t_val, frame_rot, block_scale,
                           cluster, brdf, material, order, out)
    flags = _flags(compensated, chain_rule)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_workspace(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T), flags,
                                    ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _workspace(nbytes.value, vert_rot.device)
    if workspace.dtype != torch.uint8:
        raise TypeError("workspace must be a uint8 tensor")
    if out is None:
        out = torch.empty((R.nframes, T.nvert), dtype=torch.float32, device=vert_rot.device)
    check(lib.rrt_relight(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T),
                          _dev(out, "out", torch.float32), flags, _dev(workspace, "workspace"),
                          workspace.numel(), _stream()))
    return out


def relight_noalloc(n, light_idx, light_val, vert_rot, t_idx, t_val, out, frame_rot=None,
                    block_scale=None, compensated=False, cluster=None, chain_rule=False,
                    brdf=None, material=None, order=None):
    """relight() through rrt_relight_noalloc: no workspace and no allocation,
    the caller passes the output out [F, V] float32.  The library's scratch
    array holds the workspace (n <= 256); calls that overlap on one GPU race."""
    if out is None:
        raise ValueError("relight_noalloc writes into a caller-provided out [F, V]")
    L, R, T = _descriptors(n, light_idx, light_val, vert_rot, t_idx, t_val, frame_rot, block_scale,
                           cluster, brdf, material, order, out)
    check(lib.rrt_relight_noalloc(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T),
                                  _dev(out, "out", torch.float32),
                                  _flags(compensated, chain_rule), _stream()))
    return out


class PreparedLighting:
    """Lighting whose source map P = W^T L has been reconstructed into a
    device workspace by rrt_relight_prepare (with the chain rule's block
    coefficients if chain_rule)."""

    def __init__(self, n, light_idx, light_val, workspace, chain_rule=False):
        self.n = n
        self.light_idx = light_idx
        self.light_val = light_val
        self.workspace = workspace
        self.chain_rule = chain_rule


def prepare_lighting(n, light_idx, light_val, workspace=None, chain_rule=False):
    _light_shapes(light_idx, light_val)
    L = Light(n, light_idx.numel(), _dev(light_idx, "light_idx", torch.int32).value,
              _dev(light_val, "light_val", (torch.float32, torch.float16)).value,
              _DTYPES[light_val.dtype])
    nbytes = ctypes.c_size_t(0)
    dummy_r = Rotations(1, None, 1)
    dummy_t = Transport(0, 1, 1, 1, RRT_F32, None, None, 0)
    check(lib.rrt_relight_workspace(ctypes.byref(L), ctypes.byref(dummy_r), ctypes.byref(dummy_t),
                                    0, ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _workspace(nbytes.value, light_idx.device)
    if workspace.dtype != torch.uint8:
        raise TypeError("workspace must be a uint8 tensor")
    check(lib.rrt_relight_prepare(ctypes.byref(L), _flags(False, chain_rule),
                                  _dev(workspace, "workspace"), workspace.numel(), _stream()))
    return PreparedLighting(n, light_idx, light_val, workspace, chain_rule)


def relight_prepared(prep, vert_rot, t_idx, t_val, frame_rot=None, block_scale=None,
                     compensated=False, out=None, cluster=None, brdf=None, material=None,
                     order=None):
    """relight() with a lighting already reconstructed by prepare_lighting()
    (the chain rule applies when the lighting was prepared for it)."""
    L, R, T = _descriptors(prep.n, prep.light_idx, prep.light_val, vert_rot, t_idx, t_val,
                           frame_rot, block_scale, cluster, brdf, material, order, out)
    if out is None:
        out = torch.empty((R.nframes, T.nvert), dtype=torch.float32, device=vert_rot.device)
    check(lib.rrt_relight_prepared(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T),
                                   _dev(out, "out", torch.float32),
                                   _flags(compensated, prep.chain_rule),
                                   _dev(prep.workspace, "workspace"), prep.workspace.numel(),
                                   _stream()))
    return out


def relight_latlong(H, light_idx, light_val, elev, shift, t_idx, t_val, block_scale=None,
                    compensated=False, out=None, workspace=None):
    """radiance [V] float32 on the longitude-latitude map (rrt_relight_latlong).

    light_idx [k] int32 / light_val [k] float32|float16 over [2, H, H];
    elev [V, 2] float32 (cos b, sin b); shift [V, 2] int32 (s_a, s_c);
    t_idx [V, nnz] int32 or None (dense), t_val [V, nnz] as for relight()."""
    _light_shapes(light_idx, light_val)
    if elev.dim() != 2 or elev.shape[1] != 2:
        raise ValueError(f"elev has shape {tuple(elev.shape)}, expected (V, 2)")
    _rows(shift, "shift", elev.shape[0], 2)
    nnz = _transport_shapes(elev.shape[0], t_idx, t_val, block_scale, n=H, squares=2)
    _numel(out, "out", elev.shape[0])
    L = Light(H, light_idx.numel(), _dev(light_idx, "light_idx", torch.int32).value,
              _dev(light_val, "light_val", (torch.float32, torch.float16)).value,
              _DTYPES[light_val.dtype])
    R = LatLongRotations(_dev(elev, "elev", torch.float32).value,
                         _dev(shift, "shift", torch.int32).value)
    nvert = elev.shape[0]
    T = Transport(nvert, nnz, _ptr_or_null(t_idx, "transport_idx", torch.int32).value,
                  _dev(t_val, "transport_val", _TRANSPORT_DTYPES).value,
                  _DTYPES[t_val.dtype], _ptr_or_null(block_scale, "block_scale", torch.float32).value,
                  None, 0, None, None, 0)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_latlong_workspace(ctypes.byref(L), ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _workspace(nbytes.value, elev.device)
    if workspace.dtype != torch.uint8:
        raise TypeError("workspace must be a uint8 tensor")
    if out is None:
        out = torch.empty(nvert, dtype=torch.float32, device=elev.device)
    check(lib.rrt_relight_latlong(ctypes.byref(L), ctypes.byref(R), ctypes.byref(T),
                                  _dev(out, "out", torch.float32),
                                  RRT_COMPENSATED if compensated else 0,
                                  _dev(workspace, "workspace"), workspace.numel(), _stream()))
    return out


def relight_mlp(n, light_idx, light_val, vert_rot, weights, bias, supports, scales, pos_nrm,
                cluster, frame_rot=None, compensated=False, out=None, workspace=None):
    """radiance [F, V] float32 with the learned transport (rrt_relight_mlp):
    weights RRT_MLP_WEIGHT_COUNT bfloat16 in the decoder layout (mlp_pack),
    bias RRT_MLP_BIAS_COUNT float32,
    supports [C, 256] int32, scales [C, 256] float32, pos_nrm [V, 6]
    float32, cluster [V] int32."""
    _light_shapes(light_idx, light_val)
    _mlp_shapes(weights, bias)
    if supports.dim() != 2 or supports.shape[1] != RRT_MLP_OUT:
        raise ValueError(f"supports has shape {tuple(supports.shape)}, expected (C, {RRT_MLP_OUT})")
    _rows(scales, "scales", supports.shape[0], RRT_MLP_OUT)
    nvert = _rotations(vert_rot, "vert_rot")
    _rows(pos_nrm, "pos_nrm", nvert, 6)
    _numel(cluster, "cluster", nvert)
    nframes = 1 if frame_rot is None else _rotations(frame_rot, "frame_rot")
    _numel(out, "out", nframes * nvert)
    L = Light(n, light_idx.numel(), _dev(light_idx, "light_idx", torch.int32).value,
              _dev(light_val, "light_val", (torch.float32, torch.float16)).value,
              _DTYPES[light_val.dtype])
    nframes = 1 if frame_rot is None else frame_rot.shape[0]
    R = Rotations(nframes, _ptr_or_null(frame_rot, "frame_rot", torch.float32).value,
                  _dev(vert_rot, "vert_rot", torch.float32).value)
    M = Mlp(_dev(weights, "weights", torch.bfloat16).value, _dev(bias, "bias", torch.float32).value,
            _dev(supports, "supports", torch.int32).value, _dev(scales, "scales", torch.float32).value,
            supports.shape[0])
    nvert = pos_nrm.shape[0]
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_mlp_workspace(ctypes.byref(L), ctypes.byref(R), nvert,
                                        ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _workspace(nbytes.value, pos_nrm.device)
    if workspace.dtype != torch.uint8:
        raise TypeError("workspace must be a uint8 tensor")
    if out is None:
        out = torch.empty((nframes, nvert), dtype=torch.float32, device=pos_nrm.device)
    check(lib.rrt_relight_mlp(ctypes.byref(L), ctypes.byref(R), ctypes.byref(M),
                              _dev(pos_nrm, "pos_nrm", torch.float32), _dev(cluster, "cluster", torch.int32),
                              nvert, _dev(out, "out", torch.float32),
                              RRT_COMPENSATED if compensated else 0, _dev(workspace, "workspace"),
                              workspace.numel(), _stream()))
    return out


def relight_mlp_workspace_bytes(n, light_idx, light_val, nvert):
    L = Light(n, light_idx.numel(), _dev(light_idx, "light_idx", torch.int32).value,
              _dev(light_val, "light_val", (torch.float32, torch.float16)).value,
              _DTYPES[light_val.dtype])
    R = Rotations(1, None, None)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_mlp_workspace(ctypes.byref(L), ctypes.byref(R), nvert,
                                        ctypes.byref(nbytes)))
    return nbytes.value


def relight_order(n, t_idx, cluster=None, out=None, workspace=None, nvert=None, device="cuda"):
    """Heavy-first processing order [V] int32 of transport rows t_idx [V, nnz]
    (or, with cluster [V], support rows t_idx [C, nnz]) over 6 n^2
    coefficients (rrt_relight_order); t_idx None means nvert dense rows."""
    if t_idx is None:
        if nvert is None:
            raise ValueError("dense rows (t_idx None) need nvert")
        V, nnz, dev_ = nvert, 6 * n * n, torch.device(device)
    else:
        if t_idx.dim() != 2:
            raise ValueError(f"t_idx has shape {tuple(t_idx.shape)}, expected (rows, nnz)")
        V = t_idx.shape[0] if cluster is None else cluster.numel()
        nnz, dev_ = t_idx.shape[-1], t_idx.device
    _numel(out, "order", V)
    dummy = torch.empty(1, dtype=torch.int32, device=dev_)
    L = Light(n, 1, dummy.data_ptr(), dummy.data_ptr(), RRT_F32)
    T = Transport(V, nnz, _ptr_or_null(t_idx, "t_idx", torch.int32).value, None, RRT_F32, None,
                  _ptr_or_null(cluster, "cluster", torch.int32).value,
                  0 if cluster is None else t_idx.shape[0], None, None, 0, None)
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_order_workspace(V, ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _workspace(nbytes.value, dev_)
    if out is None:
        out = torch.empty(V, dtype=torch.int32, device=dev_)
    check(lib.rrt_relight_order(ctypes.byref(L), ctypes.byref(T), _dev(out, "order", torch.int32),
                                _dev(workspace, "workspace"), workspace.numel(), _stream()))
    return out


def relight_order_workspace_bytes(nvert):
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_relight_order_workspace(nvert, ctypes.byref(nbytes)))
    return nbytes.value


def project_rows(pix, nnz):
    """Haar transform of per-vertex pixel-domain transport [B, 6, n, n]
    (float32, device) and its top-nnz truncation -> (idx [B, nnz] int32,
    values [B, nnz] float32): the stored CSR rows of the relighting path."""
    coef = haar_forward(pix)
    return topk(coef.view(pix.shape[0], -1), nnz)


def convert(x, dtype):
    """Storage conversion of a [rows, cols] float32 tensor: 'f16', 'bf16',
    'e4m3', 's16' or 's11' (the last three return (codes, block scales
    float32); 's11' codes are packed into [rows, s11_words(cols)] int32)."""
    if x.dim() != 2:
        raise ValueError(f"x has shape {tuple(x.shape)}, expected (rows, cols)")
    rows, cols = x.shape
    if dtype == "f16":
        out = torch.empty((rows, cols), dtype=torch.float16, device=x.device)
        check(lib.rrt_convert(_dev(x, "x", torch.float32), rows, cols, RRT_F16, _dev(out, "out"),
                              None, _stream()))
        return out
    if dtype == "bf16":
        out = torch.empty((rows, cols), dtype=torch.bfloat16, device=x.device)
        check(lib.rrt_convert(_dev(x, "x", torch.float32), rows, cols, RRT_BF16, _dev(out, "out"),
                              None, _stream()))
        return out
    if dtype in ("e4m3", "s16"):
        nblk = (cols + RRT_BLOCK - 1) // RRT_BLOCK
        code_t, code = (torch.uint8, RRT_E4M3) if dtype == "e4m3" else (torch.int16, RRT_S16)
        out = torch.empty((rows, cols), dtype=code_t, device=x.device)
        scale = torch.empty((rows, nblk), dtype=torch.float32, device=x.device)
        check(lib.rrt_convert(_dev(x, "x", torch.float32), rows, cols, code, _dev(out, "out"),
                              _dev(scale, "scale"), _stream()))
        return out, scale
    if dtype == "s11":
        nblk = (cols + RRT_BLOCK - 1) // RRT_BLOCK
        out = torch.empty((rows, s11_words(cols)), dtype=torch.int32, device=x.device)
        scale = torch.empty((rows, nblk), dtype=torch.float32, device=x.device)
        check(lib.rrt_convert(_dev(x, "x", torch.float32), rows, cols, RRT_S11, _dev(out, "out"),
                              _dev(scale, "scale"), _stream()))
        return out, scale
    raise ValueError(f"unknown dtype {dtype}")


# ---------------------------------------------------------------------------
# Learned transport decoder
# ---------------------------------------------------------------------------
from ._abi import (RRT_MLP_BIAS_COUNT, RRT_MLP_HIDDEN, RRT_MLP_IN, RRT_MLP_OUT,  # noqa: E402,F401
                   RRT_MLP_WEIGHT_COUNT)


def _mlp_shapes(w, bias):
    _numel(w, "weights", RRT_MLP_WEIGHT_COUNT)
    _numel(bias, "bias", RRT_MLP_BIAS_COUNT)


def mlp_encode(pos_nrm):
    """[B, 6] float32 -> [B, 128] bfloat16 positional encoding."""
    if pos_nrm.dim() != 2 or pos_nrm.shape[1] != 6:
        raise ValueError(f"pos_nrm has shape {tuple(pos_nrm.shape)}, expected (B, 6)")
    B = pos_nrm.shape[0]
    x = torch.empty((B, RRT_MLP_IN), dtype=torch.bfloat16, device=pos_nrm.device)
    check(lib.rrt_mlp_encode(_dev(pos_nrm, "pos_nrm", torch.float32), B, _dev(x, "x"), _stream()))
    return x


def mlp_pack(w_bf16, out=None):
    """The weights in the decoder layout (rrt_mlp_pack): [294912] bfloat16,
    what mlp_decode and relight_mlp take."""
    _numel(w_bf16, "weights", RRT_MLP_WEIGHT_COUNT)
    _numel(out, "out", RRT_MLP_WEIGHT_COUNT)
    out = torch.empty(RRT_MLP_WEIGHT_COUNT, dtype=torch.bfloat16, device=w_bf16.device) if out is None else out
    check(lib.rrt_mlp_pack(_dev(w_bf16, "w", torch.bfloat16), _dev(out, "out", torch.bfloat16),
                           _stream()))
    return out


def mlp_decode(w_dec, bias, scales, pos_nrm, cluster, out=None):
    """Decoded transport values [B, 256] float32 (rrt_mlp_decode): the whole
    network and the per-slot scales of each vertex's cluster in one kernel.
    w_dec: the weights in the decoder layout (mlp_pack); scales [C, 256]
    float32, pos_nrm [B, 6] float32, cluster [B] int32."""
    _mlp_shapes(w_dec, bias)
    if scales.dim() != 2 or scales.shape[1] != RRT_MLP_OUT:
        raise ValueError(f"scales has shape {tuple(scales.shape)}, expected (C, {RRT_MLP_OUT})")
    if pos_nrm.dim() != 2 or pos_nrm.shape[1] != 6:
        raise ValueError(f"pos_nrm has shape {tuple(pos_nrm.shape)}, expected (B, 6)")
    B = pos_nrm.shape[0]
    _numel(cluster, "cluster", B)
    _numel(out, "out", B * RRT_MLP_OUT)
    out = torch.empty((B, RRT_MLP_OUT), dtype=torch.float32, device=pos_nrm.device) if out is None else out
    check(lib.rrt_mlp_decode(_dev(w_dec, "w_dec", torch.bfloat16), _dev(bias, "bias", torch.float32),
                             _dev(scales, "scales", torch.float32), scales.shape[0],
                             _dev(pos_nrm, "pos_nrm", torch.float32),
                             _dev(cluster, "cluster", torch.int32), B,
                             _dev(out, "out", torch.float32), _stream()))
    return out


def mlp_workspace(B, device):
    nbytes = ctypes.c_size_t(0)
    check(lib.rrt_mlp_workspace(B, ctypes.byref(nbytes)))
    return _workspace(nbytes.value, device)


def mlp_forward(w_bf16, bias, x, workspace=None, out=None):
    """out [B, 256] float32 for packed bfloat16 weights and float32 biases."""
    _mlp_shapes(w_bf16, bias)
    if x.dim() != 2 or x.shape[1] != RRT_MLP_IN:
        raise ValueError(f"x has shape {tuple(x.shape)}, expected (B, {RRT_MLP_IN})")
    B = x.shape[0]
    _numel(out, "out", B * RRT_MLP_OUT)
    workspace = mlp_workspace(B, x.device) if workspace is None else workspace
    out = torch.empty((B, RRT_MLP_OUT), dtype=torch.float32, device=x.device) if out is None else out
    check(lib.rrt_mlp_forward(_dev(w_bf16, "w", torch.bfloat16), _dev(bias, "bias", torch.float32),
                              _dev(x, "x", torch.bfloat16), B, _dev(out, "out", torch.float32),
                              _dev(workspace, "workspace"), workspace.numel(), _stream()))
    return out


def mlp_backward(w_bf16, x, dout, workspace, dw=None, db=None):
    """(dw [294912], db [1280]) float32; workspace from the forward pass."""
    _numel(w_bf16, "weights", RRT_MLP_WEIGHT_COUNT)
    if x.dim() != 2 or x.shape[1] != RRT_MLP_IN:
        raise ValueError(f"x has shape {tuple(x.shape)}, expected (B, {RRT_MLP_IN})")
    B = x.shape[0]
    _numel(dout, "dout", B * RRT_MLP_OUT)
    _numel(dw, "dw", RRT_MLP_WEIGHT_COUNT)
    _numel(db, "db", RRT_MLP_BIAS_COUNT)
    dw = torch.empty(RRT_MLP_WEIGHT_COUNT, dtype=torch.float32, device=x.device) if dw is None else dw
    db = torch.empty(RRT_MLP_BIAS_COUNT, dtype=torch.float32, device=x.device) if db is None else db
    check(lib.rrt_mlp_backward(_dev(w_bf16, "w", torch.bfloat16), _dev(x, "x", torch.bfloat16), B,
                               _dev(dout, "dout", torch.float32), _dev(dw, "dw", torch.float32),
                               _dev(db, "db", torch.float32), _dev(workspace, "workspace"),
                               workspace.numel(), _stream()))
    return dw, db


def mse(out, target, dout=None, loss=None):
    """(dout, loss) with loss a device float64 scalar tensor (accumulated)."""
    _numel(target, "target", out.numel())
    _numel(dout, "dout", out.numel())
    _numel(loss, "loss", 1)
    dout = torch.empty_like(out) if dout is None else dout
    loss = torch.zeros((), dtype=torch.float64, device=out.device) if loss is None else loss
    check(lib.rrt_mse(_dev(out, "out", torch.float32), _dev(target, "target", torch.float32),
                      out.numel(), _dev(dout, "dout", torch.float32), _dev(loss, "loss", torch.float64),
                      _stream()))
    return dout, loss


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, param_bf16=None):
    for t, name in ((grad, "grad"), (m, "m"), (v, "v"), (param_bf16, "param_bf16")):
        _numel(t, name, param.numel())
    check(lib.rrt_adam_step(_dev(param, "param", torch.float32),
                            _ptr_or_null(param_bf16, "param_bf16", torch.bfloat16),
                            _dev(m, "m", torch.float32), _dev(v, "v", torch.float32),
                            _dev(grad, "grad", torch.float32), param.numel(), lr, beta1, beta2,
                            eps, step, _stream()))
