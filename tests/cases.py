"""Test-case assembly: seeded scene data (scenes) turned into the stored
inputs of the relighting path by the FP64 checker (oracle), plus the
checker's reference radiance.  Used by the GPU parity tests and smoke().
"""
import numpy as np

from oracle.haar import haar_forward
from oracle.relight import lighting_coefficients, relight, rel_l2, transport_rows  # noqa: F401
from scenes.scene import (Workload, frame_rotations, lighting_pixels, phong_exponents,
                          transport_pixels, vertex_rotations)


def workload(cfg, n, k_light, nverts, nnz, nframes=1, exp_lo=1.0, exp_hi=200.0,
             vertex_frames="random"):
    return Workload(cfg, f"test{cfg}", n, k_light, nverts, nframes, nnz, exp_lo, exp_hi,
                    vertex_frames)


def stored_transport(w, vertex_ids, batch=64):
    """Checker-made transport rows of the given vertices: (idx int32 [B, nnz]
    or None when dense, values float32 [B, nnz])."""
    exps = phong_exponents(w)
    vertex_ids = np.asarray(vertex_ids)
    dense = w.nnz == 6 * w.n * w.n
    idx_parts, val_parts = [], []
    for s in range(0, len(vertex_ids), batch):
        vids = vertex_ids[s:s + batch]
        T = transport_pixels(w, exps[vids], vids)
        if dense:
            val_parts.append(haar_forward(T).reshape(len(vids), -1).astype(np.float32))
        else:
            i, v = transport_rows(T, w.nnz)
            idx_parts.append(i)
            val_parts.append(v)
    vals = np.concatenate(val_parts) if val_parts else np.zeros((0, w.nnz), np.float32)
    if dense:
        return None, vals
    idx = np.concatenate(idx_parts) if idx_parts else np.zeros((0, w.nnz), np.int32)
    return idx, vals


def build_case(w, vertex_ids=None):
    """All stored inputs of a workload (for the listed vertices, default all)."""
    vertex_ids = np.arange(w.nverts) if vertex_ids is None else np.asarray(vertex_ids)
    pix = lighting_pixels(w.cfg, w.n)
    li, lv = lighting_coefficients(pix, w.k_light)
    Rv = vertex_rotations(w)[vertex_ids]
    Rf = frame_rotations(w)
    ti, tv = stored_transport(w, vertex_ids)
    return dict(n=w.n, pix=pix, light_idx=li, light_val=lv, vert_rot=Rv, frame_rot=Rf,
                t_idx=ti, t_val=tv)


def reference(case, vertices=None, frames=None, return_scale=False):
    return relight(case["light_idx"], case["light_val"], case["n"], case["vert_rot"],
                   case["frame_rot"], case["t_idx"], case["t_val"], vertices=vertices,
                   frames=frames, return_scale=return_scale)


def frame_errors(got, ref):
    """Per-frame relative L2 error of [F, V] radiance."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return [rel_l2(got[f], ref[f]) for f in range(ref.shape[0])]


def triple_case(w, materials, vertex_ids=None, batch=64):
    """Stored inputs of the triple product: the lighting and rotations of
    build_case, the materials' texel-domain BRDF factors [M, 6, n, n]
    (float32), each vertex's material, and its visibility rows (Haar
    coefficients of the binary visibility, top-nnz by the checker)."""
    from scenes.scene import brdf_pixels, material_ids, visibility_np
    vertex_ids = np.arange(w.nverts) if vertex_ids is None else np.asarray(vertex_ids)
    pix = lighting_pixels(w.cfg, w.n)
    li, lv = lighting_coefficients(pix, w.k_light)
    idx_parts, val_parts = [], []
    for s in range(0, len(vertex_ids), batch):
        vis = visibility_np(w.cfg, vertex_ids[s:s + batch], w.n, w.occlusion).astype(np.float64)
        i, v = transport_rows(vis, w.nnz)
        idx_parts.append(i)
        val_parts.append(v)
    return dict(n=w.n, light_idx=li, light_val=lv, vert_rot=vertex_rotations(w)[vertex_ids],
                frame_rot=frame_rotations(w), brdf=brdf_pixels(w, materials).astype(np.float32),
                material=material_ids(w, materials)[vertex_ids],
                t_idx=np.concatenate(idx_parts), t_val=np.concatenate(val_parts))


def latlong_case(w, vertex_ids=None):
    """Stored inputs of a longitude-latitude workload (scenes.latlong): the
    checker's top-k lighting and top-nnz transport rows over [2, H, H], and
    the vertices' (cos b, sin b) and azimuth shifts."""
    from scenes.latlong import lighting_pixels as ll_pixels
    from scenes.latlong import phong_exponents as ll_exps
    from scenes.latlong import rotations as ll_rotations
    from scenes.latlong import transport_pixels as ll_transport
    vertex_ids = np.arange(w.nverts) if vertex_ids is None else np.asarray(vertex_ids)
    li, lv = lighting_coefficients(ll_pixels(w.cfg, w.H), w.k_light)
    elev, shift = ll_rotations(w)
    exps = ll_exps(w)
    idx_parts, val_parts = [], []
    for s in range(0, len(vertex_ids), 64):
        vids = vertex_ids[s:s + 64]
        i, v = transport_rows(ll_transport(w, exps[vids], vids), w.nnz)
        idx_parts.append(i)
        val_parts.append(v)
    return dict(H=w.H, light_idx=li, light_val=lv, elev=elev[vertex_ids], shift=shift[vertex_ids],
                t_idx=np.concatenate(idx_parts), t_val=np.concatenate(val_parts))


def rotated_rows(case, frames=None):
    """The checker's rotated lighting coefficients at each stored row's
    indices: G[f, v, k] = (W S(R_fv) W^T L)[t_idx[v, k]] in FP64, so that
    the checker's radiance of any values x [V, nnz] on those rows is
    sum_k x[v, k] G[f, v, k] (the inner product of oracle.relight.relight,
    evaluated once per storage form without rotating again)."""
    from oracle.relight import frame_vertex_rotation, reconstruct_lighting
    from oracle.sphere import rotate_pixels
    n = case["n"]
    P = reconstruct_lighting(case["light_idx"], case["light_val"], n)
    nv = case["vert_rot"].shape[0]
    nf = 1 if case["frame_rot"] is None else case["frame_rot"].shape[0]
    frames = np.arange(nf) if frames is None else np.asarray(frames)
    G = np.zeros((len(frames), nv, case["t_idx"].shape[1]))
    for v in range(nv):
        for b, f in enumerate(frames):
            Rq = frame_vertex_rotation(case["vert_rot"], case["frame_rot"], v, f, n)
            G[b, v] = haar_forward(rotate_pixels(P, Rq)).ravel()[case["t_idx"][v]]
    return G


def decode_storage(form, codes, scale, nnz):
    """Host FP64 values of device storage codes [V, ...] of a form, by the
    definitions of include/rrt.h: bf16 (upper half of binary32), e4m3 (OCP
    E4M3FN code x block scale), s16 (int16 code x block scale), s11 (11-bit
    two's-complement code, packed little-endian in uint32 words, x block
    scale); blocks of 64 values."""
    import torch
    codes = codes.cpu()
    if form == "bf16":
        return codes.view(torch.bfloat16).double().numpy()
    if form == "e4m3":
        q = codes.view(torch.float8_e4m3fn).double().numpy()
    elif form == "s16":
        q = codes.numpy().astype(np.float64)
    elif form == "s11":
        words = codes.numpy().view(np.uint32).astype(np.uint64)
        e = np.arange(nnz)
        b = 11 * e
        lo = words[:, b >> 5]
        hi = np.where((b & 31) > 21, words[:, np.minimum((b >> 5) + 1, words.shape[1] - 1)], 0)
        bits = (((hi << np.uint64(32)) | lo) >> (b & 31).astype(np.uint64)) & np.uint64(0x7ff)
        q = bits.astype(np.int64)
        q = np.where(q >= 1024, q - 2048, q).astype(np.float64)
    else:
        raise ValueError(form)
    sc = np.repeat(scale.cpu().numpy().astype(np.float64), 64, axis=1)[:, :nnz]
    return q * sc


def _rows_and_reference_job(args):
    w, vids, li, lv, rot, frot, frames = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        idx, val = stored_transport(w, vids)
        case = dict(n=w.n, light_idx=li, light_val=lv, vert_rot=rot, frame_rot=frot, t_idx=idx,
                    t_val=val)
        ref, mag = reference(case, frames=frames, return_scale=True)
    return idx, val, ref, mag


def rows_and_reference(w, vids, li, lv, rot, frot, workers=8, frames=None):
    """stored_transport rows of the vertices `vids` and the checker's
    (radiance, magnitude scale) [F, len(vids)] for them (F: every frame, or
    the listed `frames`), over `workers` fresh processes (spawned: this
    process may hold a GPU context)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    vids = np.asarray(vids)
    chunks = [c for c in np.array_split(np.arange(len(vids)), 4 * workers) if len(c)]
    jobs = [(w, vids[c], li, lv, rot[c], frot, frames) for c in chunks]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_rows_and_reference_job, jobs))
    idx = np.concatenate([p[0] for p in parts])
    val = np.concatenate([p[1] for p in parts])
    ref = np.concatenate([p[2] for p in parts], axis=1)
    mag = np.concatenate([p[3] for p in parts], axis=1)
    return idx, val, ref, mag


def chain_reference(case):
    """The checker's chain-rule radiance [F, V] and its magnitude scale
    sum_k |T_k ghat_k| (FP64)."""
    from oracle.chain import chain_rotate
    from oracle.haar import haar_forward
    from oracle.relight import frame_vertex_rotation, reconstruct_lighting
    n = case["n"]
    P = reconstruct_lighting(case["light_idx"], case["light_val"], n)
    V = case["vert_rot"].shape[0]
    F = 1 if case["frame_rot"] is None else case["frame_rot"].shape[0]
    ref = np.zeros((F, V))
    scale = np.zeros((F, V))
    for v in range(V):
        idx = case["t_idx"][v].astype(np.int64)
        tv = case["t_val"][v].astype(np.float64)
        for f in range(F):
            Rq = frame_vertex_rotation(case["vert_rot"], case["frame_rot"], v, f, n)
            g = haar_forward(chain_rotate(P, Rq)).ravel()[idx]
            ref[f, v] = np.dot(tv, g)
            scale[f, v] = np.abs(tv * g).sum()
    return ref, scale
