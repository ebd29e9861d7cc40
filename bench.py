#!/usr/bin/env python3
"""Relit vertices/s of the run-time Haar-domain relighting path on one MI355X.

One step = the whole path over one lighting and one vertex batch:
  a1 forward Haar of the environment map        (rrt_haar_forward)
  a2 top-K lighting selection                    (rrt_topk)
  a3 source reconstruction P = W^T L             (rrt_relight_prepare)
  a4-a6 per-vertex Haar-domain rotation + sparse
        wavelet dot product                      (rrt_relight_prepared)
Inputs (environment pixels, vertex frames, CSR transport rows) are synthetic,
seeded, generated and projected on the device before timing.

Prints ONE JSON line.  --gpus N > 1 exits: this path is measured on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations per second: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz =
# 78.6 T (the published 157.3 TFLOP/s FP32 vector rate with an FMA counted as
# two flops).  A wave64 instruction issues in 2 cycles at that rate; many
# instructions (three-operand, cube-map, conversion) take 4 and v_rcp_f32 8,
# so the rate an instruction mix reaches lies below this peak.
PEAK_ALU_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# Algorithmic operations per rotated texel: the gfx950 instructions the
# exact source map, the gather and the texel's share of the 2x2 levels need
# (one per VALU instruction or memory access): the direction from its
# neighbour's (3 binary32 adds, exact), face, in-face coordinates and major
# component (4 cube-map instructions), the reciprocal (1), the two
# coordinates (2 fmas), the face as an integer (1), the exactness test (two
# masks, their minimum, a compare: 4), the row-major flat index from the
# significand bits (2 shifts, 2 shift-adds), the gather (1) and the share of
# the 2x2 levels (4: twelve adds per four texels per level, x 4/3 over the
# levels).  The strip layout of the source map costs 2 more instructions per
# texel, counted as overhead.
OPS_PER_TEXEL = 24
# The same count for the chain-rule rotation of the finest level: per 2x2
# destination block the map at n/2 without the levels (19), its 16-byte
# gather (1), the source face's components (9), reciprocal and square (2),
# four Jacobian entries (16), two mixed second derivatives (14), the chain
# rule (9) and the level-1 outputs with their stores (8), spread over the
# block's four texels (19.5), plus the share of the levels above level 1.
CHAIN_OPS_PER_TEXEL = 20.5
# The triple product adds the read of the BRDF factor and the product.
TRIPLE_EXTRA_OPS = 2
# Longitude-latitude rule per texel: the centre's sines and cosines (4
# reads, 2 products), the elevation rotation (6), rho (4), column select,
# shifts, flat index, gather and the levels' share (16), plus per level of
# the two binary searches 7 (two reads, two compares, two adds, one product).
LATLONG_OPS_BASE = 30
LATLONG_OPS_PER_LEVEL = 7

KERNEL_SOURCES = ["paper_1705_07272_amd/csrc/relight.hip", "paper_1705_07272_amd/csrc/geometry.h"]


def kernel_fingerprint():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# CPU baseline and accuracy clause: the FP64 checker on the GPU's own stored
# inputs for a bounded vertex sample, timed on the host cores; its result is
# also the reference of the timed GPU output on that sample.
# ----------------------------------------------------------------------------
def _cpu_relight(job):
    """One chunk of the checker's work: (kind, args) with kind the method the
    device ran (the exact rotation, the chain rule, a coarse start, the
    triple product, the lat-long map) and args its oracle function's."""
    kind, args = job
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):     # one core per worker process
        if kind == "exact":
            from oracle.relight import relight
            return relight(*args)
        if kind == "chain":
            from oracle.chain import relight_chain
            return relight_chain(*args)
        if kind == "levels":
            from oracle.levels import relight_from_level
            return relight_from_level(*args)
        if kind == "triple":
            from oracle.triple import relight_triple
            return relight_triple(*args)
        if kind == "latlong":
            from oracle.latlong import relight_latlong
            return relight_latlong(*args)
        raise ValueError(kind)


def host_cores():
    """Cores of this job: the process's CPU affinity, at most the 16 cores a
    one-GPU job is given on the benchmark machines."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _cpu_warm(_):
    import oracle.relight  # noqa: F401  (imported before the timed region)
    from threadpoolctl import threadpool_limits  # noqa: F401
    return os.getpid()


def start_cpu_pool(workers):
    """Worker processes forked before any device work in this process, with
    the checker's modules already imported in each."""
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(workers)
    pool.map(_cpu_warm, range(4 * workers))
    return pool


class PerVertex:
    """An oracle argument with one row per sampled vertex (split with them)."""

    def __init__(self, rows):
        self.rows = rows


def cpu_baseline(pool, workers, inputs, got, label, kind="exact",
                 method="FP64 pixel rotate + Haar + dense dot"):
    """inputs: the `kind` oracle's arguments in order, host copies of the
    device's stored inputs bit for bit (the lighting's top-K and FP32
    values, the vertices' rotations and FP32 rows), those with one row per
    sampled vertex wrapped in PerVertex.  got [F, S]: the timed device
    radiance of the S sampled vertices.  Returns the baseline record, the
    max frame rel-L2 of got against the checker and the checker's radiance
    [F, S]."""
    import numpy as np

    from oracle.relight import rel_l2
    S = got.shape[1]
    chunks = [c for c in np.array_split(np.arange(S), workers * 4) if len(c)]
    jobs = [(kind, tuple(x.rows[c] if isinstance(x, PerVertex) else x for x in inputs))
            for c in chunks]
    t0 = time.perf_counter()
    ref = np.concatenate(pool.map(_cpu_relight, jobs), axis=1)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()          # one process on one core, the first chunk
    _cpu_relight(jobs[0])
    dt1 = time.perf_counter() - t1
    frames = ref.shape[0]
    err = max(rel_l2(got[f], ref[f]) for f in range(frames))
    base = {"value": round(S * frames / dt, 3), "unit": "relit vertices/s",
            "cores": workers, "kind": "oracle",
            "single_core_value": round(len(chunks[0]) * frames / dt1, 3),
            "sample": f"{S} seeded vertices x {frames} frame(s) of {label}, the device's stored "
                      f"lighting and rows (FP32), {method}, "
                      f"{workers} single-threaded processes, {dt:.1f} s wall"}
    return base, err, ref


def accuracy_sample(nverts, frames, budget):
    """Seeded vertex sample of about `budget` vertex-frames (at least 64
    vertices), sorted."""
    import numpy as np
    count = min(nverts, max(64, budget // frames))
    return np.sort(np.random.default_rng(12345).choice(nverts, size=count, replace=False))


# ----------------------------------------------------------------------------
# Device inputs
# ----------------------------------------------------------------------------
def device_inputs(w, form, batch=2048, materials=0):
    """Device-resident inputs of the workload.  With materials > 0 the rows
    are the vertices' visibility (triple product) and the materials' BRDF
    factors and the vertices' material ids are added."""
    import numpy as np
    import torch

    import paper_1705_07272_amd as rrt
    from scenes.scene import (brdf_pixels, frame_rotations, lighting_pixels, material_ids,
                              phong_exponents, transport_pixels_torch, vertex_rotations,
                              visibility_torch)
    dev = torch.device("cuda")
    pix = torch.from_numpy(lighting_pixels(w.cfg, w.n)).to(dev)
    rot = torch.from_numpy(np.ascontiguousarray(vertex_rotations(w))).to(dev)
    frot = frame_rotations(w)
    frot = None if frot is None else torch.from_numpy(frot).to(dev)
    exps = phong_exponents(w)
    idx = torch.empty((w.nverts, w.nnz), dtype=torch.int32, device=dev)
    val = torch.empty((w.nverts, w.nnz), dtype=torch.float32, device=dev)
    for s in range(0, w.nverts, batch):
        e = min(w.nverts, s + batch)
        if materials:
            T = visibility_torch(w, np.arange(s, e), dev).to(torch.float32)
        else:
            T = transport_pixels_torch(w, exps[s:e], np.arange(s, e), dev, dtype=torch.float32)
        i, v = rrt.project_rows(T.contiguous(), w.nnz)
        idx[s:e] = i
        val[s:e] = v
        del T
    scale = None
    val32 = val                        # the FP32 stored rows the forms are made from
    if form == "bf16":
        val = rrt.convert(val, "bf16")
    elif form in ("e4m3", "s16", "s11"):
        val, scale = rrt.convert(val, form)
    brdf = mat = None
    if materials:
        brdf = torch.from_numpy(brdf_pixels(w, materials).astype(np.float32)).to(dev)
        mat = torch.from_numpy(material_ids(w, materials)).to(dev)
    torch.cuda.synchronize()
    return dict(pix=pix, rot=rot, frot=frot, idx=idx, val=val, val32=val32, scale=scale,
                brdf=brdf, material=mat)


def run_latlong(args, pool=None, workers=0):
    """Longitude-latitude map (Sec. V.A): the timed step is the lighting's
    Haar transform and top-k, then rrt_relight_latlong (reconstruction,
    tables, relight of every vertex under its elevation rotation and
    azimuth shifts)."""
    import numpy as np
    import torch

    import paper_1705_07272_amd as rrt
    from scenes.latlong import (LATLONG_WORKLOADS, lighting_pixels, phong_exponents, rotations,
                                transport_pixels_torch)
    w = LATLONG_WORKLOADS[args.latlong]
    dev = torch.device("cuda")
    H, V = w.H, w.nverts
    pix = torch.from_numpy(lighting_pixels(w.cfg, H)).to(dev)
    elev, shift = rotations(w)
    elev, shift = torch.from_numpy(elev).to(dev), torch.from_numpy(shift).to(dev)
    exps = phong_exponents(w)
    idx = torch.empty((V, w.nnz), dtype=torch.int32, device=dev)
    val = torch.empty((V, w.nnz), dtype=torch.float32, device=dev)
    for s in range(0, V, 2048):
        e = min(V, s + 2048)
        T = transport_pixels_torch(w, exps[s:e], np.arange(s, e), dev, dtype=torch.float32)
        idx[s:e], val[s:e] = rrt.project_rows(T.contiguous(), w.nnz)
    out = torch.empty(V, dtype=torch.float32, device=dev)
    ws = torch.empty(2 * 2 * H * H * 4 + 7 * H * 4 + 1024, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print("inputs ready", file=sys.stderr, flush=True)

    def step(ev=None):
        coef = rrt.haar_forward(pix)
        li, lv = rrt.topk(coef.view(1, -1), w.k_light)
        if ev is not None:
            ev[0].record()
        rrt.relight_latlong(H, li[0], lv[0], elev, shift, idx, val, out=out, workspace=ws)
        if ev is not None:
            ev[1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for k in range(args.steps):
        step(evs[k])
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    ms_kernel = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    faces = torch.zeros((V, 3), dtype=torch.float32, device=dev)
    fid = idx.long() // (H * H)
    faces.scatter_(1, torch.where(idx >= 0, fid, torch.full_like(fid, 2)), 1.0)
    texels = int((faces[:, :2] > 0).sum().item()) * H * H
    ops = LATLONG_OPS_BASE + LATLONG_OPS_PER_LEVEL * int(np.log2(H))
    achieved = texels * ops / (ms_kernel * 1e-3) / 1e12
    hbm = V * w.nnz * 8 + V * 16 + V * 4
    base = accuracy = None
    if pool is not None:
        # the timed output on a vertex sample against the lat-long checker fed
        # the device's stored lighting and rows
        vids = accuracy_sample(V, 1, args.cpu_sample)
        sel = torch.from_numpy(vids).cuda().long()
        coef = rrt.haar_forward(pix)
        li, lv = rrt.topk(coef.view(1, -1), w.k_light)
        inputs = (li[0].cpu().numpy(), lv[0].cpu().numpy(), H,
                  PerVertex(elev[sel].cpu().numpy()), PerVertex(shift[sel].cpu().numpy()),
                  PerVertex(idx[sel].cpu().numpy()), PerVertex(val[sel].cpu().numpy()))
        got = out[sel].cpu().numpy()[None]
        base, err, _ = cpu_baseline(pool, workers, inputs, got, w.name, "latlong",
                                    "FP64 lat-long rotation (binary32 source rule) + Haar + "
                                    "dense dot")
        pool.close()
        pool.join()
        accuracy = {"rel_l2": float(f"{err:.4g}"), "bar": 1e-5, "meets_bar": bool(err <= 1e-5),
                    "vertices": int(len(vids)), "frames": 1,
                    "reference": "FP64 lat-long oracle on the device's stored lighting and "
                                 "FP32 rows, rel-L2 over the sampled vertices"}
        print(f"accuracy: rel-L2 {err:.3e} on {len(vids)} vertices; {base['sample']}",
              file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": "relit vertices/s at rel-L2<=1e-3 vs FP64 oracle: plain FP32 vs BF16+MLP",
        "value": round(V / (ms_step * 1e-3), 1), "unit": "relit vertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "map": f"latlong {H}x{2 * H}", "light_coeffs": w.k_light,
                   "vertices": V, "frames": 1, "transport_nnz": w.nnz, "form": "f32"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_ALU_TOPS, 2), "unit": "Tops/s",
                     "frac": round(achieved / PEAK_ALU_TOPS, 4), "traffic": None,
                     "kernel": "rrt_relight_latlong (reconstruction + tables + relight_kernel)",
                     "kernel_ms": round(ms_kernel, 4), "rotated_texels": texels,
                     "ops_per_texel": ops, "hbm_algorithmic_bytes": hbm,
                     "hbm_achieved_gbs": round(hbm / (ms_kernel * 1e-3) / 1e9, 1),
                     "hbm_peak_gbs": PEAK_HBM_GBS},
        "accuracy": accuracy,
        "cpu_baseline": base}), flush=True)


def run_learned(args, w):
    """Learned-decoder form on the displaced-sphere scene (6 x 256^2, top-2,048
    lighting; the 200,000-vertex training mesh, or with --workload 5 the same
    surface at 1,000,000 vertices x 64 frames).  Setup, untimed: k-means (64
    clusters), cluster supports, targets, device training.  Accuracy on a
    seeded sample of vertices the network never saw, each against the FP64
    checker fed the device's stored per-vertex rows (timed as the CPU
    baseline): the stored rows relit on the device, the exact coefficients
    on the cluster supports (the support floor: what a perfect network
    would reach) and the decoder.  Timed: the learned step (a1-a2 +
    rrt_relight_mlp, decode and relight in one call) and, on the same scene,
    the plain FP32 stored-rows step (a1-a2 + rrt_relight)."""
    import numpy as np
    import torch

    import paper_1705_07272_amd as rrt
    from oracle.relight import rel_l2
    from paper_1705_07272_amd import learned
    from scenes.mesh import (displaced_sphere, learned_transport_pixels_torch, mesh_inputs,
                             tangent_frames)
    from scenes.scene import WORKLOADS, frame_rotations, lighting_pixels
    wt = WORKLOADS[4]                  # the training mesh
    t0 = time.perf_counter()
    p, nrm, u, rho = displaced_sphere(wt.cfg, wt.nverts)
    frames = tangent_frames(nrm)
    feats = mesh_inputs(p, nrm)
    K = args.clusters
    centres, labels = learned.kmeans(feats, K, iters=25, seed=1)

    def pixels_of(P, FR, U, RHO):
        def pixels(ids):
            ids = np.asarray(ids)
            return learned_transport_pixels_torch(w.n, P[ids], FR[ids], U[ids], RHO[ids], "cuda",
                                                  dtype=torch.float32)
        return pixels

    pixels = pixels_of(p, frames, u, rho)
    supports, scales = learned.cluster_supports(pixels, labels, K, w.nnz, sample_per_cluster=256)
    perm = np.random.default_rng(7).permutation(wt.nverts)
    held, train = np.sort(perm[: wt.nverts // 10]), np.sort(perm[wt.nverts // 10:])
    targets = learned.targets_on_supports(pixels, train, labels, supports)
    dec = learned.TransportDecoder(supports, scales, seed=3)
    hist = dec.train(torch.from_numpy(feats)[train], targets,
                     torch.from_numpy(labels.astype(np.int32))[train], steps=args.mlp_steps,
                     batch=4096, lr=2e-3, log_every=max(1, args.mlp_steps // 10))
    del targets
    print(f"learned setup {time.perf_counter() - t0:.1f} s, loss {hist[0][1]:.3e} -> "
          f"{hist[-1][1]:.3e}", file=sys.stderr, flush=True)

    # the relit scene: the training mesh itself, or the same surface sampled
    # densely (its vertices take the nearest k-means centre's cluster)
    if w.nverts != wt.nverts:
        p, nrm, u, rho = displaced_sphere(wt.cfg, w.nverts)
        frames = tangent_frames(nrm)
        feats = mesh_inputs(p, nrm)
        X = feats.astype(np.float64)
        labels = np.concatenate([np.argmin((np.sum(X[s:s + 65536] ** 2, 1)[:, None]
                                            - 2.0 * X[s:s + 65536] @ centres.T
                                            + np.sum(centres ** 2, 1)[None]), axis=1)
                                 for s in range(0, w.nverts, 65536)])
        pixels = pixels_of(p, frames, u, rho)
        unseen = np.arange(w.nverts)
    else:
        unseen = held
    V = w.nverts
    label = (w.name if w.nverts == wt.nverts else
             f"cube{w.n}_k{w.k_light}_mesh_v{V}_f{w.nframes}_mlp")
    dev = torch.device("cuda")
    pix = torch.from_numpy(lighting_pixels(w.cfg, w.n)).to(dev)
    rot = torch.from_numpy(frames.astype(np.float32)).to(dev)
    frot = frame_rotations(w) if w.nframes > 1 else None
    frot_d = None if frot is None else torch.from_numpy(frot).to(dev)
    F = 1 if frot is None else frot.shape[0]
    feats_dev = torch.from_numpy(feats).to(dev)
    lab_dev = torch.from_numpy(labels.astype(np.int32)).to(dev)

    # stored per-vertex rows (the plain path's input), projected on the device
    idx = torch.empty((V, w.nnz), dtype=torch.int32, device=dev)
    val = torch.empty((V, w.nnz), dtype=torch.float32, device=dev)
    for s in range(0, V, 512):
        idx[s:s + 512], val[s:s + 512] = rrt.project_rows(pixels(np.arange(s, min(V, s + 512)))
                                                          .contiguous(), w.nnz)
        if s % 131072 == 0:
            print(f"stored rows {s}/{V}", file=sys.stderr, flush=True)
    print("stored rows ready", file=sys.stderr, flush=True)

    # accuracy on unseen vertices: stored rows, support floor, decoder
    coef = rrt.haar_forward(pix)
    li, lv = rrt.topk(coef.view(1, -1), w.k_light)
    prep = rrt.prepare_lighting(w.n, li[0], lv[0])
    vids = np.sort(np.random.default_rng(12345).choice(
        unseen, size=min(len(unseen), max(64, args.cpu_sample // F)), replace=False))
    sel = torch.from_numpy(vids).to(dev).long()
    lab_s = lab_dev[sel].contiguous()
    ideal = learned.targets_on_supports(pixels, vids, labels, dec.supports)
    vals = dec.decode(feats_dev[sel].contiguous(), lab_s)
    kw = dict(frame_rot=frot_d)
    r_rows = rrt.relight_prepared(prep, rot[sel].contiguous(), idx[sel].contiguous(),
                                  val[sel].contiguous(), **kw).cpu().numpy()
    r_ideal = rrt.relight_prepared(prep, rot[sel].contiguous(), dec.supports, ideal.contiguous(),
                                   cluster=lab_s, **kw).cpu().numpy()
    r_dec = rrt.relight_prepared(prep, rot[sel].contiguous(), dec.supports, vals,
                                 cluster=lab_s, **kw).cpu().numpy()
    base = None
    errs = {}
    if not args.no_cpu_baseline:
        workers = host_cores()
        pool = start_cpu_pool(workers)
        inputs = (li[0].cpu().numpy(), lv[0].cpu().numpy(), w.n,
                  PerVertex(rot[sel].cpu().numpy()), frot, PerVertex(idx[sel].cpu().numpy()),
                  PerVertex(val[sel].cpu().numpy()))
        base, errs["stored_rows"], ref = cpu_baseline(pool, workers, inputs, r_rows, label)
        pool.close()
        pool.join()
    else:
        ref = r_rows.astype(np.float64)   # (no checker run: the device's stored-rows result)
    fe = lambda x: max(rel_l2(x[f], ref[f]) for f in range(F))  # noqa: E731
    errs["support_floor"] = fe(r_ideal)
    errs["decoder"] = fe(r_dec)
    errs["decoder_vs_floor"] = max(rel_l2(r_dec[f], r_ideal[f]) for f in range(F))
    form = learned.choose_form(errs["decoder"])
    print("learned accuracy " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()),
          file=sys.stderr, flush=True)

    out = torch.empty((F, V), dtype=torch.float32, device=dev)
    fused_ws = torch.empty(rrt.relight_mlp_workspace_bytes(w.n, li[0], lv[0], V),
                           dtype=torch.uint8, device=dev)
    ws = torch.empty(2 * 6 * w.n * w.n * 4 + 512, dtype=torch.uint8, device=dev)
    order = rrt.relight_order(w.n, idx)

    def timed(step, nev):
        for _ in range(args.warmup):
            step(None)
        torch.cuda.synchronize()
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(nev))
               for _ in range(args.steps)]
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(args.steps):
            step(evs[k])
        b.record()
        torch.cuda.synchronize()
        spans = [sum(e[i].elapsed_time(e[i + 1]) for e in evs) / args.steps
                 for i in range(nev - 1)]
        return a.elapsed_time(b) / args.steps, spans

    def learned_step(ev):
        # a1 + a2, then one library call: reconstruction, decode, relight
        coef = rrt.haar_forward(pix)
        li, lv = rrt.topk(coef.view(1, -1), w.k_light)
        if ev is not None:
            ev[0].record()
        dec.relight(w.n, li[0], lv[0], rot, feats_dev, lab_dev, frame_rot=frot_d, out=out,
                    workspace=fused_ws)
        if ev is not None:
            ev[1].record()

    def stored_step(ev):
        coef = rrt.haar_forward(pix)
        li, lv = rrt.topk(coef.view(1, -1), w.k_light)
        prep = rrt.prepare_lighting(w.n, li[0], lv[0], workspace=ws)
        if ev is not None:
            ev[0].record()
        rrt.relight_prepared(prep, rot, idx, val, frame_rot=frot_d, out=out, order=order)
        if ev is not None:
            ev[1].record()

    def parts_step(ev):
        # the learned call's two halves as separate calls: decode, relight
        coef = rrt.haar_forward(pix)
        li, lv = rrt.topk(coef.view(1, -1), w.k_light)
        prep = rrt.prepare_lighting(w.n, li[0], lv[0], workspace=ws)
        chunk = min(V, 200000)
        if ev is not None:
            ev[0].record()
        vals = dec.decode(feats_dev[:chunk], lab_dev[:chunk])
        if ev is not None:
            ev[1].record()
        rrt.relight_prepared(prep, rot[:chunk], dec.supports, vals, cluster=lab_dev[:chunk],
                             frame_rot=frot_d)
        if ev is not None:
            ev[2].record()

    ms, (ms_mlp_call,) = timed(learned_step, 2)
    ms_stored, (ms_stored_relight,) = timed(stored_step, 2)
    _, (ms_dec, ms_rel) = timed(parts_step, 3)
    chunk = min(V, 200000)
    flops = 2.0 * chunk * sum(o * i for (o, i) in learned.LAYER_SHAPES)
    # algorithmic relight work of the decode/relight split: texels of the
    # faces each vertex's cluster support touches
    sup_faces = torch.zeros((dec.supports.shape[0], 6), device=dev)
    sup_faces.scatter_(1, (dec.supports.long() // (w.n * w.n)).clamp(0, 5), 1.0)
    texels = int(sup_faces.sum(1)[lab_dev[:chunk].long()].sum().item()) * w.n * w.n * F
    achieved = texels * OPS_PER_TEXEL / (ms_rel * 1e-3) / 1e12
    dec_tflops = flops / (ms_dec * 1e-3) / 1e12
    row_faces = torch.zeros((V, 7), device=dev)
    row_faces.scatter_(1, torch.where(idx >= 0, idx.long() // (w.n * w.n),
                                      torch.full_like(idx.long(), 6)), 1.0)
    stored_texels = int((row_faces[:, :6] > 0).sum().item()) * w.n * w.n * F
    sup_texels_all = int(sup_faces.sum(1)[lab_dev.long()].sum().item()) * w.n * w.n * F
    print(json.dumps({
        "metric": "relit vertices/s at rel-L2<=1e-3 vs FP64 oracle: plain FP32 vs BF16+MLP",
        "value": round(V * F / (ms * 1e-3), 1), "unit": "relit vertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 decoder weights/activations, f32 accumulate, f32 relight",
        "data": "synthetic",
        "config": {"workload": label,
                   "cube_face": w.n, "light_coeffs": w.k_light, "vertices": V, "frames": F,
                   "clusters": K, "form": "mlp", "train_steps": args.mlp_steps,
                   "trained_on": wt.name},
        "accuracy": {"rel_l2": float(f"{errs['decoder']:.4g}"), "bar": 1e-3,
                     "meets_bar": bool(errs["decoder"] <= 1e-3),
                     "vertices": int(len(vids)), "frames": F,
                     "reference": "FP64 oracle on the device's stored per-vertex rows, max "
                                  "over frames of the rel-L2 over vertices the network never saw",
                     **{k: float(f"{v:.4g}") for k, v in errs.items()},
                     "form_selected": form},
        "stored_rows_fp32": {"value": round(V * F / (ms_stored * 1e-3), 1),
                             "ms_per_step": round(ms_stored, 4),
                             "relight_ms": round(ms_stored_relight, 4),
                             "rotated_texels": stored_texels,
                             "bytes": V * w.nnz * 8},
        "learned": {"decoder_bytes": dec.parameter_bytes(),
                    "relight_mlp_ms": round(ms_mlp_call, 4),
                    "rotated_texels": sup_texels_all,
                    "split_vertices": chunk, "decode_ms": round(ms_dec, 4),
                    "relight_ms": round(ms_rel, 4),
                    "workspace_bytes": fused_ws.numel()},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_ALU_TOPS, 2), "unit": "Tops/s",
                     "frac": round(achieved / PEAK_ALU_TOPS, 4), "traffic": None,
                     "kernel": "relight_kernel (cluster supports)",
                     "kernel_ms": round(ms_rel, 4), "rotated_texels": texels,
                     "ops_per_texel": OPS_PER_TEXEL},
        "roofline_decode": {"bound": "mfma", "achieved": round(dec_tflops, 2),
                            "peak": 2500.0, "unit": "TFLOP/s",
                            "frac": round(dec_tflops / 2500.0, 4),
                            "kernel": "decode_kernel (encoding, 5 BF16 MFMA layers, scaling)",
                            "kernel_ms": round(ms_dec, 4), "flops": flops},
        "cpu_baseline": base,
    }), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, help="scene configuration (2 = 6x128^2, "
                    "top-1024 lighting, 50,000 vertices, CSR-256 FP32, 1 frame)")
    ap.add_argument("--form", choices=["f32", "bf16", "s16", "s11", "e4m3", "mlp"], default="f32",
                    help="transport storage; the reduced forms also store the lighting in "
                         "binary16 and accumulate with compensation")
    ap.add_argument("--start-level", type=int, default=0,
                    help="rotate from this many levels below the finest one (Sec. V.C remark; "
                         "an approximation of the exact method, 0 = exact)")
    ap.add_argument("--nnz", type=int, default=0,
                    help="transport coefficients kept per vertex (budget sweep; 0 = the "
                         "workload's own)")
    ap.add_argument("--latlong", type=int, default=0, metavar="CFG",
                    help="longitude-latitude map workload (6: 128x256, 7: 256x512), "
                         "Sec. V.A elevation rotation plus azimuth shifts")
    ap.add_argument("--triple", type=int, default=0, metavar="M",
                    help="triple product with M materials: BRDF factors per material, the "
                         "rows hold each vertex's visibility (Sec. III)")
    ap.add_argument("--chain-rule", action="store_true",
                    help="rotate the finest level by the chain rule (Sec. V.A-V.B; an "
                         "approximation of the exact method)")
    ap.add_argument("--serial", action="store_true",
                    help="one stream: each step's lighting preparation before its relight "
                         "(default: the next lighting is prepared on a second stream)")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--mlp-steps", type=int, default=12000)
    ap.add_argument("--clusters", type=int, default=64,
                    help="learned form: k-means clusters of the mesh vertices (one shared "
                         "coefficient support each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter scale)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the path needs no collective; vertices shard trivially)", file=sys.stderr)
        sys.exit(2)

    import dataclasses

    from scenes.scene import WORKLOADS
    w = WORKLOADS[args.workload]
    if args.nnz:
        w = dataclasses.replace(w, nnz=args.nnz)

    # The checker of the method the device runs (the exact rotation, the
    # chain rule, a coarse start, the triple product, the lat-long map);
    # its worker processes start before any device work.
    pool = workers = None
    if not args.no_cpu_baseline and not args.copy_calibration and args.form != "mlp":
        workers = host_cores()
        pool = start_cpu_pool(workers)

    import torch

    import paper_1705_07272_amd as rrt

    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 5}))
        return

    if args.form == "mlp":
        run_learned(args, WORKLOADS[5] if args.workload == 5 else WORKLOADS[4])
        return
    if args.latlong:
        run_latlong(args, pool, workers)
        return

    inp = device_inputs(w, args.form, materials=args.triple)
    print("inputs ready", file=sys.stderr, flush=True)
    n, K, V = w.n, w.k_light, w.nverts
    L = args.start_level
    n_rot = n >> L                     # resolution the rotation runs at
    idx_full = inp["idx"]
    if L:
        # stored transport rows re-indexed once (a storage transformation)
        inp["idx"] = rrt.coarsen_indices(inp["idx"], n, L)
    F = 1 if inp["frot"] is None else inp["frot"].shape[0]
    out = torch.empty((F, V), dtype=torch.float32, device="cuda")
    light_f16 = args.form != "f32"
    # Pipelined steps: the next lighting's a1-a3 run on a second stream while
    # the vertices are relit under the current one (two workspace slots; each
    # step still does all of its work).  --serial runs one stream.
    slots = 1 if args.serial else 2
    main = torch.cuda.current_stream()
    side = main if args.serial else torch.cuda.Stream()
    wss = [torch.empty(2 * 6 * n * n * 4 + 512, dtype=torch.uint8, device="cuda")
           for _ in range(slots)]
    coefs = [torch.empty_like(inp["pix"]) for _ in range(slots)]
    tk_ws = [torch.empty(max(rrt.topk_workspace_bytes(1, 6 * n * n, K), 1), dtype=torch.uint8,
                         device="cuda") for _ in range(slots)]
    lis = [torch.empty((1, K), dtype=torch.int32, device="cuda") for _ in range(slots)]
    lvs = [torch.empty((1, K), dtype=torch.float32, device="cuda") for _ in range(slots)]
    keep = [None] * slots          # what the relight of a slot reads, alive until reuse
    # heavy-first processing order, recomputed from the rows in every step
    orders = [torch.empty(V, dtype=torch.int32, device="cuda") for _ in range(slots)]
    ord_ws = [torch.empty(rrt.relight_order_workspace_bytes(V), dtype=torch.uint8, device="cuda")
              for _ in range(slots)]
    prep_done = [torch.cuda.Event() for _ in range(slots)]
    rel_done = [torch.cuda.Event() for _ in range(slots)]
    counter = [0]

    def step(ev=None):
        slot = counter[0] % slots
        counter[0] += 1
        with torch.cuda.stream(side):
            side.wait_event(rel_done[slot])          # the relight that last read this slot
            if ev is not None:
                ev[2].record(side)
            coef = rrt.haar_forward(inp["pix"], out=coefs[slot])                   # a1
            li, lv = rrt.topk(coef.view(1, -1), K, out=(lis[slot], lvs[slot]),     # a2
                              workspace=tk_ws[slot])
            lv = rrt.convert(lv, "f16") if light_f16 else lv
            if L:
                li = rrt.coarsen_indices(li, n, L)
            prep = rrt.prepare_lighting(n_rot, li[0], lv[0], workspace=wss[slot],  # a3
                                        chain_rule=args.chain_rule)
            order = rrt.relight_order(n_rot, inp["idx"], out=orders[slot],
                                      workspace=ord_ws[slot])
            keep[slot] = prep
            if ev is not None:
                ev[3].record(side)
            prep_done[slot].record(side)
        main.wait_event(prep_done[slot])
        if ev is not None:
            ev[0].record(main)
        rrt.relight_prepared(prep, inp["rot"], inp["idx"], inp["val"], frame_rot=inp["frot"],
                             block_scale=inp["scale"], compensated=light_f16, out=out,
                             brdf=inp["brdf"], material=inp["material"], order=order)
        if ev is not None:
            ev[1].record(main)
        rel_done[slot].record(main)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(4)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for k in range(args.steps):
        step(evs[k])
    t_end.record()
    torch.cuda.synchronize()
    ms_step = t_start.elapsed_time(t_end) / args.steps
    ms_kernel = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    ms_prep = sum(e[2].elapsed_time(e[3]) for e in evs) / args.steps   # a1-a3 per lighting

    # Accuracy clause of the metric: the timed output of the last step on a
    # seeded vertex sample against the FP64 checker fed the device's own
    # stored lighting (its top-K, FP32) and rows (FP32, before any storage
    # form), bit for bit; the same run times the checker on the host cores.
    base = accuracy = None
    if pool is not None:
        import numpy as np
        # the literal tripling-coefficient sum costs about 6x the double product
        vids = accuracy_sample(V, F, args.cpu_sample // (4 if args.triple else 1))
        sel = torch.from_numpy(vids).cuda().long()
        last = (counter[0] - 1) % slots
        inputs = [lis[last][0].cpu().numpy(), lvs[last][0].cpu().numpy(), n,
                  PerVertex(inp["rot"][sel].cpu().numpy()),
                  None if inp["frot"] is None else inp["frot"].cpu().numpy(),
                  PerVertex(idx_full[sel].cpu().numpy()),
                  PerVertex(inp["val32"][sel].cpu().numpy())]
        kind, method = "exact", "FP64 pixel rotate + Haar + dense dot"
        if args.chain_rule:
            kind, method = "chain", "FP64 chain-rule rotation + Haar + dense dot"
        elif L:
            kind, method = "levels", f"FP64 rotation started {L} levels coarser + dense dot"
            inputs.append(L)
        elif args.triple:
            kind, method = "triple", "FP64 rotate + literal tripling-coefficient sum"
            inputs += [inp["brdf"].cpu().numpy().astype(np.float64),
                       PerVertex(inp["material"][sel].cpu().numpy())]
        got = out[:, sel].cpu().numpy()
        base, err, _ = cpu_baseline(pool, workers, inputs, got, w.name, kind, method)
        pool.close()
        pool.join()
        bar = 1e-5 if args.form == "f32" else 1e-3
        accuracy = {"rel_l2": float(f"{err:.4g}"), "bar": bar, "meets_bar": bool(err <= bar),
                    "vertices": int(len(vids)), "frames": F,
                    "reference": f"{method} on the device's stored lighting and FP32 rows, max "
                                 "over frames of the rel-L2 over the sampled vertices"}
        print(f"accuracy: rel-L2 {err:.3e} on {len(vids)} vertices x {F} frames "
              f"(bar {bar:g}); {base['sample']}", file=sys.stderr, flush=True)

    # algorithmic work of one relight launch
    faces = torch.zeros((V, 7), dtype=torch.float32, device="cuda")
    fid = inp["idx"].long() // (n_rot * n_rot)
    faces.scatter_(1, torch.where(inp["idx"] >= 0, fid, torch.full_like(fid, 6)), 1.0)
    face_count = int((faces[:, :6] > 0).sum().item())
    texels = face_count * n_rot * n_rot * F
    # stored rows: indices, values (packed words for s11), block scales
    hbm_bytes = (V * w.nnz * 4 + inp["val"].numel() * inp["val"].element_size() + V * 36 + F * V * 4
                 + (0 if inp["scale"] is None else inp["scale"].numel() * 4)
                 + (0 if inp["frot"] is None else F * 36)
                 + (0 if inp["brdf"] is None else inp["brdf"].numel() * 4 + V * 4))
    ops_texel = (CHAIN_OPS_PER_TEXEL if args.chain_rule
                 else OPS_PER_TEXEL + (TRIPLE_EXTRA_OPS if args.triple else 0))
    achieved = texels * ops_texel / (ms_kernel * 1e-3) / 1e12

    traffic = valu_util = None
    prof = os.path.join(ROOT, "profiles", f"relight_{w.name}_{args.form}_hbm.txt")
    if os.path.exists(prof):
        with open(prof) as fh:
            rec = json.load(fh)
        # counters were taken on the workload as configured, exact method
        if (rec.get("kernel_fingerprint") == kernel_fingerprint() and not args.chain_rule
                and not args.nnz and not L and not args.triple):
            traffic = rec.get("hbm_bytes_per_launch")
            valu_util = rec.get("valu_issue_util")

    line = {
        "metric": "relit vertices/s at rel-L2<=1e-3 vs FP64 oracle: plain FP32 vs BF16+MLP",
        "value": round(V * F / (ms_step * 1e-3), 1),
        "unit": "relit vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        # a1-a3 per lighting: alone on the GPU (serial), or the span of the
        # preparation while it shares the GPU with the previous relight
        ("lighting_prep_ms" if args.serial else "lighting_prep_overlapped_span_ms"):
            round(ms_prep, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 transport, f16 lighting, f32 accumulate",
                  "s16": "s16 block-scaled transport, f16 lighting, f32 accumulate",
                  "s11": "packed 11-bit block-scaled transport, f16 lighting, f32 accumulate",
                  "e4m3": "e4m3 transport, f16 lighting, f32 accumulate"}[args.form],
        "data": "synthetic",
        "config": {"workload": w.name, "cube_face": n, "light_coeffs": K, "vertices": V,
                   "frames": F, "transport_nnz": w.nnz, "form": args.form,
                   "lighting_prep": "serial" if args.serial else "overlapped (second stream)"},
        **({"start_level": {"levels": L, "rotated_face": n_rot,
                            "note": "approximation; its error against the exact FP64 oracle "
                                    "is measured by tests/test_oracle_levels.py"}} if L else {}),
        **({"triple_product": {"materials": args.triple,
                               "note": "BRDF x cosine per material, visibility rows per "
                                       "vertex; the tripling-coefficient sum evaluated as a "
                                       "texel product before the transform"}}
           if args.triple else {}),
        **({"chain_rule": {"note": "finest level rotated by the chain rule; an approximation "
                                   "whose error against the exact FP64 oracle is measured by "
                                   "tests/test_oracle_chain.py"}} if args.chain_rule else {}),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TOPS, 2),
                     "unit": "Tops/s", "frac": round(achieved / PEAK_ALU_TOPS, 4),
                     "traffic": traffic, "valu_issue_util": valu_util,
                     "kernel": "relight_kernel",
                     "kernel_ms": round(ms_kernel, 4), "rotated_texels": texels,
                     "ops_per_texel": ops_texel,
                     "hbm_algorithmic_bytes": hbm_bytes,
                     "hbm_achieved_gbs": round(hbm_bytes / (ms_kernel * 1e-3) / 1e9, 1),
                     "hbm_peak_gbs": PEAK_HBM_GBS},
        "accuracy": accuracy,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)
    # the metric holds at its accuracy bar only: the plain path at 1e-5, the
    # 16- and 11-bit fixed-point forms at 1e-3 (BF16 and E4M3 cannot meet
    # 1e-3 on this workload, whatever the arithmetic: their line says so)
    if accuracy is not None and not accuracy["meets_bar"] and args.form in ("f32", "s16", "s11"):
        sys.exit(1)


if __name__ == "__main__":
    main()
