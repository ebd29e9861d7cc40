"""Seeded synthetic inputs on the longitude-latitude map: HDR lighting,
per-vertex rotations in elevation-plus-shift form and texel-domain transport.

Inputs only: no wavelet transform, no selection, no rotation of a signal.

Map convention (Sec. V.A): direction (sin t sin f, cos t, sin t cos f), t the
elevation from +Y, f the azimuth; H rows and W = 2H columns, texel (i, j)
spans t in [i, i+1) pi/H and f in [j, j+1) pi/H; stored as two H x H squares,
square s holding columns s H .. s H + H - 1.  A vertex's local frame has its
normal on +Y (the pole t = 0).
"""
from dataclasses import dataclass

import numpy as np

from .philox import philox4x32_np, philox4x32_torch
from .scene import SEED, STREAM_EXP, STREAM_LIGHT, STREAM_ROT, STREAM_VIS, occlusion_threshold, rng

STREAM_LATLONG = 11          # offset of this module's streams


@dataclass(frozen=True)
class LatLongWorkload:
    cfg: int
    name: str
    H: int                 # rows (power of two); the map is H x 2H
    k_light: int
    nverts: int
    nnz: int
    exp_lo: float
    exp_hi: float
    occlusion: float = 0.3


LATLONG_WORKLOADS = {
    6: LatLongWorkload(6, "latlong128_k1024_csr256_v50000", 128, 1024, 50000, 256, 1.0, 200.0),
    7: LatLongWorkload(7, "latlong256_k2048_csr256_v50000", 256, 2048, 50000, 256, 1.0, 200.0),
}


def centre_angles(H):
    """(elevation [H], azimuth [2H]) of the texel centres, float64."""
    return (np.arange(H) + 0.5) * np.pi / H, (np.arange(2 * H) + 0.5) * np.pi / H


def solid_angles(H):
    """Exact solid angle of the texels of row i, [H] float64."""
    e = np.cos(np.arange(H + 1) * np.pi / H)
    return (np.pi / H) * (e[:-1] - e[1:])


def lighting_pixels(cfg, H, n_point=4, intensity=1e3):
    """HDR environment [2, H, H] float32: iid log-normal(0, 1) texels plus
    n_point point lights added to the texels hit by seeded uniform directions."""
    g = rng(cfg, STREAM_LIGHT, STREAM_LATLONG)
    L = g.lognormal(0.0, 1.0, size=(H, 2 * H))
    for d in g.normal(size=(n_point, 3)):
        d = d / np.linalg.norm(d)
        i = min(H - 1, int(np.arccos(np.clip(d[1], -1.0, 1.0)) / (np.pi / H)))
        f = np.arctan2(d[0], d[2]) % (2.0 * np.pi)
        j = min(2 * H - 1, int(f / (np.pi / H)))
        L[i, j] += intensity
    return np.stack([L[:, :H], L[:, H:]]).astype(np.float32)


def rotations(w: LatLongWorkload):
    """Per-vertex (cos b, sin b) float32 [V, 2] of the elevation rotation
    (cos b uniform in [-1, 1], the polar angle of a uniformly random
    rotation) and the two azimuth shifts (s_a, s_c) int32 [V, 2], uniform in
    [0, 2H)."""
    g = rng(w.cfg, STREAM_ROT, STREAM_LATLONG)
    b = np.arccos(g.uniform(-1.0, 1.0, size=w.nverts))
    elev = np.stack([np.cos(b), np.sin(b)], axis=1).astype(np.float32)
    shift = g.integers(0, 2 * w.H, size=(w.nverts, 2)).astype(np.int32)
    return elev, shift


def phong_exponents(w: LatLongWorkload):
    return rng(w.cfg, STREAM_EXP, STREAM_LATLONG).uniform(w.exp_lo, w.exp_hi, size=w.nverts)


def visibility_np(w: LatLongWorkload, vertex_ids):
    """bool [B, 2, H, H]: a texel (flat index over the two squares) is
    occluded when its Philox draw falls below occlusion * 2^32."""
    H = w.H
    vid = np.asarray(vertex_ids, dtype=np.uint64).reshape(-1, 1)
    tex = np.arange(2 * H * H, dtype=np.uint64).reshape(1, -1)
    r0, _, _, _ = philox4x32_np(tex, vid, STREAM_VIS + STREAM_LATLONG, 0, SEED, w.cfg)
    return (r0 >= np.uint64(occlusion_threshold(w.occlusion))).reshape(-1, 2, H, H)


def _lobe(H, exps):
    t, _ = centre_angles(H)
    c = np.maximum(np.cos(t), 0.0)
    e = np.asarray(exps, np.float64).reshape(-1, 1)
    row = (e + 2.0) / (2.0 * np.pi) * np.power(c[None], e + 1.0) * solid_angles(H)[None]   # [B, H]
    return np.broadcast_to(row[:, None, :, None], (row.shape[0], 2, H, H))


def transport_pixels(w: LatLongWorkload, exps, vertex_ids):
    """Texel-domain transport [B, 2, H, H] float64: normalised Phong lobe
    about the normal with the cosine factor, times visibility, times the
    texel solid angle."""
    return _lobe(w.H, exps) * visibility_np(w, vertex_ids)


def transport_pixels_torch(w: LatLongWorkload, exps, vertex_ids, device, dtype=None):
    """Same recipe as transport_pixels, evaluated with torch on `device`."""
    import torch
    dtype = dtype or torch.float64
    H = w.H
    t, _ = centre_angles(H)
    cos_t = torch.as_tensor(np.cos(t), device=device)
    omega = torch.as_tensor(solid_angles(H), device=device)
    e = torch.as_tensor(np.asarray(exps, dtype=np.float64), device=device).view(-1, 1)
    row = (e + 2.0) / (2.0 * np.pi) * torch.pow(cos_t.clamp_min(0.0)[None], e + 1.0) * omega[None]
    lobe = row[:, None, :, None].expand(-1, 2, H, H)
    vid = torch.as_tensor(np.asarray(vertex_ids, dtype=np.int64), device=device).view(-1, 1)
    tex = torch.arange(2 * H * H, device=device, dtype=torch.int64).view(1, -1)
    zero = torch.zeros((), dtype=torch.int64, device=device)
    r0, _, _, _ = philox4x32_torch(tex, vid, zero + STREAM_VIS + STREAM_LATLONG, zero, SEED, w.cfg)
    vis = (r0 >= occlusion_threshold(w.occlusion)).view(-1, 2, H, H)
    return (lobe * vis).to(dtype)
