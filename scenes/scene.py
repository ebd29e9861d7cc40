"""Seeded synthetic scenes: environment lighting, per-vertex frames, frame
rotations and pixel-domain transport (Phong lobe x binary visibility x texel
solid angle).

This module defines *inputs* only.  It contains no wavelet transform, no
coefficient selection and no rotation of a signal: those belong to the method
(and to the independent checker), not to the scene.

Cube-map convention used for texel directions (the paper parameterises the
sphere by a longitude-latitude map in its derivation, Sec. V.A, and notes that
the rotation applies to any explicit map; the workloads use six cube faces).
Faces 0..5 are +X, -X, +Y, -Y, +Z, -Z.  Texel (i, j) of an N x N face has
U = 2j+1-N and V = 2i+1-N; its (unnormalised) centre direction is
  +X ( N, -V, -U)   -X (-N, -V,  U)   +Y ( U,  N,  V)
  -Y ( U, -N, -V)   +Z ( U, -V,  N)   -Z (-U, -V, -N)
The local frame of a vertex has the surface normal on +Y (Sec. V, the BRDF is
expressed in a frame whose Y axis is the normal).
"""
from dataclasses import dataclass

import numpy as np

from .philox import philox4x32_np, philox4x32_torch

SEED = 1705072720
STREAM_LIGHT = 1
STREAM_ROT = 2
STREAM_FRAME = 3
STREAM_EXP = 4
STREAM_VIS = 5
STREAM_MESH = 6
STREAM_MATERIAL = 7

# Faces as signed axis permutations: direction = A_F @ (U, V, N).
FACE_AXES = np.array([
    [[0, 0, 1], [0, -1, 0], [-1, 0, 0]],    # +X: ( N, -V, -U)
    [[0, 0, -1], [0, -1, 0], [1, 0, 0]],    # -X: (-N, -V,  U)
    [[1, 0, 0], [0, 0, 1], [0, 1, 0]],      # +Y: ( U,  N,  V)
    [[1, 0, 0], [0, 0, -1], [0, -1, 0]],    # -Y: ( U, -N, -V)
    [[1, 0, 0], [0, -1, 0], [0, 0, 1]],     # +Z: ( U, -V,  N)
    [[-1, 0, 0], [0, -1, 0], [0, 0, -1]],   # -Z: (-U, -V, -N)
], dtype=np.int64)


def rng(cfg, stream, *extra):
    """numpy generator for (config, stream[, extra...])."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([SEED, int(cfg), int(stream), *[int(e) for e in extra]])))


# ----------------------------------------------------------------------------
# Workloads (synthetic stand-ins for the paper's scenes: its models, measured
# materials and light probes are not reproduced).
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    cfg: int
    name: str
    n: int                 # cube face side (power of two)
    k_light: int           # lighting coefficients kept (6 n^2 = no truncation)
    nverts: int
    nframes: int
    nnz: int               # transport coefficients per vertex (6 n^2 = dense)
    exp_lo: float
    exp_hi: float
    vertex_frames: str     # "normals" (normal + tangent) or "random"
    occlusion: float = 0.3


WORKLOADS = {
    1: Workload(1, "cube32_dense_v1000", 32, 6 * 32 * 32, 1000, 1, 6 * 32 * 32,
                1.0, 64.0, "normals"),
    2: Workload(2, "cube128_k1024_csr256_v50000", 128, 1024, 50000, 1, 256,
                1.0, 200.0, "random"),
    3: Workload(3, "cube128_k1024_csr256_v50000_f64", 128, 1024, 50000, 64, 256,
                1.0, 200.0, "random"),
    4: Workload(4, "cube256_k2048_mesh_v200000_mlp", 256, 2048, 200000, 1, 256,
                1.0, 200.0, "mesh"),
    5: Workload(5, "cube256_k2048_csr256_v1000000_f64", 256, 2048, 1000000, 64, 256,
                1.0, 500.0, "random"),
}


# ----------------------------------------------------------------------------
# Texel geometry (float64)
# ----------------------------------------------------------------------------
def texel_directions(n):
    """Unit centre directions, shape [6, n, n, 3] (float64)."""
    c = (2.0 * np.arange(n) + 1.0 - n) / n
    V, U = np.meshgrid(c, c, indexing="ij")          # V varies with row i
    uvn = np.stack([U, V, np.ones_like(U)], axis=-1)  # [n, n, 3]
    d = np.einsum("fab,ijb->fija", FACE_AXES.astype(np.float64), uvn)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def texel_solid_angles(n):
    """Exact solid angle of each texel of a face (same for every face), [n, n].

    The area of the gnomonic square [u0,u1]x[v0,v1] on the plane at distance
    1 is the signed sum of atan2(u v, sqrt(u^2 + v^2 + 1)) over its corners.
    """
    e = np.linspace(-1.0, 1.0, n + 1)

    def corner(u, v):
        return np.arctan2(u * v, np.sqrt(u * u + v * v + 1.0))

    v0, u0 = np.meshgrid(e[:-1], e[:-1], indexing="ij")
    v1, u1 = np.meshgrid(e[1:], e[1:], indexing="ij")
    return corner(u1, v1) - corner(u0, v1) - corner(u1, v0) + corner(u0, v0)


def direction_to_texel(d, n):
    """Texel (face, i, j) whose pyramid contains the direction d (float64)."""
    d = np.asarray(d, dtype=np.float64)
    a = int(np.argmax(np.abs(d)))
    face = 2 * a + (1 if d[a] < 0 else 0)
    # face coordinates (s along U, t along V) of the hit point on the face plane
    inv = np.linalg.inv(FACE_AXES[face].astype(np.float64))
    u, v, w = inv @ d
    s, t = u / w, v / w
    j = min(n - 1, int(np.floor((s + 1.0) * 0.5 * n)))
    i = min(n - 1, int(np.floor((t + 1.0) * 0.5 * n)))
    return face, max(i, 0), max(j, 0)


# ----------------------------------------------------------------------------
# Lighting
# ----------------------------------------------------------------------------
def lighting_pixels(cfg, n, n_point=4, intensity=1e3):
    """HDR environment [6, n, n] float32: iid log-normal(0, 1) texels plus
    n_point point lights of the given intensity added to the texels hit by
    seeded uniform directions."""
    g = rng(cfg, STREAM_LIGHT)
    L = g.lognormal(0.0, 1.0, size=(6, n, n))
    dirs = g.normal(size=(n_point, 3))
    for d in dirs:
        f, i, j = direction_to_texel(d / np.linalg.norm(d), n)
        L[f, i, j] += intensity
    return L.astype(np.float32)


# ----------------------------------------------------------------------------
# Rotations (local -> global, row-major 3x3, float32)
# ----------------------------------------------------------------------------
def quaternion_rotations(q):
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def random_rotations(cfg, count, stream=STREAM_ROT):
    """Uniform random rotations (normalised 4-Gaussian quaternions)."""
    q = rng(cfg, stream).normal(size=(count, 4))
    return quaternion_rotations(q).astype(np.float32)


def normal_frames(cfg, count):
    """Frames [t | n | t x n] (columns) from uniform normals and tangents."""
    g = rng(cfg, STREAM_ROT)
    nrm = g.normal(size=(count, 3))
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    a = g.normal(size=(count, 3))
    t = a - np.sum(a * nrm, axis=-1, keepdims=True) * nrm
    t /= np.linalg.norm(t, axis=-1, keepdims=True)
    b = np.cross(t, nrm)
    return np.stack([t, nrm, b], axis=-1).astype(np.float32)


def vertex_rotations(w: Workload):
    if w.vertex_frames == "normals":
        return normal_frames(w.cfg, w.nverts)
    return random_rotations(w.cfg, w.nverts, STREAM_ROT)


def frame_rotations(w: Workload):
    """Per-frame global object rotations, or None for a single unrotated frame."""
    if w.nframes == 1:
        return None
    return random_rotations(w.cfg, w.nframes, STREAM_FRAME)


def phong_exponents(w: Workload):
    return rng(w.cfg, STREAM_EXP).uniform(w.exp_lo, w.exp_hi, size=w.nverts)


# ----------------------------------------------------------------------------
# Transport: Phong lobe about the normal x visibility x solid angle
# ----------------------------------------------------------------------------
def occlusion_threshold(p):
    return int(round(p * 4294967296.0))


def visibility_np(cfg, vertex_ids, n, occlusion=0.3):
    """bool [B, 6, n, n]; a texel is occluded when its Philox draw falls below
    occlusion * 2^32.  Counter = (texel, vertex, visibility stream, 0),
    key = (seed, config)."""
    vid = np.asarray(vertex_ids, dtype=np.uint64).reshape(-1, 1)
    tex = np.arange(6 * n * n, dtype=np.uint64).reshape(1, -1)
    r0, _, _, _ = philox4x32_np(tex, vid, STREAM_VIS, 0, SEED, cfg)
    vis = r0 >= np.uint64(occlusion_threshold(occlusion))
    return vis.reshape(-1, 6, n, n)


def phong_lobe(n_exp, cos_y, omega):
    """Normalised Phong lobe about the local normal including the cosine
    factor and the texel solid angle: (n+2)/(2 pi) max(0, cos)^(n+1) Omega."""
    c = np.maximum(cos_y, 0.0)
    n_exp = np.asarray(n_exp, dtype=np.float64).reshape(-1, 1, 1, 1)
    return (n_exp + 2.0) / (2.0 * np.pi) * np.power(c[None], n_exp + 1.0) * omega[None, None]


def material_exponents(w: Workload, count):
    """Phong exponents of `count` materials, uniform in [exp_lo, exp_hi]."""
    return rng(w.cfg, STREAM_MATERIAL).uniform(w.exp_lo, w.exp_hi, size=count)


def material_ids(w: Workload, count):
    """Material of every vertex, uniform over `count` materials (int32 [V])."""
    return rng(w.cfg, STREAM_MATERIAL, 1).integers(0, count, size=w.nverts).astype(np.int32)


def brdf_pixels(w: Workload, count):
    """Texel-domain BRDF x cosine x solid angle of each material in the local
    frame, [count, 6, n, n] float64: the Phong lobe of transport_pixels
    without the visibility."""
    n = w.n
    return phong_lobe(material_exponents(w, count), texel_directions(n)[..., 1],
                      texel_solid_angles(n))


def transport_pixels(w: Workload, exps, vertex_ids):
    """Pixel-domain transport [B, 6, n, n] float64 for the given vertices."""
    n = w.n
    cos_y = texel_directions(n)[..., 1]
    omega = texel_solid_angles(n)
    lobe = phong_lobe(exps, cos_y, omega)
    vis = visibility_np(w.cfg, vertex_ids, n, w.occlusion)
    return lobe * vis


def transport_pixels_torch(w: Workload, exps, vertex_ids, device, dtype=None):
    """Same recipe as transport_pixels, evaluated with torch on `device`.
    exps / vertex_ids are 1-D sequences; returns [B, 6, n, n]."""
    import torch
    dtype = dtype or torch.float64
    n = w.n
    cos_y = torch.as_tensor(texel_directions(n)[..., 1], device=device)
    omega = torch.as_tensor(texel_solid_angles(n), device=device)
    e = torch.as_tensor(np.asarray(exps, dtype=np.float64), device=device).view(-1, 1, 1, 1)
    lobe = (e + 2.0) / (2.0 * np.pi) * torch.pow(cos_y.clamp_min(0.0)[None], e + 1.0) * omega[None, None]
    return (lobe * visibility_torch(w, vertex_ids, device)).to(dtype)


def visibility_torch(w: Workload, vertex_ids, device):
    """visibility_np(w.cfg, vertex_ids, w.n, w.occlusion) evaluated with torch
    on `device` (bool [B, 6, n, n])."""
    import torch
    n = w.n
    vid = torch.as_tensor(np.asarray(vertex_ids, dtype=np.int64), device=device).view(-1, 1)
    tex = torch.arange(6 * n * n, device=device, dtype=torch.int64).view(1, -1)
    zero = torch.zeros((), dtype=torch.int64, device=device)
    r0, _, _, _ = philox4x32_torch(tex, vid, zero + STREAM_VIS, zero, SEED, w.cfg)
    return (r0 >= occlusion_threshold(w.occlusion)).view(-1, 6, n, n)
