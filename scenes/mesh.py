"""Seeded displaced-sphere mesh and a learnable transport for the learned
decoder workload (6 x 256^2 cube map, 200,000 vertices).

Inputs only: no wavelet transform or rotation of a signal here.

Mesh: vertex directions u_i on a Fibonacci lattice (Y up), radius
rho(u) = 1 + sum_k a_k exp(kappa_k (u . c_k - 1)) with seeded bumps
(c_k uniform, a_k in [-0.15, 0.25], kappa_k in [4, 20]); position p = rho u;
normal n = normalise(rho u - grad_S rho) with the tangential gradient
grad_S rho = sum_k a_k kappa_k exp(.) (c_k - (u . c_k) u).
Frame: tangent t = normalise(e - (e . n) n) with e = +X (or +Z when n is
within 0.9 of +-X), F = [t | n | t x n] (local -> global).

Transport: T(q) = (m+2)/(2 pi) max(0, w_q . y)^(m+1) S(F w_q) Omega_q in
the vertex's local frame, with
  exponent  m(p) = 1 + 199 (0.5 + 0.5 sin(3 p_x + 2 p_y - p_z)),
  sky term  S(w) = sigmoid(10 (w . u - h)),  h = 0.1 - 1.5 (rho(u) - 1)
            (valleys see less sky, bumps more),
a smooth, deterministic function of (p, n): a network can learn it, unlike
iid visibility masks.
"""
import numpy as np

from .scene import FACE_AXES, rng, texel_directions, texel_solid_angles

STREAM_BUMPS = 11
N_BUMPS = 16


def _bumps(cfg):
    g = rng(cfg, STREAM_BUMPS)
    c = g.normal(size=(N_BUMPS, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    a = g.uniform(-0.15, 0.25, size=N_BUMPS)
    kap = g.uniform(4.0, 20.0, size=N_BUMPS)
    return c, a, kap


def fibonacci_directions(count):
    i = np.arange(count, dtype=np.float64)
    y = 1.0 - 2.0 * (i + 0.5) / count
    r = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    phi = i * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(phi), y, r * np.sin(phi)], axis=1)


def displaced_sphere(cfg, count):
    """(positions [V,3], normals [V,3], radial directions [V,3], rho [V]) FP64."""
    u = fibonacci_directions(count)
    c, a, kap = _bumps(cfg)
    dots = u @ c.T                                     # [V, K]
    e = np.exp(kap[None] * (dots - 1.0)) * a[None]     # [V, K]
    rho = 1.0 + e.sum(axis=1)
    grad = (e * kap[None]) @ c - ((e * kap[None]) * dots).sum(axis=1, keepdims=True) * u
    n = rho[:, None] * u - grad
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return rho[:, None] * u, n, u, rho


def tangent_frames(n):
    """[V, 3, 3] local -> global frames [t | n | t x n] (FP64)."""
    e = np.zeros_like(n)
    e[:, 0] = 1.0
    near = np.abs(n[:, 0]) > 0.9
    e[near] = np.array([0.0, 0.0, 1.0])
    t = e - np.sum(e * n, axis=1, keepdims=True) * n
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    b = np.cross(t, n)
    return np.stack([t, n, b], axis=-1)


def exponent_field(p):
    return 1.0 + 199.0 * (0.5 + 0.5 * np.sin(3.0 * p[:, 0] + 2.0 * p[:, 1] - p[:, 2]))


def sky_offset(rho):
    return 0.1 - 1.5 * (rho - 1.0)


def mesh_inputs(p, n):
    """Decoder inputs [V, 6] float32: position scaled to [-1, 1] (by 1.5) and
    the unit normal."""
    return np.concatenate([p / 1.5, n], axis=1).astype(np.float32)


def learned_transport_pixels(n_face, p, frames, u, rho):
    """Pixel-domain transport [B, 6, n, n] (FP64) of the given vertices."""
    w = texel_directions(n_face)                       # local directions [6,n,n,3]
    omega = texel_solid_angles(n_face)
    m = exponent_field(p)[:, None, None, None]
    cos_y = np.maximum(w[..., 1], 0.0)[None]
    lobe = (m + 2.0) / (2.0 * np.pi) * np.power(cos_y, m + 1.0) * omega[None, None]
    wg = np.einsum("bij,fxyj->bfxyi", frames, w)        # global directions
    h = sky_offset(rho)[:, None, None, None]
    sky = 1.0 / (1.0 + np.exp(-10.0 * (np.einsum("bfxyi,bi->bfxy", wg, u) - h)))
    return lobe * sky


def learned_transport_pixels_torch(n_face, p, frames, u, rho, device, dtype=None):
    """Same recipe evaluated with torch on `device` (inputs numpy FP64)."""
    import torch
    dtype = dtype or torch.float64
    t = lambda x: torch.as_tensor(np.asarray(x, np.float64), device=device)  # noqa: E731
    w = t(texel_directions(n_face))
    omega = t(texel_solid_angles(n_face))
    m = t(exponent_field(p)).view(-1, 1, 1, 1)
    cos_y = w[..., 1].clamp_min(0.0)[None]
    lobe = (m + 2.0) / (2.0 * np.pi) * torch.pow(cos_y, m + 1.0) * omega[None, None]
    F = t(frames)
    # sky argument: (F w) . u = w . (F^T u)
    Fu = torch.einsum("bij,bi->bj", F, t(u))           # [B, 3]
    arg = torch.einsum("fxyj,bj->bfxy", w, Fu) - t(sky_offset(rho)).view(-1, 1, 1, 1)
    sky = torch.sigmoid(10.0 * arg)
    return (lobe * sky).to(dtype)


__all__ = ["displaced_sphere", "tangent_frames", "mesh_inputs", "learned_transport_pixels",
           "learned_transport_pixels_torch", "fibonacci_directions", "FACE_AXES"]
