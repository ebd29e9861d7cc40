"""Learned transport decoder: host-side driver of the MLP kernels.

Not part of the paper.  Instead of storing each vertex's top-256 transport
coefficients, vertices are grouped into clusters that share one fixed
coefficient support (256 Mallat indices); a small network maps a vertex's
position and normal to its 256 coefficient values on its cluster's support.
Training (forward, backward, Adam) and inference run in librrt's kernels;
this module only drives them and holds the host-side bookkeeping:

* k-means clustering of the (position, normal) features (k-means++ seeding,
  Lloyd iterations, FP64, host);
* per-cluster supports: the 256 indices with the largest summed squared
  coefficient over a sample of the cluster's vertices;
* per (cluster, slot) output scales: the network predicts coefficient /
  scale, scale = RMS of the coefficient over the cluster's sample;
* the fallback rule: the decoder is used only when its held-out relit
  radiance is within the error budget of the stored per-vertex rows.
"""
import numpy as np
import torch

from . import (RRT_MLP_BIAS_COUNT, RRT_MLP_WEIGHT_COUNT, adam_step, mlp_backward, mlp_decode,
               mlp_encode, mlp_forward, mlp_pack, mlp_workspace, mse, relight_mlp)

LAYER_SHAPES = [(256, 128), (256, 256), (256, 256), (256, 256), (256, 256)]


def kmeans(features, k, iters=25, seed=0):
    """k-means++ seeding and Lloyd iterations (FP64).  Returns (centres, labels)."""
    X = np.asarray(features, np.float64)
    g = np.random.default_rng(seed)
    centres = [X[g.integers(len(X))]]
    d2 = np.sum((X - centres[0]) ** 2, axis=1)
    for _ in range(1, k):
        c = X[g.choice(len(X), p=d2 / d2.sum())]
        centres.append(c)
        d2 = np.minimum(d2, np.sum((X - c) ** 2, axis=1))
    C = np.stack(centres)
    labels = np.zeros(len(X), np.int64)
    for _ in range(iters):
        dist = (np.sum(X * X, 1)[:, None] - 2.0 * X @ C.T + np.sum(C * C, 1)[None])
        labels = np.argmin(dist, axis=1)
        for j in range(k):
            sel = labels == j
            if sel.any():
                C[j] = X[sel].mean(axis=0)
    return C, labels


def init_weights(seed):
    """He-normal weights (FP32 master, packed [out][in] per layer), zero biases."""
    g = np.random.default_rng(seed)
    ws = [g.normal(0.0, np.sqrt(2.0 / i), size=(o, i)).astype(np.float32) for (o, i) in LAYER_SHAPES]
    return np.concatenate([w.ravel() for w in ws]), np.zeros(RRT_MLP_BIAS_COUNT, np.float32)


class TransportDecoder:
    """Network parameters (FP32 master + BF16 copy), Adam state, supports and
    output scales, all resident on one device."""

    def __init__(self, supports, scales, device="cuda", seed=0):
        self.device = torch.device(device)
        w, b = init_weights(seed)
        self.master = torch.from_numpy(w).to(self.device)
        self.w_bf16 = self.master.to(torch.bfloat16)
        self._w_dec = None          # the decoder layout of w_bf16, made on first use
        self.bias = torch.from_numpy(b).to(self.device)
        self.mw = torch.zeros_like(self.master)
        self.vw = torch.zeros_like(self.master)
        self.mb = torch.zeros_like(self.bias)
        self.vb = torch.zeros_like(self.bias)
        self.step = 0
        self.supports = torch.as_tensor(supports).to(self.device, torch.int32).contiguous()
        self.scales = torch.as_tensor(scales).to(self.device, torch.float32).contiguous()
        assert self.master.numel() == RRT_MLP_WEIGHT_COUNT

    def train(self, inputs, targets, clusters, steps, batch=4096, lr=1e-3, lr_final=1e-5, seed=0,
              log_every=0):
        """Adam on mean squared error of target / scale.  inputs [V, 6]
        float32, targets [V, 256] float32 coefficient values on each vertex's
        cluster support, clusters [V] int.  Returns the loss history."""
        V = inputs.shape[0]
        x_all = mlp_encode(inputs.to(self.device).contiguous())
        norm = (targets.to(self.device) / self.scales[clusters.to(self.device).long()]).contiguous()
        g = torch.Generator(device="cpu").manual_seed(seed)
        ws = mlp_workspace(batch, self.device)
        out = torch.empty((batch, 256), dtype=torch.float32, device=self.device)
        losses = []
        self._w_dec = None
        for s in range(steps):
            sel = torch.randint(0, V, (batch,), generator=g).to(self.device)
            x = x_all[sel].contiguous()
            t = norm[sel].contiguous()
            mlp_forward(self.w_bf16, self.bias, x, workspace=ws, out=out)
            dout, loss = mse(out, t)
            dw, db = mlp_backward(self.w_bf16, x, dout, ws)
            self.step += 1
            rate = lr * (lr_final / lr) ** (s / max(1, steps - 1))
            adam_step(self.master, dw, self.mw, self.vw, self.step, rate, param_bf16=self.w_bf16)
            adam_step(self.bias, db, self.mb, self.vb, self.step, rate)
            if log_every and (s % log_every == 0 or s == steps - 1):
                losses.append((s, loss.item()))
        return losses

    def w_dec(self):
        """The BF16 weights in the decoder layout (rrt_mlp_pack), packed once
        after training."""
        if self._w_dec is None:
            self._w_dec = mlp_pack(self.w_bf16)
        return self._w_dec

    def decode(self, inputs, clusters):
        """Coefficient values [V, 256] float32 on each vertex's cluster support
        (rrt_mlp_decode: the network and the per-slot scales in one kernel;
        0 for a cluster outside [0, C))."""
        return mlp_decode(self.w_dec(), self.bias, self.scales,
                          inputs.to(self.device).contiguous(),
                          clusters.to(self.device, torch.int32).contiguous())

    def relight(self, n, light_idx, light_val, vert_rot, inputs, clusters, frame_rot=None,
                out=None, workspace=None):
        """Decode and relight in one library call (rrt_relight_mlp): radiance
        [F, V] with each vertex's values decoded on its cluster's support."""
        return relight_mlp(n, light_idx, light_val, vert_rot, self.w_dec(), self.bias,
                           self.supports, self.scales, inputs, clusters, frame_rot=frame_rot,
                           out=out, workspace=workspace)

    def parameter_bytes(self):
        """Device bytes of what inference needs: BF16 weights, FP32 biases,
        supports and scales."""
        return (self.w_bf16.numel() * 2 + self.bias.numel() * 4 + self.supports.numel() * 4
                + self.scales.numel() * 4)


def choose_form(decoder_error, budget=1e-3):
    """Fallback rule: the learned decoder replaces the stored rows only when
    its held-out relit error is within budget."""
    return "mlp" if decoder_error <= budget else "stored"


def cluster_supports(pixels_fn, labels, k, nnz=256, sample_per_cluster=256, batch=512, seed=0):
    """Per-cluster supports and output scales.

    pixels_fn(vertex_ids) -> [B, 6, n, n] float32 device tensor of
    pixel-domain transport.  For each cluster, a seeded sample of its
    vertices is transformed (rrt_haar_forward); the support is the nnz
    indices with the largest summed squared coefficient (rrt_topk, ascending
    indices); the scale of a slot is the RMS of its coefficient over the
    sample (1 where that is 0).  Returns (supports [k, nnz] int32,
    scales [k, nnz] float32) as device tensors."""
    from . import haar_forward, topk
    g = np.random.default_rng(seed)
    supports, scales = [], []
    for c in range(k):
        members = np.flatnonzero(labels == c)
        if len(members) == 0:
            members = np.array([0])
        pick = np.sort(g.choice(members, size=min(sample_per_cluster, len(members)), replace=False))
        acc = None
        coefs = []
        for s in range(0, len(pick), batch):
            coef = haar_forward(pixels_fn(pick[s:s + batch]).contiguous())
            coef = coef.view(coef.shape[0], -1)
            sq = (coef * coef).sum(dim=0)
            acc = sq if acc is None else acc + sq
            coefs.append(coef)
        idx, _ = topk(acc.view(1, -1).contiguous(), nnz)
        vals = torch.cat([cf[:, idx[0].long()] for cf in coefs])
        rms = torch.sqrt((vals * vals).mean(dim=0))
        supports.append(idx[0])
        scales.append(torch.where(rms > 0, rms, torch.ones_like(rms)))
    return torch.stack(supports), torch.stack(scales)


def targets_on_supports(pixels_fn, vertex_ids, labels, supports, batch=512):
    """Coefficient values [V, nnz] of the given vertices on their cluster's
    support (rrt_haar_forward, then a per-row gather)."""
    from . import haar_forward
    out = []
    lab = torch.as_tensor(np.asarray(labels)[vertex_ids]).to(supports.device).long()
    for s in range(0, len(vertex_ids), batch):
        coef = haar_forward(pixels_fn(vertex_ids[s:s + batch]).contiguous())
        coef = coef.view(coef.shape[0], -1)
        out.append(torch.gather(coef, 1, supports[lab[s:s + batch]].long()))
    return torch.cat(out)
