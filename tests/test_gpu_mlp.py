"""GPU parity of the learned decoder's kernels against the FP64 checker
(oracle/mlp.py) on the same bfloat16 weights and inputs.

Tolerances: the device keeps activations in bfloat16 between layers (each
store rounds by up to 2^-9) and accumulates in FP32, so outputs and
gradients are compared by relative L2 error: forward <= 2e-2, gradients
<= 3e-2 per tensor; the encoding within 2 bfloat16 ulps plus 1e-4 (binary32
argument rounding of the highest band); MSE and Adam (pure FP32
elementwise) within 1e-5 relative.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_07272_amd as m
    return m


def _bf16(x):
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16)


def _net(seed=0, bias_scale=0.1):
    Ws, bs = ref.init_params(seed)
    rng = np.random.default_rng(seed + 7)
    bs = [rng.normal(0, bias_scale, size=b.shape) for b in bs]
    Wq = [_bf16(W).float().numpy().astype(np.float64) for W in Ws]     # what the device sees
    bq = [np.asarray(b, np.float32).astype(np.float64) for b in bs]
    w_dev = torch.cat([_bf16(W).reshape(-1) for W in Ws]).cuda()
    b_dev = torch.from_numpy(np.concatenate([np.asarray(b, np.float32) for b in bs])).cuda()
    return Wq, bq, w_dev, b_dev


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_encode(rrt):
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, size=(1000, 6)).astype(np.float32)
    got = rrt.mlp_encode(torch.from_numpy(x).cuda()).float().cpu().numpy()
    want = ref.encode(x.astype(np.float64))
    # bfloat16 storage (half ulp 2^-8 relative) plus the binary32 rounding of
    # the argument 2^7 pi x of the highest band (about 2^7 pi 2^-24 absolute)
    ulp = np.maximum(np.abs(want), 2.0 ** -126) * 2.0 ** -7
    assert np.all(np.abs(got - want) <= 2 * ulp + 1e-4)
    assert np.all(got[:, 102:] == 0)


def test_pack_layout(rrt):
    """rrt_mlp_pack reorders the row-major weights into the documented
    decoder layout, value for value: layer by layer at the same offsets, the
    operand of rows 32 t.. and inputs 16 s.. at (t K / 16 + s) 512, lane
    m + 32 h holding w[32 t + m][16 s + 8 h + e] at 8 (m + 32 h) + e."""
    rng = np.random.default_rng(11)
    bits = rng.integers(0, 1 << 16, rrt.RRT_MLP_WEIGHT_COUNT, dtype=np.uint16)
    w = torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)
    got = rrt.mlp_pack(w).view(torch.int16).cpu().numpy().view(np.uint16)
    want = np.empty_like(bits)
    base = 0
    for K in (128, 256, 256, 256, 256):
        W = bits[base:base + 256 * K].reshape(256, K)
        S = K // 16
        # [t, s, h, m, e] <- W[32 t + m, 16 s + 8 h + e]
        frag = W.reshape(8, 32, S, 2, 8).transpose(0, 2, 3, 1, 4)
        want[base:base + 256 * K] = frag.ravel()
        base += 256 * K
    assert base == rrt.RRT_MLP_WEIGHT_COUNT
    assert np.array_equal(got, want)


@pytest.mark.parametrize("B", [1, 64, 1000, 20000])
def test_decode_kernel_equals_layered_forward(rrt, B):
    """rrt_mlp_decode (encoding, five layers and per-slot scales in one
    kernel, 64-row tiles) equals rrt_mlp_encode + rrt_mlp_forward + the
    binary32 scaling bit for bit, ragged tiles and clusters outside [0, C)
    (value 0) included; and the FP64 network on the same weights within the
    forward tolerance."""
    rng = np.random.default_rng(B)
    Wq, bq, w_dev, b_dev = _net(seed=3)
    x = np.concatenate([rng.uniform(-1, 1, size=(B, 3)),
                        rng.normal(size=(B, 3))], axis=1).astype(np.float32)
    C = 5
    cluster = rng.integers(0, C, B).astype(np.int32)
    cluster[5::97] = -1
    cluster[7::89] = C
    scales = rng.uniform(0.5, 2.0, size=(C, 256)).astype(np.float32)
    xd, cd, sd = (torch.from_numpy(a).cuda() for a in (x, cluster, scales))
    got = rrt.mlp_decode(rrt.mlp_pack(w_dev), b_dev, sd, xd, cd)
    net = rrt.mlp_forward(w_dev, b_dev, rrt.mlp_encode(xd))
    ok = (cd >= 0) & (cd < C)
    want = torch.where(ok[:, None], net * sd[cd.clamp(0, C - 1).long()], torch.zeros_like(net))
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    y, _ = ref.forward(Wq, bq, ref.encode(x.astype(np.float64)))
    keep = cluster[(cluster >= 0) & (cluster < C)]
    ref_vals = y[(cluster >= 0) & (cluster < C)] * scales[keep]
    assert _rel(got.cpu().numpy()[(cluster >= 0) & (cluster < C)], ref_vals) <= 2e-2


@pytest.mark.parametrize("B", [1, 64, 333, 4096])
def test_forward(rrt, B):
    Wq, bq, w_dev, b_dev = _net(1)
    rng = np.random.default_rng(B)
    x = _bf16(ref.encode(rng.uniform(-1, 1, size=(B, 6))))
    out = rrt.mlp_forward(w_dev, b_dev, x.cuda()).cpu().numpy()
    want, _ = ref.forward(Wq, bq, x.float().numpy().astype(np.float64))
    assert _rel(out, want) <= 2e-2, _rel(out, want)


@pytest.mark.parametrize("B", [64, 1000])
def test_backward(rrt, B):
    Wq, bq, w_dev, b_dev = _net(2)
    rng = np.random.default_rng(B + 1)
    x = _bf16(ref.encode(rng.uniform(-1, 1, size=(B, 6))))
    dout = rng.normal(size=(B, ref.OUT)).astype(np.float32)
    ws = rrt.mlp_workspace(B, "cuda")
    rrt.mlp_forward(w_dev, b_dev, x.cuda(), workspace=ws)
    dw, db = rrt.mlp_backward(w_dev, x.cuda(), torch.from_numpy(dout).cuda(), ws)
    dw, db = dw.cpu().numpy(), db.cpu().numpy()
    _, cache = ref.forward(Wq, bq, x.float().numpy().astype(np.float64))
    dWs, dbs = ref.backward(Wq, cache, dout.astype(np.float64))
    wo = bo = 0
    for l, (o, i) in enumerate(ref.shapes()):
        gw = dw[wo:wo + o * i].reshape(o, i)
        gb = db[bo:bo + o]
        assert _rel(gw, dWs[l]) <= 3e-2, (l, _rel(gw, dWs[l]))
        assert _rel(gb, dbs[l]) <= 3e-2, (l, _rel(gb, dbs[l]))
        wo += o * i
        bo += o


def test_mse_and_adam(rrt):
    rng = np.random.default_rng(9)
    out = rng.normal(size=(37, 256)).astype(np.float32)
    tgt = rng.normal(size=(37, 256)).astype(np.float32)
    dout, loss = rrt.mse(torch.from_numpy(out).cuda(), torch.from_numpy(tgt).cuda())
    l_ref, g_ref = ref.loss_and_grad(out, tgt)
    assert abs(loss.item() - l_ref) <= 1e-6 * l_ref
    np.testing.assert_allclose(dout.cpu().numpy(), g_ref, rtol=1e-5, atol=1e-9)
    p = rng.normal(size=1000).astype(np.float32)
    g = rng.normal(size=1000).astype(np.float32)
    pd, md, vd = (torch.from_numpy(p.copy()).cuda(), torch.zeros(1000, device="cuda"),
                  torch.zeros(1000, device="cuda"))
    pb = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    pr, mr, vr = p.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        gg = g * step
        rrt.adam_step(pd, torch.from_numpy(gg).cuda(), md, vd, step, 1e-3, param_bf16=pb)
        pr, mr, vr = ref.adam_step(pr, mr, vr, gg.astype(np.float64), step, 1e-3)
    np.testing.assert_allclose(pd.cpu().numpy(), pr, rtol=1e-5, atol=1e-7)
    assert torch.equal(pb, pd.to(torch.bfloat16))


def test_training_reduces_loss(rrt):
    """A few device Adam steps on a fixed smooth target lower the loss."""
    Wq, bq, w_dev, b_dev = _net(4, bias_scale=0.0)
    master = torch.cat([torch.from_numpy(np.asarray(W, np.float32)).reshape(-1) for W in Wq]).cuda()
    bias = b_dev.clone()
    mw, vw = torch.zeros_like(master), torch.zeros_like(master)
    mb, vb = torch.zeros_like(bias), torch.zeros_like(bias)
    rng = np.random.default_rng(5)
    xin = rng.uniform(-1, 1, size=(512, 6)).astype(np.float32)
    tgt = np.sin(np.pi * xin[:, :1]) * np.linspace(-1, 1, 256)[None, :].astype(np.float32)
    x = rrt.mlp_encode(torch.from_numpy(xin).cuda())
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    ws = rrt.mlp_workspace(512, "cuda")
    losses = []
    for step in range(1, 61):
        out = rrt.mlp_forward(w_dev, bias, x, workspace=ws)
        dout, loss = rrt.mse(out, t)
        dw, db = rrt.mlp_backward(w_dev, x, dout, ws)
        rrt.adam_step(master, dw, mw, vw, step, 1e-3, param_bf16=w_dev)
        rrt.adam_step(bias, db, mb, vb, step, 1e-3)
        losses.append(loss.item())
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])
