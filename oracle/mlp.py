"""FP64 reference of the learned transport decoder (not part of the paper).

Test infrastructure only (see the package docstring).

A small MLP maps a vertex's position and normal to the values of its
transport coefficients on a fixed per-cluster support:

  encode:  x in R^6 (position scaled to [-1, 1], unit normal) ->
           gamma(x) = (x, sin(2^k pi x), cos(2^k pi x) for k = 0..7)
           = 6 + 96 = 102 features, zero-padded to 128 (feature order: the six
           inputs, then for k = 0..7 the six sines followed by the six cosines)
  layers:  z_l = W_l a_{l-1} + b_l; a_l = gelu(z_l) for the 4 hidden layers of
           width 256; the output layer (256) is linear
  gelu:    0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))  (tanh form)
  loss:    mean over the batch and the 256 outputs of (out - target)^2
  Adam:    m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
           p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Weights W_l are [out, in] (row-major), matching the device layout.
"""
import numpy as np

BANDS = 8
IN_RAW = 6
IN_FEAT = IN_RAW * (1 + 2 * BANDS)       # 102
IN_PAD = 128
HIDDEN = 256
LAYERS = 4
OUT = 256
SQRT_2_OVER_PI = 0.7978845608028654
GELU_C = 0.044715


def encode(x):
    """[B, 6] -> [B, 128] positional encoding (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    feats = [x]
    for k in range(BANDS):
        w = (2.0 ** k) * np.pi
        feats.append(np.sin(w * x))
        feats.append(np.cos(w * x))
    f = np.concatenate(feats, axis=1)
    out = np.zeros((x.shape[0], IN_PAD))
    out[:, :IN_FEAT] = f
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(SQRT_2_OVER_PI * (z + GELU_C * z ** 3)))


def gelu_grad(z):
    u = SQRT_2_OVER_PI * (z + GELU_C * z ** 3)
    t = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3.0 * GELU_C * z ** 2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def shapes():
    dims = [IN_PAD] + [HIDDEN] * LAYERS + [OUT]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def init_params(seed):
    """He-style init: W ~ N(0, 2 / fan_in), b = 0 (FP64)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for (o, i) in shapes():
        Ws.append(rng.normal(0.0, np.sqrt(2.0 / i), size=(o, i)))
        bs.append(np.zeros(o))
    return Ws, bs


def forward(Ws, bs, x_enc):
    """Returns (out, cache) with cache = list of (input, pre-activation)."""
    a = np.asarray(x_enc, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = a @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        cache.append((a, z))
        a = gelu(z) if l < len(Ws) - 1 else z
    return a, cache


def loss_and_grad(out, target):
    d = np.asarray(out, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return float(np.sum(d * d) / n), 2.0 * d / n


def backward(Ws, cache, dout):
    """Gradients (dWs, dbs) of a scalar whose gradient w.r.t. out is dout."""
    dWs = [None] * len(Ws)
    dbs = [None] * len(Ws)
    g = np.asarray(dout, np.float64)
    for l in range(len(Ws) - 1, -1, -1):
        a_in, z = cache[l]
        dz = g if l == len(Ws) - 1 else g * gelu_grad(z)
        dWs[l] = dz.T @ a_in
        dbs[l] = dz.sum(axis=0)
        g = dz @ np.asarray(Ws[l], np.float64)
    return dWs, dbs


def adam_step(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (arrays updated and returned)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
