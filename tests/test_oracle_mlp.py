"""Pins of the checker's MLP (no GPU): central-difference gradients of the
loss for every parameter tensor, the GELU derivative, the encoding's
closed-form values, and Adam's first step (|update| = lr exactly)."""
import numpy as np

from oracle import mlp


def _small_net(seed=0):
    Ws, bs = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    bs = [rng.normal(0, 0.1, size=b.shape) for b in bs]
    return Ws, bs


def test_encoding_values():
    x = np.array([[0.0, 0.5, -1.0, 0.25, 1.0, -0.5]])
    e = mlp.encode(x)
    assert e.shape == (1, 128)
    np.testing.assert_allclose(e[0, :6], x[0])
    # band 0: sin(pi x), cos(pi x); band 1: sin(2 pi x) ...
    np.testing.assert_allclose(e[0, 6:12], np.sin(np.pi * x[0]), atol=1e-15)
    np.testing.assert_allclose(e[0, 12:18], np.cos(np.pi * x[0]), atol=1e-15)
    np.testing.assert_allclose(e[0, 18:24], np.sin(2 * np.pi * x[0]), atol=1e-15)
    assert e[0, 6 + 2] == np.sin(-np.pi) and abs(e[0, 12 + 1]) < 1e-15   # sin(-pi), cos(pi/2)
    assert np.all(e[0, 102:] == 0)


def test_gelu_grad_central_difference():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([10.0])), [10.0], rtol=1e-12)


def test_backward_central_difference():
    Ws, bs = _small_net(3)
    rng = np.random.default_rng(4)
    x = mlp.encode(rng.uniform(-1, 1, size=(5, 6)))
    target = rng.normal(size=(5, mlp.OUT))

    def loss(Ws_, bs_):
        out, _ = mlp.forward(Ws_, bs_, x)
        return mlp.loss_and_grad(out, target)[0]

    out, cache = mlp.forward(Ws, bs, x)
    _, dout = mlp.loss_and_grad(out, target)
    dWs, dbs = mlp.backward(Ws, cache, dout)
    h = 1e-6
    for l in range(len(Ws)):
        for (i, j) in [(0, 0), (7, 3), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1), (100, 101)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (loss(Wp, bs) - loss(Wm, bs)) / (2 * h)
            assert abs(fd - dWs[l][i, j]) <= 1e-6 * max(1e-6, abs(fd)) + 1e-10, (l, i, j)
        for i in (0, 31, bs[l].size - 1):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[l][i] += h
            bm[l][i] -= h
            fd = (loss(Ws, bp) - loss(Ws, bm)) / (2 * h)
            assert abs(fd - dbs[l][i]) <= 1e-6 * max(1e-6, abs(fd)) + 1e-10, (l, i)


def test_adam_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 0.0])
    p1, m, v = mlp.adam_step(p, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # bias-corrected first step moves each parameter by lr * sign(g) (eps aside)
    np.testing.assert_allclose(p1[:2], p[:2] - 0.01 * np.sign(g[:2]), rtol=1e-6)
    assert p1[2] == p[2]


def test_parameter_count():
    assert sum(o * i + o for (o, i) in mlp.shapes()) == 296192
