"""Pins for the FP64 reference of the cost-model network (no GPU)."""
import numpy as np

from oracle import mlp


def _setup(seed, n=40):
    rng = np.random.default_rng(seed)
    w = np.zeros(mlp.N_PARAMS)
    w[mlp.OFF_W1:mlp.OFF_B1] = rng.normal(0, 0.5, mlp.H * mlp.F)
    w[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, 0.3, mlp.H)
    w[mlp.OFF_W2:mlp.OFF_B2] = rng.normal(0, 0.2, mlp.H * mlp.H)
    w[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0, 0.3, mlp.H)
    w[mlp.OFF_W3:mlp.OFF_B3] = rng.normal(0, 0.3, mlp.H)
    w[mlp.OFF_B3] = 0.7
    X = rng.normal(0, 1, (n, mlp.F))
    Y = rng.normal(0, 1, n)
    return w, X, Y


def test_gradient_matches_central_differences():
    w, X, Y = _setup(1)
    g = mlp.grad(w, X, Y)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 120, replace=False),
                          [mlp.OFF_B3, mlp.OFF_W1, mlp.OFF_B1, mlp.OFF_W2, mlp.OFF_B2, mlp.OFF_W3]])
    h = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (mlp.loss(wp, X, Y) - mlp.loss(wm, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_closed_form_special_cases():
    """All-zero hidden layers give the output bias; a single active path is
    a product of the weights along it."""
    w = np.zeros(mlp.N_PARAMS)
    w[mlp.OFF_B3] = 1.25
    X = np.random.default_rng(3).normal(size=(5, mlp.F))
    np.testing.assert_allclose(mlp.forward(w, X), 1.25)
    w[mlp.OFF_W1 + 0 * mlp.F + 2] = 2.0      # h1[0] = relu(2 x2)
    w[mlp.OFF_W2 + 5 * mlp.H + 0] = 3.0      # h2[5] = relu(3 h1[0])
    w[mlp.OFF_W3 + 5] = -0.5
    x = np.zeros((2, mlp.F)); x[0, 2] = 1.0; x[1, 2] = -1.0
    np.testing.assert_allclose(mlp.forward(w, x), [1.25 - 0.5 * 6.0, 1.25])


def test_bf16_rounding():
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3, 65504.0], np.float32)
    r = mlp.bf16_round(a)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins -> 1
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0 + 2 ** -7)
    assert r[3] == -2.5
    assert (r.view(np.uint32) & 0xFFFF).max() == 0
    assert abs(r[4] - 3.0e-3) / 3.0e-3 < 2 ** -8
