"""Pins of the fp64 network reference (CPU): finite differences, ReLU homogeneity, hidden-unit
permutation invariance, zero weights, masking, and Adam's closed-form first step."""
import numpy as np

from oracle import mlp_ref as R


def data(n=40, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 32))
    T = rng.normal(size=(n, 6))
    M = (rng.random(size=(n, 6)) < 0.8).astype(np.float64)
    return X, T, M


def test_sizes():
    assert R.NPARAM == 6662


def test_gradient_central_differences():
    X, T, M = data()
    theta = R.init(3)
    theta[[64 * 32 + 1, 6000, 6661]] += 0.1  # nonzero biases too
    L, g = R.loss_grad(theta, X, T, M)
    assert abs(L - R.loss(theta, X, T, M)) < 1e-12
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(R.NPARAM, 300, replace=False), [0, 2047, 2048, 2111, 6655, 6661]])
    h = 1e-6
    for i in idx:
        e = np.zeros(R.NPARAM)
        e[i] = h
        fd = (R.loss(theta + e, X, T, M) - R.loss(theta - e, X, T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_relu_positive_homogeneity_without_biases():
    X, _, _ = data()
    theta = R.init(4)  # biases are zero at init
    out1, _ = R.forward(theta, X)
    out2, _ = R.forward(theta, 3.5 * X)
    assert np.allclose(out2, 3.5 * out1, rtol=1e-12, atol=1e-12)


def test_hidden_permutation_invariance():
    X, _, _ = data()
    theta = R.init(5)
    W1, b1, W2, b2, W3, b3 = R.unflatten(theta)
    b1 = b1 + 0.3
    b2 = b2 - 0.2
    p = np.random.default_rng(0).permutation(64)
    q = np.random.default_rng(1).permutation(64)
    a = R.forward(R.flatten([W1, b1, W2, b2, W3, b3]), X)[0]
    b = R.forward(R.flatten([W1[p], b1[p], W2[q][:, p], b2[q], W3[:, q], b3]), X)[0]
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_zero_weights_give_bias_and_known_gradient():
    X, T, M = data()
    theta = np.zeros(R.NPARAM)
    b3 = np.arange(6, dtype=np.float64)
    theta[-6:] = b3
    out, _ = R.forward(theta, X)
    assert np.array_equal(out, np.tile(b3, (X.shape[0], 1)))
    L, g = R.loss_grad(theta, X, T, M)
    assert np.allclose(g[-6:], ((b3 - T) * M).sum(axis=0) / X.shape[0])
    assert np.all(g[:-6] == 0)  # ReLU(0) blocks every other gradient


def test_mask_removes_terms():
    X, T, M = data()
    theta = R.init(6)
    T2 = T + (1 - M) * 1e6  # masked targets may be anything
    assert abs(R.loss(theta, X, T, M) - R.loss(theta, X, T2, M)) < 1e-9


def test_adam_first_step_is_lr_times_sign():
    opt = R.Adam(5, lr=0.01)
    theta = np.zeros(5)
    g = np.array([3.0, -2.0, 1e-3, -7.0, 0.5])
    new = opt.step(theta, g)
    assert np.allclose(new, -0.01 * np.sign(g), rtol=1e-4)
