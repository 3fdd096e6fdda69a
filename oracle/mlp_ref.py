"""ORACLE -- test infrastructure only.

fp64 reference of the learned format selector's network: a 3-layer
perceptron 32 -> 64 -> 64 -> 6 (ReLU hidden layers, linear output) that
predicts, for one row block, the log2 time of each of the 6 storage formats.
Training minimises the masked squared error

    loss = 1/(2N) * sum_i sum_f mask[i,f] * (out[i,f] - target[i,f])^2

with Adam (Kingma and Ba, ICLR 2015: beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
bias-corrected moments). This model is not in the paper: the paper's chooser
is a hand heuristic whose thresholds it says need per-machine tuning
(Section 2.4, "Heuristic format chooser"); the network replaces that tuning.

Parameter layout (also the flat vector order of the GPU kernels):
W1 (64x32, row-major), b1 (64), W2 (64x64), b2 (64), W3 (6x64), b3 (6):
6,662 values.
"""
import numpy as np

SIZES = (32, 64, 64, 6)
SHAPES = [(64, 32), (64,), (64, 64), (64,), (6, 64), (6,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unflatten(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in parts])


def init(seed=0):
    """He-uniform weights (bound sqrt(6/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            b = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-b, b, size=s))
        else:
            parts.append(np.zeros(s))
    return flatten(parts)


def forward(theta, X):
    """Predictions (N x 6) for inputs X (N x 32), and the activations."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3.T + b3
    return out, (X, z1, h1, z2, h2)


def loss(theta, X, T, M):
    out, _ = forward(theta, X)
    N = out.shape[0]
    d = (out - T) * M
    return 0.5 * float(np.sum(d * d)) / N


def loss_grad(theta, X, T, M):
    """Loss and its gradient with respect to the flat parameter vector (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta)
    out, (X, z1, h1, z2, h2) = forward(theta, X)
    N = out.shape[0]
    d = (out - np.asarray(T, np.float64)) * np.asarray(M, np.float64)
    L = 0.5 * float(np.sum(d * d)) / N
    g_out = d / N                        # dL/dout
    gW3 = g_out.T @ h2
    gb3 = g_out.sum(axis=0)
    g_h2 = g_out @ W3
    g_z2 = g_h2 * (z2 > 0)
    gW2 = g_z2.T @ h1
    gb2 = g_z2.sum(axis=0)
    g_h1 = g_z2 @ W2
    g_z1 = g_h1 * (z1 > 0)
    gW1 = g_z1.T @ X
    gb1 = g_z1.sum(axis=0)
    return L, flatten([gW1, gb1, gW2, gb2, gW3, gb3])


class Adam:
    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
