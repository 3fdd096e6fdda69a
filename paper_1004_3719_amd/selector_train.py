"""Training and evaluation of the learned per-block format selector.

Labels come from the library itself: every training window (a run of row
blocks of one generated matrix, so of one row-length law, +-1 fraction and
band) is built once per format, with all blocks forced to that format, and
its whole product y = A x is timed on the GPU; the label of (block, format)
is log2 of that time per block in microseconds. Timing the product in place
keeps x at its real size, so gathers cost what they cost in use; a block
timed alone (ffx_matrix_block_times) finds its x entries in cache and
favours the wrong formats. Features are the builder's own 32 block features
(ffx_block_features). The network is trained with the library's forward,
backward and Adam kernels (Selector.train_step); nothing here computes a
gradient. Input standardisation (mean, scale) is taken from the training
features and stored with the model.

The paper's chooser is a hand heuristic whose thresholds need tuning per
machine (Section 2.4, "Heuristic format chooser"); this replaces the tuning by
measurement. Whatever the network predicts, products are unchanged: it only
picks formats.
"""
import time

import numpy as np

from .ffx import FORMATS, Matrix, Selector, block_features

NF = len(FORMATS)


def window_labels(A, x_dev, y_dev, reps=6, opts=None):
    """(features (nb x 32), log2 microseconds per block (nb x 6), the heuristic's formats (nb)) of a
    window A whose blocks share one generator: each format's label is the in-place product time of the
    whole window divided by its block count."""
    opts = dict(opts or {})
    F = block_features(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, **opts)
    nb = F.shape[0]
    T = np.zeros((nb, NF), np.float32)
    for f in range(NF):
        M = Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, fixed_format=f, **opts)
        T[:, f] = np.log2(max(time_product(M, x_dev, y_dev, reps) / nb, 1e-3))
        M.close()
    M = Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, **opts)
    H = M.block_formats()
    M.close()
    return F, T, H


def choice_cost(T, choice):
    """Summed block time of a per-block format choice, relative to the best choice (1 = best)."""
    t = np.exp2(T.astype(np.float64))
    return float(t[np.arange(len(t)), choice].sum() / t.min(axis=1).sum())


def shift_columns(A, r0):
    """Rows r0.. of a matrix taken as a matrix of their own keep their diagonals only if the columns
    move with the rows: column c becomes (c - r0) mod ncols, a cyclic permutation of the columns that
    keeps every diagonal, band and block structure relative to the new row numbers."""
    A.col = ((A.col.astype(np.int64) - r0) % A.ncols).astype(np.int32)
    return A


def standardisation(X):
    mean = X.mean(axis=0).astype(np.float32)
    sd = X.std(axis=0)
    scale = np.where(sd > 1e-6, 1.0 / np.maximum(sd, 1e-6), 1.0).astype(np.float32)
    return mean, scale


def relative(T):
    """log2 times relative to the STREAM format of the same block: the choice only depends on the
    differences between formats, which are small beside the spread of block times, so the network
    learns them directly."""
    return T - T[:, :1]


def fit(X, T, M=None, epochs=60, batch=512, lr=2e-3, seed=0, device="cuda:0", val=None, log=None):
    """Train a Selector on features X and log-time targets T (numpy, trained relative to STREAM);
    M masks missing labels. Returns (selector, history)."""
    import torch
    dev = torch.device(device)
    T = relative(T)
    if val is not None:
        val = (val[0], relative(val[1]))
    if M is None:
        M = np.ones_like(T)
    mean, scale = standardisation(X)
    S = Selector(seed=seed)
    S.set_params(mean=mean, scale=scale)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    Td = torch.from_numpy(np.ascontiguousarray(T, np.float32)).to(dev)
    Md = torch.from_numpy(np.ascontiguousarray(M, np.float32)).to(dev)
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            if idx.numel() < 2:
                continue
            step_lr = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))  # cosine decay
            S.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), Md[idx].contiguous(), lr=step_lr)
        if ep % 10 == 9 or ep == epochs - 1:
            loss, _ = S.gradient(Xd, Td, Md)
            rec = {"epoch": ep + 1, "train_loss": loss}
            if val is not None:
                Xv, Tv = val
                Xvd = torch.from_numpy(np.ascontiguousarray(Xv, np.float32)).to(dev)
                Tvd = torch.from_numpy(np.ascontiguousarray(Tv, np.float32)).to(dev)
                lv, _ = S.gradient(Xvd, Tvd, torch.ones_like(Tvd))
                rec["val_loss"] = lv
            hist.append(rec)
            if log:
                log(rec)
    return S, hist


def apply_margin(S, mu):
    """Fold a decision margin into the output biases: every format other than STREAM (output 0) is
    predicted mu (log2 units) slower, so a block leaves STREAM only when the network predicts a gain
    larger than mu. Predicted differences smaller than the network's error then cost nothing."""
    th, mean, scale = S.get_params()
    th = th.copy()
    th[-5:] += np.float32(mu)  # b3[1..5]
    S.set_params(theta=th, mean=mean, scale=scale)


def pick_margin(S, X, T, margins=(0.0, 0.05, 0.1, 0.2, 0.3, 0.5)):
    """The margin with the lowest summed block time on (X, T), applied to S; returns (mu, costs)."""
    base, mean, scale = S.get_params()
    costs = {}
    for mu in margins:
        S.set_params(theta=base, mean=mean, scale=scale)
        apply_margin(S, mu)
        costs[mu] = choice_cost(T, choose(S, X)[0])
    best = min(margins, key=lambda m: (round(costs[m], 4), m))
    S.set_params(theta=base, mean=mean, scale=scale)
    apply_margin(S, best)
    return best, costs


def choose(S, X, device="cuda:0"):
    """Predicted fastest format per row (argmin of the predicted log times)."""
    import torch
    P = S.predict(torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(torch.device(device))).cpu().numpy()
    return P.argmin(axis=1), P


def time_product(M, x, y, reps=10):
    """Median microseconds of y = A x with HIP events."""
    import torch
    for _ in range(2):
        M.spmv(x, y=y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        M.spmv(x, y=y)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e3)
    return float(np.median(ts))


def evaluate(A, model_path, x, reps=10, fixed=()):
    """Whole-product time with the heuristic's and the learned formats (and whether the results agree),
    and with each format of `fixed` forced on every block (key "fixed_<name>_us")."""
    import torch
    y1 = torch.empty(A.nrows, dtype=x.dtype, device=x.device)
    y2 = torch.empty_like(y1)
    t0 = time.perf_counter()
    Mh = Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m)
    Ml = Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, selector="learned", model_path=model_path)
    build_s = time.perf_counter() - t0
    th = time_product(Mh, x, y1, reps)
    tl = time_product(Ml, x, y2, reps)
    same = bool(torch.equal(y1, y2))
    out = {"heuristic_us": th, "learned_us": tl, "same_result": same, "build_s": build_s,
           "heuristic_formats": Mh.info()["format_blocks"], "learned_formats": Ml.info()["format_blocks"]}
    Mh.close()
    Ml.close()
    for f in fixed:
        Mf = Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, fixed_format=f)
        out["fixed_%s_us" % f] = time_product(Mf, x, y2, reps)
        out["same_result"] = out["same_result"] and bool(torch.equal(y1, y2))
        Mf.close()
    return out
