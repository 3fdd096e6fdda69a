"""Driver of the learned per-block format selector: training windows, labels, training, evaluation.

Every measurement and every training step runs in the library:
- ffx_selector_label builds a training window once per format (every block forced to it), times its
  whole product y = A x in place on the GPU and returns the block features, the labels (log2 of the
  window time per block in microseconds) and the heuristic's formats;
- ffx_selector_train standardises the features, trains the network relative to STREAM with the
  library's forward, backward and Adam kernels (minibatches, cosine-decayed rate), picks the decision
  margin on held-out samples and writes the model.
This module only chooses the windows (rows of generated matrices) and marshals arrays.

The paper's chooser is a hand heuristic whose thresholds need tuning per machine (Section 2.4,
"Heuristic format chooser"); this replaces the tuning by measurement. Whatever the network predicts,
products are unchanged: it only picks formats.
"""
import time

import numpy as np

from .ffx import FORMATS, Matrix, selector_label, selector_train

NF = len(FORMATS)


def window_labels(A, reps=6, seed=0, opts=None):
    """(features (nb x 32), log2 microseconds per block (nb x 6), the heuristic's formats (nb)) of the
    training window A, measured by the library."""
    return selector_label(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, reps=reps, seed=seed, **dict(opts or {}))


def shift_columns(A, r0):
    """Rows r0.. of a matrix taken as a matrix of their own keep their diagonals only if the columns
    move with the rows: column c becomes (c - r0) mod ncols, a cyclic permutation of the columns that
    keeps every diagonal, band and block structure relative to the new row numbers."""
    A.col = ((A.col.astype(np.int64) - r0) % A.ncols).astype(np.int32)
    return A


def train(X, T, H=None, epochs=60, lr=2e-3, seed=0, n_val=None, out_model=None):
    """The library's training (ffx_selector_train); the first n_val samples (default n/10) are held out.
    Returns (Selector, report)."""
    return selector_train(X, T, heur=H, epochs=epochs, lr=lr, seed=seed,
                          n_val=-1 if n_val is None else n_val, out_model=out_model)


def choice_cost(T, choice):
    """Summed block time of a per-block format choice, relative to the best choice (1 = best)."""
    t = np.exp2(T.astype(np.float64))
    return float(t[np.arange(len(t)), choice].sum() / t.min(axis=1).sum())


def choose(S, X, device="cuda:0"):
    """Predicted fastest format per row (argmin of the network's outputs)."""
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


def evaluate(A, model_path, x, reps=10, fixed=(), rounds=1):
    """Whole-product time with the heuristic's formats, the learned formats and each format of `fixed`
    forced on every block (key "fixed_<name>_us"); each the median over `rounds` interleaved rounds of
    `reps` launches. Returns the times and every product's result (device tensors, for the caller's
    oracle check)."""
    import torch
    t0 = time.perf_counter()
    # the block formats are what is compared, so the one-vector products run on the tiles (col_sorted 0)
    mats = {"heuristic": Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, col_sorted=0),
            "learned": Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, selector="learned",
                                       model_path=model_path, col_sorted=0)}
    build_s = time.perf_counter() - t0
    for f in fixed:
        mats["fixed_" + f] = Matrix.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, fixed_format=f,
                                             col_sorted=0)
    ys = {k: torch.empty(A.nrows, dtype=x.dtype, device=x.device) for k in mats}
    times = {k: [] for k in mats}
    for _ in range(rounds):
        for k, M in mats.items():
            times[k].append(time_product(M, x, ys[k], reps))
    out = {k + "_us": float(np.median(v)) for k, v in times.items()}
    out["build_s"] = build_s
    out["heuristic_formats"] = mats["heuristic"].info()["format_blocks"]
    out["learned_formats"] = mats["learned"].info()["format_blocks"]
    out["results"] = ys
    for M in mats.values():
        M.close()
    return out
