"""Seeded synthetic workloads shared by the tests, the bench and the oracle runs.

This module only draws inputs: sparse patterns (CSR with raw, unreduced
integer values), dense vectors and block operands. It contains none of the
method's modular arithmetic, so both the oracle and the GPU library receive
exactly the same raw data and each reduces it on its own.

The recipes below stand in for the paper's matrices (Table "Matrices
overview", Section 2.2), which are not available; they follow the shapes of
the five benchmark configurations: plain uniform rows, a power-law hybrid with
a band overlay and many +-1 entries, a block-Wiedemann operand with a planted
rank deficiency, a batch of uneven matrices, and generated matrices for
format selection.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_gen.so")
SEED0 = 0x10043719

LEN_FIXED, LEN_UNIFORM, LEN_ZIPF, LEN_BIMODAL = 0, 1, 2, 3
COL_UNIFORM, COL_LIVE, COL_BANDED, COL_BLOCKDIAG = 0, 1, 2, 3


class Spec(ctypes.Structure):
    _fields_ = [
        ("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("seed", ctypes.c_uint64),
        ("len_kind", ctypes.c_int32), ("len_a", ctypes.c_int32), ("len_b", ctypes.c_int32),
        ("len_c", ctypes.c_int32), ("len_d", ctypes.c_int32),
        ("len_alpha", ctypes.c_double), ("len_p", ctypes.c_double),
        ("col_kind", ctypes.c_int32), ("band_lo", ctypes.c_int32), ("band_hi", ctypes.c_int32),
        ("ndead", ctypes.c_int64), ("block", ctypes.c_int64),
        ("p_pm1", ctypes.c_double), ("val_lo", ctypes.c_int64), ("val_hi", ctypes.c_int64),
    ]


def build(force=False):
    """Compile gen.c into _gen.so (gcc, OpenMP)."""
    src = os.path.join(HERE, "gen.c")
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(src):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.synth_count.restype = ctypes.c_int64
        L.synth_count.argtypes = [P(Spec), ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        L.synth_fill.restype = ctypes.c_int
        L.synth_fill.argtypes = [P(Spec), ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.synth_vector.restype = None
        L.synth_vector.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        L.synth_unit.restype = None
        L.synth_unit.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        L.synth_raw.restype = None
        L.synth_raw.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        _lib = L
    return _lib


def spec(nrows, ncols, seed, **kw):
    s = Spec()
    s.nrows, s.ncols, s.seed = int(nrows), int(ncols), int(seed) & (2**64 - 1)
    s.band_lo, s.band_hi = 0, -1  # no band overlay by default
    s.val_lo, s.val_hi = 1, 1
    for k, v in kw.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


class Csr:
    """A generated CSR matrix: rowptr int64[nrows+1], col int32[nnz], raw values int64[nnz]."""

    def __init__(self, nrows, ncols, rowptr, col, val, m=None, name=""):
        self.nrows, self.ncols = int(nrows), int(ncols)
        self.rowptr, self.col, self.val = rowptr, col, val
        self.m = m
        self.name = name

    @property
    def nnz(self):
        return int(self.rowptr[-1] - self.rowptr[0])

    def __repr__(self):
        return "Csr(%s %dx%d nnz=%d m=%s)" % (self.name, self.nrows, self.ncols, self.nnz, self.m)


def rows(s, r0=0, r1=None):
    """Rows [r0, r1) of the matrix described by spec s, as a Csr whose rowptr starts at 0."""
    if r1 is None:
        r1 = s.nrows
    L = lib()
    cnt = np.empty(r1 - r0, dtype=np.int64)
    nnz = L.synth_count(ctypes.byref(s), r0, r1, cnt.ctypes.data)
    if nnz < 0:
        raise ValueError("bad synthetic spec")
    rowptr = np.zeros(r1 - r0 + 1, dtype=np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.int64)
    rc = L.synth_fill(ctypes.byref(s), r0, r1, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    if rc != 0:
        raise RuntimeError("synth_fill failed (%d)" % rc)
    return Csr(r1 - r0, s.ncols, rowptr, col, val)


def vector(seed, tag, count, lo, hi, dtype=np.int64):
    """count integers uniform in [lo, hi]."""
    out = np.empty(int(count), dtype=np.int64)
    lib().synth_vector(int(seed) & (2**64 - 1), int(tag), int(count), int(lo), int(hi), out.ctypes.data)
    return out.astype(dtype, copy=False)


def unit(seed, tag, count):
    out = np.empty(int(count), dtype=np.float64)
    lib().synth_unit(int(seed) & (2**64 - 1), int(tag), int(count), out.ctypes.data)
    return out


def raw(key, count):
    out = np.empty(int(count), dtype=np.uint64)
    lib().synth_raw(int(key) & (2**64 - 1), int(count), out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Benchmark workloads
# ---------------------------------------------------------------------------
M_C1, M_C2, M_C3, M_C4, M_C5 = 65521, 32749, 2**31 - 1, 65521, 65521


def c1(seed=SEED0 + 0, n=10_000, k=10, m=M_C1):
    """Plain SpMV: square n x n, k distinct uniform columns per row, values in [1, m-1]."""
    s = spec(n, n, seed, len_kind=LEN_FIXED, len_a=k, col_kind=COL_UNIFORM, val_lo=1, val_hi=m - 1)
    A = rows(s)
    A.m, A.name = m, "c1"
    return A


def c2_spec(seed=SEED0 + 1, n=2_000_000, zipf_alpha=1.8, kmax=5000, band=2, p_pm1=0.6):
    """Power-law rows (truncated discrete Zipf on [1, kmax]) at distinct uniform columns, with the
    diagonals -band..+band overlaid; each entry is +-1 w.p. p_pm1, else a uniform int32."""
    return spec(n, n, seed, len_kind=LEN_ZIPF, len_a=1, len_b=kmax, len_alpha=zipf_alpha,
                col_kind=COL_UNIFORM, band_lo=-band, band_hi=band,
                p_pm1=p_pm1, val_lo=-(2**31), val_hi=2**31 - 1)


def c2(seed=SEED0 + 1, n=2_000_000, m=M_C2, **kw):
    A = rows(c2_spec(seed, n, **kw))
    A.m, A.name = m, "c2"
    return A


def c3_spec(seed=SEED0 + 2, n=200_000, k=15, ndead=1000, m=M_C3):
    """k distinct columns per row drawn from n - ndead live columns (so at least ndead columns are
    empty and rank <= n - ndead), values uniform in [1, m-1]."""
    return spec(n, n, seed, len_kind=LEN_FIXED, len_a=k, col_kind=COL_LIVE, ndead=ndead,
                val_lo=1, val_hi=m - 1)


def c3(seed=SEED0 + 2, n=200_000, k=15, ndead=1000, m=M_C3):
    A = rows(c3_spec(seed, n, k, ndead, m))
    A.m, A.name = m, "c3"
    return A


def c3_blocks(seed=SEED0 + 2, n=200_000, s=8, m=M_C3):
    """Projection U and start block V, both n x s interleaved (row j holds s residues), in [0, m-1]."""
    U = vector(seed, 11, n * s, 0, m - 1).reshape(n, s)
    V = vector(seed, 12, n * s, 0, m - 1).reshape(n, s)
    return U, V


def c3_length(n, s):
    """Sequence length covering i = 0 .. 2n/s + 2."""
    return 2 * n // s + 3


def c4_params(k, seed=SEED0 + 3, nmin=2000, nmax=500_000):
    """Parameters of matrix k of the uneven batch."""
    u = unit(seed, 1000 + k, 8)
    n = int(round(math.exp(math.log(nmin) + u[0] * (math.log(nmax) - math.log(nmin)))))
    d = 3 + min(57, int(u[1] * 58))               # mean nnz/row uniform in 3..60
    structure = min(2, int(u[2] * 3))             # 0 uniform random, 1 banded, 2 block-diagonal
    block = 256 + min(3840, int(u[3] * 3841))     # block size for block-diagonal
    s = 1 + min(15, int(u[4] * 16))               # right-hand sides 1..16
    return dict(n=n, d=d, structure=structure, block=block, s=s, seed=(seed * 1000003 + k) & (2**64 - 1))


def c4_matrix(k, seed=SEED0 + 3, m=M_C4, p_pm1=0.7, **kw):
    p = c4_params(k, seed, **kw)
    n, d = p["n"], p["d"]
    common = dict(p_pm1=p_pm1, val_lo=1, val_hi=m - 1)
    if p["structure"] == 0:
        sp = spec(n, n, p["seed"], len_kind=LEN_FIXED, len_a=d, col_kind=COL_UNIFORM, **common)
    elif p["structure"] == 1:
        lo = -((d - 1) // 2)
        sp = spec(n, n, p["seed"], col_kind=COL_BANDED, band_lo=lo, band_hi=lo + d - 1, **common)
    else:
        sp = spec(n, n, p["seed"], len_kind=LEN_FIXED, len_a=min(d, p["block"]), col_kind=COL_BLOCKDIAG,
                  block=p["block"], **common)
    A = rows(sp)
    A.m, A.name = m, "c4[%d]" % k
    A.s = p["s"]
    A.params = p
    return A


def c4_rhs(k, A, seed=SEED0 + 3, m=M_C4):
    return vector(seed, 5000 + k, A.ncols * A.s, 0, m - 1).reshape(A.ncols, A.s)


def c5_params(k, seed=SEED0 + 4, nmin=50_000, nmax=4_000_000):
    """Parameters of generated matrix k for format selection (k < 1800 training, else held out)."""
    u = unit(seed, 2000 + k, 12)
    n = int(round(math.exp(math.log(nmin) + u[0] * (math.log(nmax) - math.log(nmin)))))
    family = min(2, int(u[1] * 3))                # 0 uniform, 1 zipf, 2 bimodal row lengths
    mean = 2 + u[2] * 62                          # mean row length in [2, 64]
    alpha = 1.5 + u[3]                            # zipf exponent in [1.5, 2.5]
    p_pm1 = u[4]
    band = min(64, int(u[5] * 65))                # band width 0..64
    return dict(n=n, family=family, mean=mean, alpha=alpha, p_pm1=p_pm1, band=band, u=u,
                seed=(seed * 1000003 + k) & (2**64 - 1))


def c5_spec(k, seed=SEED0 + 4, m=M_C5, **kw):
    p = c5_params(k, seed, **kw)
    n, mean = p["n"], p["mean"]
    u = p["u"]
    common = dict(p_pm1=p["p_pm1"], val_lo=1, val_hi=m - 1, col_kind=COL_UNIFORM)
    # band overlay: the diagonals -band//2 .. band - band//2 - 1 (none when band == 0)
    if p["band"] > 0:
        common.update(band_lo=-(p["band"] // 2), band_hi=p["band"] - p["band"] // 2 - 1)
    if p["family"] == 0:
        half = max(0, int(mean * u[6]))
        a = max(0, int(round(mean)) - half)
        sp = spec(n, n, p["seed"], len_kind=LEN_UNIFORM, len_a=a, len_b=int(round(mean)) + half, **common)
    elif p["family"] == 1:
        sp = spec(n, n, p["seed"], len_kind=LEN_ZIPF, len_a=1, len_b=4096, len_alpha=p["alpha"], **common)
    else:
        lo_mean = max(1.0, mean * (0.1 + 0.4 * u[6]))
        hi_mean = mean * (1.5 + 3.0 * u[7])
        pl = 0.5 + 0.45 * u[8]
        sp = spec(n, n, p["seed"], len_kind=LEN_BIMODAL, len_p=pl,
                  len_a=max(0, int(lo_mean) - 1), len_b=int(lo_mean) + 1,
                  len_c=max(1, int(hi_mean * 0.75)), len_d=max(2, int(hi_mean * 1.25)), **common)
    return sp, p


def c5_matrix(k, seed=SEED0 + 4, m=M_C5, r0=0, r1=None, **kw):
    sp, p = c5_spec(k, seed, m, **kw)
    A = rows(sp, r0, r1)
    A.m, A.name = m, "c5[%d]" % k
    A.params = p
    A.row0 = r0
    return A


def stencil(seed=SEED0 + 5, width=2048, height=1024, p_pm1=0.6, shuffle=True, m=M_C2):
    """A 9-point stencil on a width x height grid: node (x, y) is coupled to itself and to its up to 8
    grid neighbours (so rows hold 4, 6 or 9 entries and the pattern is symmetric). With shuffle, the
    nodes are numbered by a seeded uniformly random permutation (the order of counter-based random
    keys), so the grid's locality is present but hidden by the numbering; without, node (x, y) is
    row y*width + x (a band of half-width width + 1). Each entry is +-1 with probability p_pm1 (fair
    sign), else a uniform int32."""
    n = width * height
    g = np.arange(n, dtype=np.int64)
    gx, gy = g % width, g // width
    if shuffle:
        order = np.argsort(raw(seed, n), kind="stable")  # order[label] = grid node
        label = np.empty(n, np.int64)
        label[order] = np.arange(n, dtype=np.int64)
    else:
        order, label = g, g
    nb = np.full((n, 9), -1, np.int64)
    q = 0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            x, y = gx + dx, gy + dy
            ok = (x >= 0) & (x < width) & (y >= 0) & (y < height)
            nb[ok, q] = label[(y * width + x)[ok]]
            q += 1
    nb = nb[order]  # row r is grid node order[r]
    nb[nb < 0] = n  # absent neighbours sort last
    nb.sort(axis=1)
    lens = (nb < n).sum(axis=1)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = nb[nb < n].astype(np.int32)
    nnz = len(col)
    u = unit(seed, 1, nnz)
    sign = vector(seed, 2, nnz, 0, 1)
    val = np.where(u < p_pm1, 2 * sign - 1, vector(seed, 3, nnz, -(2**31), 2**31 - 1))
    A = Csr(n, n, rowptr, col, val, m=m, name="stencil%dx%d%s" % (width, height, "-shuffled" if shuffle else ""))
    A.grid = (width, height)
    return A
