"""ORACLE -- test infrastructure only.

Python access to the plain C oracle (oracle.c) and to the fp64 reference of
the format-selection network (mlp_ref.py). Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import this package; the
library under paper_1004_3719_amd/ never does, and this package imports
nothing from it.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")
OMP_PATH = os.path.join(HERE, "liboracle_omp.so")  # the same source, rows of a product over all cores


def build(force=False, src=SRC, out=LIB_PATH, extra=()):
    """Compile oracle.c (single-threaded, -O2) into a shared library; with force, also the OpenMP build."""
    if force and out == LIB_PATH and src == SRC and not extra:
        build(True, src, OMP_PATH, ("-fopenmp",))
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", *extra, "-o", tmp, src])
    os.replace(tmp, out)
    return out


def _bind(path):
    L = ctypes.CDLL(path)
    i64, u64, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    sig = {
        "oracle_spmm": [i64, i64, vp, vp, vp, u64, i64, u64, vp, i64, u64, vp, i64],
        "oracle_spmm_t": [i64, i64, vp, vp, vp, u64, i64, u64, vp, i64, u64, vp, i64],
        "oracle_spmv": [i64, i64, vp, vp, vp, u64, u64, vp, u64, vp],
        "oracle_spmv_t": [i64, i64, vp, vp, vp, u64, u64, vp, u64, vp],
        "oracle_power": [i64, vp, vp, vp, u64, i64, i64, vp, i64, vp, i64],
        "oracle_sequence": [i64, vp, vp, vp, u64, i64, vp, i64, vp, i64, i64, vp, vp],
        "oracle_canon": [i64, vp, u64, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    return L


class Oracle:
    """The oracle entry points on numpy arrays (int64 values, int32 columns)."""

    def __init__(self, path=None):
        if path is None:
            path = LIB_PATH if os.path.exists(LIB_PATH) else build()
        self.L = _bind(path)
        self.path = path

    @staticmethod
    def _csr(A):
        rp = np.ascontiguousarray(A.rowptr, dtype=np.int64)
        rp = rp - rp[0]
        return rp, np.ascontiguousarray(A.col, dtype=np.int32), np.ascontiguousarray(A.val, dtype=np.int64)

    @staticmethod
    def _mat(v, rows, s):
        v = np.ascontiguousarray(np.asarray(v, dtype=np.int64).reshape(rows, s))
        return v

    def _check(self, rc, what):
        if rc != 0:
            raise ValueError("oracle %s rejected its arguments" % what)

    def spmm(self, A, X, alpha=1, beta=0, Y=None, m=None):
        m = A.m if m is None else m
        X = np.asarray(X, dtype=np.int64)
        s = 1 if X.ndim == 1 else X.shape[1]
        Xm = self._mat(X, A.ncols, s)
        Ym = np.zeros((A.nrows, s), np.int64) if Y is None else self._mat(Y, A.nrows, s).copy()
        rp, c, v = self._csr(A)
        rc = self.L.oracle_spmm(A.nrows, A.ncols, rp.ctypes.data, c.ctypes.data, v.ctypes.data, m, s,
                                alpha, Xm.ctypes.data, s, beta, Ym.ctypes.data, s)
        self._check(rc, "spmm")
        return Ym if X.ndim == 2 else Ym.reshape(-1)

    def spmv(self, A, x, alpha=1, beta=0, y=None, m=None):
        return self.spmm(A, np.asarray(x).reshape(-1), alpha, beta, y, m)

    def spmm_t(self, A, X, alpha=1, beta=0, Y=None, m=None):
        m = A.m if m is None else m
        X = np.asarray(X, dtype=np.int64)
        s = 1 if X.ndim == 1 else X.shape[1]
        Xm = self._mat(X, A.nrows, s)
        Ym = np.zeros((A.ncols, s), np.int64) if Y is None else self._mat(Y, A.ncols, s).copy()
        rp, c, v = self._csr(A)
        rc = self.L.oracle_spmm_t(A.nrows, A.ncols, rp.ctypes.data, c.ctypes.data, v.ctypes.data, m, s,
                                  alpha, Xm.ctypes.data, s, beta, Ym.ctypes.data, s)
        self._check(rc, "spmm_t")
        return Ym if X.ndim == 2 else Ym.reshape(-1)

    def spmv_t(self, A, x, alpha=1, beta=0, y=None, m=None):
        return self.spmm_t(A, np.asarray(x).reshape(-1), alpha, beta, y, m)

    def power(self, A, k, V, m=None):
        m = A.m if m is None else m
        V = np.asarray(V, dtype=np.int64)
        s = 1 if V.ndim == 1 else V.shape[1]
        Vm = self._mat(V, A.nrows, s)
        W = np.zeros_like(Vm)
        rp, c, v = self._csr(A)
        rc = self.L.oracle_power(A.nrows, rp.ctypes.data, c.ctypes.data, v.ctypes.data, m, k, s,
                                 Vm.ctypes.data, s, W.ctypes.data, s)
        self._check(rc, "power")
        return W if V.ndim == 2 else W.reshape(-1)

    def sequence(self, A, U, V, L, m=None, want_last=False):
        """S[i] = U^T A^i V for i < L (shape L x s x s); with want_last also A^L V."""
        m = A.m if m is None else m
        U = np.asarray(U, dtype=np.int64)
        s = U.shape[1]
        Um, Vm = self._mat(U, A.nrows, s), self._mat(V, A.nrows, s)
        S = np.zeros((L, s, s), np.int64)
        W = np.zeros((A.nrows, s), np.int64) if want_last else None
        rp, c, v = self._csr(A)
        rc = self.L.oracle_sequence(A.nrows, rp.ctypes.data, c.ctypes.data, v.ctypes.data, m, s,
                                    Um.ctypes.data, s, Vm.ctypes.data, s, L, S.ctypes.data,
                                    W.ctypes.data if want_last else None)
        self._check(rc, "sequence")
        return (S, W) if want_last else S

    def canon(self, vals, m):
        v = np.ascontiguousarray(vals, dtype=np.int64)
        out = np.empty_like(v)
        self._check(self.L.oracle_canon(v.size, v.ctypes.data, m, out.ctypes.data), "canon")
        return out


_default = None
_omp = None


def get():
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def get_all_cores():
    """The oracle built with OpenMP: product rows split over every core (OMP_NUM_THREADS)."""
    global _omp
    if _omp is None:
        path = OMP_PATH if os.path.exists(OMP_PATH) and os.path.getmtime(OMP_PATH) >= os.path.getmtime(SRC) \
            else build(True, SRC, OMP_PATH, ("-fopenmp",))
        _omp = Oracle(path)
    return _omp
