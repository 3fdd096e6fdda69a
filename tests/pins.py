"""Pins of the oracle: checks against what the paper and the mathematics fix.

Each pin takes an oracle object (the real one, or a copy with a planted
mistake) and raises AssertionError on a mismatch. The pins are:
  * the paper's worked example (Section 2.4, "Base case: JIT");
  * dense brute force in Python integers on tiny random inputs, for every
    entry point, with raw values that are negative, zero, +-1 or near +-2^63;
  * invariants: adjointness, linearity, sequence shift symmetry and the
    Cayley-Hamilton recurrence of the projected sequence;
  * closed forms: identity, permutation, diagonal, nilpotent shift, the
    all-(m-1) worst case of the reduction bound and all-+-1 matrices.
"""
import json
import os

import numpy as np

import _brute as bf
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
MODULI = [2, 3, 27, 32749, 65521, 2**31 - 1]


def _eq(got, want, what):
    got = np.asarray(got, dtype=object).reshape(-1).tolist()
    want = np.asarray(want, dtype=object).reshape(-1).tolist()
    assert [int(v) for v in got] == [int(v) for v in want], what


def _vec(rng, rows, s, m):
    return rng.integers(0, m, size=(rows, s), dtype=np.int64)


def pin_worked_example(orc):
    g = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    D = g["A"]
    rp = np.array([0, 2, 3], dtype=np.int64)
    A = synth.Csr(2, 2, rp, np.array([0, 1, 1], np.int32), np.array([D[0][0], D[0][1], D[1][1]], np.int64))
    for case in g["cases"]:
        y = orc.spmv(A, case["x"], alpha=1, beta=1, y=case["y_in"], m=g["m"])
        _eq(y, case["y_out"], "worked example %s" % case)


def pin_spmv_brute(orc, seed=1):
    rng = np.random.default_rng(seed)
    for m in MODULI:
        for (r, c) in [(1, 1), (7, 5), (5, 9), (16, 16), (33, 20)]:
            A = bf.random_csr(rng, r, c, 0.35)
            x = _vec(rng, c, 1, m).reshape(-1)
            y = _vec(rng, r, 1, m).reshape(-1)
            a, b = int(rng.integers(0, m)), int(rng.integers(0, m))
            _eq(orc.spmv(A, x, a, b, y, m=m), bf.spmm(A, x, m, a, b, y), "spmv m=%d %dx%d" % (m, r, c))
            _eq(orc.spmv(A, x, 1, 0, None, m=m), bf.spmm(A, x, m), "apply m=%d" % m)


def pin_spmv_t_brute(orc, seed=2):
    rng = np.random.default_rng(seed)
    for m in MODULI:
        for (r, c) in [(1, 3), (6, 4), (4, 11), (20, 20)]:
            A = bf.random_csr(rng, r, c, 0.4)
            x = _vec(rng, r, 1, m).reshape(-1)
            y = _vec(rng, c, 1, m).reshape(-1)
            a, b = int(rng.integers(0, m)), int(rng.integers(0, m))
            _eq(orc.spmv_t(A, x, a, b, y, m=m), bf.spmm_t(A, x, m, a, b, y), "spmv_t m=%d" % m)


def pin_spmm_brute(orc, seed=3):
    rng = np.random.default_rng(seed)
    for m in [3, 65521, 2**31 - 1]:
        for s in [1, 2, 3, 8, 16]:
            A = bf.random_csr(rng, 9, 7, 0.4)
            X = _vec(rng, 7, s, m)
            Y = _vec(rng, 9, s, m)
            a, b = int(rng.integers(0, m)), int(rng.integers(0, m))
            _eq(orc.spmm(A, X, a, b, Y, m=m), bf.spmm(A, X, m, a, b, Y), "spmm m=%d s=%d" % (m, s))
            Xt = _vec(rng, 9, s, m)
            Yt = _vec(rng, 7, s, m)
            _eq(orc.spmm_t(A, Xt, a, b, Yt, m=m), bf.spmm_t(A, Xt, m, a, b, Yt), "spmm_t m=%d s=%d" % (m, s))


def pin_power_brute(orc, seed=4):
    rng = np.random.default_rng(seed)
    for m in [2, 27, 65521, 2**31 - 1]:
        A = bf.random_csr(rng, 12, 12, 0.3)
        V = _vec(rng, 12, 3, m)
        for k in [0, 1, 2, 5]:
            _eq(orc.power(A, k, V, m=m), bf.power(A, k, V, m), "power m=%d k=%d" % (m, k))


def pin_sequence_brute(orc, seed=5):
    rng = np.random.default_rng(seed)
    for m in [3, 32749, 2**31 - 1]:
        for s in [1, 2, 4]:
            n = 10
            A = bf.random_csr(rng, n, n, 0.3)
            U, V = _vec(rng, n, s, m), _vec(rng, n, s, m)
            L = 2 * n // s + 3
            S, W = orc.sequence(A, U, V, L, m=m, want_last=True)
            want = bf.sequence(A, U, V, L + 1, m)
            for i in range(L):
                _eq(S[i], want[i], "sequence m=%d s=%d i=%d" % (m, s, i))
            _eq(W, bf.power(A, L, V, m), "sequence last block m=%d" % m)


def _c1_small(m, seed=7, n=300, k=6):
    s = synth.spec(n, n, seed, len_kind=synth.LEN_FIXED, len_a=k, col_kind=synth.COL_UNIFORM,
                   p_pm1=0.3, val_lo=-(2**40), val_hi=2**40)
    A = synth.rows(s)
    A.m = m
    return A


def pin_adjoint(orc, seed=6):
    """y . (A x) = (A^T y) . x (mod m)."""
    rng = np.random.default_rng(seed)
    for m in [65521, 2**31 - 1]:
        A = _c1_small(m)
        x, y = _vec(rng, A.ncols, 1, m).reshape(-1), _vec(rng, A.nrows, 1, m).reshape(-1)
        Ax = orc.spmv(A, x, m=m)
        Aty = orc.spmv_t(A, y, m=m)
        lhs = sum(int(a) * int(b) for a, b in zip(y, Ax)) % m
        rhs = sum(int(a) * int(b) for a, b in zip(Aty, x)) % m
        assert lhs == rhs, "adjoint m=%d" % m


def pin_linearity(orc, seed=8):
    """A(a x + b z) = a A x + b A z, and the alpha/beta form is that combination."""
    rng = np.random.default_rng(seed)
    for m in [32749, 2**31 - 1]:
        A = _c1_small(m, seed=9)
        x, z = _vec(rng, A.ncols, 1, m).reshape(-1), _vec(rng, A.ncols, 1, m).reshape(-1)
        a, b = int(rng.integers(1, m)), int(rng.integers(1, m))
        comb = np.array([(a * int(u) + b * int(v)) % m for u, v in zip(x, z)], dtype=np.int64)
        lhs = orc.spmv(A, comb, m=m)
        Ax, Az = orc.spmv(A, x, m=m), orc.spmv(A, z, m=m)
        rhs = [(a * int(u) + b * int(v)) % m for u, v in zip(Ax, Az)]
        _eq(lhs, rhs, "linearity m=%d" % m)
        y = _vec(rng, A.nrows, 1, m).reshape(-1)
        _eq(orc.spmv(A, x, a, b, y, m=m), [(a * int(u) + b * int(v)) % m for u, v in zip(Ax, y)],
            "alpha/beta m=%d" % m)


def pin_sequence_shift(orc, seed=10):
    """S_{i+j} = ((A^T)^i U)^T (A^j V)."""
    rng = np.random.default_rng(seed)
    m, s = 65521, 3
    A = _c1_small(m, seed=11, n=120, k=5)
    U, V = _vec(rng, A.nrows, s, m), _vec(rng, A.nrows, s, m)
    S = orc.sequence(A, U, V, 9, m=m)
    for i, j in [(0, 3), (2, 2), (3, 5), (1, 0)]:
        Ui = U.copy()
        for _ in range(i):
            Ui = orc.spmm_t(A, Ui, m=m)
        Vj = orc.power(A, j, V, m=m)
        want = [[sum(int(Ui[k, a]) * int(Vj[k, b]) for k in range(A.nrows)) % m for b in range(s)]
                for a in range(s)]
        _eq(S[i + j], want, "shift i=%d j=%d" % (i, j))


def pin_cayley_hamilton(orc, seed=12):
    """sum_k c_k S_{i+k} = 0 for the characteristic polynomial c of A (checked first by c(A) = 0)."""
    rng = np.random.default_rng(seed)
    for p in [32749, 65521]:
        n, s = 14, 2
        A = bf.random_csr(rng, n, n, 0.3, dup=False)
        D = bf.mod(bf.dense(A), p)
        c = bf.charpoly(D, p)
        assert all(v == 0 for row in bf.poly_at_matrix(c, D, p) for v in row), "charpoly"
        U, V = _vec(rng, n, s, p), _vec(rng, n, s, p)
        S = orc.sequence(A, U, V, 2 * n + 2, m=p)
        for i in range(0, n + 2):
            acc = sum(c[k] * S[i + k].astype(object) for k in range(n + 1))
            assert all(int(v) % p == 0 for v in np.asarray(acc).reshape(-1)), "Cayley-Hamilton p=%d i=%d" % (p, i)


def _from_dense_pattern(rows, ncols, vals):
    rp = np.zeros(len(rows) + 1, np.int64)
    for i, r in enumerate(rows):
        rp[i + 1] = rp[i] + len(r)
    col = np.array([c for r in rows for c in r], np.int32)
    return synth.Csr(len(rows), ncols, rp, col, np.asarray(vals, np.int64))


def pin_closed_forms(orc, seed=13):
    rng = np.random.default_rng(seed)
    n = 40
    for m in [2, 65521, 2**31 - 1]:
        x = _vec(rng, n, 1, m).reshape(-1)
        y0 = _vec(rng, n, 1, m).reshape(-1)
        # identity: y = alpha x + beta y0, S_i = U^T V for all i
        I = _from_dense_pattern([[i] for i in range(n)], n, np.ones(n))
        a, b = int(rng.integers(0, m)), int(rng.integers(0, m))
        _eq(orc.spmv(I, x, a, b, y0, m=m), [(a * int(u) + b * int(v)) % m for u, v in zip(x, y0)], "identity")
        U, V = _vec(rng, n, 2, m), _vec(rng, n, 2, m)
        UtV = [[sum(int(U[k, p]) * int(V[k, q]) for k in range(n)) % m for q in range(2)] for p in range(2)]
        for Si in orc.sequence(I, U, V, 4, m=m):
            _eq(Si, UtV, "identity sequence")
        # permutation: y[i] = x[perm[i]]; transpose applies the inverse
        perm = rng.permutation(n)
        P = _from_dense_pattern([[int(perm[i])] for i in range(n)], n, np.ones(n))
        _eq(orc.spmv(P, x, m=m), x[perm], "permutation")
        inv = np.empty(n, int)
        inv[perm] = np.arange(n)
        _eq(orc.spmv_t(P, x, m=m), x[inv], "permutation transpose")
        # diagonal: S_i = U^T D^i V
        d = _vec(rng, n, 1, m).reshape(-1)
        Dm = _from_dense_pattern([[i] for i in range(n)], n, d)
        S = orc.sequence(Dm, U, V, 5, m=m)
        for i in range(5):
            want = [[sum(int(U[k, p]) * pow(int(d[k]), i, m) * int(V[k, q]) for k in range(n)) % m
                     for q in range(2)] for p in range(2)]
            _eq(S[i], want, "diagonal sequence i=%d" % i)
        # nilpotent shift (row i has a 1 at column i+1): A^i = 0 for i >= n
        N = _from_dense_pattern([[i + 1] if i + 1 < n else [] for i in range(n)], n, np.ones(n - 1))
        S = orc.sequence(N, U, V, n + 3, m=m)
        assert all(int(v) == 0 for v in S[n:].reshape(-1)), "nilpotent tail"
        _eq(orc.spmv(N, x, m=m), list(x[1:]) + [0], "shift")
        # worst case of the reduction bound: every value and x entry is m-1, so each product is 1
        lens = rng.integers(0, 30, size=n)
        rows = [sorted(rng.choice(n, size=int(L), replace=False).tolist()) for L in lens]
        W = _from_dense_pattern(rows, n, np.full(int(lens.sum()), m - 1))
        _eq(orc.spmv(W, np.full(n, m - 1), m=m), [int(L) % m for L in lens], "all m-1")
        # all +-1 with x = 1: y = (#plus - #minus) mod m
        signs = rng.choice([-1, 1], size=int(lens.sum()))
        Pm = _from_dense_pattern(rows, n, signs)
        want, k = [], 0
        for L in lens:
            want.append(int(signs[k:k + int(L)].sum()) % m)
            k += int(L)
        _eq(orc.spmv(Pm, np.ones(n, np.int64), m=m), want, "all +-1")


def pin_rejects(orc):
    A = _from_dense_pattern([[0], [1]], 2, [1, 1])
    for bad in [lambda: orc.spmv(A, [0, 1], m=1), lambda: orc.spmv(A, [0, 5], m=5),
                lambda: orc.spmv(A, [0, -1], m=5), lambda: orc.spmv(A, [0, 1], alpha=5, m=5),
                lambda: orc.spmv(_from_dense_pattern([[2]], 2, [1]), [0, 1], m=5),
                lambda: orc.spmv(A, [0, 1], m=2**31)]:
        try:
            bad()
        except ValueError:
            continue
        raise AssertionError("bad argument accepted")


ALL_PINS = [pin_worked_example, pin_spmv_brute, pin_spmv_t_brute, pin_spmm_brute, pin_power_brute,
            pin_sequence_brute, pin_adjoint, pin_linearity, pin_sequence_shift, pin_cayley_hamilton,
            pin_closed_forms, pin_rejects]
