"""Dense brute force in Python integers (arbitrary precision), for tiny inputs.

Independent of the oracle: matrices are expanded to dense lists of Python
ints with raw (unreduced) values, products are exact, and a single `% m`
(Python's, always in [0, m-1] for m > 0) is taken at the very end. Used to
pin the oracle, never the other way round.
"""
import numpy as np

import synth


def dense(A):
    """Dense raw matrix (list of lists of Python ints); duplicate coordinates add."""
    D = [[0] * A.ncols for _ in range(A.nrows)]
    rp = [int(v) for v in A.rowptr]
    for i in range(A.nrows):
        for k in range(rp[i] - rp[0], rp[i + 1] - rp[0]):
            D[i][int(A.col[k])] += int(A.val[k])
    return D


def transpose(D, ncols):
    return [[D[i][j] for i in range(len(D))] for j in range(ncols)]


def matmul(P, Q):
    """P (r x t) times Q (t x c), exact."""
    t = len(Q)
    c = len(Q[0]) if t else 0
    return [[sum(P[i][k] * Q[k][j] for k in range(t)) for j in range(c)] for i in range(len(P))]


def mod(P, m):
    return [[v % m for v in row] for row in P]


def as_rows(v, rows, s):
    v = np.asarray(v, dtype=object).reshape(rows, s)
    return [[int(v[i, b]) for b in range(s)] for i in range(rows)]


def spmm(A, X, m, alpha=1, beta=0, Y=None):
    D = dense(A)
    s = 1 if np.ndim(X) == 1 else np.shape(X)[1]
    Xl = as_rows(X, A.ncols, s)
    Yl = as_rows(np.zeros(A.nrows * s, dtype=np.int64) if Y is None else Y, A.nrows, s)
    P = matmul(D, Xl)
    return [[(alpha * P[i][b] + beta * Yl[i][b]) % m for b in range(s)] for i in range(A.nrows)]


def spmm_t(A, X, m, alpha=1, beta=0, Y=None):
    Dt = transpose(dense(A), A.ncols)
    s = 1 if np.ndim(X) == 1 else np.shape(X)[1]
    Xl = as_rows(X, A.nrows, s)
    Yl = as_rows(np.zeros(A.ncols * s, dtype=np.int64) if Y is None else Y, A.ncols, s)
    P = matmul(Dt, Xl)
    return [[(alpha * P[j][b] + beta * Yl[j][b]) % m for b in range(s)] for j in range(A.ncols)]


def power(A, k, V, m):
    D = mod(dense(A), m)
    s = np.shape(V)[1]
    W = as_rows(V, A.nrows, s)
    for _ in range(k):
        W = mod(matmul(D, W), m)
    return W


def sequence(A, U, V, L, m):
    """[U^T A^i V mod m for i < L], each s x s, computed with dense powers."""
    D = mod(dense(A), m)
    s = np.shape(U)[1]
    Ul = as_rows(U, A.nrows, s)
    Ut = transpose(Ul, s)
    W = as_rows(V, A.nrows, s)
    out = []
    for _ in range(L):
        out.append(mod(matmul(Ut, W), m))
        W = mod(matmul(D, W), m)
    return out


def charpoly(D, p):
    """Characteristic polynomial coefficients c[0..n] (c[n] = 1) of the square matrix D over
    Z/pZ, p prime > n, by the Faddeev-LeVerrier recurrence."""
    n = len(D)
    D = mod(D, p)
    c = [0] * (n + 1)
    c[n] = 1
    M = [[0] * n for _ in range(n)]
    for k in range(1, n + 1):
        AM = matmul(D, M) if k > 1 else [[0] * n for _ in range(n)]
        M = [[(AM[i][j] + (c[n - k + 1] if i == j else 0)) % p for j in range(n)] for i in range(n)]
        AM = matmul(D, M)
        tr = sum(AM[i][i] for i in range(n)) % p
        c[n - k] = (-tr * pow(k, p - 2, p)) % p
    return c


def poly_at_matrix(c, D, p):
    n = len(D)
    R = [[0] * n for _ in range(n)]
    P = [[int(i == j) for j in range(n)] for i in range(n)]
    for k in range(len(c)):
        R = [[(R[i][j] + c[k] * P[i][j]) % p for j in range(n)] for i in range(n)]
        P = mod(matmul(D, P), p)
    return R


def random_csr(rng, nrows, ncols, density, raw="mixed", dup=True, empty_rows=True):
    """A tiny random CSR with unreduced values (negative, huge, zero, +-1), optional duplicates."""
    rows = []
    for i in range(nrows):
        if empty_rows and rng.random() < 0.15:
            rows.append([])
            continue
        k = int(rng.binomial(ncols, density)) if ncols else 0
        cols = sorted(rng.choice(ncols, size=min(k, ncols), replace=False).tolist()) if k else []
        if dup and cols and rng.random() < 0.3:
            cols.append(cols[int(rng.integers(len(cols)))])
            rng.shuffle(cols)
        rows.append(cols)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    for i, r in enumerate(rows):
        rp[i + 1] = rp[i] + len(r)
    col = np.array([c for r in rows for c in r], dtype=np.int32)
    nnz = len(col)
    if raw == "mixed":
        kinds = rng.integers(0, 6, size=nnz)
        v = rng.integers(-(2**62), 2**62, size=nnz, dtype=np.int64)
        v = np.where(kinds == 0, 1, v)
        v = np.where(kinds == 1, -1, v)
        v = np.where(kinds == 2, rng.integers(-100, 100, size=nnz), v)
        v = np.where(kinds == 3, 0, v)
        ext = rng.integers(0, 4, size=nnz)
        v = np.where((kinds == 4) & (ext == 0), np.iinfo(np.int64).min, v)
        v = np.where((kinds == 4) & (ext == 1), np.iinfo(np.int64).max, v)
        val = v.astype(np.int64)
    else:
        val = rng.integers(raw[0], raw[1] + 1, size=nnz, dtype=np.int64)
    return synth.Csr(nrows, ncols, rp, col, val)


def rank_mod_p(D, p):
    """Rank of a matrix of Python ints over the prime field F_p, by Gauss-Jordan elimination."""
    A = [[int(v) % p for v in row] for row in D]
    rows, cols = len(A), len(A[0]) if A else 0
    r = 0
    for c in range(cols):
        piv = next((i for i in range(r, rows) if A[i][c]), None)
        if piv is None:
            continue
        A[r], A[piv] = A[piv], A[r]
        inv = pow(A[r][c], p - 2, p)
        A[r] = [v * inv % p for v in A[r]]
        for i in range(rows):
            if i != r and A[i][c]:
                f = A[i][c]
                A[i] = [(a - f * b) % p for a, b in zip(A[i], A[r])]
        r += 1
    return r


def shifted_leading_matrix(M, d, shift):
    """Leading coefficient matrix of a polynomial matrix M (rows x cols x coefficients) with respect
    to the shifted row degrees d: entry (i, j) is the coefficient of x^(d_i - shift_j) in M[i][j]
    (0 when that exponent is negative or beyond the stored coefficients). M is reduced with respect
    to the shift, with shifted row degrees d, exactly when every row stays within d and this matrix
    is nonsingular."""
    rows, cols, ln = M.shape
    out = [[0] * cols for _ in range(rows)]
    for i in range(rows):
        for j in range(cols):
            e = int(d[i]) - int(shift[j])
            if 0 <= e < ln:
                out[i][j] = int(M[i, j, e])
    return out


def within_shifted_degrees(M, d, shift):
    """Every entry M[i][j] has degree at most d_i - shift_j (the zero polynomial counts)."""
    rows, cols, ln = M.shape
    for i in range(rows):
        for j in range(cols):
            top = int(d[i]) - int(shift[j])
            if top < 0:
                if M[i, j].any():
                    return False
            elif top + 1 < ln and M[i, j, top + 1:].any():
                return False
    return True
