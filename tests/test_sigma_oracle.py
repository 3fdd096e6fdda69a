"""Pins of the block-Wiedemann oracle (oracle/sigma.py) against definitions and textbook routines
written here on their own: the order condition M G = 0 mod x^sigma by direct convolution,
Berlekamp-Massey for one vector (s = 1), the generator identity sum_k F_k S_{t+k} = 0, the
determinant valuation by cofactor expansion, and the rank by Gaussian elimination over F_p."""
import itertools

import numpy as np
import pytest

import _brute as bf
import oracle
import synth
from oracle import sigma

P = 65521


def conv_coeff(M, G, k, p):
    """[x^k] of M(x) G(x), by the definition."""
    m, n = M.shape[0], G.shape[1]
    out = np.zeros((m, n), dtype=object)
    for j in range(k + 1):
        if j < M.shape[2] and k - j < G.shape[2]:
            out = out + M[:, :, j].astype(object).dot(G[:, :, k - j].astype(object))
    return np.vectorize(lambda v: int(v) % p)(out)


def gauss_rank(D, p):
    A = [list(map(int, r)) for r in D]
    rows, cols = len(A), len(A[0]) if A else 0
    r = 0
    for c in range(cols):
        piv = next((i for i in range(r, rows) if A[i][c] % p), None)
        if piv is None:
            continue
        A[r], A[piv] = A[piv], A[r]
        inv = pow(A[r][c], p - 2, p)
        A[r] = [v * inv % p for v in A[r]]
        for i in range(rows):
            if i != r and A[i][c] % p:
                f = A[i][c]
                A[i] = [(a - f * b) % p for a, b in zip(A[i], A[r])]
        r += 1
    return r


def dense(A):
    D = np.zeros((A.nrows, A.ncols), np.int64)
    for i in range(A.nrows):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            D[i, A.col[k]] = (D[i, A.col[k]] + A.val[k]) % A.m
    return D


def berlekamp_massey(a, p):
    """Connection polynomial C (C[0] = 1) of least degree L with sum_k C[k] a[i-k] = 0 for i >= L."""
    C, B = [1], [1]
    L, mgap, b = 0, 1, 1
    for i in range(len(a)):
        d = a[i]
        for k in range(1, L + 1):
            d = (d + C[k] * a[i - k]) % p
        if d == 0:
            mgap += 1
            continue
        coef = d * pow(b, p - 2, p) % p
        T = list(C)
        C = C + [0] * max(0, len(B) + mgap - len(C))
        for k in range(len(B)):
            C[k + mgap] = (C[k + mgap] - coef * B[k]) % p
        if 2 * L <= i:
            L, B, b, mgap = i + 1 - L, T, d, 1
        else:
            mgap += 1
    return C[:L + 1] + [0] * max(0, L + 1 - len(C)), L


def c3_case(n, s, ndead, seed, p=P):
    A = synth.c3(seed=seed, n=n, k=4, ndead=ndead, m=p)
    U = synth.vector(seed, 1, n * s, 0, p - 1).reshape(n, s)
    V = synth.vector(seed, 2, n * s, 0, p - 1).reshape(n, s)
    return A, U, V


@pytest.mark.parametrize("m,n,sigma_,shift", [(2, 1, 9, [0, 0]), (4, 2, 17, [0, 0, 1, 1]), (6, 3, 12, [2, 0, 1, 0, 3, 1]),
                                              (16, 8, 6, [0] * 8 + [1] * 8)])
def test_order_condition(m, n, sigma_, shift):
    """M G = 0 mod x^sigma, M has m rows of shifted degree d, and it is a basis: det M is
    c x^(sum of degree increases) (the increases add up to n * sigma for a G of full rank)."""
    G = synth.vector(m * 7 + n, 3, m * n * sigma_, 0, P - 1).reshape(m, n, sigma_)
    M, d = sigma.mbasis(G, sigma_, shift, P)
    for k in range(sigma_):
        assert not conv_coeff(M, G, k, P).any(), k
    assert sum(d) - sum(shift) == n * sigma_
    # row i of M has degree at most d_i - min(shift)
    for i in range(m):
        nz = np.nonzero(M[i].any(axis=0))[0]
        assert nz.max() <= d[i] - min(shift)
    # reduced with respect to the shift: entries within the shifted degrees and a nonsingular
    # shifted leading coefficient matrix
    assert bf.within_shifted_degrees(M, d, shift)
    assert bf.rank_mod_p(bf.shifted_leading_matrix(M, d, shift), P) == m


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_scalar_generator_is_berlekamp_massey(seed):
    """One vector (s = 1): the generator is the minimal polynomial of the scalar sequence
    u^T A^i v, as Berlekamp-Massey finds it (reversed and made monic)."""
    n = 30
    A, U, V = c3_case(n, 1, 2, seed)
    L = 2 * n + 3
    S = oracle.get().sequence(A, U, V, L) % P
    a = [int(S[i, 0, 0]) for i in range(L)]
    Cbm, Lbm = berlekamp_massey(a, P)
    Frev, deg = sigma.generator(S, P)
    assert deg[0] == Lbm
    f = [int(v) for v in Frev[0, 0, :deg[0] + 1]]  # reversed generator: f(x) = x^deg F(1/x)
    inv = pow(f[0], P - 2, P)
    assert [v * inv % P for v in f] == Cbm


@pytest.mark.parametrize("n,s,ndead,seed", [(40, 1, 3, 1), (60, 2, 5, 2), (80, 4, 7, 3), (120, 4, 10, 4),
                                            (90, 3, 0, 5), (64, 8, 6, 6)])
def test_generator_and_rank(n, s, ndead, seed):
    """The generator F annihilates the sequence (sum_k F_k S_{t+k} = 0 for every t that fits), its
    reversed form has a nonsingular constant term (so deg det F is the sum of the row degrees),
    and deg det F - codeg det F is the rank found by Gaussian elimination."""
    A, U, V = c3_case(n, s, ndead, seed)
    L = 2 * n // s + 3
    S = oracle.get().sequence(A, U, V, L) % P
    Frev, deg = sigma.generator(S, P)
    for i in range(s):
        for t in range(L - deg[i]):
            acc = np.zeros(s, dtype=object)
            for k in range(deg[i] + 1):
                acc = acc + Frev[i, :, deg[i] - k].astype(object).dot(S[t + k].astype(object))
            assert all(int(v) % P == 0 for v in acc), (i, t)
    assert gauss_rank(Frev[:, :, 0], P) == s
    r, D, e = sigma.rank(S, P)
    assert D == sum(deg)
    assert r == gauss_rank(dense(A), P)


def _poly_det(F, p):
    """det of a small polynomial matrix by cofactor expansion (Leibniz), coefficients as lists."""
    s = F.shape[0]

    def pmul(a, b):
        out = [0] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                out[i + j] = (out[i + j] + x * y) % p
        return out

    total = [0]
    for perm in itertools.permutations(range(s)):
        sign = 1
        for i in range(s):
            for j in range(i + 1, s):
                if perm[i] > perm[j]:
                    sign = -sign
        term = [1]
        for i in range(s):
            term = pmul(term, [int(v) for v in F[i, perm[i]]])
        if len(term) > len(total):
            total = total + [0] * (len(term) - len(total))
        for k, v in enumerate(term):
            total[k] = (total[k] + sign * v) % p
    return total


@pytest.mark.parametrize("seed", range(6))
def test_det_valuation_brute(seed):
    """x-adic valuation of det F against the determinant expanded in full, on small matrices with
    factors of x planted in rows and columns."""
    s, ln = 3, 5
    F = synth.vector(100 + seed, 1, s * s * ln, 0, P - 1).reshape(s, s, ln)
    F[0, :, :2] = 0         # row 0 divisible by x^2
    F[:, 1, 0] = 0          # column 1 divisible by x
    if seed % 2:
        F[2] = (F[0] * 3 + F[1]) % P  # singular
    det = _poly_det(F, P)
    nz = [k for k, v in enumerate(det) if v]
    want = nz[0] if nz else None
    assert (want is None) == bool(seed % 2)
    assert sigma.det_valuation(F, P, K=4) == want


def test_reducedness_check_rejects_degenerate():
    """The reducedness check that the order-basis tests apply fails a degenerate basis with the
    right degrees (all zero, or one row a multiple of another) and passes the oracle's."""
    m, n, sig, shift = 4, 2, 9, [0, 0, 1, 1]
    G = synth.vector(77, 3, m * n * sig, 0, P - 1).reshape(m, n, sig)
    M, d = sigma.mbasis(G, sig, shift, P)
    assert bf.rank_mod_p(bf.shifted_leading_matrix(M, d, shift), P) == m
    Z = np.zeros_like(M)
    assert bf.rank_mod_p(bf.shifted_leading_matrix(Z, d, shift), P) < m
    D = M.copy()
    i, j = sorted(range(m), key=lambda r: d[r])[:2]
    D[j] = 0
    D[j, :, d[j] - d[i]:] = M[i, :, :M.shape[2] - (d[j] - d[i])]  # row j = x^(d_j - d_i) row i
    assert bf.within_shifted_degrees(D, d, shift)
    assert bf.rank_mod_p(bf.shifted_leading_matrix(D, d, shift), P) < m
