"""ORACLE -- test infrastructure only: block Wiedemann steps 2 and 3 over a prime field.

Plain numpy (int64, every product reduced at once) for small orders. Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

* ``mbasis``: an order basis (sigma-basis) of an m x n power series G, computed
  one order at a time (the M-Basis algorithm of Giorgi, Jeannerod and Villard,
  ISSAC 2003, on which the paper's PM-Basis rests, Section 3.2): at order k the
  residual coefficient Delta = [x^k](M G) is put in echelon form taking the
  rows by increasing shifted degree (ties by index); every row is reduced by
  the pivot rows before it, and each row that keeps a nonzero residual becomes
  a pivot and is multiplied by x (its shifted degree grows by one). After sigma
  orders, M G = 0 mod x^sigma and M is reduced with respect to the degrees.
* ``generator``: a minimal left matrix generator of the sequence S_i (Section
  3, step 2) from the order basis of [S(x); -I] with shifts 0 on the first s
  rows and 1 on the last s: a row [a, b] then has shifted degree
  max(deg a, deg b + 1), so for the rows of a generator in reversed form
  (a S = b mod x^L with deg b < deg F) it is the generator's degree. The s rows
  of smallest shifted degree give the generator.
* ``rank``: Section 3, step 3: rank = deg det F - codeg det F for the
  generator F, the degree of the determinant being the sum of the row degrees
  (the basis is row reduced) and the co-degree its x-adic valuation.
"""
import numpy as np


def _inv(a, p):
    return pow(int(a) % p, p - 2, p)


def mbasis(G, sigma, shift, p):
    """Order basis of G (m x n x >= sigma coefficients, residues mod the prime p) to order sigma
    with the given shifted degrees. Returns (M, d): M is m x m x (sigma + 1), d the final shifted
    degrees."""
    G = np.asarray(G, np.int64) % p
    m, n = G.shape[0], G.shape[1]
    M = np.zeros((m, m, sigma + 1), np.int64)
    for i in range(m):
        M[i, i, 0] = 1
    d = [int(v) for v in shift]
    for k in range(sigma):
        # residual coefficient [x^k](M G)
        delta = np.zeros((m, n), np.int64)
        for j in range(k + 1):
            delta = (delta + ((M[:, :, j][:, :, None] * G[None, :, :, k - j]) % p).sum(axis=1)) % p
        order = sorted(range(m), key=lambda i: (d[i], i))
        pivots = []  # (row, column) in the order they were found
        for i in order:
            for (r, c) in pivots:
                if delta[i, c]:
                    f = delta[i, c] * _inv(delta[r, c], p) % p
                    delta[i] = (delta[i] - f * delta[r]) % p
                    M[i] = (M[i] - f * M[r]) % p
            nz = np.nonzero(delta[i])[0]
            if len(nz):
                pivots.append((i, int(nz[0])))
        for (r, _) in pivots:
            M[r, :, 1:] = M[r, :, :-1].copy()
            M[r, :, 0] = 0
            d[r] += 1
    return M, d


def sequence_series(S, p):
    """[S(x); -I] as a 2s x s x L power series from the L terms S_i (L x s x s)."""
    S = np.asarray(S, np.int64) % p
    L, s = S.shape[0], S.shape[1]
    G = np.zeros((2 * s, s, L), np.int64)
    G[:s] = np.transpose(S, (1, 2, 0))
    for i in range(s):
        G[s + i, i, 0] = p - 1
    return G


def generator(S, p):
    """Minimal left generator of S_0..S_{L-1}: (Frev, deg) with Frev s x s x (max deg + 1) the
    generator in reversed form (row i of F(lambda) is lambda^deg[i] Frev_i(1/lambda)) and deg
    its row degrees."""
    S = np.asarray(S, np.int64)
    L, s = S.shape[0], S.shape[1]
    M, d = mbasis(sequence_series(S, p), L, [0] * s + [1] * s, p)
    rows = sorted(range(2 * s), key=lambda i: (d[i], i))[:s]
    deg = [d[i] for i in rows]
    top = max(deg) + 1
    return M[rows, :s, :top].copy(), deg


def det_valuation(F, p, K=8):
    """x-adic valuation of det F for a square polynomial matrix F (s x s x len) over F_p, by
    Gaussian elimination over the truncated power series F_p[[x]]/x^K, K doubling until the
    determinant is nonzero mod x^K. det F is a polynomial of degree at most s * (len - 1), so once
    K exceeds that degree a determinant that vanishes mod x^K is zero: None (F singular)."""
    s = F.shape[0]
    limit = s * max(F.shape[2] - 1, 0) + 1
    while True:
        A = np.zeros((s, s, K), np.int64)
        t = min(K, F.shape[2])
        A[:, :, :t] = F[:, :, :t] % p
        val, ok = 0, True
        for c in range(s):
            # pivot: the entry of column c (rows c..) of least valuation
            best, bv = -1, K
            for r in range(c, s):
                nz = np.nonzero(A[r, c])[0]
                if len(nz) and nz[0] < bv:
                    best, bv = r, int(nz[0])
            if best < 0:
                ok = False
                break
            if best != c:
                A[[c, best]] = A[[best, c]]
            val += bv
            # A[c, c] = x^bv * u with u a unit; eliminate below: row_r -= (A[r,c] / A[c,c]) row_c,
            # where A[r,c] has valuation >= bv so the quotient is a power series
            u = np.zeros(K, np.int64)
            u[:K - bv] = A[c, c, bv:]
            uinv = _series_inv(u, p, K)
            for r in range(c + 1, s):
                q = np.zeros(K, np.int64)
                q[:K - bv] = A[r, c, bv:]
                f = _series_mul(q, uinv, p, K)
                for cc in range(c, s):
                    A[r, cc] = (A[r, cc] - _series_mul(f, A[c, cc], p, K)) % p
        if ok and val < K:
            return val
        if K >= limit:
            return None
        K *= 2


def _series_mul(a, b, p, K):
    out = np.zeros(K, np.int64)
    for i in np.nonzero(a)[0]:
        out[i:] = (out[i:] + a[i] * b[:K - i]) % p
    return out


def _series_inv(u, p, K):
    inv0 = _inv(u[0], p)
    out = np.zeros(K, np.int64)
    out[0] = inv0
    for k in range(1, K):
        acc = sum(int(u[j]) * int(out[k - j]) for j in range(1, k + 1)) % p
        out[k] = (-acc * inv0) % p
    return out


def rank(S, p):
    """Section 3, step 3: (rank, deg det F, codeg det F) from the sequence S (L x s x s)."""
    Frev, deg = generator(S, p)
    s = Frev.shape[0]
    # F(lambda): row i reversed to its degree
    F = np.zeros((s, s, max(deg) + 1), np.int64)
    for i in range(s):
        F[i, :, :deg[i] + 1] = Frev[i, :, :deg[i] + 1][:, ::-1]
    D = int(sum(deg))
    e = det_valuation(F, p)
    return D - e, D, e
