"""GPU parity of block Wiedemann steps 2-3: the order basis (PM-Basis with M-Basis leaves) against
the oracle's one-order-at-a-time M-Basis bit for bit, and the rank from the generator against the
oracle's and the planted rank."""
import numpy as np
import pytest

import _brute as bf
import oracle
import synth
from oracle import sigma as osig

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M31 = 2**31 - 1


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("m,n,sig,shift_kind,p", [
    (2, 1, 1, "zero", 65521), (2, 1, 40, "zero", M31), (4, 2, 33, "gen", 65521), (16, 8, 31, "gen", M31),
    (16, 8, 32, "gen", M31), (16, 8, 33, "gen", 65521), (16, 8, 64, "zero", M31), (16, 8, 100, "gen", M31),
    (6, 3, 257, "rand", 65521), (16, 8, 300, "gen", M31), (5, 5, 70, "rand", 3), (16, 1, 90, "rand", 65521),
    (16, 8, 600, "gen", M31), (16, 8, 1100, "gen", 65521)])
def test_sigma_basis_matches_oracle(dev, m, n, sig, shift_kind, p):
    """Random series of every shape the entry point takes, orders around the leaf size (32) and
    across several levels of the recursion, zero / generator / random shifts, small and large p.
    Orders 600 and 1,100 reach the levels whose lengths come from the degrees read back (above 256)
    below ones queued with bound lengths, the small-product kernel with several output tiles and
    the tile kernel for A entries of more than 257 coefficients."""
    from paper_1004_3719_amd import sigma_basis
    G = synth.vector(m * 1000 + n * 10 + sig, 7, m * n * sig, 0, p - 1).reshape(m, n, sig)
    shift = {"zero": [0] * m, "gen": [0] * (m // 2) + [1] * (m - m // 2),
             "rand": list(synth.vector(sig, 8, m, 0, 5))}[shift_kind]
    print("[case] sigma basis", m, n, sig, shift_kind, p, flush=True)
    M, d = sigma_basis(torch.from_numpy(G.astype(np.int32)).to(dev), p, shift)
    Mo, do = osig.mbasis(G, sig, shift, p)
    assert d == do
    assert np.array_equal(M.cpu().numpy().astype(np.int64), Mo)


@pytest.mark.parametrize("threshold", [1, 40, 0])
@pytest.mark.parametrize("m,n,sig,shift_kind,p", [
    (16, 8, 300, "gen", M31), (16, 8, 257, "zero", 65521), (6, 3, 200, "rand", 3), (16, 1, 130, "rand", M31)])
def test_sigma_basis_ntt_products(dev, threshold, m, n, sig, shift_kind, p):
    """The polynomial-matrix products through the NTT over three primes with a CRT (the paper's DFT
    multiplication) at every level of the recursion (threshold 1), at the larger levels only (40), or
    none (0, schoolbook): the basis is the oracle's M-Basis bit for bit either way."""
    from paper_1004_3719_amd import sigma_basis
    from paper_1004_3719_amd.ffx import set_ntt_threshold
    G = synth.vector(m * 1000 + n * 10 + sig, 9, m * n * sig, 0, p - 1).reshape(m, n, sig)
    shift = {"zero": [0] * m, "gen": [0] * (m // 2) + [1] * (m - m // 2),
             "rand": list(synth.vector(sig, 10, m, 0, 5))}[shift_kind]
    print("[case] sigma basis ntt", threshold, m, n, sig, shift_kind, p, flush=True)
    set_ntt_threshold(threshold)
    try:
        M, d = sigma_basis(torch.from_numpy(G.astype(np.int32)).to(dev), p, shift)
    finally:
        set_ntt_threshold(1024)
    Mo, do = osig.mbasis(G, sig, shift, p)
    assert d == do
    assert np.array_equal(M.cpu().numpy().astype(np.int64), Mo)


def test_sigma_basis_rejects(dev):
    from paper_1004_3719_amd import sigma_basis
    G = torch.zeros((4, 2, 8), dtype=torch.int32, device=dev)
    for p in (65520, 1):  # not prime
        with pytest.raises(Exception):
            sigma_basis(G, p, [0] * 4)
    with pytest.raises(Exception):
        sigma_basis(torch.zeros((18, 9, 8), dtype=torch.int32, device=dev), 65521, [0] * 18)


@pytest.mark.parametrize("n,s,ndead,seed,p", [(40, 1, 3, 1, 65521), (60, 2, 5, 2, M31), (200, 4, 7, 3, M31),
                                              (300, 8, 12, 4, M31), (257, 3, 0, 5, 65521), (500, 8, 20, 6, 65521)])
def test_sequence_rank_small(dev, n, s, ndead, seed, p):
    """Rank from the oracle's sequence through the GPU steps 2-3 equals the oracle's rank (itself
    pinned to Gaussian elimination), with the same generator degrees; the GPU sequence of the same
    operands gives the same answer."""
    from paper_1004_3719_amd import Matrix, sequence_rank
    A = synth.c3(seed=seed, n=n, k=4, ndead=ndead, m=p)
    U = synth.vector(seed, 1, n * s, 0, p - 1).reshape(n, s)
    V = synth.vector(seed, 2, n * s, 0, p - 1).reshape(n, s)
    L = 2 * n // s + 3
    print("[case] rank", n, s, ndead, p, flush=True)
    So = oracle.get().sequence(A, U, V, L)
    want = osig.rank(So, p)
    _, dego = osig.generator(So, p)
    r, D, e, deg = sequence_rank(torch.from_numpy(So).to(dev), p)
    assert (r, D, e) == want and deg == dego
    M = Matrix.from_synth(A)
    Sg = M.sequence(torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev), L)
    assert sequence_rank(Sg, p)[:3] == want


@pytest.mark.parametrize("kind", ["zero", "rank1", "zero_s2"])
def test_sequence_rank_tiny(dev, kind):
    """Degenerate operands whose generator has degree at most 2 (the co-degree search must still
    run): the zero matrix (F = lambda for s = 1, rank 0) and a dense rank-1 matrix, against the
    oracle's rank and Gaussian elimination."""
    from paper_1004_3719_amd import Matrix, sequence_rank
    p = 65521
    n, s = (6, 2) if kind == "zero_s2" else (6, 1)
    if kind == "rank1":
        u = synth.vector(31, 1, n, 1, p - 1)
        v = synth.vector(31, 2, n, 1, p - 1)
        rp = np.arange(0, n * n + 1, n, dtype=np.int64)
        col = np.tile(np.arange(n, dtype=np.int32), n)
        val = (u[:, None] * v[None, :] % p).reshape(-1).astype(np.int64)
    else:
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(0, np.int32)
        val = np.zeros(0, np.int64)
    A = synth.Csr(n, n, rp, col, val, m=p, name=kind)
    want_rank = 1 if kind == "rank1" else 0
    U = synth.vector(32, 1, n * s, 0, p - 1).reshape(n, s)
    V = synth.vector(32, 2, n * s, 0, p - 1).reshape(n, s)
    L = 2 * n // s + 3
    print("[case] rank tiny", kind, flush=True)
    So = oracle.get().sequence(A, U, V, L)
    want = osig.rank(So, p)
    assert want[0] == want_rank
    assert sequence_rank(torch.from_numpy(So).to(dev), p)[:3] == want
    M = Matrix.from_synth(A)
    Sg = M.sequence(torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev), L)
    assert sequence_rank(Sg, p)[:3] == want


def test_c3_rank_full_size(dev):
    """The block-Wiedemann operand at full size (n = 200,000, 15 entries per row drawn from
    n - 1,000 live columns, m = 2^31 - 1, s = 8, L = 50,003): the GPU sequence and steps 2-3 give
    the planted rank n - 1,000, with one factor x per row of the generator (the 1,000 empty columns
    make 0 an eigenvalue of geometric multiplicity 1,000 >= s)."""
    from paper_1004_3719_amd import Matrix, sequence_rank
    A = synth.c3()
    U, V = synth.c3_blocks()
    L = synth.c3_length(A.nrows, 8)
    M = Matrix.from_synth(A)
    print("[case] c3 full rank", flush=True)
    S = M.sequence(torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev), L)
    r, D, e, deg = sequence_rank(S, A.m)
    assert r == A.nrows - 1000
    assert e == 8 and D == sum(deg)


@pytest.mark.parametrize("p", [M31, 65521])
@pytest.mark.parametrize("ntt", [1024, 0])
def test_sigma_basis_large_order(dev, p, ntt):
    """Order 3,000 (several levels of 1,024-coefficient product tiles): M G = 0 mod x^3000 at sampled
    coefficients computed here from the definition, every row within its degree bound, and the
    degrees rising by n per order in all (G of full rank)."""
    from paper_1004_3719_amd import sigma_basis
    m, n, sig = 16, 8, 3000
    G = synth.vector(p, 9, m * n * sig, 0, p - 1).reshape(m, n, sig)
    shift = [0] * 8 + [1] * 8
    print("[case] sigma basis large", p, ntt, flush=True)
    from paper_1004_3719_amd.ffx import set_ntt_threshold
    set_ntt_threshold(ntt)  # 1024: the top products through the NTT; 0: all schoolbook
    try:
        Mt, d = sigma_basis(torch.from_numpy(G.astype(np.int32)).to(dev), p, shift)
    finally:
        set_ntt_threshold(1024)
    M = Mt.cpu().numpy().astype(np.int64)
    assert sum(d) - sum(shift) == n * sig
    for i in range(m):
        assert not M[i, :, d[i] + 1:].any()
    # reduced: within the shifted degrees, with a nonsingular shifted leading coefficient matrix
    # (with the order condition and the degree sum, this makes M an order basis)
    assert bf.within_shifted_degrees(M, d, shift)
    assert bf.rank_mod_p(bf.shifted_leading_matrix(M, d, shift), p) == m
    for k in [0, 1, 31, 32, 33, 1023, 1024, 1500, 2047, 2048, 2999]:
        Grev = G[:, :, k::-1]  # G[.., k - j] for j = 0..k
        prod = (M[:, :, None, :k + 1] * Grev[None, :, :, :]) % p
        assert not (prod.sum(axis=(1, 3)) % p).any(), k


def _coeff_mod(M, G, k, p):
    """[x^k](M G) mod p exactly in int64: B split into 16-bit halves keeps every sum below 2^63."""
    m, n = M.shape[0], G.shape[1]
    out = np.zeros((m, n), np.int64)
    for q in range(M.shape[1]):
        A = M[:, q, :k + 1]
        B = G[q, :, k::-1][:, :A.shape[1]]
        lo = (A @ (B & 0xFFFF).T) % p
        hi = (A @ (B >> 16).T) % p
        out = (out + lo + hi * 65536 % p) % p
    return out


@pytest.mark.parametrize("p", [M31, 65521])
@pytest.mark.parametrize("ntt", [1024, 0])
def test_sigma_basis_order_40k(dev, p, ntt):
    """Order 40,000, where the top products of the recursion run on the four-coefficients-per-lane
    tiles: the order condition at sampled coefficients (computed here from the definition), the
    degree bounds and the total degree increase."""
    from paper_1004_3719_amd import sigma_basis
    m, n, sig = 16, 8, 40_000
    G = synth.vector(p + 1, 10, m * n * sig, 0, p - 1).reshape(m, n, sig)
    shift = [0] * 8 + [1] * 8
    print("[case] sigma basis 40k", p, ntt, flush=True)
    from paper_1004_3719_amd.ffx import set_ntt_threshold
    set_ntt_threshold(ntt)  # 1024: the top products through the NTT; 0: the four-per-lane schoolbook tiles
    try:
        Mt, d = sigma_basis(torch.from_numpy(G.astype(np.int32)).to(dev), p, shift)
    finally:
        set_ntt_threshold(1024)
    M = Mt.cpu().numpy().astype(np.int64)
    assert sum(d) - sum(shift) == n * sig
    top = max(d) + 1
    assert not M[:, :, top:].any()
    assert bf.within_shifted_degrees(M, d, shift)
    assert bf.rank_mod_p(bf.shifted_leading_matrix(M, d, shift), p) == m
    M = M[:, :, :top]
    for k in [0, 20_000, 20_001, 31_999, 39_999]:
        assert not _coeff_mod(M, G, k, p).any(), k
