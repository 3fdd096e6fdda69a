"""The seeded generators: determinism, row-range independence and the workload shapes."""
import numpy as np

import synth


def test_splitmix_reference_values():
    # splitmix64 with state 0 and gamma 0x9E3779B97F4A7C15: the first outputs are the published
    # test vector of the generator (seed 0): e220a8397b1dcdaf, 6e789e6aa1b965f4, 06c45d188009454f
    r = synth.raw(0, 3)
    assert [int(v) for v in r] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_deterministic_and_row_ranges():
    s = synth.c2_spec(n=50_000)
    A = synth.rows(s)
    B = synth.rows(s)
    assert np.array_equal(A.rowptr, B.rowptr) and np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)
    P = synth.rows(s, 12_345, 23_456)
    k0, k1 = A.rowptr[12_345], A.rowptr[23_456]
    assert np.array_equal(P.col, A.col[k0:k1]) and np.array_equal(P.val, A.val[k0:k1])
    assert np.array_equal(P.rowptr, A.rowptr[12_345:23_457] - k0)


def test_rows_sorted_distinct_in_range():
    for A in [synth.c1(), synth.c2(n=20_000), synth.c3(n=5_000, ndead=50), synth.c4_matrix(3)]:
        for i in range(0, A.nrows, max(1, A.nrows // 500)):
            c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
            assert np.all(np.diff(c) > 0)
        assert A.col.min() >= 0 and A.col.max() < A.ncols


def test_c1_shape():
    A = synth.c1()
    assert A.nrows == 10_000 and A.nnz == 100_000
    assert A.val.min() >= 1 and A.val.max() <= 65520


def test_c2_shape():
    A = synth.c2(n=400_000)
    L = np.diff(A.rowptr)
    assert L.max() <= 5000 + 5 and L.min() >= 3  # band rows at the edge have 3 band entries
    pm = np.isin(A.val, (-1, 1)).mean()
    assert abs(pm - 0.6) < 0.01
    # truncated Zipf(1.8) on [1,5000] has mean ~12.2; plus ~5 band entries, minus overlaps
    assert 16.0 < L.mean() < 18.5


def test_c3_dead_columns():
    A = synth.c3(n=20_000, ndead=100)
    used = np.unique(A.col)
    assert len(used) <= 20_000 - 100
    assert np.all(np.diff(A.rowptr) == 15)
    assert A.val.min() >= 1 and A.val.max() <= 2**31 - 2


def test_vectors_in_range():
    v = synth.vector(1, 2, 100_000, 0, 65520)
    assert v.min() == 0 and v.max() == 65520


def test_stencil_shape():
    """The 9-point stencil: rows of 4 (corners), 6 (edges) or 9 entries, a symmetric pattern with the
    diagonal, a band of half-width width + 1 in grid order, and the same pattern up to a relabelling
    when shuffled."""
    W, H = 37, 23
    for shuffle in (False, True):
        A = synth.stencil(width=W, height=H, shuffle=shuffle)
        n = W * H
        lens = np.diff(A.rowptr)
        assert sorted(np.unique(lens)) == [4, 6, 9]
        assert (lens == 4).sum() == 4 and (lens == 6).sum() == 2 * (W - 2) + 2 * (H - 2)
        rows = np.repeat(np.arange(n), lens)
        pairs = set(zip(rows.tolist(), A.col.tolist()))
        assert all((j, i) in pairs for i, j in pairs)
        assert all((i, i) in pairs for i in range(n))
        bw = int(np.abs(A.col - rows).max())
        if shuffle:
            assert bw > 10 * (W + 1)
        else:
            assert bw == W + 1
        assert np.all(np.diff(A.col)[np.diff(rows) == 0] > 0)  # sorted, distinct columns per row
    u = synth.stencil(width=W, height=H, shuffle=False)
    s = synth.stencil(width=W, height=H, shuffle=True)
    assert u.nnz == s.nnz
    assert np.array_equal(np.sort(np.diff(u.rowptr)), np.sort(np.diff(s.rowptr)))
    frac = np.mean(np.isin(s.val, [1, -1]))
    assert 0.5 < frac < 0.7
