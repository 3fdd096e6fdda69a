"""The C ABI without a GPU: the library loads, exports every declared symbol, and rejects bad input."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_1004_3719_amd as P
from paper_1004_3719_amd import ffx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(ffx_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    L = P.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_build_opts_defaults():
    """ffx_build_opts_default gives the documented defaults (a C caller that only fills `size` and
    calls it gets the same behaviour as the Python binding's defaults)."""
    o = ffx.BuildOpts()
    P.lib().ffx_build_opts_default(ctypes.byref(o))
    assert o.size == ctypes.sizeof(ffx.BuildOpts)
    assert (o.acc, o.selector, o.split_pm1, o.block_rows, o.build_transpose, o.tile_entries) == (
        ffx.ACC["auto"], ffx.SEL["heuristic"], 1, 4096, 0, 0)
    assert (o.compact_x, o.reorder, o.col_sorted) == (-1, 0, -1)
    assert o.model_path is None


def test_status_strings():
    L = P.lib()
    assert L.ffx_status_str(2) == b"FFX_EBOUND"
    assert P.version().startswith("ffx")


def _csr():
    return np.array([0, 2, 3], np.int64), np.array([0, 1, 1], np.int32), np.array([2, -1, 3], np.int64)


@pytest.mark.parametrize("m", [0, 1, 2**31, 2**32 - 1])
def test_bad_modulus(m):
    rp, c, v = _csr()
    with pytest.raises(P.FfxError) as e:
        P.Matrix.from_csr(2, 2, rp, c, v, m)
    assert e.value.status == ffx.FFX_EINVAL


def test_bad_indices_and_pointers():
    rp, c, v = _csr()
    with pytest.raises(P.FfxError) as e:
        P.Matrix.from_csr(2, 2, rp, np.array([0, 2, 1], np.int32), v, 7)
    assert e.value.status == ffx.FFX_EINVAL and "column index" in str(e.value)
    with pytest.raises(P.FfxError) as e:
        P.Matrix.from_csr(2, 2, np.array([0, 2, 1], np.int64), c, v, 7)
    assert e.value.status == ffx.FFX_EINVAL
    with pytest.raises(P.FfxError) as e:
        P.Matrix.from_coo(2, 2, [0, 5], [0, 1], np.array([1, 1], np.int64), 7)
    assert e.value.status == ffx.FFX_EINVAL


def test_fp64_bound_refused():
    # (m-1)^2 >= 2^53 when m > 94906266: one product alone is not exact in a double
    rp, c, v = _csr()
    with pytest.raises(P.FfxError) as e:
        P.Matrix.from_csr(2, 2, rp, c, v, 2**31 - 1, acc="fp64")
    assert e.value.status == ffx.FFX_EBOUND


@pytest.mark.parametrize("acc,largest", [("fp64", 94_906_266), ("fp64c", 189_812_531), ("fp32", 4096),
                                         ("fp32c", 8191)])
def test_float_bounds(acc, largest):
    """Each floating accumulator is refused just above the largest modulus whose product of two
    extreme operands (m-1 canonical, floor(m/2) centered), plus a reduced accumulator, is exact;
    at that modulus the bound check passes (a later device step may still fail without a GPU)."""
    rp, c, v = _csr()
    for m in (largest + 1, largest + 2):
        with pytest.raises(P.FfxError) as e:
            P.Matrix.from_csr(2, 2, rp, c, v, m, acc=acc)
        assert e.value.status == ffx.FFX_EBOUND, m
    try:
        P.Matrix.from_csr(2, 2, rp, c, v, largest, acc=acc).close()
    except P.FfxError as e:
        assert e.status != ffx.FFX_EBOUND


def test_bad_options():
    rp, c, v = _csr()
    for kw in [dict(block_rows=100), dict(block_rows=0), dict(tile_entries=100), dict(fixed_format=9)]:
        with pytest.raises(P.FfxError) as e:
            P.Matrix.from_csr(2, 2, rp, c, v, 7, **kw)
        assert e.value.status == ffx.FFX_EINVAL, kw


def test_null_out_pointer():
    L = P.lib()
    rp, c, v = _csr()
    st = L.ffx_matrix_create_csr(2, 2, rp.ctypes.data, c.ctypes.data, v.ctypes.data, 1, 7, None, None, None)
    assert st == ffx.FFX_EINVAL


def test_sequence_graph_batch_range():
    with pytest.raises(P.FfxError):
        P.set_sequence_graph_batch(-1)
    with pytest.raises(P.FfxError):
        P.set_sequence_graph_batch(4097)
    P.set_sequence_graph_batch(0)
    P.set_sequence_graph_batch(64)


def test_check_block_argument_errors():
    L = P.lib()
    bad = ctypes.c_int64(7)
    assert L.ffx_check_block(1, None, 0, 1, 1, 0, None, ctypes.byref(bad)) == 1  # modulus
    assert L.ffx_check_block(65521, None, 10, 1, 1, 0, None, ctypes.byref(bad)) == 1  # NULL block
    assert L.ffx_check_block(65521, ctypes.c_void_p(16), 10, 4, 2, 0, None, ctypes.byref(bad)) == 1  # ld < s
    assert L.ffx_check_block(65521, ctypes.c_void_p(16), 10, 1, 1, 7, None, ctypes.byref(bad)) == 1  # dtype
    assert bad.value == -1
    assert L.ffx_check_block(65521, None, 0, 1, 1, 0, None, ctypes.byref(bad)) == 0  # empty block


# ---------------------------------------------------------------- reordering --
def _bandwidth(rowptr, col, perm):
    n = len(perm)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    return int(np.abs(inv[rows] - inv[col]).max()) if len(col) else 0


def _shuffled(rowptr, col, seed):
    """The same pattern with its nodes renumbered by a seeded permutation."""
    import synth
    n = len(rowptr) - 1
    lab = np.empty(n, np.int64)
    lab[np.argsort(synth.raw(seed, n), kind="stable")] = np.arange(n)
    rows = lab[np.repeat(np.arange(n), np.diff(rowptr))]
    cols = lab[col]
    o = np.lexsort((cols, rows))
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return rp, cols[o].astype(np.int32)


def _path(n, parts=1):
    """parts disjoint paths of n nodes each (tridiagonal blocks)."""
    rows, cols = [], []
    for b in range(parts):
        for i in range(n):
            for j in (i - 1, i, i + 1):
                if 0 <= j < n:
                    rows.append(b * n + i)
                    cols.append(b * n + j)
    N = n * parts
    rp = np.zeros(N + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=rp[1:])
    return rp, np.array(cols, np.int32)


@pytest.mark.parametrize("parts", [1, 3])
def test_rcm_recovers_a_shuffled_path(parts):
    """A path graph renumbered at random has bandwidth ~n; reverse Cuthill-McKee from a
    pseudo-peripheral node (an end of the path) puts it back in path order: bandwidth exactly 1."""
    rp, col = _shuffled(*_path(500, parts), seed=3)
    assert _bandwidth(rp, col, np.arange(500 * parts)) > 100
    perm = P.reorder_rcm(500 * parts, rp, col)
    assert np.array_equal(np.sort(perm), np.arange(500 * parts))
    assert _bandwidth(rp, col, perm) == 1


def test_rcm_stencil_against_scipy():
    """On a shuffled 9-point stencil and on a random sparse pattern, the bandwidth after the
    ordering is within 25% of scipy's reverse Cuthill-McKee."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    import synth
    A = synth.stencil(width=60, height=45, shuffle=True)
    R = synth.rows(synth.spec(3000, 3000, 5, len_kind=synth.LEN_UNIFORM, len_a=0, len_b=3,
                              col_kind=synth.COL_BANDED, band_lo=-40, band_hi=40))
    for rp, col, n in [(A.rowptr, A.col, A.nrows), (*_shuffled(R.rowptr, R.col, 9), R.nrows)]:
        perm = P.reorder_rcm(n, rp, col)
        assert np.array_equal(np.sort(perm), np.arange(n))
        M = sp.csr_matrix((np.ones(len(col)), col, rp), shape=(n, n))
        ref = reverse_cuthill_mckee((M + M.T).tocsr(), symmetric_mode=True)
        assert _bandwidth(rp, col, perm) <= 1.25 * _bandwidth(rp, col, ref) + 2
        assert _bandwidth(rp, col, perm) < _bandwidth(rp, col, np.arange(n)) / 10


def test_rcm_edge_cases():
    assert len(P.reorder_rcm(0, np.zeros(1, np.int64), np.zeros(0, np.int32))) == 0
    assert list(P.reorder_rcm(1, np.array([0, 0], np.int64), np.zeros(0, np.int32))) == [0]
    # isolated nodes, self loops and a one-way entry: still a permutation
    rp = np.array([0, 1, 1, 2, 3], np.int64)
    col = np.array([0, 3, 3], np.int32)
    perm = P.reorder_rcm(4, rp, col)
    assert sorted(perm) == [0, 1, 2, 3]
    with pytest.raises(P.FfxError) as e:
        P.reorder_rcm(2, np.array([0, 1, 2], np.int64), np.array([0, 2], np.int32))
    assert e.value.status == ffx.FFX_EINVAL
    with pytest.raises(P.FfxError) as e:
        P.reorder_rcm(2, np.array([0, 2, 1], np.int64), np.array([0, 1], np.int32))
    assert e.value.status == ffx.FFX_EINVAL


def test_reorder_needs_square():
    rp, c, v = np.array([0, 1, 2], np.int64), np.array([0, 2], np.int32), np.array([5, 6], np.int64)
    with pytest.raises(P.FfxError) as e:
        P.Matrix.from_csr(2, 3, rp, c, v, 7, reorder=True)
    assert e.value.status == ffx.FFX_EINVAL


def test_sigma_and_rank_argument_errors():
    """Bad arguments of the order basis and the rank are refused before any device work."""
    L = P.lib()
    sh = (ctypes.c_int32 * 16)()
    d = (ctypes.c_int32 * 16)()
    G = ctypes.c_void_p(16)
    M = ctypes.c_void_p(32)
    cases = [
        (65520, 4, 2, 8, 8, 9),   # modulus not prime
        (4294967291, 4, 2, 8, 8, 9),  # prime above 2^31 - 1: the leaf's 32-bit sums would wrap
        (2147483659, 4, 2, 8, 8, 9),  # the smallest prime above 2^31
        (65521, 17, 8, 8, 8, 9),  # too many rows
        (65521, 4, 9, 8, 8, 9),   # too many columns
        (65521, 2, 3, 8, 8, 9),   # n > m
        (65521, 4, 2, 0, 8, 9),   # empty order
        (65521, 4, 2, 8, 7, 9),   # ldg < sigma
        (65521, 4, 2, 8, 8, 8),   # ldm < sigma + 1
    ]
    for p, m, n, sig, ldg, ldm in cases:
        st = L.ffx_sigma_basis(p, m, n, sig, G, ldg, sh, M, ldm, d, None)
        assert st == ffx.FFX_EINVAL, (p, m, n, sig, ldg, ldm)
    r, D, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    deg = (ctypes.c_int32 * 16)()
    S = ctypes.c_void_p(16)
    for p, s, Ln, dt in [(65521, 9, 10, 0), (65521, 0, 10, 0), (65521, 2, 0, 0), (65520, 2, 10, 0), (65521, 2, 10, 7),
                         (4294967291, 2, 10, 0), (2147483659, 2, 10, 0)]:
        st = L.ffx_sequence_rank(p, s, Ln, S, dt, deg, ctypes.byref(r), ctypes.byref(D), ctypes.byref(e), None)
        assert st == ffx.FFX_EINVAL, (p, s, Ln, dt)
    st = L.ffx_sequence_rank(65521, 2, 10, S, 0, None, ctypes.byref(r), ctypes.byref(D), ctypes.byref(e), None)
    assert st == ffx.FFX_EINVAL
