"""ffx_spmv_noalloc: the product through the library's static scratch, called
through the C ABI, against ffx_spmv on the same inputs (and the oracle).

Two calls in a row share one GPU's static array; the second is on a smaller
input, so it must not read anything the first one left behind. Collected last:
a failure here hides no other test.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def note(*a):
    print("[case]", *a, flush=True)


def tdev(a, dev, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(dev)


def _noalloc(M, x, y, alpha, beta):
    from paper_1004_3719_amd import ffx
    L = ffx.lib()
    st = torch.cuda.current_stream().cuda_stream
    return L.ffx_spmv_noalloc(M.handle, alpha, ctypes.c_void_p(x.data_ptr()), beta, ctypes.c_void_p(y.data_ptr()),
                              ffx._dt(x), ctypes.c_void_p(st))


def _cases():
    # large then small: power-law rows mod 32749 (16-bit x copy in the scratch), the plain workload
    return [("powerlaw 200k", synth.c2(n=200_000), {}),
            ("plain 7k", synth.c1(n=7000), {})]


@pytest.mark.parametrize("dt", [torch.int32, torch.int64])
@pytest.mark.parametrize("opts", [{}, {"reorder": True}, {"compact_x": 0, "reorder": True}, {"col_sorted": 1},
                                  {"col_sorted": 1, "reorder": True}])
def test_noalloc_matches_spmv(dev, dt, opts):
    from paper_1004_3719_amd import Matrix
    orc = oracle.get()
    for name, A, _ in _cases():
        note("noalloc", name, dt, opts)
        M = Matrix.from_synth(A, **opts)
        x = synth.vector(71, 1, A.ncols, 0, A.m - 1)
        y0 = synth.vector(71, 2, A.nrows, 0, A.m - 1)
        for alpha, beta in ((1, 0), (5, A.m - 2)):
            ya = tdev(y0, dev, dt)
            yb = tdev(y0, dev, dt)
            M.spmv(tdev(x, dev, dt), alpha=alpha, beta=beta, y=ya)
            assert _noalloc(M, tdev(x, dev, dt), yb, alpha, beta) == 0
            torch.cuda.synchronize()
            a, b = ya.cpu().numpy(), yb.cpu().numpy()
            assert np.array_equal(a, b), (name, alpha, beta)
            assert np.array_equal(b, orc.spmv(A, x, alpha, beta, y0)), (name, alpha, beta)
        M.close()


def test_noalloc_large_modulus_needs_no_scratch(dev):
    """m > 65536: no 16-bit copy, the call runs the tiles directly."""
    from paper_1004_3719_amd import Matrix
    A = synth.c3(n=6000, ndead=40)
    M = Matrix.from_synth(A)
    x = synth.vector(72, 1, A.ncols, 0, A.m - 1)
    ya = M.spmv(tdev(x, dev, torch.int64))
    yb = torch.empty_like(ya)
    assert _noalloc(M, tdev(x, dev, torch.int64), yb, 1, 0) == 0
    torch.cuda.synchronize()
    assert np.array_equal(ya.cpu().numpy(), yb.cpu().numpy())
    assert np.array_equal(yb.cpu().numpy(), oracle.get().spmv(A, x))
    M.close()


def test_noalloc_refuses_beyond_the_scratch(dev):
    """A 16-bit copy of more than 16 Mi columns does not fit the 32 MiB array: FFX_EINVAL, nothing enqueued,
    y untouched; ffx_spmv still computes the product."""
    from paper_1004_3719_amd import Matrix, ffx
    ncols = (32 << 20) // 2 + 64
    rp = np.array([0, 2, 3], np.int64)
    col = np.array([5, ncols - 1, 17], np.int32)
    val = np.array([3, 4, -1], np.int64)
    m = 65521
    M = Matrix.from_csr(2, ncols, rp, col, val, m)
    x = torch.zeros(ncols, dtype=torch.int32, device=dev)
    x[5], x[ncols - 1], x[17] = 10, 20, 30
    y = torch.full((2,), 77, dtype=torch.int32, device=dev)
    st = _noalloc(M, x, y, 1, 0)
    assert st == ffx.FFX_EINVAL
    assert b"static scratch" in ffx.lib().ffx_last_error()
    torch.cuda.synchronize()
    assert y.cpu().tolist() == [77, 77]
    assert M.spmv(x).cpu().tolist() == [(3 * 10 + 4 * 20) % m, (m - 30) % m]
    M.close()


def test_noalloc_argument_errors(dev):
    from paper_1004_3719_amd import Matrix, ffx
    A = synth.c1(n=500)
    M = Matrix.from_synth(A)
    x = tdev(synth.vector(73, 1, A.ncols, 0, A.m - 1), dev)
    L = ffx.lib()
    st = torch.cuda.current_stream().cuda_stream
    assert L.ffx_spmv_noalloc(None, 1, ctypes.c_void_p(x.data_ptr()), 0, ctypes.c_void_p(x.data_ptr()), 0,
                              ctypes.c_void_p(st)) == ffx.FFX_EINVAL
    y = torch.empty_like(x)
    assert L.ffx_spmv_noalloc(M.handle, A.m, ctypes.c_void_p(x.data_ptr()), 0, ctypes.c_void_p(y.data_ptr()), 0,
                              ctypes.c_void_p(st)) == ffx.FFX_EINVAL  # alpha not a residue
    assert L.ffx_spmv_noalloc(M.handle, 1, ctypes.c_void_p(x.data_ptr()), 0, ctypes.c_void_p(x.data_ptr()), 0,
                              ctypes.c_void_p(st)) == ffx.FFX_EINVAL  # x and y alias
    M.close()
