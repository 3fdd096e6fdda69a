"""Products captured in a HIP graph (torch.cuda.graph) and replayed: ffx_spmv on a handle that keeps
no temporary, and ffx_spmv_noalloc on handles whose product stages x in the library's static
scratch (the 16-bit copy of the column-sorted groups, x in the stored order of a reordered handle).
Each graph is replayed several times with eager work (a new x, a cleared y) and synchronisations
between the replays, and every replay is checked against the oracle."""
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


CASES = {
    "plain": (lambda: synth.c1(n=10_000), {}, False),
    "powerlaw column-sorted": (lambda: synth.c2(n=200_000), {"col_sorted": 1}, True),
    "powerlaw reordered": (lambda: synth.c2(n=200_000), {"reorder": True}, True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_graph_replays(dev, case):
    from paper_1004_3719_amd import Matrix
    make, opts, noalloc = CASES[case]
    A = make()
    note("graph", case, A.nnz)
    M = Matrix.from_synth(A, **opts)
    if "col_sorted" in opts:
        assert M.info()["sg_groups"] > 0
    orc = oracle.get()
    xs = [synth.vector(60 + k, 1, A.ncols, 0, A.m - 1) for k in range(2)]
    x = torch.from_numpy(xs[0].astype(np.int32)).to(dev)
    y = torch.empty(A.nrows, dtype=torch.int32, device=dev)

    def call():
        return M.spmv_noalloc(x, y=y) if noalloc else M.spmv(x, y=y)

    # one call before the capture, on a side stream (the library sets its kernels' LDS limits once)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            call()
    for rep in range(4):
        xv = xs[rep % 2]
        x.copy_(torch.from_numpy(xv.astype(np.int32)))
        y.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), orc.spmv(A, xv)), (case, rep)
    del g
    M.close()
