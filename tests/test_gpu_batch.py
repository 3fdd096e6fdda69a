"""GPU parity of the batched launch: every matrix of an uneven batch against the oracle."""
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


def small_batch(count, nmax=30_000, seed=synth.SEED0 + 3):
    mats = [synth.c4_matrix(k, seed=seed, nmax=nmax) for k in range(count)]
    return mats


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("order,chunk,wpc", [(0, 8, 4), (1, 4, 1), (0, 4, 8)])
@pytest.mark.parametrize("xcd,x16", [(1, -1), (0, 0), (1, 0), (0, 1)])
def test_batch_matches_oracle(dev, graph, order, chunk, wpc, xcd, x16):
    from paper_1004_3719_amd import Batch, Matrix
    mats = small_batch(24)
    print("[case] batch", graph, order, chunk, wpc, xcd, x16, [A.params["structure"] for A in mats], flush=True)
    Ms = [Matrix.from_synth(A) for A in mats]
    B = Batch(Ms, [A.s for A in mats], wg_per_cu=wpc, order=order, max_chunk=chunk, use_graph=graph, xcd=xcd,
              compact_x=x16)
    Xs = [torch.from_numpy(synth.c4_rhs(k, A).astype(np.int32)).to(dev) for k, A in enumerate(mats)]
    Ys = [torch.full((A.nrows, A.s), -5, dtype=torch.int32, device=dev) for A in mats]
    orc = oracle.get()
    for rep in range(2):  # the second launch replays the graph
        B.spmm(Xs, Ys)
        torch.cuda.synchronize()
        for k, A in enumerate(mats):
            want = orc.spmm(A, synth.c4_rhs(k, A))
            assert np.array_equal(Ys[k].cpu().numpy(), want), (rep, k, A.params)


@pytest.mark.parametrize("x16", [1, 0])
def test_batch_strided_operands(dev, x16):
    """X and Y with leading dimensions above s (views into wider blocks), int64: the 16-bit copy
    follows the caller's leading dimension, and the columns outside the views stay untouched."""
    from paper_1004_3719_amd import Batch, Matrix
    mats = small_batch(10, nmax=15_000)
    Ms = [Matrix.from_synth(A) for A in mats]
    B = Batch(Ms, [A.s for A in mats], compact_x=x16)
    rhs = [synth.c4_rhs(k, A) for k, A in enumerate(mats)]
    Xw = [torch.zeros((A.ncols, A.s + 3), dtype=torch.int64, device=dev) for A in mats]
    for X, R in zip(Xw, rhs):
        X[:, 1:1 + R.shape[1]] = torch.from_numpy(R).to(dev)
    Yw = [torch.full((A.nrows, A.s + 5), 7, dtype=torch.int64, device=dev) for A in mats]
    B.spmm([X[:, 1:1 + A.s] for X, A in zip(Xw, mats)], [Y[:, 2:2 + A.s] for Y, A in zip(Yw, mats)])
    torch.cuda.synchronize()
    orc = oracle.get()
    for k, A in enumerate(mats):
        Y = Yw[k].cpu().numpy()
        assert np.array_equal(Y[:, 2:2 + A.s], orc.spmm(A, rhs[k])), k
        assert (Y[:, :2] == 7).all() and (Y[:, 2 + A.s:] == 7).all()


def test_batch_full_size(dev):
    """The 256-matrix batch at its stated size (n up to 500,000, 1..16 right-hand sides, 70% +-1,
    m = 65521), default parameters, every Y_k against the oracle (all cores), twice (the second
    launch replays the graph)."""
    from paper_1004_3719_amd import Batch, Matrix
    mats, Ms = [], []
    for k in range(256):
        A = synth.c4_matrix(k)
        mats.append(A)
        Ms.append(Matrix.from_synth(A))
        if k % 32 == 31:
            print("[case] c4 full: built %d matrices" % (k + 1), flush=True)
    B = Batch(Ms, [A.s for A in mats])
    rhs = [synth.c4_rhs(k, A) for k, A in enumerate(mats)]
    Xs = [torch.from_numpy(R.astype(np.int32)).to(dev) for R in rhs]
    Ys = [torch.full((A.nrows, A.s), -1, dtype=torch.int32, device=dev) for A in mats]
    orc = oracle.get_all_cores()
    for rep in range(2):
        B.spmm(Xs, Ys)
        torch.cuda.synchronize()
        for k, A in enumerate(mats):
            assert np.array_equal(Ys[k].cpu().numpy(), orc.spmm(A, rhs[k])), (rep, k, A.params)
        print("[case] c4 full: launch %d equal to the oracle on all 256 matrices" % rep, flush=True)
        for Y in Ys:
            Y.fill_(-1)


def test_batch_tune_and_cache(dev, tmp_path):
    """The tuner's choice is stored in and read back from its JSON cache; 48 matrices give a cache key
    of well over 512 characters."""
    from paper_1004_3719_amd import Batch, Matrix
    mats = small_batch(48, nmax=8_000)
    Ms = [Matrix.from_synth(A) for A in mats]
    B = Batch(Ms, [A.s for A in mats])
    Xs = [torch.from_numpy(synth.c4_rhs(k, A).astype(np.int64)).to(dev) for k, A in enumerate(mats)]
    Ys = [torch.zeros((A.nrows, A.s), dtype=torch.int64, device=dev) for A in mats]
    cache = str(tmp_path / "tune.json")
    best = B.tune(Xs, Ys, reps=2, cache_path=cache)
    assert best["max_chunk"] in (4, 8) and 1 <= best["wg_per_cu"] <= 8
    assert best["xcd"] in (0, 1) and best["compact_x"] in (0, 1)
    B2 = Batch(Ms, [A.s for A in mats])
    assert len(open(cache).read()) > 600
    assert B2.tune(Xs, Ys, cache_path=cache) == best  # read back from the cache
    B2.spmm(Xs, Ys)
    orc = oracle.get()
    for k, A in enumerate(mats):
        assert np.array_equal(Ys[k].cpu().numpy(), orc.spmm(A, synth.c4_rhs(k, A)))


@pytest.mark.parametrize("acc,m", [("fp32", 4093), ("fp32c", 8191), ("fp64c", 65521)])
def test_batch_float_accumulators(dev, acc, m):
    """A batch built with a floating accumulator (reductions after every term for fp32 at 4093
    and centered fp32 at 8191) against the oracle."""
    from paper_1004_3719_amd import Batch, Matrix
    mats = [synth.c4_matrix(k, nmax=20_000, m=m) for k in range(10)]
    print("[case] batch acc", acc, m, flush=True)
    Ms = [Matrix.from_synth(A, acc=acc) for A in mats]
    B = Batch(Ms, [A.s for A in mats])
    rhs = [synth.c4_rhs(k, A, m=m) for k, A in enumerate(mats)]
    Xs = [torch.from_numpy(X.astype(np.int32)).to(dev) for X in rhs]
    Ys = [torch.full((A.nrows, A.s), -5, dtype=torch.int32, device=dev) for A in mats]
    B.spmm(Xs, Ys)
    torch.cuda.synchronize()
    orc = oracle.get()
    for k, A in enumerate(mats):
        assert np.array_equal(Ys[k].cpu().numpy(), orc.spmm(A, rhs[k])), (k, A.params)


@pytest.mark.parametrize("s", [1, 8])
def test_tune_tile_entries(dev, s):
    """The build-time tile tuner times each candidate tile size on the matrix itself; the matrix
    built with its choice (STREAM tiles throughout) still equals the oracle."""
    from paper_1004_3719_amd import Matrix
    from paper_1004_3719_amd.ffx import tune_tile_entries
    A = synth.c4_matrix(5, nmax=40_000)
    print("[case] tune tile entries", s, A.nrows, A.nnz, flush=True)
    best, us = tune_tile_entries(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, s=s, reps=3,
                                 fixed_format="STREAM")
    assert best in (512, 1024, 2048, 4096)
    assert all(t > 0 for t in us.values()) and us[best] == min(us.values())
    M = Matrix.from_synth(A, fixed_format="STREAM", tile_entries=best)
    X = synth.vector(synth.SEED0 + 3, 9000 + s, A.ncols * s, 0, A.m - 1).reshape(A.ncols, s)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.int64)).to(dev)
    Y = torch.zeros((A.nrows, s), dtype=torch.int64, device=dev)
    M.spmm(Xd, Y=Y)
    torch.cuda.synchronize()
    assert np.array_equal(Y.cpu().numpy(), oracle.get().spmm(A, X))
