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
def test_batch_matches_oracle(dev, graph, order, chunk, wpc):
    from paper_1004_3719_amd import Batch, Matrix
    mats = small_batch(24)
    print("[case] batch", graph, order, chunk, wpc, [A.params["structure"] for A in mats], flush=True)
    Ms = [Matrix.from_synth(A) for A in mats]
    B = Batch(Ms, [A.s for A in mats], wg_per_cu=wpc, order=order, max_chunk=chunk, use_graph=graph)
    Xs = [torch.from_numpy(synth.c4_rhs(k, A).astype(np.int32)).to(dev) for k, A in enumerate(mats)]
    Ys = [torch.full((A.nrows, A.s), -5, dtype=torch.int32, device=dev) for A in mats]
    orc = oracle.get()
    for rep in range(2):  # the second launch replays the graph
        B.spmm(Xs, Ys)
        torch.cuda.synchronize()
        for k, A in enumerate(mats):
            want = orc.spmm(A, synth.c4_rhs(k, A))
            assert np.array_equal(Ys[k].cpu().numpy(), want), (rep, k, A.params)


def test_batch_tune_and_cache(dev, tmp_path):
    from paper_1004_3719_amd import Batch, Matrix
    mats = small_batch(12, nmax=20_000)
    Ms = [Matrix.from_synth(A) for A in mats]
    B = Batch(Ms, [A.s for A in mats])
    Xs = [torch.from_numpy(synth.c4_rhs(k, A).astype(np.int64)).to(dev) for k, A in enumerate(mats)]
    Ys = [torch.zeros((A.nrows, A.s), dtype=torch.int64, device=dev) for A in mats]
    cache = str(tmp_path / "tune.json")
    best = B.tune(Xs, Ys, reps=2, cache_path=cache)
    assert best["max_chunk"] in (4, 8) and 1 <= best["wg_per_cu"] <= 8
    B2 = Batch(Ms, [A.s for A in mats])
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
