"""GPU checks of the learned selector: the network kernels against the fp64 reference, the model
file, the heuristic fallback, and that the selector never changes a product."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp_ref as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 32)).astype(np.float32)
    T = rng.normal(size=(n, 6)).astype(np.float32)
    M = (rng.random(size=(n, 6)) < 0.85).astype(np.float32)
    return X, T, M


def test_forward_and_gradient_match_reference(dev):
    from paper_1004_3719_amd import Selector
    S = Selector(seed=7)
    theta, mean, scale = S.get_params()
    theta = theta + np.random.default_rng(3).normal(scale=0.05, size=theta.shape).astype(np.float32)
    S.set_params(theta=theta)
    X, T, M = data(512, 1)
    Xd, Td, Md = (torch.from_numpy(a).to(dev) for a in (X, T, M))
    out = S.predict(Xd).cpu().numpy()
    ref, _ = R.forward(theta.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(out - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    loss, g = S.gradient(Xd, Td, Md)
    Lr, gr = R.loss_grad(theta.astype(np.float64), X, T, M)
    g = g.cpu().numpy()
    assert abs(loss - Lr) <= 1e-4 * abs(Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    assert np.max(np.abs(g - gr)) <= 1e-4 * np.max(np.abs(gr)) + 1e-7


def test_standardisation_is_applied(dev):
    from paper_1004_3719_amd import Selector
    S = Selector(seed=8)
    theta, _, _ = S.get_params()
    rng = np.random.default_rng(5)
    mean = rng.normal(size=32).astype(np.float32)
    scale = (0.5 + rng.random(size=32)).astype(np.float32)
    S.set_params(mean=mean, scale=scale)
    X, _, _ = data(64, 2)
    out = S.predict(torch.from_numpy(X).to(dev)).cpu().numpy()
    ref, _ = R.forward(theta.astype(np.float64), (X.astype(np.float64) - mean) * scale)
    assert np.max(np.abs(out - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))


def test_adam_steps_match_reference(dev):
    from paper_1004_3719_amd import Selector
    S = Selector(seed=9)
    theta0, _, _ = S.get_params()
    X, T, M = data(256, 3)
    Xd, Td, Md = (torch.from_numpy(a).to(dev) for a in (X, T, M))
    opt = R.Adam(R.NPARAM, lr=1e-3)
    th = theta0.astype(np.float64)
    for _ in range(3):
        S.train_step(Xd, Td, Md, lr=1e-3)
        _, g = R.loss_grad(th, X, T, M)
        th = opt.step(th, g)
    got, _, _ = S.get_params()
    # Adam moves each weight by about lr per step; compare the moves
    assert np.max(np.abs((got - theta0) - (th - theta0))) <= 2e-5


def test_training_reduces_loss(dev):
    from paper_1004_3719_amd import Selector
    rng = np.random.default_rng(4)
    X = rng.normal(size=(2048, 32)).astype(np.float32)
    W = rng.normal(size=(32, 6)).astype(np.float32) / 6
    T = (np.tanh(X @ W) + 0.1 * X[:, :6]).astype(np.float32)
    M = np.ones_like(T)
    Xd, Td, Md = (torch.from_numpy(a).to(dev) for a in (X, T, M))
    S = Selector(seed=1)
    l0 = S.train_step(Xd, Td, Md, lr=3e-3, want_loss=True)
    for _ in range(300):
        S.train_step(Xd, Td, Md, lr=3e-3)
    l1, _ = S.gradient(Xd, Td, Md)
    assert l1 < 0.2 * l0


def test_model_file_roundtrip_and_fallback(dev, tmp_path):
    from paper_1004_3719_amd import FfxError, Matrix, Selector
    S = Selector(seed=11)
    path = str(tmp_path / "sel.bin")
    S.save(path)
    S2 = Selector.load(path)
    a, b = S.get_params(), S2.get_params()
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    bad = str(tmp_path / "bad.bin")
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0xFF
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(FfxError):
        Selector.load(bad)
    A = synth.c2(n=50_000)
    heur = Matrix.from_synth(A).block_formats()
    for p in [bad, str(tmp_path / "missing.bin")]:  # corrupt or missing model: the heuristic's formats
        assert np.array_equal(Matrix.from_synth(A, selector="learned", model_path=p).block_formats(), heur)


def test_learned_selection_never_changes_a_result(dev, tmp_path):
    from paper_1004_3719_amd import Matrix, Selector
    A = synth.c2(n=80_000)
    x = synth.vector(21, 1, A.ncols, 0, A.m - 1)
    want = oracle.get().spmv(A, x)
    xd = torch.from_numpy(x.astype(np.int32)).to(dev)
    for seed in range(4):  # arbitrary networks pick arbitrary formats
        path = str(tmp_path / ("s%d.bin" % seed))
        Selector(seed=100 + seed).save(path)
        M = Matrix.from_synth(A, selector="learned", model_path=path)
        assert np.array_equal(M.spmv(xd).cpu().numpy(), want), M.info()["format_blocks"]


def test_block_times(dev):
    from paper_1004_3719_amd import Matrix
    A = synth.c2(n=40_000)
    x = torch.from_numpy(synth.vector(22, 1, A.ncols, 0, A.m - 1).astype(np.int32)).to(dev)
    M = Matrix.from_synth(A)
    t = M.block_times(x, reps=4)
    assert t.shape == (M.info()["nblocks"],) and np.all(t > 0) and np.all(np.isfinite(t))
    y = M.spmv(x)
    assert np.array_equal(y.cpu().numpy(), oracle.get().spmv(A, x.cpu().numpy()))


def _rule_data(n, seed):
    """Blocks whose fastest format is a known function of two features (a rule the network can learn):
    labels log2 microseconds, with format 3 fastest where feature 7 is large and format 1 where
    feature 9 is small, STREAM otherwise."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 32)).astype(np.float32)
    T = np.full((n, 6), 3.0, np.float32) + rng.normal(scale=0.02, size=(n, 6)).astype(np.float32)
    T[:, 0] -= 0.3
    T[X[:, 7] > 0.8, 3] -= 1.0
    T[X[:, 9] < -0.8, 1] -= 1.0
    H = rng.integers(0, 6, size=n).astype(np.int32)
    return X, T, H


def test_train_through_the_abi(dev, tmp_path):
    """ffx_selector_train learns the rule, reports held-out costs, writes a model that loads and that
    the builder uses; training is deterministic for a seed."""
    from paper_1004_3719_amd import Selector
    from paper_1004_3719_amd import selector_train as ST
    from paper_1004_3719_amd.ffx import selector_train
    X, T, H = _rule_data(6000, 3)
    path = str(tmp_path / "m.bin")
    S, rep = selector_train(X, T, heur=H, epochs=40, lr=3e-3, seed=11, n_val=1000, out_model=path)
    print("[case] train report", rep, flush=True)
    assert rep["steps"] == 40 * 10 and np.isfinite(rep["train_loss"]) and rep["train_loss"] < 0.1
    assert rep["val_cost"] < rep["val_cost_stream"] and rep["val_cost"] < rep["val_cost_heuristic"]
    assert rep["val_cost"] < 1.1
    ch, _ = ST.choose(S, X[:1000])
    assert abs(ST.choice_cost(T[:1000], ch) - rep["val_cost"]) < 1e-6
    L = Selector.load(path)
    a = S.predict(torch.from_numpy(X[:256]).to(dev)).cpu().numpy()
    b = L.predict(torch.from_numpy(X[:256]).to(dev)).cpu().numpy()
    assert np.array_equal(a, b)
    S2, rep2 = selector_train(X, T, heur=H, epochs=40, lr=3e-3, seed=11, n_val=1000)
    assert np.array_equal(S2.get_params()[0], S.get_params()[0]) and rep2 == rep
    # the builder takes the model from the file; products stay exact
    A = synth.c1(n=9000)
    from paper_1004_3719_amd import Matrix
    M = Matrix.from_synth(A, selector="learned", model_path=path)
    x = synth.vector(5, 1, A.ncols, 0, A.m - 1)
    y = M.spmv(torch.from_numpy(x.astype(np.int32)).to(dev)).cpu().numpy()
    assert np.array_equal(y, oracle.get().spmv(A, x))


def test_train_argument_errors(dev):
    from paper_1004_3719_amd import FfxError
    from paper_1004_3719_amd.ffx import selector_train
    X, T, H = _rule_data(100, 4)
    for kw in ({"epochs": 0}, {"lr": -1.0}, {"n_val": 100}, {"n_val": 99}):
        with pytest.raises(FfxError):
            selector_train(X, T, **kw)
    Tn = T.copy()
    Tn[5, 2] = np.nan
    with pytest.raises(FfxError):
        selector_train(X, Tn)


def test_decision_margin_shifts_non_default_outputs(dev):
    """The margin is folded into the output biases of the five non-STREAM formats: with the same seed
    and samples, a margin of 0.25 moves their predictions by exactly 0.25 against a margin of 0, and
    STREAM's not at all; a block leaves STREAM only for a larger predicted gain."""
    from paper_1004_3719_amd import selector_train as ST
    from paper_1004_3719_amd.ffx import selector_train
    X, T, _ = _rule_data(2000, 7)
    S0, r0 = selector_train(X, T, epochs=5, seed=5, margins=[0.0])
    S1, r1 = selector_train(X, T, epochs=5, seed=5, margins=[0.25])
    assert r0["margin"] == 0.0 and r1["margin"] == 0.25
    Xd = torch.from_numpy(X[:300]).to(dev)
    before = S0.predict(Xd).cpu().numpy()
    after = S1.predict(Xd).cpu().numpy()
    assert np.array_equal(after[:, 0], before[:, 0])
    assert np.allclose(after[:, 1:] - before[:, 1:], 0.25, atol=1e-5)
    ch, _ = ST.choose(S1, X[:300])
    rel = before[:, 1:].min(axis=1) - before[:, 0]
    far = np.abs(rel + 0.25) > 1e-3  # away from the tie at exactly mu
    assert np.array_equal((ch == 0)[far], (rel > -0.25)[far])


def test_label_window(dev):
    """ffx_selector_label: the builder's features, finite labels (equal over the blocks of the window),
    the heuristic's formats."""
    from paper_1004_3719_amd import Matrix, block_features
    from paper_1004_3719_amd import selector_train as ST
    sp, _ = synth.c5_spec(3)
    A = ST.shift_columns(synth.rows(sp, 4096, 4096 * 5), 4096)
    A.m = synth.M_C5
    F, T, H = ST.window_labels(A, reps=3, seed=9)
    assert F.shape == (4, 32) and T.shape == (4, 6) and H.shape == (4,)
    assert np.array_equal(F, block_features(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m))
    assert np.all(np.isfinite(T)) and np.all(T == T[0])
    M = Matrix.from_synth(A)
    assert np.array_equal(H, M.block_formats())
    M.close()


MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1004_3719_amd", "models",
                     "selector.bin")


@pytest.mark.skipif(not os.path.exists(MODEL), reason="no trained model in the package")
def test_trained_model_gain(dev):
    """The committed network, trained on in-place product timings of generated training windows, on
    held-out generated matrices (first 65,536 rows of each; tile formats, so col_sorted is off):
    every product equal to the oracle, and the summed time of the learned formats below the plain
    heuristic's and within 3% (the run-to-run spread) of the best single fixed format. Each matrix's
    time is the median of 3 interleaved rounds."""
    from paper_1004_3719_amd import selector_train as ST
    from paper_1004_3719_amd.ffx import FORMATS
    orc = oracle.get()
    tot = {}
    for k in range(1800, 1816):
        sp, _ = synth.c5_spec(k)
        A = synth.rows(sp, 0, min(sp.nrows, 65536))
        A.m = synth.M_C5
        xh = synth.vector(k, 8, A.ncols, 0, A.m - 1)
        x = torch.from_numpy(xh.astype(np.int32)).to(dev)
        r = ST.evaluate(A, MODEL, x, reps=10, fixed=FORMATS, rounds=3)
        want = orc.spmv(A, xh)
        for name, y in r["results"].items():
            assert np.array_equal(y.cpu().numpy(), want), (k, name)
        for key, v in r.items():
            if key.endswith("_us"):
                tot[key] = tot.get(key, 0.0) + v
    best = min(tot["fixed_%s_us" % f] for f in FORMATS)
    print("[case] held-out product time: heuristic %.1f us, learned %.1f us, best fixed %.1f us"
          % (tot["heuristic_us"], tot["learned_us"], best), flush=True)
    assert tot["learned_us"] < tot["heuristic_us"]
    assert tot["learned_us"] <= 1.03 * best


@pytest.mark.skipif(not os.path.exists(MODEL), reason="no trained model in the package")
@pytest.mark.parametrize("k", [1808, 1840, 1875, 1926])
def test_held_out_whole_matrices(dev, k):
    """Whole held-out selection matrices (three of the smallest, 50k rows each, one row-length family
    each, and one of about 3.9 M rows): the products built with the learned and the heuristic formats
    (tiles) and with the column-sorted groups all equal the oracle's."""
    from paper_1004_3719_amd import Matrix
    sp, _ = synth.c5_spec(k)
    A = synth.rows(sp)
    A.m = synth.M_C5
    print("[case] held-out whole", k, A.nrows, A.nnz, flush=True)
    xh = synth.vector(k, 8, A.ncols, 0, A.m - 1)
    x = torch.from_numpy(xh.astype(np.int32)).to(dev)
    want = oracle.get_all_cores().spmv(A, xh)
    for opts in ({"selector": "learned", "model_path": MODEL, "col_sorted": 0}, {"col_sorted": 0},
                 {"col_sorted": 1}):
        M = Matrix.from_synth(A, **opts)
        assert np.array_equal(M.spmv(x).cpu().numpy(), want), opts
        M.close()
