"""GPU checks of the learned cost model and the learned schedule."""
import os
import tempfile

import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from oracle import mlp
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _weights(seed):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.3, mlp.N_PARAMS).astype(np.float32)
    return mlp.bf16_round(w)


def test_forward_and_gradient_match_fp64_reference():
    rng = np.random.default_rng(7)
    w = _weights(1)
    for n in (1, 63, 64, 65, 1000, 4096):
        X = mlp.bf16_round(rng.normal(0, 1, (n, mlp.F)).astype(np.float32))
        Y = rng.normal(0, 2, n).astype(np.float32)
        y_gpu = A.amlm_mlp_forward(w, X)
        y_ref = mlp.forward(w.astype(np.float64), X.astype(np.float64))
        np.testing.assert_allclose(y_gpu, y_ref, rtol=1e-4, atol=1e-4)
        g_gpu, loss = A.amlm_mlp_grad(w, X, Y)
        g_ref = mlp.grad(w.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
        tol = 1e-3 * np.maximum(1.0, np.abs(g_ref))
        bad = np.abs(g_gpu - g_ref) > tol
        assert not bad.any(), (n, np.nonzero(bad)[0][:5], g_gpu[bad][:5], g_ref[bad][:5])
        assert abs(loss - mlp.loss(w, X, Y)) <= 1e-4 * max(1.0, loss)


def test_matrix_core_inference_matches_reference():
    """The MFMA path (16x16x32 BF16 tiles) against the FP64 reference with the
    same BF16 rounding of inputs and activations; sizes cover partial tiles."""
    rng = np.random.default_rng(11)
    w = _weights(3)
    for n in (1, 15, 16, 17, 100, 4097):
        X = rng.normal(0, 1, (n, mlp.F)).astype(np.float32)
        y = A.amlm_mlp_predict(w, X)
        ref = mlp.forward_bf16_act(w.astype(np.float64), X)
        np.testing.assert_allclose(y, ref, rtol=2e-2, atol=2e-2 * max(1.0, np.abs(ref).max()))
        # and it tracks the FP32-activation forward closely
        full = mlp.forward(w.astype(np.float64), mlp.bf16_round(X).astype(np.float64))
        assert np.corrcoef(y, full)[0, 1] > 0.999 if n > 16 else True


def test_gradient_is_deterministic():
    rng = np.random.default_rng(9)
    w = _weights(2)
    X = rng.normal(0, 1, (3000, mlp.F)).astype(np.float32)
    Y = rng.normal(0, 1, 3000).astype(np.float32)
    g1, _ = A.amlm_mlp_grad(w, X, Y)
    g2, _ = A.amlm_mlp_grad(w, X, Y)
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32))


@pytest.fixture(scope="module")
def trained():
    gs = [W.mid(202 + i, scale=0.1) for i in range(2)]
    Gs = [A.Graph(g.src, g.dst, g.ts, g.n_vertices) for g in gs]
    ps = [A.params(A.AMLM_ALL, 86400, 6, 2)] * len(Gs)
    A.amlm_costmodel_train(Gs, ps, epochs=4, batch=4096, seed=5)
    w, mean, inv_std = A.amlm_costmodel_get()
    for G in Gs:
        G.close()
    return w, mean, inv_std


def _spearman(a, b):
    from scipy.stats import spearmanr
    return float(spearmanr(a, b).correlation)


def test_heldout_rank_correlation(trained):
    """On a graph the model never saw (another seed of the generator), the
    predicted scatter-gather bytes rank the anchors by their true bytes
    (counted by the plain miner): the deterministic training gives a fixed
    correlation, checked against a floor and against the length rule (the
    sender-window length alone, which is what the schedule would use without
    the network)."""
    g = W.mid(209, scale=0.03)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    pred, lab, wl = A.amlm_costmodel_eval(G, A.params(A.AMLM_ALL, 86400, 6, 2))
    G.close()
    assert pred.shape[0] > 10000 and np.isfinite(pred).all()
    rho_model = _spearman(pred, lab)
    rho_len = _spearman(wl, lab)
    print(f"held-out Spearman: model {rho_model:.4f}, window length {rho_len:.4f} over {pred.shape[0]} anchors")
    # measured on MI355X with this training (deterministic): model 0.678,
    # window length 0.480 (a smaller model, 2 x 100k-edge graphs and 3
    # epochs, gave 0.465: no better than the length)
    assert rho_model >= 0.60
    assert rho_model >= rho_len + 0.10
    assert A.amlm_costmodel_length_coef() > 0


def test_training_is_deterministic(trained):
    w, mean, inv_std = trained
    assert np.isfinite(w).all() and np.isfinite(mean).all()
    # retrain with the same seed: identical weights
    gs = [W.mid(202 + i, scale=0.1) for i in range(2)]
    Gs = [A.Graph(g.src, g.dst, g.ts, g.n_vertices) for g in gs]
    A.amlm_costmodel_train(Gs, [A.params(A.AMLM_ALL, 86400, 6, 2)] * 2, epochs=4, batch=4096, seed=5)
    w2, _, _ = A.amlm_costmodel_get()
    assert np.array_equal(w.view(np.uint32), w2.view(np.uint32))
    for G in Gs:
        G.close()


def test_learned_schedule_counts_equal_static_and_oracle(trained):
    g = W.mid(210, scale=0.03)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    ps = A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_STATIC)
    pl = A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_LEARNED)
    a = A.to_u32(A.amlm_mine(G, ps))
    b = A.to_u32(A.amlm_mine(G, pl))
    A.amlm_graph_sync(G)
    np.testing.assert_array_equal(a, b)
    ref = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 86400, 6, 2)
    np.testing.assert_array_equal(b, ref)
    G.close()


def test_length_and_given_schedules_equal_static(trained):
    """The ablation schedules (sender-window length rule, caller-given true
    costs) slice the same anchors differently and give the same counts,
    with slices forced by a small split size too."""
    g = W.mid(211, scale=0.03)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    base = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_STATIC)))
    _, work = A.amlm_mine_work(G, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_LEARNED))
    torch.cuda.synchronize()
    cost = torch.log1p(work[3].view(torch.int64).to(torch.float64)).to(torch.float32).contiguous()
    A.amlm_graph_set_costs(G, cost)
    for split in (0, 512):
        A.amlm_tune_set(G, split_bytes=split)
        for sched in (A.AMLM_SCHED_LEARNED, A.AMLM_SCHED_LENGTH, A.AMLM_SCHED_GIVEN):
            c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 6, 2, sched)))
            A.amlm_graph_sync(G)
            np.testing.assert_array_equal(c, base, err_msg=f"schedule {sched} split {split}")
    A.amlm_graph_set_costs(G, None)
    with pytest.raises(A.AmlmError):
        A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_GIVEN))
    G.close()


def test_save_load_roundtrip(trained):
    w, mean, inv_std = trained
    coef = A.amlm_costmodel_length_coef()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        A.amlm_costmodel_save(path)
        A.amlm_costmodel_load(path)
        w2, m2, s2 = A.amlm_costmodel_get()
    assert np.array_equal(w, w2) and np.array_equal(mean, m2) and np.array_equal(inv_std, s2)
    assert A.amlm_costmodel_length_coef() == coef
