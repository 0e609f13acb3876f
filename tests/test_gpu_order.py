"""GPU root orders and the root-scoring model, through the C ABI, against the
CPU oracle: per-root features and labels of the trace, the MLP's scores,
gradient and Adam step, graph-replayed training against eager launches, and
the invariance of the exhaustive result under every root order."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import enum as E
from oracle import lattice as L
from oracle import mlp as N
from oracle import roots as RT

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4   # norm-wise relative, per parameter tensor (FP32 accumulation vs FP64)


@pytest.fixture(scope="module")
def M():
    import paper_2508_08702_amd as M
    return M


@pytest.fixture(scope="module")
def ctx(M):
    c = M.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("m,D,seed,split", [(3, 100, 1001, 4), (4, 50, 7, 6), (4, 100, 11, 9), (5, 200, 13, 8),
                                            (5, 50, 17, 12)])
def test_trace_features_and_labels_match_oracle(M, ctx, m, D, seed, split):
    inst = mi.single_small(seed) if m == 3 else mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    print(f"  trace m={m} D={D} seed={seed} split={split}", flush=True)
    prm = M.msp_params_default(split_depth=split, time_cap_ms=60000.0)
    tr = M.msp_root_trace(ctx, _dev(inst.A), _dev(inst.d), _dev(P.basis), params=prm)
    torch.cuda.synchronize()
    roots = RT.roots_dfs(P, split)
    ref = E.enumerate_prepared(P, split=split)
    Lv = P.k - split
    assert tr.stats["split_depth"] == split and tr.feat.shape[0] == len(roots) == ref.n_roots
    assert tr.n_found == ref.n_found
    Fo = RT.features(P, roots, Lv)
    Fg = tr.feat.cpu().numpy()
    # features from the prefix and the partial norm are the same FP64 values
    # rounded to FP32; those from w (columns 1, 2, 13) see the w recurrence
    np.testing.assert_allclose(Fg, Fo, rtol=1e-6, atol=1e-6)
    assert np.array_equal(tr.label.cpu().numpy(), RT.labels(P, roots, Lv, ref.solutions))


def _tensor_slices():
    o, out = 0, []
    for name, size in (("W1", 64 * 16), ("b1", 64), ("W2", 64 * 64), ("b2", 64), ("W3", 64), ("b3", 1)):
        out.append((name, slice(o, o + size)))
        o += size
    assert o == N.NPARAM
    return out


@pytest.mark.parametrize("count", [1, 1000, 100003])
def test_model_scores_and_gradient_match_oracle(M, ctx, count):
    rng = np.random.default_rng(count)
    w32 = (rng.standard_normal(N.NPARAM) * 0.25).astype(np.float32)
    M.msp_model_set(ctx, w32)
    assert np.array_equal(M.msp_model_get(ctx), w32)
    X = rng.standard_normal((count, N.NFEAT)).astype(np.float32)
    y = (rng.random(count) < 0.1).astype(np.uint8)
    we = N.effective(w32)
    z = M.msp_model_score(ctx, _dev(X)).cpu().numpy().astype(np.float64)
    zo = N.forward(we, X.astype(np.float64))
    assert np.max(np.abs(z - zo)) <= 1e-4 * max(1.0, np.max(np.abs(zo)))
    g, loss = M.msp_model_grad(ctx, _dev(X), _dev(y), pos_weight=5.0)
    Lo, go = N.loss_and_grad(we, X.astype(np.float64), y, 5.0)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - Lo) <= 1e-5 * max(1.0, abs(Lo))
    for name, sl in _tensor_slices():
        ref = np.linalg.norm(go[sl])
        assert np.linalg.norm(g[sl] - go[sl]) <= GRAD_TOL * max(ref, 1e-12), name


def test_one_adam_step_matches_oracle(M, ctx):
    rng = np.random.default_rng(11)
    count = 3000
    w32 = (rng.standard_normal(N.NPARAM) * 0.25).astype(np.float32)
    X = rng.standard_normal((count, N.NFEAT)).astype(np.float32)
    y = (rng.random(count) < 0.2).astype(np.uint8)
    M.msp_model_set(ctx, w32)
    lr = 1e-3
    tp = M.msp_train_params_default(epochs=1, batch=3008, lr=lr, pos_weight=2.0, use_graph=0)
    losses = M.msp_model_train(ctx, _dev(X), _dev(y), tp)
    w1 = M.msp_model_get(ctx).astype(np.float64)
    Lo, go = N.loss_and_grad(N.effective(w32), X.astype(np.float64), y, 2.0)
    wo, _, _ = N.adam_step(w32.astype(np.float64), 0.0, 0.0, go, 1, lr)
    assert abs(losses[0] - Lo) <= 1e-5 * max(1.0, abs(Lo))
    sig = np.abs(go) > 1e-3 * np.max(np.abs(go))       # the step is lr * sign(g) there
    assert np.max(np.abs(w1[sig] - wo[sig])) <= 1e-6
    assert np.max(np.abs(w1 - w32)) <= lr * 1.001


def test_training_graph_replays_match_eager_launches(M, ctx):
    rng = np.random.default_rng(5)
    count = 5000                                       # 19 full batches of 256 and a ragged one
    X = _dev(rng.standard_normal((count, N.NFEAT)).astype(np.float32))
    y = _dev((rng.random(count) < 0.05).astype(np.uint8))
    M.msp_model_init(ctx, 42)
    w0 = M.msp_model_get(ctx)
    for epochs in (1, 3, 4):
        res = {}
        for graph in (0, 1):
            M.msp_model_set(ctx, w0)
            tp = M.msp_train_params_default(epochs=epochs, batch=256, lr=3e-3, seed=9, use_graph=graph)
            losses = M.msp_model_train(ctx, X, y, tp)
            torch.cuda.synchronize()
            res[graph] = (losses, M.msp_model_get(ctx))
        assert res[0][0] == res[1][0], epochs
        assert np.array_equal(res[0][1], res[1][1]), epochs
        assert not np.array_equal(res[1][1], w0)


@pytest.mark.parametrize("seed,m,D", [(2001, 6, 100), (2002, 6, 50), (4100, 7, 100), (4101, 7, 200)])
def test_orders_keep_the_exhaustive_result(M, ctx, seed, m, D):
    inst = mi.msp_class(m, D, seed)
    A, d = _dev(inst.A), _dev(inst.d)
    prm = M.msp_params_default(time_cap_ms=60000.0)
    Bk = M.msp_reduce(ctx, A, d, prm)
    M.msp_model_init(ctx, 3)
    runs = {}
    for order in (M.MSP_PLAIN, M.MSP_LEARNED, M.MSP_DISCREPANCY):
        print(f"  order {order} m={m} seed={seed}", flush=True)
        r = M.msp_enumerate(ctx, A, d, Bk, params=prm, order=order)
        assert r.status == M.MSP_OK
        runs[order] = (E.sort_rows(r.x.cpu().numpy()), r.stats)
    x0, s0 = runs[M.MSP_PLAIN]
    assert E.verify(inst.A, inst.d, x0)
    for order in (M.MSP_LEARNED, M.MSP_DISCREPANCY):
        x, s = runs[order]
        assert np.array_equal(x, x0)
        for key in ("evals", "nodes", "expansions", "leaves", "roots"):
            assert s[key] == s0[key], (order, key)
        assert s["ordering_ms"] > 0.0


@pytest.mark.parametrize("order", [1, 2])
def test_first_mode_with_orders_returns_verified_solutions(M, ctx, order):
    M.msp_model_init(ctx, 4)
    for seed in (4102, 4105):
        inst = mi.msp_class(7, 100, seed)
        A, d = _dev(inst.A), _dev(inst.d)
        prm = M.msp_params_default(time_cap_ms=60000.0)
        Bk = M.msp_reduce(ctx, A, d, prm)
        r = M.msp_enumerate(ctx, A, d, Bk, params=prm, mode=M.MSP_FIRST, order=order, cap=64)
        assert r.status == M.MSP_OK and r.n_found >= 1
        assert E.verify(inst.A, inst.d, r.x.cpu().numpy())
        assert r.stats["ttfs_ms"] >= r.stats["ordering_ms"] > 0.0


def test_learned_order_needs_a_model(M):
    c = M.Context(0)
    try:
        inst = mi.msp_class(5, 100, 3)
        A, d = _dev(inst.A), _dev(inst.d)
        Bk = M.msp_reduce(c, A, d)
        with pytest.raises(M.MspError) as ei:
            M.msp_enumerate(c, A, d, Bk, order=M.MSP_LEARNED)
        assert ei.value.code == M.MSP_E_ARG
        with pytest.raises(M.MspError):
            M.msp_model_get(c)
        with pytest.raises(M.MspError):
            M.msp_model_set(c, np.full(N.NPARAM, np.nan, dtype=np.float32))
    finally:
        c.close()


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("m,seed,feasible", [(6, 31, True), (7, 32, True), (6, 33, False), (7, 34, False)])
def test_refined_first_search_stays_exhaustive(M, ctx, order, m, seed, feasible):
    """Best-first refinement reorders the tree but covers it exactly once:
    with refinement forced through several stages, first mode returns an
    oracle solution where there is one, and where there is none (d_0 beyond
    the row sum) it walks exactly the nodes of the plain exhaustive run."""
    M.msp_model_init(ctx, 6)
    inst = mi.cornuejols_dawande(m, seed)
    A_np, d_np = inst.A, inst.d.copy()
    if not feasible:
        d_np[0] = int(A_np[0].astype(np.int64).sum()) + 1
    P = L.prepare(A_np, d_np)
    ref = E.enumerate_prepared(P, split=6, threads=8)
    assert (ref.n_found > 0) == feasible
    A, d, Bk = _dev(A_np), _dev(d_np), _dev(P.basis)
    base = M.msp_params_default(time_cap_ms=60000.0)
    plain = M.msp_enumerate(ctx, A, d, Bk, params=base)
    assert plain.status == M.MSP_OK and plain.n_found == ref.n_found
    prm = M.msp_params_default(time_cap_ms=60000.0, target_roots=2048, refine=-1, refine_keep=64)
    print(f"  refined first m={m} seed={seed} order={order} oracle solutions={ref.n_found}", flush=True)
    r = M.msp_enumerate(ctx, A, d, Bk, params=prm, mode=M.MSP_FIRST, order=order, cap=64)
    assert r.status == M.MSP_OK
    assert r.stats["stages"] >= 1 and r.stats["root_level"] < P.k - r.stats["split_depth"]
    if not feasible:
        assert r.n_found == 0
        for key in ("evals", "nodes", "expansions", "leaves"):
            assert r.stats[key] == plain.stats[key], key
    else:
        x = r.x.cpu().numpy()
        assert 1 <= x.shape[0] and E.verify(A_np, d_np, x)
        rows = {tuple(row) for row in ref.solutions}
        assert all(tuple(row) in rows for row in x)
