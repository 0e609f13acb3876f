"""CPU pins of the oracle's root-ordering parts: BF16 rounding, the MLP's
forward pass, gradient and Adam step, and the subtree roots, features and
labels of tree partitioning."""
from __future__ import annotations

import numpy as np
import pytest

import msp_instances as mi
from oracle import enum as E
from oracle import lattice as L
from oracle import mlp as N
from oracle import roots as RT


def test_bf16_round_hand_values():
    one = 1.0
    cases = [
        (one, one),
        (one + 2.0 ** -8, one),                        # halfway, ties to even (down)
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),        # halfway, ties to even (up)
        (one + 2.0 ** -8 + 2.0 ** -20, one + 2.0 ** -7),
        (-(one + 2.0 ** -8 + 2.0 ** -20), -(one + 2.0 ** -7)),
        (3.0, 3.0),
        (0.1, 0.10009765625),
        (0.0, 0.0),
    ]
    for x, want in cases:
        got = N.bf16_round(np.array([x], dtype=np.float32))[0]
        assert got == np.float32(want), (x, got, want)
    sp = N.bf16_round(np.array([np.inf, -np.inf, np.nan], dtype=np.float32))
    assert np.isinf(sp[0]) and sp[0] > 0 and np.isinf(sp[1]) and sp[1] < 0 and np.isnan(sp[2])
    # every result has 16 zero low bits and is within half a bf16 ulp
    rng = np.random.default_rng(5)
    x = rng.standard_normal(10000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 10000)
    r = N.bf16_round(x)
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
    ulp = np.abs(x.astype(np.float64)) * 2.0 ** -7
    assert np.all(np.abs(r.astype(np.float64) - x) <= 0.5 * ulp * 1.0001)


def test_forward_closed_form_l1_norm():
    # h1 = (relu(x), relu(-x), 0..), h2 = h1, z = sum h2 + b3 = ||x||_1 + b3
    W1 = np.zeros((N.HID, N.NFEAT))
    W1[:16] = np.eye(16)
    W1[16:32] = -np.eye(16)
    W2 = np.eye(N.HID)
    W3 = np.zeros(N.HID)
    W3[:32] = 1.0
    w = N.pack(W1, np.zeros(N.HID), W2, np.zeros(N.HID), W3, 0.5)
    X = np.random.default_rng(1).standard_normal((9, 16))
    assert np.allclose(N.forward(w, X), np.abs(X).sum(axis=1) + 0.5, rtol=0, atol=1e-12)
    # a transposed W2 changes the answer once W2 is not symmetric
    W2b = np.eye(N.HID)
    W2b[0, 20] = 1.0
    wb = N.pack(W1, np.zeros(N.HID), W2b, np.zeros(N.HID), W3, 0.5)
    want = np.abs(X).sum(axis=1) + 0.5 + np.maximum(-X[:, 4], 0.0)
    assert np.allclose(N.forward(wb, X), want, atol=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    w = rng.standard_normal(N.NPARAM) * 0.3
    X = rng.standard_normal((7, N.NFEAT))
    y = np.array([1, 0, 0, 1, 0, 0, 0])
    L0, g = N.loss_and_grad(w, X, y, pos_weight=3.0)
    assert abs(L0 - N.loss(w, X, y, 3.0)) < 1e-14
    h = 1e-6
    fd = np.empty_like(w)
    for p in range(N.NPARAM):
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd[p] = (N.loss(wp, X, y, 3.0) - N.loss(wm, X, y, 3.0)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))
    assert np.count_nonzero(g) > N.NPARAM // 4


def test_adam_closed_form_first_steps():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w0 = np.zeros(4)
    w1, m, v = N.adam_step(w0, np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(w1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # with a constant gradient the corrected moments stay g and g^2
    w2, m, v = N.adam_step(w1, m, v, g, 2, lr=0.01)
    assert np.allclose(w2 - w1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)


def test_zigzag_rank_against_listed_sequence():
    rng = np.random.default_rng(3)
    for _ in range(200):
        y = float(rng.uniform(-5, 5))
        c = -y
        u1 = int(np.rint(c))
        s = 1 if u1 - c <= 0 else -1
        seq, off = [u1], 0
        for _ in range(20):
            off = RT._zig_next(off, s)
            seq.append(u1 + off)
        assert sorted(seq[:21]) == list(range(min(seq[:21]), max(seq[:21]) + 1))  # no repeats, no gaps
        for idx, val in enumerate(seq):
            assert RT.zigzag_rank(val, y, False) == idx
    for uj in range(6):
        assert RT.zigzag_rank(uj, 0.3, True) == uj


@pytest.mark.parametrize("m,D,seed,split", [(3, 100, 1001, 4), (4, 50, 7, 6), (4, 100, 11, 9), (5, 200, 13, 8)])
def test_roots_match_recursive_enumerator_and_partition_solutions(m, D, seed, split):
    inst = mi.single_small(seed) if m == 3 else mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    roots = RT.roots_dfs(P, split)
    ref = E.enumerate_prepared(P, split=split)
    assert len(roots) == ref.n_roots
    Lv = P.k - split
    lab = RT.labels(P, roots, Lv, ref.solutions)
    # every solution lies below exactly one root: the subtrees partition the tree
    pref = [tuple(rt.u[Lv:]) for rt in roots]
    assert len(set(pref)) == len(pref)
    index = {p: i for i, p in enumerate(pref)}
    hits = [index.get(tuple(int(c) for c in RT.coefficients(P, x)[Lv:])) for x in ref.solutions]
    assert all(h is not None for h in hits)
    assert int(lab.sum()) == len(set(hits)) and 1 <= lab.sum() <= ref.n_found
    # the planted solution's root is labelled
    up = RT.coefficients(P, inst.x_planted)
    assert lab[index[tuple(int(c) for c in up[Lv:])]] == 1
    F = RT.features(P, roots, Lv)
    R = P.n + 1
    for r, rt in enumerate(roots):
        # partial norm = ||w||^2 up to rounding
        assert abs(float(F[r, 0]) * R - float(rt.w @ rt.w)) <= 1e-6 * R
        assert abs(F[r, 12] - r / len(roots)) < 1e-7
    assert np.all(F[:, 0] <= 1.0 + 1e-6) and np.all(F[:, 1] <= 1.0 + 1e-6)
    assert np.all((F[:, 4] >= 0) & (F[:, 4] <= 1))


def test_root_features_hand_computed_fixture():
    """All 16 root features of three hand-made roots on a k=3, n=3, m=1
    lattice (L = 1, R = 4), each value worked out by hand from the feature
    definitions, independently of the oracle's code."""
    import math
    from types import SimpleNamespace

    mu = np.zeros((3, 3))
    mu[1, 0], mu[2, 0], mu[2, 1] = 0.5, 0.25, -0.5
    P = SimpleNamespace(k=3, dim=4, m=1, n=3, mu=mu, beta=np.array([2.0, 3.0, 4.0]))
    roots = [
        # u_2 = 1 (top-zero level: rank 1); y_1 = 1 * -0.5, c = 0.5, u1 = rint(0.5) = 0,
        # s = +1 (0 - 0.5 <= 0), u_1 = 1 is u1 + 1 on the side of s: rank 1; x_L = 0.5
        RT.Root(u=[0, 1, 1], l=3.5, w=np.array([1.0, -1.0, 0.5, 0.0])),
        # u_2 = 2 (rank 2); y_1 = -1, c = 1, u1 = 1, s = +1, u_1 = -1 = u1 - 2: rank 4; x_L = -2
        RT.Root(u=[0, -1, 2], l=2.0, w=np.array([0.25, 2.0, -3.0, 5.0])),
        # both levels top-zero with value 0: every rank, value and norm is 0
        RT.Root(u=[0, 0, 0], l=0.0, w=np.zeros(4)),
    ]
    want = np.array([
        [3.5 / 4, 3.5 / 2.5, 1 / 4, 1.0, 1.0, 1 / 8, 1.0, 1.0, 1 / 4,
         0.25 * 3 / 4, 0.5 / 2, (1 / 3) * math.log(0.5 / 4) / 8, 0.0, 0.0, 1 / 3, 1 / 16],
        [2 / 4, 2 / 10.25, 1.0, 3.0, 1.0, 4 / 8, 1.0, 1.5, 2 / 4,
         4 * 3 / 4, 1.0, (1 / 3) * math.log(2 / 4) / 8, 1 / 3, 3 / 4, 1 / 3, 1 / 16],
        [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
         0.0, 0.0, 0.0, 2 / 3, 0.0, 1 / 3, 1 / 16],
    ], dtype=np.float32)
    got = RT.features(P, roots, 1)
    assert got.dtype == np.float32 and got.shape == (3, RT.NFEAT)
    np.testing.assert_array_equal(got, want)
