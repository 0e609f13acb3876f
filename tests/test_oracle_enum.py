"""Pins of the oracle's enumeration (Algorithm 1) against what the problem
definition and the mathematics fix, independently of any lattice code:
brute force over 2^n, meet-in-the-middle, DP counts, a closed form, the
planted solution, exact A x = d, basis independence, exact-rational
soundness of both pruning tests on solution paths (Thm 2), and invariance of
the search-tree counters under the root split."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import msp_instances as mi
from oracle import brute as B
from oracle import enum as E
from oracle import lattice as L

SMALL = [(m, n, D) for (m, n, D) in [(1, 14, 20), (1, 18, 100), (2, 16, 5), (2, 18, 10), (2, 20, 5),
                                     (3, 20, 20), (3, 20, 100), (4, 22, 10)]]


@pytest.mark.parametrize("m,n,D", SMALL)
def test_enumerator_equals_brute_force(m, n, D):
    multi = 0
    for seed in range(6):
        inst = mi.planted(m, n, D, 100 + seed)
        _, r = E.solve(inst.A, inst.d, threads=2, split=2)
        bf = B.brute_force(inst.A, inst.d)
        assert r.solutions.shape == bf.shape
        assert (r.solutions == bf).all()
        multi += bf.shape[0] > 1
    if D <= 10:
        assert multi > 0  # the small-D classes exercise many-solution instances


def test_config1_instance_brute_force():
    inst = mi.single_small()
    _, r = E.solve(inst.A, inst.d)
    bf = B.brute_force(inst.A, inst.d)
    assert (r.solutions == bf).all() and r.n_found == bf.shape[0] >= 1


@pytest.mark.parametrize("seed", [1, 2])
def test_enumerator_equals_meet_in_middle_m5(seed):
    inst = mi.msp_class(5, 50, seed)  # n = 40
    _, r = E.solve(inst.A, inst.d, threads=4, split=6)
    mm = B.meet_in_middle(inst.A, inst.d)
    assert (r.solutions == mm).all() and r.n_found == mm.shape[0]


@pytest.mark.parametrize("m,n,D,seed", [(1, 28, 10000, 3), (2, 32, 200, 4), (2, 30, 30, 7), (2, 24, 5, 8)])
def test_counts_equal_dp(m, n, D, seed):
    inst = mi.planted(m, n, D, seed)
    _, r = E.solve(inst.A, inst.d, threads=4, split=4, cap=1 << 20)
    assert r.n_found == B.count_dp(inst.A, inst.d)
    assert E.verify(inst.A, inst.d, r.solutions)


@pytest.mark.parametrize("n,c,a", [(12, 4, 7), (16, 8, 3), (14, 1, 5), (18, 9, 1)])
def test_binomial_closed_form(n, c, a):
    """m = 1, every a_j = a, d = a c: the solutions are the C(n, c) subsets of size c."""
    A = np.full((1, n), a, dtype=np.int32)
    d = np.array([a * c], dtype=np.int64)
    _, r = E.solve(A, d, cap=1 << 16)
    assert r.n_found == math.comb(n, c)
    assert (r.solutions.sum(axis=1) == c).all()
    assert len({row.tobytes() for row in r.solutions}) == r.n_found


@pytest.mark.parametrize("m,D", [(4, 100), (5, 200), (6, 100)])
def test_planted_solution_found_and_verified(m, D):
    for seed in range(3):
        inst = mi.msp_class(m, D, 300 + seed)
        _, r = E.solve(inst.A, inst.d, threads=4, split=6)
        assert E.verify(inst.A, inst.d, r.solutions)
        assert any((row == inst.x_planted).all() for row in r.solutions)


def _random_unimodular(k, rng, steps=60):
    U = np.eye(k, dtype=np.int64)
    for _ in range(steps):
        i, j = rng.choice(k, 2, replace=False)
        U[i] += int(rng.integers(-1, 2)) * U[j]
    perm = rng.permutation(k)
    return U[perm]


def test_basis_independence():
    inst = mi.msp_class(4, 50, 17)
    P = L.prepare(inst.A, inst.d)
    r0 = E.enumerate_prepared(P)
    rng = np.random.default_rng(0)
    for _ in range(3):
        U = _random_unimodular(P.k, rng)
        Bt = U @ P.basis
        P2 = L.prepare_from_basis(inst.A, inst.d, Bt)
        r2 = E.enumerate_prepared(P2)
        assert (r2.solutions == r0.solutions).all()


def test_shuffled_variables_same_solutions():
    inst = mi.planted(3, 20, 10, 23)
    _, r0 = E.solve(inst.A, inst.d)
    perm = np.random.default_rng(1).permutation(inst.n)
    _, r1 = E.solve(inst.A[:, perm], inst.d)
    back = np.zeros_like(r1.solutions)
    back[:, perm] = r1.solutions
    assert (E.sort_rows(back) == r0.solutions).all()


def test_split_depth_and_threads_leave_counters_unchanged():
    inst = mi.msp_class(6, 100, 2000)
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P)
    for s in (1, 3, 8, 15, 30):
        for th in (1, 3):
            r = E.enumerate_prepared(P, split=s, threads=th)
            assert (r.evals, r.nodes, r.expansions, r.leaves) == (ref.evals, ref.nodes, ref.expansions, ref.leaves)
            assert (r.solutions == ref.solutions).all()


def test_pruning_variants_keep_the_solution_set():
    """The one-direction cut and the Hoelder test only remove subtrees without
    solutions: turning them off must give the same set with more nodes."""
    for seed, (m, n, D) in enumerate([(3, 20, 10), (4, 30, 20), (2, 20, 5)]):
        inst = mi.planted(m, n, D, 40 + seed)
        P = L.prepare(inst.A, inst.d)
        full = E.enumerate_prepared(P)
        no_cut = E.enumerate_prepared(P, onedir=False)
        no_h = E.enumerate_prepared(P, hoelder=False)
        assert (no_cut.solutions == full.solutions).all()
        assert (no_h.solutions == full.solutions).all()
        assert no_h.nodes >= no_cut.nodes >= full.nodes


def test_solution_paths_pass_both_tests_exactly():
    """Thm 2 with y = e_t and the l2 bound, in exact rationals: for every
    solution v and every level t >= 1, ||pi_t v||^2 <= R and
    ||pi_t v||^2 <= r_max ||pi_t v||_1 (l1 over all n+1 coordinates)."""
    for seed in range(3):
        inst = mi.planted(3, 14, 20, 70 + seed)
        P = L.prepare(inst.A, inst.d)
        gs = P.gs
        r = E.enumerate_prepared(P)
        R = inst.n + 1
        bh = [gs.bhat(i) for i in range(gs.k)]
        for x in r.solutions:
            v = [2 * int(c) - 1 for c in x] + [1]
            # coordinates of v along b_hat_j: <v, b_hat_j> / beta_j
            coef = [sum(Fraction(a) * b for a, b in zip(v, bh[j])) / gs.beta(j) for j in range(gs.k)]
            for t in range(1, gs.k):
                proj = [sum(coef[j] * bh[j][c] for j in range(t, gs.k)) for c in range(gs.dim)]
                l2 = sum(p * p for p in proj)
                l1 = sum(abs(p) for p in proj)
                assert l2 <= R
                assert l2 <= l1
            assert sum(c * c for c in v) == R  # a solution sits exactly on the l2 bound


def test_first_mode_returns_a_verified_solution():
    inst = mi.msp_class(5, 50, 3)
    P = L.prepare(inst.A, inst.d)
    full = E.enumerate_prepared(P, threads=4, split=5)
    r = E.enumerate_prepared(P, threads=4, split=5, mode="first")
    assert r.n_found >= 1
    allset = {row.tobytes() for row in full.solutions}
    assert all(row.tobytes() in allset for row in r.solutions)


def test_time_cap_gives_a_subset():
    inst = mi.msp_class(7, 50, 5)
    P = L.prepare(inst.A, inst.d)
    r = E.enumerate_prepared(P, threads=2, split=6, time_cap_s=0.05)
    assert E.verify(inst.A, inst.d, r.solutions)
