"""CPU pins of the oracle for bounded variables 0 <= x_j <= r_j (eq. (2) with
r_max = lcm(r_j), c_j = r_max / r_j, and Thm 1's box |v_j| <= r_max)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import brute as B
from oracle import enum as E
from oracle import lattice as L


def test_bounded_embedding_hand_fixture():
    # A = [[3, 5]], d = [8], r = (2, 3): r_max = 6, c = (3, 2), N = 4
    vecs = L.embedding(np.array([[3, 5]]), np.array([8]), N=4, r=[2, 3])
    assert vecs == [[-32, -6, -6, 6], [12, 6, 0, 0], [20, 0, 4, 0]]
    assert L.bounds_scale([1, 2, 3, 4]) == (12, [12, 6, 4, 3])
    assert L.embedding(np.array([[3, 5]]), np.array([8]), N=4, r=[1, 1]) == \
        L.embedding(np.array([[3, 5]]), np.array([8]), N=4)


@pytest.mark.parametrize("seed", range(8))
def test_bounded_sets_match_box_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    m = 1 + seed % 2
    n = 7 + seed % 3
    r = rng.integers(1, 4, size=n)
    A = rng.integers(0, 10, size=(m, n)).astype(np.int32)
    x = np.array([rng.integers(0, rj + 1) for rj in r], dtype=np.int64)
    d = A.astype(np.int64) @ x
    P, res = E.solve(A, d, r=r, split=2)
    want = B.brute_force_bounded(A, d, r)
    assert res.n_found == want.shape[0] and np.array_equal(res.solutions, E.sort_rows(want))
    assert any(np.array_equal(row, x) for row in res.solutions)
    assert E.verify(A, d, res.solutions, r)
    # the one-direction cut and the Hoelder test remove no solution here either
    for hoelder, onedir in ((False, False), (True, False)):
        res2 = E.enumerate_prepared(P, hoelder=hoelder, onedir=onedir)
        assert np.array_equal(res2.solutions, res.solutions)


def test_unit_bounds_are_the_binary_problem():
    rng = np.random.default_rng(7)
    A = rng.integers(0, 50, size=(3, 20)).astype(np.int32)
    d = A.astype(np.int64) @ rng.integers(0, 2, size=20)
    Pb, rb = E.solve(A, d)
    Pr, rr = E.solve(A, d, r=np.ones(20, dtype=np.int64))
    assert np.array_equal(Pb.basis, Pr.basis)
    assert np.array_equal(rb.solutions, rr.solutions)
    assert (rb.nodes, rb.evals) == (rr.nodes, rr.evals)
