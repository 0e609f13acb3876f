"""CPU pins of the oracle's BKZ block condition (oracle/bkz.py): the exact
shortest vector of a projected block against brute force over small
coefficient boxes, the closed form of an orthogonal block, and a basis built
to violate the condition."""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

from oracle import bkz as K
from oracle import lattice as L


def _proj_len(gs, j, h, u):
    """||pi_j(sum u_i b_i)||^2 in exact arithmetic, straight from b_hat."""
    total = Fraction(0)
    for i in range(j, h + 1):
        x = sum((u[l - j] * gs.mu(l, i) for l in range(i, h + 1)), Fraction(0))
        total += x * x * gs.beta(i)
    return total


def test_block_shortest_matches_brute_force():
    rng = np.random.default_rng(5)
    for trial in range(6):
        k = 5
        B = rng.integers(-4, 5, size=(k, 7))
        B[np.arange(k), np.arange(k)] += 9          # full rank
        gs = L.gram_schmidt_exact(B.tolist())
        for j, h in ((0, 2), (1, 3), (2, 4), (0, 4)):
            lam, u = K.block_shortest(gs, j, h)
            assert lam == _proj_len(gs, j, h, u) and any(u)
            best = min(_proj_len(gs, j, h, v)
                       for v in itertools.product(range(-3, 4), repeat=h - j + 1) if any(v))
            assert lam == best, (trial, j, h)


def test_orthogonal_block_closed_form():
    # an orthogonal basis: lambda_1 of every projected block is its shortest row
    B = np.diag([5, 3, 7, 2, 6])
    gs = L.gram_schmidt_exact(B.tolist())
    lam, _ = K.block_shortest(gs, 0, 4)
    assert lam == 4
    lam, _ = K.block_shortest(gs, 1, 2)
    assert lam == 9


def test_violation_is_found():
    # b_1 = (1, 0, ..) is much shorter than b_0 = (20, 1, ..): block [0, 1] holds it
    B = np.array([[20, 1, 0], [1, 0, 0], [0, 0, 3]])
    v = K.bkz_violations(B, 2)
    assert v and v[0][0] == 0 and v[0][1] == 1
    # swapped, the same lattice satisfies the condition
    assert K.bkz_violations(B[[1, 0, 2]], 2) == []
