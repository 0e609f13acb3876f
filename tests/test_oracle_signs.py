"""CPU pins of the oracle with entries of either sign and with general box
bounds (paper, Section 2: A and d may hold negative entries; a lower bound l
is moved to 0 by x := x - l, d := d - A l, r := u - l): the enumerator's
solution sets equal brute force over {0,1}^n, and over the box l <= x <= u."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import msp_instances as mi
from oracle import brute as B
from oracle import enum as E


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_signed_binary_instances_match_brute_force(seed):
    inst = mi.signed_planted(3, 18, -50, 50, seed)
    assert (inst.A < 0).any() and (inst.A > 0).any()
    _, r = E.solve(inst.A, inst.d, split=4, threads=2)
    want = B.brute_force(inst.A, inst.d)
    assert np.array_equal(r.solutions, E.sort_rows(want))
    assert any(np.array_equal(x, inst.x_planted) for x in r.solutions)


def box_brute_force(A, d, lo, hi) -> np.ndarray:
    """Every integer x with lo <= x <= hi and A x = d (sorted rows, int64)."""
    ranges = [range(int(l), int(u) + 1) for l, u in zip(lo, hi)]
    X = np.array(list(itertools.product(*ranges)), dtype=np.int64)
    keep = np.all(X @ np.asarray(A, dtype=np.int64).T == np.asarray(d, dtype=np.int64)[None, :], axis=1)
    X = X[keep]
    return X[np.lexsort(X.T[::-1])] if X.shape[0] else X


def shifted_oracle(A, d, lo, hi) -> np.ndarray:
    """The oracle on the shifted problem (x' = x - l in [0, u - l]), shifted back."""
    lo64 = np.asarray(lo, dtype=np.int64)
    d2 = np.asarray(d, dtype=np.int64) - np.asarray(A, dtype=np.int64) @ lo64
    r = (np.asarray(hi, dtype=np.int64) - lo64).astype(np.int64)
    _, res = E.solve(A, d2, r=r, split=3, threads=2)
    X = res.solutions.astype(np.int64) + lo64[None, :]
    return X[np.lexsort(X.T[::-1])] if X.shape[0] else X


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_box_bounds_with_negative_entries_match_brute_force(seed):
    b = mi.box_planted(2, 8, -6, 7, -2, 2, 2, seed)
    assert (b.lo < 0).any()
    want = box_brute_force(b.A, b.d, b.lo, b.hi)
    got = shifted_oracle(b.A, b.d, b.lo, b.hi)
    assert np.array_equal(got, want)
    assert any(np.array_equal(x, b.x_planted) for x in got)
