"""CPU oracle, part 4: solution sets computed without any lattice.

TEST INFRASTRUCTURE ONLY (see the package docstring).

These pin the enumerator's output against the plain definition of the
feasibility problem (Section 1): S(A, d) = {x in {0,1}^n : A x = d}.

  * ``brute_force``  -- all 2^n vectors, n <= 24 (chunked numpy).
  * ``meet_in_middle`` -- the textbook two-list method: split the variables
    into halves, tabulate A x_L for every left half, and look up d - A x_R
    for every right half.  Exact, n <= ~40.
  * ``count_dp``     -- number of solutions by dynamic programming over a
    dense table of partial sums (m = 1 is subset sum, Section 1; m = 2 uses a
    2-D table).
"""
from __future__ import annotations

import numpy as np


def _bits(n: int, start: int, count: int) -> np.ndarray:
    idx = np.arange(start, start + count, dtype=np.int64)
    return ((idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.uint8)


def sort_rows(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint8)
    if x.shape[0] == 0:
        return x.reshape(0, x.shape[1] if x.ndim == 2 else 0)
    return x[np.lexsort(x.T[::-1])]


def brute_force(A, d, chunk: int = 1 << 16) -> np.ndarray:
    """Every x in {0,1}^n with A x = d, by exhaustive search (n <= 24)."""
    A = np.asarray(A, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    m, n = A.shape
    if n > 24:
        raise ValueError("brute force is limited to n <= 24")
    total = 1 << n
    hits = []
    for start in range(0, total, chunk):
        cnt = min(chunk, total - start)
        X = _bits(n, start, cnt)
        ok = np.all(X.astype(np.int64) @ A.T == d[None, :], axis=1)
        if ok.any():
            hits.append(X[ok])
    if not hits:
        return np.zeros((0, n), dtype=np.uint8)
    return sort_rows(np.concatenate(hits))


def meet_in_middle(A, d) -> np.ndarray:
    """Exact solution set by a two-list split (n <= ~40)."""
    A = np.asarray(A, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    m, n = A.shape
    nl = n // 2
    nr = n - nl
    if max(nl, nr) > 21:
        raise ValueError("meet-in-the-middle is limited to n <= 42")
    XL = _bits(nl, 0, 1 << nl)
    XR = _bits(nr, 0, 1 << nr)
    SL = XL.astype(np.int64) @ A[:, :nl].T  # (2^nl, m)
    SR = d[None, :] - XR.astype(np.int64) @ A[:, nl:].T
    # match rows of SL against rows of SR exactly via a structured view
    def key(M):
        M = np.ascontiguousarray(M)
        return M.view(np.dtype((np.void, M.dtype.itemsize * M.shape[1]))).ravel()
    kl, kr = key(SL), key(SR)
    order = np.argsort(kl, kind="stable")
    kl_sorted = kl[order]
    lo = np.searchsorted(kl_sorted, kr, side="left")
    hi = np.searchsorted(kl_sorted, kr, side="right")
    rows = []
    for j in np.nonzero(hi > lo)[0]:
        for i in order[lo[j]:hi[j]]:
            rows.append(np.concatenate([XL[i], XR[j]]))
    if not rows:
        return np.zeros((0, n), dtype=np.uint8)
    return sort_rows(np.array(rows, dtype=np.uint8))


def count_dp(A, d) -> int:
    """Number of x in {0,1}^n with A x = d (m <= 2, entries >= 0), by dynamic
    programming over a dense table of reachable sums: after column j,
    table[s] = number of x_1..x_j with partial sums s.  Exact in int64 for
    n <= 62 (counts never exceed 2^n)."""
    A = np.asarray(A, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    m, n = A.shape
    if m > 2 or n > 62 or (A < 0).any() or (d < 0).any():
        raise ValueError("count_dp handles m <= 2, n <= 62, non-negative data")
    if m == 1:
        S = int(d[0])
        tab = np.zeros(S + 1, dtype=np.int64)
        tab[0] = 1
        for j in range(n):
            a = int(A[0, j])
            if a == 0:
                tab = tab * 2
            elif a <= S:
                tab[a:] = tab[a:] + tab[:-a].copy()
        return int(tab[S])
    S1, S2 = int(d[0]), int(d[1])
    tab = np.zeros((S1 + 1, S2 + 1), dtype=np.int64)
    tab[0, 0] = 1
    for j in range(n):
        a, b = int(A[0, j]), int(A[1, j])
        if a > S1 or b > S2:
            continue
        shifted = np.zeros_like(tab)
        shifted[a:, b:] = tab[: S1 + 1 - a, : S2 + 1 - b]
        tab = tab + shifted
    return int(tab[S1, S2])


def brute_force_bounded(A, d, r) -> np.ndarray:
    """All x with 0 <= x_j <= r_j and A x = d, by trying every point of the
    box (prod (r_j + 1) points; small boxes only).  Rows sorted
    lexicographically, uint8."""
    import itertools
    A = np.asarray(A, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    r = [int(v) for v in r]
    total = 1
    for v in r:
        total *= v + 1
    assert total <= 1 << 22, "box too large for brute force"
    pts = np.array(list(itertools.product(*[range(v + 1) for v in r])), dtype=np.int64)
    ok = np.all(pts @ A.T == d[None, :], axis=1)
    return pts[ok].astype(np.uint8)
