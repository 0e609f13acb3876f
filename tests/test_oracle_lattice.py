"""Pins of the oracle's lattice set-up (embedding, exact LLL, kernel
extraction, exact Gram-Schmidt) against facts the paper and linear algebra
fix: eq. (2) entry by entry, the LLL conditions and unimodularity checked
exactly, the kernel property of Section 2, and the Gram-Schmidt invariants of
eq. (4)."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import msp_instances as mi
from oracle import lattice as L

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {"vec": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            vals = [int(v) for v in vals]
            if key == "vec":
                out["vec"].append(vals)
            else:
                out[key] = vals
    return out


def test_embedding_matches_hand_written_eq2():
    g = _read_golden("tiny_embedding.txt")
    A = np.array([g["A"]], dtype=np.int32)
    d = np.array(g["d"], dtype=np.int64)
    assert L.embedding(A, d, N=g["N"][0]) == g["vec"]


def test_embedding_layout_general():
    inst = mi.planted(3, 7, 20, 5)
    N = 1024
    vecs = L.embedding(inst.A, inst.d, N)
    m, n = 3, 7
    assert len(vecs) == n + 1 and all(len(v) == m + n + 1 for v in vecs)
    # column 0: -N d, then -r_max n times, then r_max
    assert vecs[0][:m] == [-N * int(x) for x in inst.d]
    assert vecs[0][m:m + n] == [-1] * n and vecs[0][-1] == 1
    for j in range(n):
        v = vecs[j + 1]
        assert v[:m] == [N * int(inst.A[i, j]) for i in range(m)]
        assert v[m:m + n] == [2 if c == j else 0 for c in range(n)]
        assert v[-1] == 0


def _rank_and_solve(B, target):
    """Solve x B = target exactly (B rows independent); returns x as Fractions."""
    rows = [[Fraction(c) for c in r] for r in B]
    k, dim = len(rows), len(rows[0])
    # Gaussian elimination on the transpose system B^T x = target
    M = [[rows[i][j] for i in range(k)] + [Fraction(target[j])] for j in range(dim)]
    piv_cols = []
    r = 0
    for c in range(k):
        p = next((i for i in range(r, dim) if M[i][c] != 0), None)
        if p is None:
            continue
        M[r], M[p] = M[p], M[r]
        inv = 1 / M[r][c]
        M[r] = [v * inv for v in M[r]]
        for i in range(dim):
            if i != r and M[i][c] != 0:
                f = M[i][c]
                M[i] = [a - f * b for a, b in zip(M[i], M[r])]
        piv_cols.append(c)
        r += 1
    # consistency
    for i in range(r, dim):
        assert M[i][k] == 0, "target not in the row span"
    x = [Fraction(0)] * k
    for i, c in enumerate(piv_cols):
        x[c] = M[i][k]
    return x


def _det(M):
    M = [[Fraction(v) for v in row] for row in M]
    n = len(M)
    det = Fraction(1)
    for c in range(n):
        p = next((i for i in range(c, n) if M[i][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for i in range(c + 1, n):
            f = M[i][c] / M[c][c]
            M[i] = [a - f * b for a, b in zip(M[i], M[c])]
    return det


@pytest.mark.parametrize("seed,m,n,D", [(1, 2, 8, 10), (2, 3, 10, 20), (3, 1, 9, 50)])
def test_lll_exact_conditions_and_unimodular(seed, m, n, D):
    inst = mi.planted(m, n, D, seed)
    B = L.embedding(inst.A, inst.d, 64)
    R = L.lll_exact(B)
    size_ok, lov_ok = L.check_lll_reduced(R)
    assert size_ok and lov_ok
    # R = U B with U integral and det U = +-1: solve each row of R in terms of B
    U = [_rank_and_solve(B, r) for r in R]
    assert all(x.denominator == 1 for row in U for x in row)
    assert abs(_det(U)) == 1


def test_check_lll_detects_unreduced_basis():
    # a basis that is not size reduced and violates Lovász
    B = [[1, 0, 0], [5, 1, 0], [0, 0, 7]]
    size_ok, _ = L.check_lll_reduced(B)
    assert not size_ok
    B2 = [[10, 0], [0, 1]]
    _, lov_ok = L.check_lll_reduced(B2)
    assert not lov_ok


@pytest.mark.parametrize("seed,m,D", [(1001, 3, 100), (7, 4, 50), (11, 5, 200)])
def test_kernel_vectors_encode_the_kernel(seed, m, D):
    """Each extracted vector v = (2u'_1 - u_0, ..., 2u'_n - u_0, u_0) with
    A u' = u_0 d (Section 2: a basis of the kernel of A x - d x_{n+1} = 0)."""
    inst = mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    n = inst.n
    assert P.k == n - m + 1 and P.dim == n + 1
    for v in P.basis.tolist():
        u0 = v[n]
        up = []
        for j in range(n):
            assert (v[j] + u0) % 2 == 0
            up.append((v[j] + u0) // 2)
        lhs = inst.A.astype(object) @ np.array(up, dtype=object)
        assert list(lhs) == [u0 * int(x) for x in inst.d]


def test_too_small_N_is_reported():
    inst = mi.msp_class(4, 100, 3)
    with pytest.raises(L.NotIsolated):
        L.prepare(inst.A, inst.d, N=1)


def test_dependent_rows_are_reported_as_rank_deficient():
    # a repeated row leaves rank A = m - 1: the kernel has n - m + 2 vectors
    inst = mi.msp_class(4, 100, 3)
    A2 = np.vstack([inst.A, inst.A[:1]]).astype(np.int32)
    d2 = np.concatenate([inst.d, inst.d[:1]])
    with pytest.raises(L.RankDeficient):
        L.prepare(A2, d2)


@pytest.mark.parametrize("seed,m,D", [(1001, 3, 100), (21, 4, 50)])
def test_gram_schmidt_exact_invariants(seed, m, D):
    inst = mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    gs = P.gs
    bh = [gs.bhat(i) for i in range(gs.k)]
    # orthogonality, exactly
    for i in range(gs.k):
        for j in range(i):
            assert sum(a * b for a, b in zip(bh[i], bh[j])) == 0
    # b_i = b_hat_i + sum_j mu_ij b_hat_j, exactly
    for i in range(gs.k):
        for c in range(gs.dim):
            rec = bh[i][c] + sum(gs.mu(i, j) * bh[j][c] for j in range(i))
            assert rec == int(P.basis[i][c])
    # beta_i = ||b_hat_i||^2 and prod beta = det(Gram), computed independently
    for i in range(gs.k):
        assert gs.beta(i) == sum(x * x for x in bh[i])
    G = [[int(np.dot(P.basis[i].astype(object), P.basis[j].astype(object))) for j in range(gs.k)] for i in range(gs.k)]
    prod = Fraction(1)
    for i in range(gs.k):
        prod *= gs.beta(i)
    assert prod == _det(G)


def test_float64_roundings_are_nearest():
    inst = mi.msp_class(3, 100, 1001)
    P = L.prepare(inst.A, inst.d)
    gs = P.gs
    for i in range(gs.k):
        assert P.beta[i] == float(gs.beta(i))
        for j in range(i):
            assert P.mu[i, j] == float(gs.mu(i, j))
        for c in range(gs.dim):
            assert P.bhat[i, c] == float(gs.bhat(i)[c])
