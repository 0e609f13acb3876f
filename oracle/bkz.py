"""CPU oracle, part 7: the block condition of BKZ reduction (the paper's
"blockwise Korkine-Zolotarev" reduction, Section 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a basis b_0..b_{k-1} with exact Gram-Schmidt data (mu, beta = ||b_hat||^2)
and a block [j, h], the projected block lattice is
    L_j,h = { pi_j(sum_{i=j}^{h} u_i b_i) : u integer },
whose vectors have squared length
    sum_{i=j}^{h} beta_i (u_i + sum_{l=i+1}^{h} u_l mu_{l,i})^2.
``block_shortest`` finds its shortest non-zero vector by exhaustive
depth-first enumeration (levels h down to j, every integer u_i whose
partial length stays within the best length so far), with every length in
exact rationals, so the minimum it returns is exact.  A basis is BKZ-reduced
with block size beta and insertion threshold delta when, for every j,
    delta * beta_j <= lambda_1(L_j,min(j+beta-1,k-1))^2,
i.e. no vector of a projected block is shorter than delta * ||b_hat_j||^2.
"""
from __future__ import annotations

import math
from fractions import Fraction

from .lattice import GSExact, gram_schmidt_exact


def block_shortest(gs: GSExact, j: int, h: int):
    """Exact (lambda_1^2, u) of the projected block lattice L_j,h (u indexed
    from j; the sign of u is normalised so its last non-zero entry is > 0)."""
    beta = [gs.beta(i) for i in range(j, h + 1)]
    mu = [[gs.mu(l, i) for i in range(j, h + 1)] for l in range(j, h + 1)]  # mu[l-j][i-j]
    size = h - j + 1
    best = [beta[0], [1] + [0] * (size - 1)]      # b_hat_j itself lies in the block
    u = [0] * size

    def rec(i: int, partial: Fraction):
        # centre of level i from the levels above it in the block
        c = -sum((u[l] * mu[l][i] for l in range(i + 1, size)), Fraction(0))
        room = best[0] - partial
        if room < 0:
            return
        # every integer x with beta_i (x - c)^2 <= room
        span = math.isqrt(int(room / beta[i]) + 1) + 1
        base = math.floor(c)
        for x in range(base - span, base + span + 2):
            t = partial + beta[i] * (x - c) ** 2
            if t > best[0]:
                continue
            u[i] = x
            if i == 0:
                if any(u) and t < best[0]:
                    best[0], best[1] = t, list(u)
            else:
                rec(i - 1, t)
        u[i] = 0

    rec(size - 1, Fraction(0))
    v = best[1]
    nz = [q for q in v if q != 0]
    if nz and nz[-1] < 0:
        v = [-q for q in v]
    return best[0], v


def bkz_violations(basis, block: int, delta: Fraction = Fraction(999, 1000)):
    """Blocks [j, min(j + block - 1, k - 1)] of an integer basis that hold a
    vector shorter than delta * ||b_hat_j||^2: list of (j, lambda_1^2, beta_j)."""
    gs = gram_schmidt_exact([[int(c) for c in row] for row in basis])
    out = []
    for j in range(gs.k - 1):
        h = min(j + block - 1, gs.k - 1)
        lam, _ = block_shortest(gs, j, h)
        if lam < delta * gs.beta(j):
            out.append((j, lam, gs.beta(j)))
    return out
