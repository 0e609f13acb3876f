"""CPU oracle, part 1: the lattice set-up in exact integer arithmetic.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

What is here (paper, Section 2):
  * ``embedding``      -- the generator matrix of eq. (2), binary case
                          (r_max = c_i = 1), stored as n+1 basis vectors.
  * ``lll_exact``      -- integral LLL (all quantities are exact integers:
                          Gram determinants d_i and lambda_ij = d_j mu_ij),
                          the reduction of step 1 of Algorithm 1.
  * ``extract_kernel`` -- keep the n-m+1 reduced vectors whose first m
                          entries vanish and drop those m entries (step 2).
  * ``gram_schmidt_exact`` -- eq. (4) in exact rationals (fraction-free
                          integer recurrences), with float64 roundings of
                          mu, beta = ||b_hat||^2 and b_hat (step 3).

Nothing here depends on floating point except the final rounding of exact
rationals to the nearest float64.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import math

import numpy as np

DEFAULT_N = 1 << 10  # Section 2: N = 2^10 suffices for the market split classes


class NotIsolated(Exception):
    """N was too small: fewer than n - m + 1 reduced vectors are zero in their
    first m entries, so the basis does not split into kernel vectors and
    others the way Section 2 describes."""


class RankDeficient(Exception):
    """More than n - m + 1 reduced vectors are zero in their first m entries:
    the kernel has dimension n - rank(A) + 1 > n - m + 1, i.e. the rows of A
    are dependent (rank A < m)."""


def bounds_scale(r) -> tuple[int, list[int]]:
    """r_max = lcm(r_1..r_n) and c_j = r_max / r_j (Section 2, under eq. (2))."""
    rmax = 1
    for rj in r:
        rj = int(rj)
        if rj < 1:
            raise ValueError("upper bounds must be >= 1")
        rmax = rmax * rj // math.gcd(rmax, rj)
    return rmax, [rmax // int(rj) for rj in r]


def embedding(A: np.ndarray, d: np.ndarray, N: int = DEFAULT_N, r=None) -> list[list[int]]:
    """Basis vectors (the columns of eq. (2)).

    With upper bounds 0 <= x_j <= r_j (r = None: binary, r_max = c_j = 1):
    vector 0 = (-N d_1..-N d_m, -r_max (n times), r_max); vector j (1..n) =
    (N a_{1j}..N a_{mj}, 2 c_j e_j, 0).  Each vector has m + n + 1 entries:
    the m scaled equation rows, the n variable rows, the r_max row last.
    Returned as Python ints (exact).
    """
    A = np.asarray(A)
    m, n = A.shape
    rmax, c = bounds_scale(r) if r is not None else (1, [1] * n)
    vecs = []
    v0 = [-N * int(d[i]) for i in range(m)] + [-rmax] * n + [rmax]
    vecs.append(v0)
    for j in range(n):
        v = [N * int(A[i, j]) for i in range(m)] + [0] * n + [0]
        v[m + j] = 2 * c[j]
        vecs.append(v)
    return vecs


def _dot(a, b) -> int:
    return sum(x * y for x, y in zip(a, b))


def _round_div(a: int, b: int) -> int:
    """Nearest integer to a / b for b > 0, ties rounded up (exact)."""
    return (2 * a + b) // (2 * b)


def lll_exact(basis: list[list[int]], delta: Fraction = Fraction(99, 100)) -> list[list[int]]:
    """Integral LLL reduction (Lovász parameter delta, exact size reduction).

    Integer formulation: d_i is the Gram determinant of the first i+1 vectors
    (d_{-1} = 1) and lam[i][j] = d_j * mu_ij for j < i.  Every update is an
    exact integer operation, so the output is size-reduced (|mu_ij| <= 1/2)
    and satisfies the Lovász condition exactly.  The input vectors must be
    linearly independent.
    """
    b = [list(v) for v in basis]
    nv = len(b)
    if nv <= 1:
        return b
    p, q = delta.numerator, delta.denominator
    # dd[i+1] = d_i ; dd[0] = d_{-1} = 1
    dd = [1] + [0] * nv
    lam = [[0] * nv for _ in range(nv)]

    def gram_row(kk: int) -> None:
        # fill lam[kk][0..kk-1] and dd[kk+1]
        for j in range(kk + 1):
            u = _dot(b[kk], b[j])
            for i in range(j):
                u = (dd[i + 1] * u - lam[kk][i] * lam[j][i]) // dd[i]
            if j < kk:
                lam[kk][j] = u
            else:
                if u == 0:
                    raise ValueError("basis vectors are linearly dependent")
                dd[kk + 1] = u

    def red(kk: int, l: int) -> None:
        if 2 * abs(lam[kk][l]) > dd[l + 1]:
            r = _round_div(lam[kk][l], dd[l + 1])
            bk, bl = b[kk], b[l]
            for c in range(len(bk)):
                bk[c] -= r * bl[c]
            lam[kk][l] -= r * dd[l + 1]
            lk, ll = lam[kk], lam[l]
            for i in range(l):
                lk[i] -= r * ll[i]

    def swap(kk: int, kmax: int) -> None:
        b[kk], b[kk - 1] = b[kk - 1], b[kk]
        for j in range(kk - 1):
            lam[kk][j], lam[kk - 1][j] = lam[kk - 1][j], lam[kk][j]
        la = lam[kk][kk - 1]
        B = (dd[kk - 1] * dd[kk + 1] + la * la) // dd[kk]
        for i in range(kk + 1, kmax + 1):
            t = lam[i][kk]
            lam[i][kk] = (dd[kk + 1] * lam[i][kk - 1] - la * t) // dd[kk]
            lam[i][kk - 1] = (B * t + la * lam[i][kk]) // dd[kk + 1]
        dd[kk] = B

    gram_row(0)
    kk, kmax = 1, 0
    while kk < nv:
        if kk > kmax:
            kmax = kk
            gram_row(kk)
        red(kk, kk - 1)
        # swap when q d_k d_{k-2} < p d_{k-1}^2 - q lam^2   (Lovász fails)
        if q * dd[kk + 1] * dd[kk - 1] < p * dd[kk] * dd[kk] - q * lam[kk][kk - 1] ** 2:
            swap(kk, kmax)
            kk = max(1, kk - 1)
        else:
            for l in range(kk - 2, -1, -1):
                red(kk, l)
            kk += 1
    return b


def extract_kernel(reduced: list[list[int]], m: int) -> list[list[int]]:
    """Step 2 of Algorithm 1: keep the vectors whose first m entries are all
    zero (in reduced order) and drop those m entries.

    Exactly n - m + 1 such vectors must exist (Section 2); they then form a
    basis of the kernel of A x - d x_{n+1} = 0 (restricted to the lattice).
    Fewer means N did not isolate the kernel; more means the kernel is larger
    than n - m + 1, because A has dependent rows.
    """
    nv = len(reduced)
    n = nv - 1
    k_expected = n - m + 1
    kern = [v[m:] for v in reduced if all(c == 0 for c in v[:m])]
    if len(kern) < k_expected:
        raise NotIsolated(f"{len(kern)} zero-top vectors, expected {k_expected}")
    if len(kern) > k_expected:
        raise RankDeficient(f"{len(kern)} zero-top vectors, expected {k_expected}")
    return kern


@dataclass
class GSExact:
    """Exact Gram-Schmidt data of a basis b_0..b_{k-1} (rows), eq. (4).

    d[i]   = Gram determinant of b_0..b_i   (d[-1] := 1, stored as dm1)
    lam[i][j] = d[j] * mu_ij   (j < i), integer
    num[i] = d[i-1] * b_hat_i  (integer vector)
    """

    k: int
    dim: int
    d: list[int]
    lam: list[list[int]]
    num: list[list[int]]

    def dm1(self, i: int) -> int:
        return 1 if i == 0 else self.d[i - 1]

    def mu(self, i: int, j: int) -> Fraction:
        if j == i:
            return Fraction(1)
        if j > i:
            return Fraction(0)
        return Fraction(self.lam[i][j], self.d[j])

    def beta(self, i: int) -> Fraction:
        return Fraction(self.d[i], self.dm1(i))

    def bhat(self, i: int) -> list[Fraction]:
        den = self.dm1(i)
        return [Fraction(c, den) for c in self.num[i]]

    # float64 roundings (correctly rounded: int / int is exact-rounded)
    def mu_f64(self) -> np.ndarray:
        out = np.zeros((self.k, self.k), dtype=np.float64)
        for i in range(self.k):
            out[i, i] = 1.0
            for j in range(i):
                out[i, j] = self.lam[i][j] / self.d[j]
        return out

    def beta_f64(self) -> np.ndarray:
        return np.array([self.d[i] / self.dm1(i) for i in range(self.k)], dtype=np.float64)

    def bhat_f64(self) -> np.ndarray:
        out = np.zeros((self.k, self.dim), dtype=np.float64)
        for i in range(self.k):
            den = self.dm1(i)
            out[i] = [c / den for c in self.num[i]]
        return out


def gram_schmidt_exact(basis: list[list[int]]) -> GSExact:
    """Eq. (4) in exact arithmetic, fraction free.

    With a_i^(0) = b_i and a_i^(j+1) = (d_j a_i^(j) - lam_ij a_j^(j)) / d_{j-1}
    every division is exact and a_i^(i) = d_{i-1} b_hat_i.  Then
    lam_ij = d_j mu_ij = d_{j-1} <b_i, b_hat_j> = <b_i, a_j^(j)> and
    d_i = d_{i-1} beta_i = <b_i, a_i^(i)>.
    """
    k = len(basis)
    dim = len(basis[0]) if k else 0
    d: list[int] = [0] * k
    lam = [[0] * k for _ in range(k)]
    num: list[list[int]] = []
    for i in range(k):
        a = list(basis[i])
        for j in range(i):
            dj_1 = 1 if j == 0 else d[j - 1]
            lij = _dot(basis[i], num[j])
            lam[i][j] = lij
            dj = d[j]
            aj = num[j]
            a = [(dj * x - lij * y) // dj_1 for x, y in zip(a, aj)]
        num.append(a)
        di = _dot(basis[i], a)
        if di == 0:
            raise ValueError("basis vectors are linearly dependent")
        d[i] = di
    return GSExact(k=k, dim=dim, d=d, lam=lam, num=num)


@dataclass
class Prepared:
    """Everything the enumeration needs for one instance."""

    m: int
    n: int
    A: np.ndarray
    d: np.ndarray
    basis: np.ndarray  # int64 (k, n+1): reduced kernel basis, r_max coordinate last
    gs: GSExact
    mu: np.ndarray  # float64 (k, k) lower triangle, unit diagonal
    beta: np.ndarray  # float64 (k,)
    bhat: np.ndarray  # float64 (k, n+1)
    r: np.ndarray | None = None  # upper bounds (None: binary)
    rmax: int = 1
    cvec: np.ndarray | None = None  # int64 c_j = r_max / r_j (None: binary)

    @property
    def k(self) -> int:
        return int(self.basis.shape[0])

    @property
    def dim(self) -> int:
        return int(self.basis.shape[1])


def prepare_from_basis(A, d, kernel_basis, r=None) -> Prepared:
    """Exact GS of a given kernel basis (k x (n+1) integer rows)."""
    A = np.asarray(A)
    kb = [[int(c) for c in row] for row in np.asarray(kernel_basis).tolist()]
    gs = gram_schmidt_exact(kb)
    m, n = A.shape
    rmax, c = bounds_scale(r) if r is not None else (1, None)
    return Prepared(m=m, n=n, A=A, d=np.asarray(d), basis=np.array(kb, dtype=np.int64),
                    gs=gs, mu=gs.mu_f64(), beta=gs.beta_f64(), bhat=gs.bhat_f64(),
                    r=None if r is None else np.asarray(r, dtype=np.int64), rmax=rmax,
                    cvec=None if c is None else np.asarray(c, dtype=np.int64))


def prepare(A, d, N: int = DEFAULT_N, delta: Fraction = Fraction(99, 100), r=None) -> Prepared:
    """Steps 1-3 of Algorithm 1 in exact arithmetic (r: upper bounds, None = binary)."""
    A = np.asarray(A)
    m, n = A.shape
    if m > n:
        raise ValueError("m must not exceed n")
    red = lll_exact(embedding(A, d, N, r), delta)
    kern = extract_kernel(red, m)
    return prepare_from_basis(A, d, kern, r)


def check_lll_reduced(basis: list[list[int]], delta: Fraction = Fraction(99, 100),
                      eta: Fraction = Fraction(1, 2)) -> tuple[bool, bool]:
    """Exact test: (size reduced |mu_ij| <= eta, Lovász condition holds)."""
    gs = gram_schmidt_exact(basis)
    size_ok = all(abs(gs.mu(i, j)) <= eta for i in range(gs.k) for j in range(i))
    lov_ok = True
    for i in range(1, gs.k):
        if gs.beta(i) < (delta - gs.mu(i, i - 1) ** 2) * gs.beta(i - 1):
            lov_ok = False
            break
    return size_ok, lov_ok
