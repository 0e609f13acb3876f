"""GPU parity for bounded variables 0 <= x_j <= r_j (eq. (2) in its general
form): the GPU reduction and enumeration against the oracle, search counters
on the oracle's basis, the binary special case, and argument errors."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

from oracle import brute as B
from oracle import enum as E
from oracle import lattice as L

pytestmark = pytest.mark.gpu


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


def _instance(seed, m, n, rhi, D=50):
    rng = np.random.default_rng(seed)
    r = rng.integers(1, rhi + 1, size=n).astype(np.int32)
    A = rng.integers(0, D, size=(m, n)).astype(np.int32)
    x = np.array([rng.integers(0, rj + 1) for rj in r], dtype=np.int64)
    return A, A.astype(np.int64) @ x, r, x


@pytest.mark.parametrize("seed,m,n,rhi", [(200, 3, 20, 3), (201, 4, 24, 3), (202, 5, 40, 2), (203, 5, 30, 4), (205, 6, 40, 3)])
def test_bounded_matches_oracle(M, ctx, seed, m, n, rhi):
    A, d, r, x = _instance(seed, m, n, rhi)
    P = L.prepare(A, d, r=r)
    ref = E.enumerate_prepared(P, split=6, threads=os.cpu_count() or 1)
    print(f"  bounded seed={seed} m={m} n={n} r_max={P.rmax} oracle solutions={ref.n_found}", flush=True)
    prm = M.msp_params_default(time_cap_ms=60000.0)
    Ad, dd, rd = _dev(A), _dev(d), _dev(r)
    # on the oracle's basis: the same set and the same search counters
    g = M.msp_enumerate_bounded(ctx, Ad, dd, rd, _dev(P.basis), params=prm)
    assert g.status == M.MSP_OK and g.n_found == ref.n_found
    assert np.array_equal(E.sort_rows(g.x.cpu().numpy()), ref.solutions)
    for key in ("evals", "nodes", "expansions", "leaves"):
        assert g.stats[key] == getattr(ref, key), key
    # the whole GPU path
    Bk = M.msp_reduce_bounded(ctx, Ad, dd, rd, prm)
    assert Bk.shape[0] == n - m + 1
    g2 = M.msp_enumerate_bounded(ctx, Ad, dd, rd, Bk, params=prm)
    xs = E.sort_rows(g2.x.cpu().numpy())
    assert g2.status == M.MSP_OK and np.array_equal(xs, ref.solutions)
    assert E.verify(A, d, xs, r) and any(np.array_equal(row, x) for row in xs)


def test_bounded_small_box_brute_force(M, ctx):
    A, d, r, _ = _instance(7, 2, 9, 3, D=9)
    Ad, dd, rd = _dev(A), _dev(d), _dev(r)
    Bk = M.msp_reduce_bounded(ctx, Ad, dd, rd)
    g = M.msp_enumerate_bounded(ctx, Ad, dd, rd, Bk)
    assert np.array_equal(E.sort_rows(g.x.cpu().numpy()), E.sort_rows(B.brute_force_bounded(A, d, r)))


def test_unit_bounds_equal_the_binary_path(M, ctx):
    rng = np.random.default_rng(9)
    A = rng.integers(0, 100, size=(5, 40)).astype(np.int32)
    d = A.astype(np.int64) @ rng.integers(0, 2, size=40)
    Ad, dd, rd = _dev(A), _dev(d), _dev(np.ones(40, dtype=np.int32))
    B0 = M.msp_reduce(ctx, Ad, dd)
    B1 = M.msp_reduce_bounded(ctx, Ad, dd, rd)
    assert torch.equal(B0, B1)
    a = M.msp_enumerate(ctx, Ad, dd, B0)
    b = M.msp_enumerate_bounded(ctx, Ad, dd, rd, B0)
    assert np.array_equal(E.sort_rows(a.x.cpu().numpy()), E.sort_rows(b.x.cpu().numpy()))
    assert a.stats["nodes"] == b.stats["nodes"]


def test_bounded_argument_errors(M, ctx):
    A, d, r, _ = _instance(3, 3, 20, 3)
    Ad, dd = _dev(A), _dev(d)
    bad = r.copy()
    bad[4] = 0
    with pytest.raises(M.MspError) as e:
        M.msp_reduce_bounded(ctx, Ad, dd, _dev(bad))
    assert e.value.code == M.MSP_E_ARG
    primes = np.array([251, 241, 239, 233, 229] + [1] * 15, dtype=np.int32)   # lcm > 2^20
    with pytest.raises(M.MspError) as e:
        M.msp_reduce_bounded(ctx, Ad, dd, _dev(primes))
    assert e.value.code == M.MSP_E_OVERFLOW
