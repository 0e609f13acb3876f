"""GPU reduction (msp_reduce: eq. (2) embedding, LLL, kernel extraction)
checked exactly on the host: every output vector encodes a kernel vector of
A x = d x_{n+1}, the output spans the same lattice as the oracle's kernel
basis (equal Gram determinants of two sets of kernel-lattice vectors), the
basis is LLL reduced, and enumeration on it returns the oracle's set."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest
import torch

import msp_instances as mi
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


def _is_kernel_vector(inst, v):
    n = inst.n
    u0 = int(v[n])
    up = []
    for j in range(n):
        if (int(v[j]) + u0) % 2:
            return False
        up.append((int(v[j]) + u0) // 2)
    lhs = inst.A.astype(object) @ np.array(up, dtype=object)
    return list(lhs) == [u0 * int(x) for x in inst.d]


CASES = [(3, 100, 1001), (4, 50, 7), (5, 200, 11), (6, 100, 2000), (7, 50, 3), (8, 100, 7), (9, 200, 4508), (11, 100, 5004)]


@pytest.mark.parametrize("m,D,seed", CASES)
def test_reduce_spans_the_kernel_lattice(M, ctx, m, D, seed):
    inst = mi.single_small(seed) if m == 3 else mi.msp_class(m, D, seed)
    print(f"  msp_reduce m={m} D={D} seed={seed}", flush=True)
    Bg = M.msp_reduce(ctx, _dev(inst.A), _dev(inst.d)).cpu().numpy()
    n = inst.n
    assert Bg.shape == (n - m + 1, n + 1)
    assert all(_is_kernel_vector(inst, v) for v in Bg)
    P = L.prepare(inst.A, inst.d)
    gs_gpu = L.gram_schmidt_exact(Bg.tolist())
    assert gs_gpu.d[-1] == P.gs.d[-1]  # det Gram: same lattice
    # LLL reduced (FP reduction: |mu| <= 0.51, Lovász with a little slack)
    for i in range(gs_gpu.k):
        for j in range(i):
            assert abs(gs_gpu.mu(i, j)) <= Fraction(51, 100) + Fraction(1, 10**6)
        if i:
            assert gs_gpu.beta(i) >= (Fraction(98, 100) - gs_gpu.mu(i, i - 1) ** 2) * gs_gpu.beta(i - 1)


@pytest.mark.parametrize("m,D,seed", [(3, 100, 1001), (6, 100, 2001), (7, 200, 6)])
def test_enumeration_on_gpu_basis(M, ctx, m, D, seed):
    inst = mi.single_small(seed) if m == 3 else mi.msp_class(m, D, seed)
    A, d = _dev(inst.A), _dev(inst.d)
    Bt = M.msp_reduce(ctx, A, d)
    r = M.msp_enumerate(ctx, A, d, Bt, params=M.msp_params_default(time_cap_ms=60000.0))
    x = E.sort_rows(r.x.cpu().numpy())
    P_or, ref = E.solve(inst.A, inst.d, split=6, threads=4)
    assert (x == ref.solutions).all()
    # node parity on the GPU's basis
    Pg = L.prepare_from_basis(inst.A, inst.d, Bt.cpu().numpy())
    ref_g = E.enumerate_prepared(Pg, split=6, threads=4)
    assert r.stats["nodes"] == ref_g.nodes and r.stats["evals"] == ref_g.evals


def test_reduce_errors(M, ctx):
    inst = mi.msp_class(4, 100, 3)
    A, d = _dev(inst.A), _dev(inst.d)
    with pytest.raises(M.MspError) as e:
        M.msp_reduce(ctx, A, d, M.msp_params_default(N=1))
    assert e.value.code == M.MSP_E_NOT_ISOLATED
    # dependent rows: the kernel has more than n - m + 1 dimensions
    A2 = np.vstack([inst.A, inst.A[:1]]).astype(np.int32)
    d2 = np.concatenate([inst.d, inst.d[:1]])
    with pytest.raises(M.MspError) as e:
        M.msp_reduce(ctx, _dev(A2), _dev(d2))
    assert e.value.code == M.MSP_E_RANK
    # entries too large for exact int64 Gram arithmetic
    A3 = np.full((2, 10), 1 << 20, dtype=np.int32)
    d3 = np.array([5 << 20, 5 << 20], dtype=np.int64)
    with pytest.raises(M.MspError) as e:
        M.msp_reduce(ctx, _dev(A3), _dev(d3))
    assert e.value.code == M.MSP_E_OVERFLOW
