"""Parity of the benchmark's headline workload: one planted m=9, n=80, D=200
instance (seed 4508) reduced on the GPU with LLL and BKZ-16, walked
exhaustively.  The oracle's recursive enumerator walks the same BKZ basis at
test time (search counters equal); the solution set also equals the stored
oracle run on the oracle's own exact-LLL basis (tests/golden/m9_seed4508.json),
which owes nothing to the GPU, and the BKZ basis spans the same lattice as that
basis (equal Gram determinant, every vector in the kernel of A x = d x_n)."""
from __future__ import annotations

import json
import os
import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import enum as E
from oracle import lattice as L

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m9_seed4508.json")


def _coordinates(B0, v):
    """Integer u with u B0 = v, or None if v is not in the lattice of B0."""
    u = np.rint(np.linalg.lstsq(B0.T.astype(np.float64), v.astype(np.float64), rcond=None)[0]).astype(np.int64)
    return u if np.array_equal(u @ B0, v) else None


def test_bench_workload_bkz16_basis_matches_oracle():
    import paper_2508_08702_amd as M
    inst = mi.msp_class(9, 200, 4508)
    g = json.load(open(GOLDEN))
    dev = torch.device("cuda", 0)
    A = torch.from_numpy(inst.A).to(dev)
    d = torch.from_numpy(inst.d).to(dev)
    with M.Context(0) as ctx:
        print("  gpu BKZ-16 reduction and exhaustive walk, m=9 D=200 seed 4508", flush=True)
        prm = M.msp_params_default(bkz_block=16, time_cap_ms=110000.0)
        Bz = M.msp_reduce(ctx, A, d, prm)
        r = M.msp_enumerate(ctx, A, d, Bz, params=prm)
        torch.cuda.synchronize()
        assert r.status == M.MSP_OK
        x = E.sort_rows(r.x.cpu().numpy())
        Bn = Bz.cpu().numpy()
    # the same lattice as the oracle's exact-LLL basis: every BKZ vector has
    # integer coordinates in it, and the Gram determinants are equal
    P0 = L.prepare(inst.A, inst.d)
    B0 = np.asarray(P0.basis, dtype=np.int64)
    assert all(_coordinates(B0, row) is not None for row in Bn.astype(np.int64))
    assert L.gram_schmidt_exact([[int(v) for v in row] for row in Bn]).d[-1] == P0.gs.d[-1]
    # set: the stored oracle run on the oracle's own basis
    want = E.sort_rows(np.array(g["solutions"], dtype=np.uint8))
    assert np.array_equal(x, want)
    # counters: the oracle on the GPU's BKZ basis
    P = L.prepare_from_basis(inst.A, inst.d, Bn)
    print(f"  oracle exhaustive walk on the BKZ-16 basis ({os.cpu_count()} threads)", flush=True)
    ref = E.enumerate_prepared(P, split=12, threads=os.cpu_count() or 1)
    assert np.array_equal(ref.solutions, want)
    for key in ("evals", "nodes", "expansions", "leaves"):
        assert r.stats[key] == getattr(ref, key), key
