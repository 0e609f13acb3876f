"""The widest walker variants (n + 1 = 85 .. 127 coordinates: register
widths 88, 96, 102, 112 and 128) against stored oracle runs
(tests/golden/wide_shapes.json, written by tests/golden/make_wide_golden.py
from oracle/ alone): the exhaustive GPU walk of the oracle's exact-LLL basis
(stored with the run, checked by hash) gives the same solution set and the
same four search counters."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import enum as E

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wide_shapes.json")
CASES = json.load(open(GOLDEN))["cases"]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c['instance']['n']}" for c in CASES])
@pytest.mark.parametrize("split", [-1, 20])
def test_wide_walker_matches_stored_oracle_run(case, split):
    import paper_2508_08702_amd as M
    g = case["instance"]
    inst = mi.planted(g["m"], g["n"], g["D"], g["seed"])
    basis = np.array(case["basis"], dtype=np.int64)
    assert hashlib.sha256(basis.tobytes()).hexdigest() == case["basis_sha256"]
    dev = torch.device("cuda", 0)
    print(f"  wide walk n={g['n']} m={g['m']} k={case['k']} split {split}", flush=True)
    with M.Context(0) as ctx:
        r = M.msp_enumerate(ctx, torch.from_numpy(inst.A).to(dev), torch.from_numpy(inst.d).to(dev),
                            torch.from_numpy(basis).to(dev),
                            params=M.msp_params_default(split_depth=split, time_cap_ms=60000.0))
        torch.cuda.synchronize()
    assert r.status == M.MSP_OK and r.n_found == case["n_found"]
    want = E.sort_rows(np.array(case["solutions"], dtype=np.uint8))
    assert np.array_equal(E.sort_rows(r.x.cpu().numpy()), want)
    for key in ("evals", "nodes", "expansions", "leaves"):
        assert r.stats[key] == case[key], key
