"""Write exhaustive oracle runs of wide planted instances (n + 1 = 85 .. 127
coordinates, the widest walker variants) to tests/golden/wide_shapes.json.

    python tests/golden/make_wide_golden.py [--threads N]

Only oracle/ computes anything here: the exact-integer LLL basis (stored, so
that the GPU test walks the same basis without redoing the slow exact
reduction), the recursive enumeration (all solutions, search-tree counters)
and the exact A x = d check.  The instances have m well above the market
split classes' (n = 10(m-1)), which keeps each tree at 1e5 .. 4e7 nodes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import msp_instances as mi  # noqa: E402
from oracle import enum as E  # noqa: E402
from oracle import lattice as L  # noqa: E402

# (n, m): dim = n + 1 -> walker widths 88, 96, 102, 112, 128
SHAPES = [(84, 20), (92, 24), (100, 26), (110, 30), (126, 36)]
D = 50


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    cases = []
    for n, m in SHAPES:
        seed = 7000 + n
        inst = mi.planted(m, n, D, seed)
        t0 = time.time()
        P = L.prepare(inst.A, inst.d)
        t_lll = time.time() - t0
        r = E.enumerate_prepared(P, split=8, threads=args.threads)
        assert not r.timed_out and E.verify(inst.A, inst.d, r.solutions)
        assert any(np.array_equal(x, inst.x_planted) for x in r.solutions)
        basis = np.ascontiguousarray(P.basis, dtype=np.int64)
        cases.append({
            "instance": {"m": m, "n": n, "D": D, "seed": seed},
            "k": P.k,
            "basis": basis.tolist(),
            "basis_sha256": hashlib.sha256(basis.tobytes()).hexdigest(),
            "n_found": r.n_found,
            "solutions": [[int(v) for v in row] for row in r.solutions],
            "evals": r.evals, "nodes": r.nodes, "expansions": r.expansions, "leaves": r.leaves,
            "oracle_seconds": round(r.seconds, 2), "lll_seconds": round(t_lll, 1),
        })
        print(json.dumps({k: v for k, v in cases[-1].items() if k not in ("basis", "solutions")}), flush=True)
    out = {"centre_sum": "one running sum over i = t+1 .. k-1", "cases": cases}
    with open(os.path.join(HERE, "wide_shapes.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
