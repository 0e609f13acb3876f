"""Write the exhaustive oracle result of one m=9 instance (a parity case at
full size) to tests/golden/m9_seed<seed>.json.

    python tests/golden/make_m9_golden.py [--threads N] [--seed 4508 --D 200]

Only oracle/ computes anything here: the exact-integer LLL basis, the
recursive enumeration (all solutions, search-tree counters) and the exact
A x = d check.  At m=9, n=80 the tree has about 1e11 to 1e12 nodes, so this
takes hours on a few cores; the stored result is what the GPU test compares
with, bit for bit (solution set and counters on the same basis).
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


def basis_digest(basis) -> str:
    return hashlib.sha256(np.ascontiguousarray(basis, dtype=np.int64).tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=4508)
    ap.add_argument("--D", type=int, default=200)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--split", type=int, default=14)
    args = ap.parse_args()
    inst = mi.msp_class(9, args.D, args.seed)
    t0 = time.time()
    P = L.prepare(inst.A, inst.d)
    t_lll = time.time() - t0
    r = E.enumerate_prepared(P, split=args.split, threads=args.threads)
    assert not r.timed_out
    assert E.verify(inst.A, inst.d, r.solutions)
    out = {
        "instance": {"m": 9, "n": inst.n, "D": args.D, "seed": args.seed},
        "basis_sha256": basis_digest(P.basis),
        "k": P.k,
        "n_found": r.n_found,
        "solutions": [[int(v) for v in row] for row in r.solutions],
        "evals": r.evals, "nodes": r.nodes, "expansions": r.expansions, "leaves": r.leaves,
        "oracle_seconds": round(r.seconds, 1), "lll_seconds": round(t_lll, 1), "threads": r.threads,
        "centre_sum": "one running sum over i = t+1 .. k-1",
    }
    path = os.path.join(HERE, f"m9_seed{args.seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "solutions"}))


if __name__ == "__main__":
    main()
