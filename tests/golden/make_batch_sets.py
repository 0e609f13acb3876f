"""Write the oracle's solution sets of the uneven batch's m = 7 and m = 8
instances (seeds 3000-3095 of msp_instances.mixed_batch) to
tests/golden/batch_sets.json.

    python tests/golden/make_batch_sets.py [--threads N]

Only oracle/ computes anything here: the exact-integer LLL basis, the
recursive enumeration of all solutions and the exact A x = d check.  The
m <= 6 instances are cheap enough for the GPU test to run the oracle itself.
"""
from __future__ import annotations

import argparse
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    out = {}
    t0 = time.time()
    for inst in mi.mixed_batch():
        if inst.m < 7:
            continue
        _, r = E.solve(inst.A, inst.d, split=10, threads=args.threads)
        assert not r.timed_out and E.verify(inst.A, inst.d, r.solutions)
        assert any(np.array_equal(x, inst.x_planted) for x in r.solutions)
        out[str(inst.seed)] = {"m": inst.m, "n": inst.n, "D": int(inst.D), "n_found": r.n_found,
                               "solutions": [[int(v) for v in row] for row in r.solutions],
                               "oracle_seconds": round(r.seconds, 1)}
        print(inst.seed, inst.m, inst.D, r.n_found, round(r.seconds, 1), round(time.time() - t0), flush=True)
    with open(os.path.join(HERE, "batch_sets.json"), "w") as f:
        json.dump({"instances": out}, f)


if __name__ == "__main__":
    main()
