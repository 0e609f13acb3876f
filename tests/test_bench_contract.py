"""bench.py host-side contract: more than one GPU is refused with a message,
and the HBM traffic figure it reports comes from a committed profile of the
same walk-kernel source (its hash and byte count are written there)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_traffic_figure_matches_its_profile():
    import bench
    for (workload, bkz), tr in bench.WALK_TRAFFIC.items():
        assert workload in bench.WORKLOADS and bkz >= 0
        path = os.path.join(ROOT, tr["profile"])
        txt = open(path).read()
        assert tr["sha256"] in txt
        # the profile states the per-launch bytes that bench.py reports
        assert f"{tr['bytes']:.3e}".replace("e+", "e") in txt.replace("e+", "e")


def test_traffic_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    """The traffic figure is keyed by the walk kernel's code: editing a comment
    or a blank line keeps the hash, editing code changes it."""
    import shutil

    import bench
    src = os.path.join(ROOT, "paper_2508_08702_amd", "csrc")
    fake = tmp_path / "paper_2508_08702_amd" / "csrc"
    fake.mkdir(parents=True)
    for f in ("walk.hip", "enum_rules.h", "msp_internal.h"):
        shutil.copy(os.path.join(src, f), fake / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.walk_source_hash()
    walk = fake / "walk.hip"
    txt = walk.read_text()
    walk.write_text(txt.replace("namespace msp {", "// a new comment line\n\nnamespace msp {  /* and a block */", 1))
    assert bench.walk_source_hash() == h0
    walk.write_text(txt.replace("namespace msp {", "namespace msp {\nstatic const int unused_marker = 1;", 1))
    assert bench.walk_source_hash() != h0
