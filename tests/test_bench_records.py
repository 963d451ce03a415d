"""The benchmark's reading of committed counter records (no GPU needed)."""
import hashlib
import json
import os

import bench


def _record(workload, prec, leaf_sha, kern_sha, fetch, write):
    return {"workload": workload, "prec": prec, "leaf_gemm_sha256": leaf_sha, "kernels_sha256": kern_sha,
            "launches": 1, "fetch_factor": 2.0, "write_factor": 1.0,
            "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write}


def test_traffic_record_matches_only_the_current_sources(tmp_path, monkeypatch):
    sha = {name: hashlib.sha256(open(os.path.join(bench.CSRC, name), "rb").read()).hexdigest()
           for name in ("leaf_gemm.hip", "kernels.hip")}
    good = _record("w", "f64", sha["leaf_gemm.hip"], sha["kernels.hip"], 3.0, 1.0)
    stale = _record("w", "f32", "0" * 64, sha["kernels.hip"], 5.0, 1.0)
    (tmp_path / "a.md").write_text("text\n```json\n" + json.dumps(good) + "\n```\n")
    (tmp_path / "b.md").write_text("```json\n" + json.dumps(stale) + "\n```\n```json\nnot json\n```\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.committed_traffic("w", "f64") == 4.0
    assert bench.committed_traffic("w", "f32") is None   # taken with another leaf-product source
    assert bench.committed_traffic("x", "f64") is None   # another workload

