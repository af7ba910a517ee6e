"""CPU: host logic of bench.py -- the counter-traffic record is summed over
the polar groups at the chosen sweep_unroll, and refused when a choice was
not recorded or the sweep sources changed."""
import json
import os

import pytest

import bench


def _record():
    rec = {}
    for line in open(bench.TRAFFIC_RECORD).read().splitlines():
        if line and not line.startswith("#"):
            k, v = line.split(" ", 1)
            rec[k] = v
    return rec


def _current_hash():
    import hashlib
    h = hashlib.sha256()
    for f in bench.SWEEP_SOURCES:
        with open(os.path.join(bench.ROOT, "paper_2305_11998_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _current_record(tmp_path, monkeypatch):
    """The committed record with the hash of the sources as they are (the
    summing logic is tested whether or not the counters are current)."""
    rec = _record()
    lines = [f"{k} {v}" for k, v in rec.items() if k != "source_sha256"] + [f"source_sha256 {_current_hash()}"]
    p = tmp_path / "traffic.txt"
    p.write_text("\n".join(lines) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(p))


def test_traffic_is_the_sum_over_polar_groups(tmp_path, monkeypatch):
    _current_record(tmp_path, monkeypatch)
    per = json.loads(_record()["traffic_bytes_per_launch"])
    tuning = {pm: {"sweep_unroll": int(sorted(v)[0])} for pm, v in per.items()}
    want = sum(per[pm][str(t["sweep_unroll"])] for pm, t in tuning.items())
    assert bench.recorded_traffic(tuning) == pytest.approx(want, rel=0, abs=0)
    assert want > 0


def test_traffic_refused_for_an_unrecorded_choice(tmp_path, monkeypatch):
    _current_record(tmp_path, monkeypatch)
    per = json.loads(_record()["traffic_bytes_per_launch"])
    pm = sorted(per)[0]
    assert bench.recorded_traffic({pm: {"sweep_unroll": 3}}) is None
    assert bench.recorded_traffic({"64": {"sweep_unroll": 16}}) is None


def test_traffic_refused_when_the_sources_change(tmp_path, monkeypatch):
    rec = open(bench.TRAFFIC_RECORD).read().replace("source_sha256 ", "source_sha256 0")
    p = tmp_path / "traffic.txt"
    p.write_text(rec)
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(p))
    per = json.loads(_record()["traffic_bytes_per_launch"])
    tuning = {pm: {"sweep_unroll": int(sorted(v)[0])} for pm, v in per.items()}
    assert bench.recorded_traffic(tuning) is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_refinement_norms_of_the_multilevel_study():
    """bench's refinement rows: cell-average restriction of the finer grid,
    area-weighted L2 differences and their ratios."""
    import numpy as np
    import bench
    n = 8
    x = (np.arange(n) + 0.5) / n
    fine = np.add.outer(x, x).ravel()                        # linear: restriction is exact
    xc = (np.arange(n // 2) + 0.5) / (n // 2)
    assert np.allclose(bench._restrict(fine, n), np.add.outer(xc, xc).ravel())
    runs = [dict(h_mat=3.0, h_moc=0.1, T=np.full(4, 1.0), E=np.full(4, 2.0)),
            dict(h_mat=1.5, h_moc=0.1, T=np.full(16, 1.2), E=np.full(16, 2.0)),
            dict(h_mat=0.75, h_moc=0.1, T=np.full(64, 1.3), E=np.full(64, 2.5))]
    rows = bench._refinement_rows(runs, "h_mat")
    assert np.isclose(rows[0]["dT"], 0.2 * 6.0) and np.isclose(rows[1]["dT"], 0.1 * 6.0)
    assert np.isclose(rows[1]["rho_T"], 2.0) and np.isclose(rows[0]["dT_rel"], 0.2 / 1.2)
    assert rows[0]["dE"] == 0.0 and "rho_E" not in rows[1] and np.isclose(rows[1]["dE"], 0.5 * 6.0)
