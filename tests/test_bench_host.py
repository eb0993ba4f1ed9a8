"""Host-side logic of bench.py (no GPU): the counter record that gates the
`traffic` field, the contributions-per-determinant count, and the refusal of
more than one GPU."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write_record(tmp, src_text, sha=None):
    os.makedirs(os.path.join(tmp, "profiles"), exist_ok=True)
    src = os.path.join(tmp, "k.hip")
    with open(src, "w") as f:
        f.write(src_text)
    digest = sha or hashlib.sha256(src_text.encode()).hexdigest()
    with open(os.path.join(tmp, "profiles", "finish_16e20o_pmc.md"), "w") as f:
        f.write("# summary\n\n    traffic_record kernel=finish fetch_kib=1000.0 write_kib=500.0 "
                "fetch_scale=2.0 write_scale=1.0 sources=k.hip sha256=%s\n" % digest)


def test_traffic_record_used_while_sources_match(tmp_path, monkeypatch):
    _write_record(str(tmp_path), "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("finish", "16e20o") == pytest.approx(1024.0 * (1000.0 * 2.0 + 500.0 * 1.0))


def test_traffic_record_dropped_once_sources_change(tmp_path, monkeypatch):
    _write_record(str(tmp_path), "kernel v1\n")
    with open(os.path.join(str(tmp_path), "k.hip"), "w") as f:
        f.write("kernel v2\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("finish", "16e20o") is None


def test_traffic_record_missing(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("finish", "16e20o") is None


def test_committed_record_names_existing_sources():
    # the committed summary lists files of this repository (whether or not the
    # hash still matches the current sources)
    path = os.path.join(ROOT, "profiles", "finish_16e20o_pmc.md")
    recs = [ln.split() for ln in open(path) if ln.split()[:1] == ["traffic_record"]]
    assert len(recs) == 1
    rec = dict(p.split("=", 1) for p in recs[0][1:])
    for f in rec["sources"].split(","):
        assert os.path.exists(os.path.join(ROOT, f)), f
    assert len(rec["sha256"]) == 64


@pytest.mark.parametrize("n,na,nb", [(6, 2, 3), (7, 3, 3), (8, 4, 2), (5, 0, 2), (6, 1, 1)])
def test_contributions_per_determinant_brute_force(n, na, nb):
    # every determinant of the space at excitation level 1 or 2 from a
    # reference one, counted by enumeration
    from itertools import combinations

    def strings(k):
        return [sum(1 << p for p in c) for c in combinations(range(n), k)]

    ra, rb = (1 << na) - 1, (1 << nb) - 1
    count = 0
    for a in strings(na):
        da = bin(a ^ ra).count("1") // 2
        if da > 2:
            continue
        for b in strings(nb):
            lvl = da + bin(b ^ rb).count("1") // 2
            count += lvl in (1, 2)
    assert bench.sd_per_det(n, na, nb) == count


def test_contributions_of_the_16e20o_workload():
    assert 10000 * bench.sd_per_det(20, 8, 8) == 131_040_000


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
