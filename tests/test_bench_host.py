"""Host logic of bench.py (no GPU): the single-GPU guard, the counter-summary lookup tied to the
kernel source, and the algorithmic byte and FLOP model of the roofline entries."""
import hashlib
import importlib.util
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_measured_traffic_follows_the_source_hash(bench, tmp_path, monkeypatch):
    """The composite's counters are reported only while the projection (whose binning rule makes
    the tile lists) and the compositing source both hash to what they were taken on."""
    text = open(os.path.join(ROOT, "profiles", "composite_1M_1080p_hbm_traffic.md")).read()
    stored = float(re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text).group(1))
    taken_on = re.search(r"source_sha256:\s*([0-9a-f]{64})", text).group(1)
    csrc_root = os.path.join(ROOT, "paper_2409_16504_amd", "csrc")
    h = hashlib.sha256()
    for f in ("project.hip", "composite.hip"):
        h.update(open(os.path.join(csrc_root, f), "rb").read())
    assert bench.sources_sha256("composite") == h.hexdigest()
    assert bench.measured_traffic("composite") == (stored if h.hexdigest() == taken_on else None)
    assert bench.measured_traffic("no_such_stage") is None
    sources = {"project.hip": b"// projection\n", "composite.hip": b"// compositing\n"}
    want = hashlib.sha256(sources["project.hip"] + sources["composite.hip"]).hexdigest()
    # the summary against the sources it was taken on is reported; a change to either is not
    for changed in (None, "project.hip", "composite.hip"):
        root = tmp_path / str(changed)
        (root / "profiles").mkdir(parents=True)
        (root / "profiles" / "composite_1M_1080p_hbm_traffic.md").write_text(text.replace(taken_on, want))
        csrc = root / "paper_2409_16504_amd" / "csrc"
        csrc.mkdir(parents=True)
        for f, body in sources.items():
            (csrc / f).write_bytes(body if f != changed else b"// another source\n")
        monkeypatch.setattr(bench, "ROOT", str(root))
        assert bench.measured_traffic("composite") == (stored if changed is None else None), changed
        monkeypatch.undo()


def _bins(n_tiles, tile_ids, depth_bits_values, vals):
    keys = (np.asarray(tile_ids, np.uint64) << np.uint64(32)) | np.asarray(depth_bits_values, np.uint64)
    return dict(keys=keys, vals=np.asarray(vals, np.uint32), ranges=np.zeros((2, n_tiles), np.uint32))


def test_stage_bytes(bench):
    # 10 splats, 6 of them visible; 8 instances over 300 tiles (9 tile bits: two 8-bit passes);
    # depth bits spanning 2^17 (18 bits: three passes)
    n, m = 10, 8
    bins = _bins(300, [0, 0, 1, 5, 5, 7, 299, 299], [100, 100 + (1 << 17), 5, 7, 9, 11, 13, 15],
                 [0, 1, 2, 3, 4, 5, 5, 1])
    per_stage = dict(project=1e-6, binning=1e-6, sort=1e-6, ranges=1e-6)    # ms
    out = bench.stage_rooflines(per_stage, n, m, bins, 64, 64)
    vis = 6
    # a 64 x 64 frame stores its tile rectangles in 4 bytes
    assert out["project"]["bytes"] == n * 68 + vis * 72 + (n - vis) * 8
    assert out["binning"]["bytes"] == n * 8 + m * 8
    assert out["sort"]["bytes"] == n * (12 + 16 * 3) + m * 16 * 2
    assert out["ranges"]["bytes"] == 300 * 24
    # bytes over the stage time as GB/s, and the fraction of the 8 TB/s peak
    assert out["binning"]["gbs"] == pytest.approx((n * 8 + m * 8) / 1e-9 / 1e9, rel=1e-3)
    # 257 tile columns: the 8-byte form
    wide = bench.stage_rooflines(per_stage, n, m, bins, 4112, 64)
    assert wide["project"]["bytes"] == n * 68 + vis * 76 + (n - vis) * 12
    assert wide["binning"]["bytes"] == n * 12 + m * 8
    assert bench.rect_bytes(4080, 4080) == 4 and bench.rect_bytes(64, 4112) == 8
    assert out["binning"]["frac"] == pytest.approx(out["binning"]["gbs"] / 8000.0, rel=1e-3)


def test_composite_roofline_is_alu_bound(bench):
    bins = _bins(4, [0, 1], [3, 4], [0, 1])
    per_stage = dict(project=0.01, binning=0.01, sort=0.02, ranges=0.005, composite=0.5)
    visits, blends = 1_000_000, 250_000
    r = bench.roofline(per_stage, 2, 2, bins, visits, blends)
    # 25 FLOP per evaluated (pixel, list entry) pair against the 157.3 TFLOP/s FP32 peak
    assert r["kernel"] == "composite" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(25 * visits / 0.5e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["avg_ms"] == 0.5
    # beside it the finer count (9 per visit, 21 per blend) against the peak without packed FP32
    fine = 9 * visits + 21 * blends
    assert r["fine_model"]["achieved"] == pytest.approx(fine / 0.5e-3 / 1e12)
    assert r["fine_model"]["frac"] == pytest.approx(r["fine_model"]["achieved"] / 78.6)


def test_composite_roofline_without_visit_counts_reports_no_figure(bench):
    """Without the CPU baseline leg there are no visit counts: the entry stays ALU-bound and
    gives no achieved figure rather than a bytes-based one."""
    bins = _bins(4, [0, 1], [3, 4], [0, 1])
    per_stage = dict(project=0.01, binning=0.01, sort=0.02, ranges=0.005, composite=0.5)
    r = bench.roofline(per_stage, 2, 2, bins, None, None)
    assert r["kernel"] == "composite" and r["bound"] == "alu"
    assert r["achieved"] is None and r["frac"] is None and r["avg_ms"] == 0.5
