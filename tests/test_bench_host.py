"""Host logic of the benchmark (no GPU): the one-GPU contract, the readers of
the committed counter summaries and their staleness check, and the
algorithmic bytes the traffic ratio divides by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1901_04200_amd import roofline  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_pass2_algorithmic_bytes():
    # 2^20 paths, K = 16: 16 segments x 2 state values x 4 bytes per path,
    # 4096 workgroups x 5 FP64 partials, 40 FP32 seeds
    assert roofline.pass2_bytes(1 << 20, 16, 4096, 40, 256) == 16 * 2 * 4 * (1 << 20) + 4096 * 5 * 8 + 40 * 4
    # a ragged last segment still counts once
    assert roofline.pass2_bytes(100, 16, 1, 1, 17) == 2 * 2 * 4 * 100 + 5 * 8 + 4


def test_profile_readers_match_the_sources():
    """The committed summaries carry the hashes of the sources they were
    taken with; while those are unchanged the readers return their figures."""
    t = bench.pass2_traffic(16, 1)
    if t is None or bench.counted_slots("lv", "pass2", 16) is None:
        pytest.skip("the counter summaries predate the current kernel sources: take them again")
    assert 1.0 <= t / roofline.pass2_bytes(1 << 20, 16, 4096, 40, 256) < 1.02
    assert bench.pass2_traffic(24, 1) is None          # spacing never measured
    assert bench.counted_slots("lv", "pass2", 16) > 0
    assert bench.counted_slots("slv", "pass2", 8) > 0
    assert bench.counted_slots("lv", "pass2", 24) is None


def test_profile_readers_drop_stale_figures(monkeypatch):
    """A changed source (any hash mismatch) makes the figures unavailable
    instead of wrong."""
    monkeypatch.setattr(bench, "code_hash", lambda path: "0" * 64)
    assert bench.pass2_traffic(16, 1) is None
    assert bench.counted_slots("lv", "pass2", 16) is None
    r = bench.grid_roofline("lv", "k_lv_pass2", 16, 1 << 30, 3.0)
    assert r["frac"] is None and r["bound"] == "alu"


def test_code_hash_ignores_comments_and_layout(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f(int x) { return x + 1; }  // one\n/* block */\n")
    b.write_text("int f(int x)\n{\n    return x + 1;   // another comment\n}\n")
    assert bench.code_hash(str(a)) == bench.code_hash(str(b))
    b.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_hash(str(a)) != bench.code_hash(str(b))


@pytest.mark.parametrize("achieved_frac", [0.5, 0.875])
def test_grid_roofline_arithmetic(achieved_frac):
    sl = bench.counted_slots("slv", "pass2", 8)
    if sl is None:
        pytest.skip("the counter summaries predate the current kernel sources: take them again")
    ps = 1 << 28
    ms = sl * ps / (achieved_frac * roofline.PEAK_SLOTS) * 1e3
    r = bench.grid_roofline("slv", "k_slv_pass2", 8, ps, ms)
    assert abs(r["frac"] - achieved_frac) < 1e-12
    assert r["slots_per_path_step"] == sl
