"""Host-side logic of bench.py that runs without a GPU: the one-GPU guard and
the rule that the profiled HBM traffic is reported only while the transport
kernel's sources are the ones the counters were taken on."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_profiled_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    good = tmp_path / "good.md"
    good.write_text(f"- hbm_bytes_per_launch: 1.5e+10\n- kernel_source_sha256: {bench.kernel_source_sha256()}\n")
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(good))
    assert bench.profiled_traffic() == 1.5e10
    stale = tmp_path / "stale.md"
    stale.write_text("- hbm_bytes_per_launch: 1.5e+10\n- kernel_source_sha256: 00\n")
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(stale))
    assert bench.profiled_traffic() is None
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic() is None


def test_ledger_totals():
    """The VALU ledger's per-scattering totals that the roofline uses: 508
    slots with the dipole phase and the emissivity tally, 486 isotropic with
    the emissivity tally."""
    assert bench.ledger_per_scatter(True, True) == 508
    assert bench.ledger_per_scatter(False, True) == 486


def test_call_ledger_total_and_per_packet_traffic(tmp_path, monkeypatch):
    """The learned kernel's call ledger sums to the 2818 lane-slots its
    roofline uses, and a counter summary taken at fewer packets than the timed
    launch scales its traffic per packet."""
    assert sum(bench.LEDGER_CALL.values()) == 2818
    s = tmp_path / "learned.md"
    s.write_text(f"- kernel_source_sha256: `{bench.kernel_source_sha256()}`\n- hbm_bytes_per_launch: `2e+9`\n"
                 "- hbm_bytes_per_packet: `200`\n")
    assert bench.profiled_traffic(str(s), 10 ** 8) == 2e10
    assert bench.profiled_traffic(str(s)) == 2e9


def test_unknown_leg_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--legs", "nope", "--legs-only"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "unknown legs" in r.stderr
