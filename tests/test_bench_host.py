"""Host-side logic of bench.py (no GPU): the one-GPU contract and the rule
that counter traffic is reported only for the kernel sources it was taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_source_hash_is_stable_and_hex():
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 64 and int(h, 16) >= 0


def _fake_profile(tmp_path, sha, traffic):
    p = tmp_path / "hopping_h16r12_stoch_16x16x16x32.md"
    p.write_text(f"# summary\n\n    kernel_source_sha256: {sha}\n    traffic_bytes_per_launch: {traffic}\n")
    return str(p)


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    good = _fake_profile(tmp_path, bench.kernel_source_hash(), 3478292881)
    monkeypatch.setattr(bench, "traffic_profile", lambda prec: good)
    assert bench.profiled_traffic("h16") == 3478292881.0
    stale = _fake_profile(tmp_path, "0" * 64, 3478292881)
    monkeypatch.setattr(bench, "traffic_profile", lambda prec: stale)
    assert bench.profiled_traffic("h16") is None
    monkeypatch.setattr(bench, "traffic_profile", lambda prec: str(tmp_path / "missing.md"))
    assert bench.profiled_traffic("h16") is None


def test_committed_profiles_carry_machine_readable_fields():
    for prec in ("h16", "f32"):
        txt = open(bench.traffic_profile(prec)).read()
        assert "kernel_source_sha256:" in txt and "traffic_bytes_per_launch:" in txt
        assert "rocprofv3 --kernel-trace --stats" in txt


def test_iteration_roofline_counts_passes_and_links():
    """16-bit CGNR: 16 vector passes of 52 bytes per site and system-iteration
    plus 8 links of 24 bytes per site and hopping launch, over the step time."""
    r = bench.iteration_roofline("cgnr", "h16", 65536, 384 * 400, 4 * 400, 2.5)
    want = (16 * 52 * 65536 * 384 * 400 + 8 * 24 * 65536 * 4 * 400) / 2.5 / 1e9
    assert abs(r["achieved"] - want) <= 0.05 and r["bytes_per_site_and_system_iteration"] == 832
    assert abs(r["frac"] - want / 8000.0) <= 1e-4


def test_traffic_of_each_timed_hop(tmp_path, monkeypatch):
    p = tmp_path / "hopping_h16r12_stoch_16x16x16x32.md"
    p.write_text(f"    kernel_source_sha256: {bench.kernel_source_hash()}\n"
                 "    traffic_bytes_per_launch: 3480000000\n    traffic_bytes_per_launch_end_hop: 6110000000\n")
    monkeypatch.setattr(bench, "traffic_profile", lambda prec: str(p))
    assert bench.profiled_traffic("h16") == 3.48e9
    assert bench.profiled_traffic("h16", "first_hop") == 3.48e9
    assert bench.profiled_traffic("h16", "end_hop") == 6.11e9
