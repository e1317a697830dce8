"""Host logic of bench.py, no GPU: the one-GPU guard, the algorithmic-byte
model (the per-round formula written out for a two-round example), the choice
of the rounds whose insert phase is one launch, and the rule that a traffic
figure is used only while the kernel source (the round kernels and their device
header) is the one it was measured on."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench as B  # noqa: E402


def _stats(rows):
    st = np.zeros((len(rows), 16), np.uint64)
    for i, (n, d, u, q, mode) in enumerate(rows):
        st[i, :4] = (n, d, u, q)
        st[i, 15] = mode
    return st


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU only" in r.stderr


@pytest.mark.parametrize("args", [["--steps", "0"], ["--phase-builds", "0"]])
def test_no_timed_or_phase_builds_is_refused(args):
    """The roofline needs timed builds and the phase table an untimed one."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "must be at least 1" in r.stderr


def test_algorithmic_bytes_of_two_rounds():
    st = _stats([(100, 30, 10, 40, 0), (30, 10, 5, 12, 0)])
    # round 1 (bytes, s = 1): n + 12 d + 16 u + q; round 2 (ranks, s = 4, F read): 8 n + 12 d + 16 u + 4 q
    r1 = 100 + 12 * 30 + 16 * 10 + 40
    r2 = 8 * 30 + 12 * 10 + 16 * 5 + 4 * 12
    assert B.path_alg_bytes(st) == r1 + r2
    ph = B.phase_alg_bytes(st)
    assert ph["classify"] == 100 + 4 * 30 and ph["emit"] == 4 * 30
    assert sum(ph.values()) == B.path_alg_bytes(st)
    assert ph["insert"] == 8 * (30 + 10) + 8 * (10 + 5)
    assert ph["commit"] == (8 * 10 + 40 + 4 * 30) + (8 * 5 + 4 * 12 + 4 * 10)


def test_single_launch_insert_rounds():
    st = _stats([(100, 30, 10, 40, 0), (30, 10, 5, 12, 0), (10, 3, 3, 6, 1), (3, 0, 0, 0, 0)])
    rows = B.insert_rounds(st)
    assert len(rows) == 1 and int(rows[0][0]) == 30  # round 2 only: not round 1, tail, or empty


def test_traffic_needs_the_measured_source(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "PROFILE_DIR", str(tmp_path))
    f = tmp_path / "k_insert_unsigned_int__false_demo_traffic.txt"
    f.write_text("kernel_source_sha256: %s\ntraffic_bytes_per_launch: 123\n" % B.source_digest())
    assert B.profile_traffic("k_insert<unsigned int, false>", "demo") == 123.0
    f.write_text("kernel_source_sha256: 00\ntraffic_bytes_per_launch: 123\n")
    assert B.profile_traffic("k_insert<unsigned int, false>", "demo") is None
    assert B.profile_traffic("k_insert<unsigned int, false>", "absent") is None


def test_path_traffic_needs_the_measured_source(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "PROFILE_DIR", str(tmp_path))
    f = tmp_path / "path_demo_traffic.txt"
    f.write_text("# header\nkernel_source_sha256: %s\npath_bytes_per_build: 4.5e9\n" % B.source_digest())
    assert B.profile_value("path_demo_traffic.txt", "path_bytes_per_build") == 4.5e9
    assert B.profile_value("path_demo_traffic.txt", "missing_field") is None
    f.write_text("kernel_source_sha256: 00\npath_bytes_per_build: 4.5e9\n")
    assert B.profile_value("path_demo_traffic.txt", "path_bytes_per_build") is None


def test_cpu_baselines_name_the_host():
    """Both oracle timings record the host CPU beside their core count."""
    from oracle import oracle as O
    from paper_2411_12439_amd import datagen as D
    text, off = O.pack([b"ACGTACGGTACA" * 20, b"ACGTTCGGTACA" * 20, b"GATTACA" * 30])
    one = B.cpu_baseline(text, off, D.HASH_SEED, 2)
    par = B.cpu_baseline_parallel(text, off, D.HASH_SEED, 1)
    for r in (one, par):
        assert r["kind"] == "oracle" and r["value"] > 0
        assert "logical CPUs visible" in r["host_cpu"] and r["host_cpu"].split(",")[0]
    assert one["cores"] == 1 and 1 <= par["cores"] <= 3
