"""Host logic of the benchmark (no GPU): the stored counter record is used only for the kernel
sources it was measured on, the roofline helpers scale it as documented, and the one-GPU
guard refuses more GPUs before touching the device."""
import hashlib
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEY = ("f32", 16384, 5000, 192)


def test_counter_record_matches_the_committed_kernel_sources():
    """The stored counters describe the kernel as committed: a change to these sources must
    come with counters taken again (or the record removed, when the bench reports null)."""
    rec = bench.MEASURED_TRAFFIC[KEY]
    for path, digest in rec["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            assert hashlib.sha256(f.read()).hexdigest() == digest, path
    assert bench._counters(*KEY) is rec


def test_traffic_and_valu_follow_the_documented_scaling():
    rec = bench.MEASURED_TRAFFIC[KEY]
    want = rec["fetch_kib"] * 1024 * 2.0 + rec["write_kib"] * 1024 * 1.0
    assert bench.measured_traffic(*KEY) == pytest.approx(want, rel=1e-15)
    v = bench.valu_utilisation(*KEY, kernel_s=0.5)
    assert v["issue_frac"] == pytest.approx(rec["valu_insts"] / (256 * 4 * 2.4e9 / 4 * 0.5), rel=1e-15)
    assert bench.measured_traffic("f32", 123, 5000, 192) is None          # no record for this launch


def test_counter_record_is_dropped_when_a_source_changes(monkeypatch):
    rec = dict(bench.MEASURED_TRAFFIC[KEY])
    rec["sources"] = dict(rec["sources"])
    first = next(iter(rec["sources"]))
    rec["sources"][first] = "0" * 64
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, KEY, rec)
    assert bench.measured_traffic(*KEY) is None
    assert bench.valu_utilisation(*KEY, kernel_s=0.5) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_learned_gain_with_training_counts_the_training_time_against_the_learned_form():
    cmp = {"learned": {"distinct_minima": 86, "seconds": 2.88}, "uniform": {"minima_per_s": 58 / 2.82},
           "training": {"train_s": 0.61}}
    assert bench._gain_with_training(cmp) == pytest.approx((86 / (2.88 + 0.61)) / (58 / 2.82), rel=1e-15)


def test_alu_peaks_follow_from_the_unit_counts():
    """FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop per FMA x 2.4 GHz in scalar
    instructions, twice that with packed FP32."""
    unpacked = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
    assert bench.FP32_UNPACKED_PEAK_TFLOPS == pytest.approx(unpacked, rel=1e-3)
    assert bench.FP32_PEAK_TFLOPS == pytest.approx(2 * unpacked, rel=1e-3)
    # the issue-slot peak the VALU utilisation is taken against: one wave64 FP32 instruction
    # per SIMD every 4 cycles
    assert bench.VALU_ISSUE_PEAK * 64 * 2 / 1e12 == pytest.approx(unpacked, rel=1e-12)
