"""Host-side checks of bench.py: the one-GPU contract, the algorithmic operation counts and
the gating of recorded HBM traffic on the kernel sources.  No GPU is used."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_ops_per_word_matches_its_terms():
    # n = 64, L = 4: 2n + n*6 + n + 3n + (2L+4) + n(L+8) + 2n
    assert bench.ops_per_word(64, 4) == 128 + 384 + 64 + 192 + 12 + 768 + 128
    assert bench.ops_per_word(128, 1) == 256 + 896 + 128 + 384 + 6 + 1152 + 256
    w = dict(words=10, queries=100, ranks=300)
    assert bench.algorithmic_ops(w, 64, 4) == 10 * bench.ops_per_word(64, 4) + 200 + 600


def test_wilson_interval_brackets_the_estimate():
    lo, hi = bench.wilson(13, 10000)
    assert lo < 13 / 10000 < hi
    assert bench.wilson(0, 100)[0] == 0.0
    assert bench.wilson(0, 0) == (0.0, 1.0)


def test_recorded_traffic_requires_matching_kernel_sources(tmp_path, monkeypatch):
    f = tmp_path / "t.md"
    f.write_text(f"bytes_per_launch[plain_f32]: 1.5e9\nsource_sha256: {bench.kernel_digest()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic("plain_f32") == pytest.approx(1.5e9)
    assert bench.recorded_traffic("plain_f64") is None
    f.write_text("bytes_per_launch[plain_f32]: 1.5e9\nsource_sha256: " + "0" * 64 + "\n")
    assert bench.recorded_traffic("plain_f32") is None


def _form(ms, blers):
    return dict(ms_per_step=ms, info_bits_per_s=1e3 / ms,
                per_snr={str(s): dict(bler=b, bler_ci95=bench.wilson(int(round(b * 10000)), 10000))
                         for s, b in blers.items()})


def test_choose_form_takes_the_fastest_form_at_matched_bler():
    forms = {"plain_f64": _form(23.0, {2.5: 0.88, 3.0: 0.0133}),
             "plain_f32": _form(22.0, {2.5: 0.88, 3.0: 0.0133}),
             "batched_f32": _form(19.0, {2.5: 0.88, 3.0: 0.0133}),
             "batched_f64": _form(18.0, {2.5: 0.88, 3.0: 0.05})}     # faster, but its BLER is off
    name, best = bench.choose_form(forms)
    assert name == "batched_f32" and best is forms["batched_f32"]
    assert forms["batched_f64"]["bler_matches_plain_f64"] is False
    assert forms["batched_f32"]["speedup_vs_plain"] == pytest.approx(22.0 / 19.0)
    assert forms["batched_f64"]["speedup_vs_plain"] == pytest.approx(23.0 / 18.0)


def test_every_workload_is_selectable():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0
    for w in ("headline", "product", "mixed", "component", "serve", "gldpc", "rician"):
        assert w in r.stdout
