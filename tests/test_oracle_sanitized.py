"""The oracle built with the address and undefined-behaviour sanitizers, and separately with the
thread sanitizer (host gcc, no GPU): its component, product and QC-GLDPC entry points run clean on
[16,11] words and frames, the frame loops on three threads, and give exactly the regular build's
results."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import synth  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ODIR = os.path.join(ROOT, "oracle")


@pytest.fixture(scope="module", params=["address,undefined", "thread"])
def driver(request, tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_check")
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + request.param,
           "-fno-sanitize-recover=all", "-o", exe, os.path.join(ODIR, "sanitize_check.c"),
           os.path.join(ODIR, "sogrand_oracle.c"), "-lm", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return exe


def test_sanitized_oracle_runs_clean_and_agrees(driver, tmp_path):
    code = synth.ebch(16, 11)
    n, k, L, qcap, iters, W, F, nthreads = code.n, code.k, 4, 3000, 4, 300, 6, 3
    pstop, alpha = 0.0, 0.5
    words = np.ascontiguousarray(synth.component_words(code, 2.0, 17, np.arange(W))[0], dtype=np.float64)
    pf = np.ascontiguousarray(synth.product_frames(code, 2.0, 18, np.arange(F))[0], dtype=np.float64)
    gf = np.ascontiguousarray(synth.gldpc_frames(synth.gldpc(code), 2.0, 19, np.arange(F))[0], dtype=np.float64)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([n, k, L, iters, nthreads], np.int32).tobytes())
        f.write(np.array([qcap, W, F], np.int64).tobytes())
        f.write(np.array([pstop, alpha], np.float64).tobytes())
        f.write(np.asarray(code.hcols, np.uint64).tobytes())
        f.write(words.tobytes())
        f.write(pf.tobytes())
        f.write(gf.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([driver, str(inp), str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    for report in ("runtime error", "AddressSanitizer", "ThreadSanitizer", "LeakSanitizer"):
        assert report not in r.stderr, r.stderr[-2000:]

    buf = open(out, "rb").read()
    pos = 0

    def take(dtype, count):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a

    ref = oracle.decode_component(code, words, L, qcap)
    np.testing.assert_array_equal(take(np.float64, W * n).reshape(W, n), ref["llr_app"])
    np.testing.assert_array_equal(take(np.float64, W * n).reshape(W, n), ref["llr_ext"])
    np.testing.assert_array_equal(take(np.uint8, W * n).reshape(W, n), ref["hard"])
    np.testing.assert_array_equal(take(np.uint32, W), ref["n_queries"])
    np.testing.assert_array_equal(take(np.int32, W), ref["n_found"])
    np.testing.assert_array_equal(take(np.uint32, W * L).reshape(W, L), ref["found_q"])
    np.testing.assert_array_equal(take(np.float64, W * L).reshape(W, L), ref["p_found"])
    np.testing.assert_array_equal(take(np.float64, W), ref["p_notfound"])
    for fn, frames in ((oracle.decode_product, pf), (oracle.decode_gldpc, gf)):
        r2 = fn(code, frames, L, qcap, iters, alpha, want_app=True, want_last_diag=True, nthreads=1)
        np.testing.assert_array_equal(take(np.uint8, F * n * n).reshape(F, n, n), r2["hard"])
        np.testing.assert_array_equal(take(np.float64, F * n * n).reshape(F, n, n), r2["llr_app"])
        np.testing.assert_array_equal(take(np.uint8, F), r2["success"])
        np.testing.assert_array_equal(take(np.uint16, F), r2["half_iters"])
        np.testing.assert_array_equal(take(np.uint64, F), r2["sum_queries"])
        np.testing.assert_array_equal(take(np.uint64, F), r2["sum_max_queries"])
        np.testing.assert_array_equal(take(np.float64, F), r2["kappa_max"])
    assert pos == len(buf)
