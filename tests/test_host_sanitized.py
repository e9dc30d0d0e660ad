"""The library's host code under the address and undefined-behaviour sanitizers (no GPU): a
copy of libsogrand built with the sanitizers on its host side only runs the C-ABI tests
(argument checks before device work, code construction, the tuned-shape table, plans' argument
checks) in a child process with the sanitizer runtime preloaded, and must pass them with no
sanitizer report."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_host_code_under_sanitizers(tmp_path):
    from paper_2310_10737_amd import build as B
    rt = asan_runtime()
    if rt is None or not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc or no sanitizer runtime")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + san

    def comp(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.check_call([B.HIPCC] + flags + ["-c", "-o", obj, os.path.join(B.CSRC, src)],
                              stderr=subprocess.DEVNULL)
        return obj
    with ThreadPoolExecutor(len(B.SOURCES)) as ex:
        objs = list(ex.map(comp, B.SOURCES))
    lib = str(tmp_path / "libsogrand_sanitized.so")
    subprocess.check_call([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + san + ["-o", lib] + objs +
                          ["-lpthread"])
    env = dict(os.environ, SOGRAND_TEST_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider"], capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    for report in ("runtime error", "AddressSanitizer"):
        assert report not in out, out[-3000:]
