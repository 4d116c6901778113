"""The CPU checks of the C ABI (tests/test_abi_cpu.py) rerun in a subprocess
against libcosim_asan.so, the same sources built with the host code under
AddressSanitizer (device code is not instrumented), with the compiler's ASan
runtime preloaded: argument validation, geometry creation, plan bookkeeping
and error reporting on the host must not read or write out of bounds or use
freed memory.  No GPU is needed."""
import os
import subprocess
import sys

from paper_2503_18479_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale() -> bool:
    if not os.path.exists(B.ASAN_LIB):
        return True
    t = os.path.getmtime(B.ASAN_LIB)
    srcs = [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC)]
    srcs += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return any(os.path.getmtime(p) > t for p in srcs)


def test_abi_host_code_under_asan():
    if _stale():
        B.build(asan=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = B.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["COSIM_LIBRARY"] = B.ASAN_LIB
    env["COSIM_EXPECT_ASAN"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_cpu.py"),
                        "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
