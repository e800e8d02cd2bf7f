"""Host code under sanitizers, on the CPU.

* The host tests of the C ABI, the streaming runtime and the sensing host
  helpers (tests/test_abi_host.py, test_stream_host.py, test_sense_host.py)
  run again in a child process against librxphy built with AddressSanitizer
  and UndefinedBehaviorSanitizer on its host code (build.py build_sanitized;
  the sanitizer runtime preloaded, leak checks off because the Python
  interpreter and the HIP runtime are not instrumented).  Any report fails.
* The streaming runtime's slot ring and completion thread
  (csrc/stream_ring.h, the state machine the library's streams use) is
  stress-tested by tests/sanitize/ring_stress.cpp with a simulated device,
  built with g++ under ThreadSanitizer and under AddressSanitizer +
  UndefinedBehaviorSanitizer.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_abi_host.py", "tests/test_stream_host.py", "tests/test_sense_host.py"]
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer")


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_host_tests_under_address_and_ub_sanitizers():
    rt = asan_runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no hipcc / clang sanitizer runtime")
    sys.path.insert(0, ROOT)
    from paper_2603_20481_amd.csrc import build
    lib = build.build_sanitized()
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "RXPHY_LIBRARY": lib,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0:verify_asan_link_order=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
                "PYTHONDONTWRITEBYTECODE": "1"})
    rc, out = run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]
                  + HOST_TESTS, env=env)
    print(out[-3000:])
    assert rc == 0, out[-3000:]
    assert not any(k in out for k in REPORTS), out[-3000:]
    assert "passed" in out


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_stream_ring_stress_under_sanitizers(san, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "ring_stress")
    flags = ["-fsanitize=" + san] + (["-fno-sanitize-recover=undefined"] if "undefined" in san else [])
    rc, out = run([gxx, "-std=c++17", "-O1", "-g", "-pthread"] + flags +
                  [os.path.join(ROOT, "tests", "sanitize", "ring_stress.cpp"), "-o", exe])
    assert rc == 0, out
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["ASAN_OPTIONS"] = "halt_on_error=1"
    rc, out = run(["timeout", "-k", "5", "120", exe], env=env, timeout=180)
    print(out)
    assert rc == 0, out
    assert not any(k in out for k in REPORTS), out
    assert "all checks passed" in out
