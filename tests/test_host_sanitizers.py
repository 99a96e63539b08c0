"""Host code under the sanitizers, on the CPU.

The precompute of many handles runs the layout build, the caching device
allocator and the worker pool on several host threads at once; the FP64
oracle runs its element and node loops with OpenMP.  These tests build
those host paths with ThreadSanitizer and with AddressSanitizer +
UndefinedBehaviorSanitizer and run them:

- tests/native/host_check.cpp: the library's layout.cpp, devcache.cpp and
  pool.cpp with the HIP runtime calls replaced by host stubs
  (tests/native/hip_stub.cpp); layout invariants, the fan mesh's tile
  valence, and layouts built concurrently by the pool equal to serial ones.
- tests/native/oracle_threads.c: the oracle's OpenMP loops (geometry,
  lumping, consistent source, time steps) with 4 threads and with 1, which
  must agree bit for bit.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1909_05098_amd", "csrc")
LLVM = "/opt/rocm/llvm"

HOST_SOURCES = [os.path.join(NATIVE, "host_check.cpp"), os.path.join(NATIVE, "hip_stub.cpp")] + \
    [os.path.join(CSRC, f) for f in ("layout.cpp", "devcache.cpp", "pool.cpp")]


def _build_host(tmp_path, flags):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/hip"):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           *HOST_SOURCES, "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, env=None):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={**os.environ, **(env or {})})
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "runtime error" not in r.stderr, r.stderr
    return r.stdout


def test_host_paths_under_thread_sanitizer(tmp_path):
    out = _run(_build_host(tmp_path, ["-fsanitize=thread"]))
    assert "host_check: ok" in out


def test_host_paths_under_address_and_ub_sanitizers(tmp_path):
    out = _run(_build_host(tmp_path, ["-fsanitize=address,undefined",
                                      "-fno-sanitize-recover=undefined"]),
               {"ASAN_OPTIONS": "detect_leaks=1"})
    assert "host_check: ok" in out


def test_oracle_openmp_loops_under_thread_sanitizer(tmp_path):
    clang = os.path.join(LLVM, "bin", "clang")
    archer = os.path.join(LLVM, "lib", "libarcher.so")
    if not (os.path.exists(clang) and os.path.exists(archer)):
        pytest.skip("clang with the Archer OpenMP tool is missing")
    exe = str(tmp_path / "oracle_threads")
    r = subprocess.run([clang, "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=thread",
                        os.path.join(NATIVE, "oracle_threads.c"), "-lm", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = _run(exe, {"TSAN_OPTIONS": "ignore_noninstrumented_modules=1",
                     "OMP_TOOL_LIBRARIES": archer,
                     "LD_LIBRARY_PATH": os.path.join(LLVM, "lib")})
    assert "bit-identical" in out
