"""The serving loop's scheduling core on the CPU, with no GPU: tests/serve_fake.cpp drives
hav_serve::Server (paper_2305_14306_amd/csrc/server_core.hpp, the same core the library
runs over HIP) with an executor over the CPU oracle. It covers admission by footprint,
queueing under a one-slot budget, release of idle slots of other classes, rejection of
requests that can never fit, result routing under continuous batching, recovery after a
failed batch, and shutdown with requests queued.

The driver is built twice: with AddressSanitizer + UndefinedBehaviorSanitizer (g++), which
also runs the oracle under them, and with ThreadSanitizer. The TSan build uses ROCm's
clang++: GCC 11's libtsan does not intercept pthread_cond_clockwait, which libstdc++'s
condition_variable::wait_for calls, so under it every wait looks like the mutex is still
held and the run reports false races and stalls."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "serve_fake.cpp"), os.path.join(ROOT, "oracle", "hav_oracle.cpp")]
INC = os.path.join(ROOT, "include")
ROCM_CLANG = "/opt/rocm/llvm/bin/clang++"

BUILDS = {
    "asan_ubsan": ("g++", ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=undefined"]),
    "tsan": (ROCM_CLANG, ["-fsanitize=thread"]),
}


@pytest.mark.parametrize("build", sorted(BUILDS))
def test_server_core_with_oracle_executor(tmp_path, build):
    cxx, flags = BUILDS[build]
    if shutil.which(cxx) is None and not os.path.exists(cxx):
        pytest.skip(f"{cxx} not found")
    exe = str(tmp_path / f"serve_fake_{build}")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-pthread", *flags, "-I", INC, *SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ALL PASS" in r.stdout, out[-4000:]
    assert "Sanitizer" not in out, out[-4000:]
