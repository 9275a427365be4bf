"""Host code under the compiler's sanitizers (CPU only).

- The oracle (every entry point of oracle.h on RAMBO events of each process)
  under AddressSanitizer and UndefinedBehaviorSanitizer.
- The serving scheduler (csrc/serve.cpp) with its test double, several
  submitting threads, splits, injected failures and bounded pass-over, under
  ThreadSanitizer and under AddressSanitizer + UndefinedBehaviorSanitizer.

Built with ROCm's clang: the ThreadSanitizer runtime of the system gcc does
not intercept pthread_cond_clockwait (used by std::condition_variable's timed
waits), so it reports every lock taken after such a wait as a double lock."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = os.path.join(ROOT, "tests", "sanitize")

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="no clang++ with sanitizer runtimes")


def _build_and_run(tmp_path, name, sources, flags, libs=(), timeout=600):
    exe = str(tmp_path / name)
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, *sources, "-pthread", "-o", exe,
           *libs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    return r.stdout


_HIP = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
_HIPLIB = ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
_SERVE = [os.path.join(ROOT, "paper_2303_18244_amd", "csrc", "serve.cpp"), os.path.join(SAN, "serve_driver.cpp")]


@pytest.mark.slow
def test_oracle_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "oracle_asan",
                         [os.path.join(ROOT, "oracle", "oracle.cpp"), os.path.join(SAN, "oracle_driver.cpp")],
                         ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    assert "all checks passed" in out


def test_serve_scheduler_tsan(tmp_path):
    out = _build_and_run(tmp_path, "serve_tsan", _SERVE, ["-fsanitize=thread", *_HIP], _HIPLIB)
    assert "all checks passed" in out


def test_serve_scheduler_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "serve_asan", _SERVE,
                         ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", *_HIP], _HIPLIB)
    assert "all checks passed" in out
