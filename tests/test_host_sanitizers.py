"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a build with both on the host side (device code unchanged) runs
every host-side call over the benchmark workloads (tests/sanitize_driver.py)
with the ASan runtime preloaded; any report aborts the run."""
import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.mark.slow
def test_host_calls_are_clean_under_asan_and_ubsan(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("no ASan runtime in this ROCm installation")
    from paper_2111_06893_amd import build
    lib = build.build(sanitize=True, out=str(tmp_path / "libdgtn_sanitized.so"))
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitize_driver.py"), lib], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "SANITIZED HOST CALLS DONE" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
