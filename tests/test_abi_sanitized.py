"""The C ABI's host paths (argument validation, status strings, error
messages, struct layouts) under AddressSanitizer and
UndefinedBehaviorSanitizer: the library is built with both on its host code
and tests/test_abi_cpu.py runs against it in a child process with the clang
ASan runtime preloaded. No GPU is used."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_abi_host_paths_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    sys.path.insert(0, ROOT)
    from paper_1707_02245_amd import build as B
    lib = B.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=rt, PAT_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    check = ("from paper_1707_02245_amd import _lib; _lib.load(); "
             "maps = open('/proc/self/maps').read(); "
             f"assert {lib!r} in maps, 'sanitized library not mapped'; print('sanitized library loaded')")
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_abi_cpu.py", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
