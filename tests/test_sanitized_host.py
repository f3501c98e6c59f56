"""The host C++ of libivde (argument validation, FP64 composition, layout,
graph-cut optimisation, server bookkeeping) under AddressSanitizer and
UndefinedBehaviorSanitizer: the CPU suites that exercise it without a GPU run
in a subprocess against libivde_san.so (built by build() with host-only
sanitizers), with any report fatal."""
import os
import subprocess
import sys

import pytest

from paper_1909_02294_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(not os.path.exists(build.SAN_LIB), reason="libivde_san.so not built")
def test_host_code_under_asan_and_ubsan():
    env = build.sanitize_env()
    probe = ("import ctypes, sys; from paper_1909_02294_amd import ivde; ivde.load(); "
             "maps = open('/proc/self/maps').read(); "
             "assert 'libivde_san.so' in maps and 'libclang_rt.asan' in maps, 'sanitizer build not loaded'; "
             "print(ivde.LIB_PATH)")
    r = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip() == build.SAN_LIB
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi_cpu.py", "tests/test_graphcut_parity.py"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
