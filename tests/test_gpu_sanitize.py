"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host pass only; the GPU kernels are the product's): tests/host/abi_sanitize,
built by __graft_entry__.build() (tests/host/build_sanitize.py), drives every
entry point of the C ABI and a server with its driver thread on the GPU.  The
sanitizers abort the program at the first error; leak checking is off (the
HIP runtime keeps allocations until exit)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "host", "abi_sanitize")


def test_host_code_under_sanitizers():
    assert os.path.exists(EXE), "build() builds tests/host/abi_sanitize"
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    p = subprocess.run([EXE], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       timeout=280)
    out = p.stdout.decode(errors="replace")
    print(out[-3000:], flush=True)
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert p.returncode == 0 and "all checks held" in out
