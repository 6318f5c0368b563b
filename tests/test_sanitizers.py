"""The oracle and the library's host code (argument checks, planners,
workspace layout) under AddressSanitizer and UBSan, on the CPU: sanitized
builds of both run existing tests in child processes under their
sanitizer runtime (gcc's for the oracle, clang's for the HIP library's host
code); any finding aborts the child. No kernel runs here."""
import glob
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _run(cmd, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout, cwd=ROOT)


def test_oracle_pins_under_asan_ubsan():
    so = oracle.build_sanitized()
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.exists(libasan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    r = _run([sys.executable, os.path.join(HERE, "mutant_pins.py"), so], {"LD_PRELOAD": libasan}, 600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


def test_host_code_under_asan_ubsan():
    from paper_2307_15255_amd import build
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    so = build.build(sanitize=True)
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", os.path.join(HERE, "test_abi.py"),
              os.path.join(HERE, "test_autotune_host.py")],
             {"LD_PRELOAD": rts[-1], "PT_LIB_PATH": so}, 900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
