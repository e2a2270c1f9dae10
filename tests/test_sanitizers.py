"""The oracle and the C ABI's host code under AddressSanitizer + UBSan (no
GPU).  Each runs a set of CPU tests in a child process that preloads the
matching ASan runtime (g++'s for the oracle, the HIP compiler's for libhp's
host code); any sanitizer report fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_child(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan():
    import oracle
    oracle.build(sanitize=True)
    out = _run_child({"LD_PRELOAD": oracle.asan_runtime(), "HP_ORACLE_SANITIZED": "1", "OMP_NUM_THREADS": "4"},
                     ["tests/test_oracle_render.py", "tests/test_oracle_hssim.py", "tests/test_oracle_query.py",
                      "tests/test_oracle_healpix.py", "tests/test_oracle_interp.py", "tests/test_oracle_depth.py"])
    assert " passed" in out


def test_abi_host_checks_under_asan_ubsan():
    from paper_2606_29794_amd import build
    build.build(sanitize=True)
    out = _run_child({"LD_PRELOAD": build.asan_runtime(), "HP_SANITIZED": "1"}, ["tests/test_abi.py"])
    assert " passed" in out
