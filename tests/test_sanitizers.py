"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) built with gcc's sanitizers, its pins run in a child
  process that preloads gcc's runtime.
* The library's host half (argument validation, planners' host checks, sizing
  rules, regressor files and their checksums) built by build_sanitize.py with
  the compiler's sanitizers, the host-only ABI and sizing tests run against it
  in a child process that preloads that runtime.

Any sanitizer report fails the test (the children halt on the first one).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

OPTS = {
    # Python and torch keep allocations alive at exit and mix allocators in
    # their own code; neither is what is checked here.
    "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:detect_odr_violation=0:alloc_dealloc_mismatch=0",
    "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
}


def _run(env_extra, tests):
    env = dict(os.environ)
    env.update(OPTS)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def _gcc_runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc has no {name}")
    return path


def test_oracle_under_sanitizers():
    pre = f"{_gcc_runtime('libasan.so')}:{_gcc_runtime('libubsan.so')}"
    out = _run({"TN_ORACLE_SANITIZE": "1", "LD_PRELOAD": pre},
               ["tests/test_oracle.py", "tests/test_oracle_torus.py", "tests/test_oracle_prior.py",
                "tests/test_oracle_partial.py"])
    assert " passed" in out


def test_host_library_under_sanitizers():
    from paper_2603_07387_amd import build_sanitize as B
    lib = B.build()
    rt = B.runtime()
    if not rt:
        pytest.skip("no ASan runtime next to hipcc")
    out = _run({"TN_SKETCH_LIB": lib, "LD_PRELOAD": rt}, ["tests/test_abi.py", "tests/test_sizing_host.py"])
    assert " passed" in out
