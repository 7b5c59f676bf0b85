"""The host plan code (csrc/plan.cpp: pattern validation, merge, N(J),
scatter map, combination, chunking) built with AddressSanitizer and
UndefinedBehaviorSanitizer, and the plan tests of tests/test_abi.py run
against that build in a child process (the sanitizer runtime preloaded,
any report fatal). No GPU and no HIP code are involved: the library holds
plan.cpp and a host-only plan destructor written here."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_08245_amd", "csrc")

DESTROY = r'''
#include "plan.h"
// host-only: an unbound plan owns no HIP objects
extern "C" void nolsm_plan_destroy(nolsm_plan *p) { delete p; }
'''

PLAN_TESTS = ("plan_equals_oracle_merge or plan_merges_different_patterns or malformed_patterns or "
              "configure_chunks or bad_options or combination_equals_oracle or default_route or "
              "pipeline_schedule_splits or switch_point")


def gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_plan_code_under_address_sanitizer(tmp_path):
    asan = gcc_runtime("libasan.so")
    ubsan = gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    stub = tmp_path / "destroy.cpp"
    stub.write_text(DESTROY)
    lib = tmp_path / "libnolsm_plan_asan.so"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-shared", "-fPIC", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "plan.cpp"), str(stub), "-o", str(lib)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env.update(NOLSM_LIB=str(lib), LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), "-k", PLAN_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail, tail
    npass = int(r.stdout.strip().splitlines()[-1].split(" passed")[0].split()[-1])
    assert npass >= 10, tail
