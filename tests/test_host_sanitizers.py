"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

* The library's host orchestration (validation, workspace, every GEMM descriptor and launch
  argument of all entry points) is built with the sanitizers in its host code
  (`build(sanitize=True)`) and driven through the dry-run bounds tests (MLCC3_DRYRUN=1: fake
  device addresses, no kernel launched) in a child process with clang's ASan runtime preloaded.
* The C oracle is built with gcc's sanitizers and runs the brute-force pins at tiny sizes in a
  child process with gcc's ASan runtime preloaded.
A sanitizer report aborts the child (-fno-sanitize-recover), which fails the test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def _run(env_extra, args, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *args], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=timeout)
    out = p.stdout + p.stderr
    assert p.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_library_host_code_under_asan_ubsan():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang ASan runtime not found")
    from paper_2202_08612_amd import build
    so = build.build(sanitize=True)
    out = _run({"LD_PRELOAD": rt[-1], "MLCC3_HOST_LIB": so, "MLCC3_DRYRUN": "1"},
               ["tests/test_dryrun_bounds.py", "-m", "not gpu"], 900)
    assert " passed" in out


def test_oracle_under_asan_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.exists(asan):
        pytest.skip("gcc ASan runtime not found")
    from oracle import oracle
    so = oracle.build(sanitize=True)
    out = _run({"LD_PRELOAD": os.path.realpath(asan), "MLCC3_ORACLE_SO": so},
               ["tests/test_oracle_pins.py", "-m", "not gpu", "-k",
                "brute_force_equals or densities_brute or cvs_brute or triple_range or ccsd_reduction"], 900)
    assert " passed" in out
