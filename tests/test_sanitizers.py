"""AddressSanitizer and UndefinedBehaviorSanitizer over the CPU-side code.

* The oracle (``oracle/oracle.c``) built with gcc's ASan + UBSan runs the
  oracle's own pin tests in a child process with the sanitizer runtime
  preloaded.
* The library's host code (request validation, table building, output
  layout, request sizes; the device code is left alone) built with clang's
  ASan + UBSan on the host pass only runs the ABI, serving-scheduler and
  generator tests in another child process (the two runtimes cannot share a
  process).

Any sanitizer report aborts the child (halt_on_error, no UBSan recovery), so
a clean exit means a clean run.  Built under _build/san (not committed).
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "san")

pytestmark = pytest.mark.slow

ORACLE_TESTS = ["tests/test_oracle_ball.py", "tests/test_oracle_robot.py",
                "tests/test_oracle_sbip.py", "tests/test_oracle_angle.py",
                "tests/test_oracle_worked.py", "tests/test_oracle_invariants.py",
                "tests/test_oracle_scenarios.py", "tests/test_golden.py"]
HOST_TESTS = ["tests/test_abi_cpu.py", "tests/test_serving.py", "tests/test_zones_host.py"]


def _run_child(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow"] + tests, cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_asan_and_ubsan():
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                           "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    pre = ":".join(subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
                   for n in ("libasan.so", "libubsan.so"))
    out = _run_child({"ORACLE_LIB": lib, "LD_PRELOAD": pre}, ORACLE_TESTS)
    assert " passed" in out


def test_library_host_code_under_asan_and_ubsan():
    os.makedirs(OUT, exist_ok=True)
    sys.path.insert(0, ROOT)
    from paper_1909_07717_amd import build as Bd
    lib = os.path.join(OUT, "libdpps_san.so")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    Bd.build(extra=host_san, out=lib, link_extra=["-shared-libsan"] + host_san)
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    assert rt, "clang ASan runtime not found"
    out = _run_child({"DPPS_LIB": lib, "LD_PRELOAD": rt[-1]}, HOST_TESTS)
    assert " passed" in out
