"""The oracle's C code and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

Each check builds a sanitizer build into a temporary directory and runs CPU
test files against it in a child process (the sanitizer runtime preloaded,
leak detection off: the Python interpreter is not instrumented); any report
fails the check, as does any failing test.  No GPU is touched: the library's
host paths exercised are argument and option validation, the planner, the
workspace sizes, the tuning table and its files.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("AddressSanitizer", "runtime error:", "UndefinedBehaviorSanitizer")


def _run_child(files, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=99"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=98"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
           "-m", "not gpu"] + [os.path.join(ROOT, f) for f in files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    bad = [line for line in out.splitlines() if any(k in line for k in REPORTS)]
    assert r.returncode == 0 and not bad, "\n".join(bad[:20]) + "\n" + out[-3000:]


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True,
                       check=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("gcc has no %s" % name)
    return p


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "signtri_oracle.c")
    subprocess.run(["gcc", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-std=c99", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", lib, src, "-lm"],
                   check=True)
    _run_child(["tests/test_oracle_pins.py", "tests/test_oracle_reorder.py",
                "tests/test_oracle_mutations.py"],
               {"SIGNTRI_ORACLE_LIB": lib, "LD_PRELOAD": _gcc_runtime("libasan.so")})


def test_host_code_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1607_06303_amd import build

    lib = build.build_host_sanitized(str(tmp_path / "san"))
    _run_child(["tests/test_abi_cpu.py", "tests/test_tune_cpu.py"],
               {"SIGNTRI_LIB": lib, "LD_PRELOAD": build.sanitizer_runtime()})
