"""Host-side sanitizer runs (CPU only): the oracle built with
AddressSanitizer and UndefinedBehaviorSanitizer runs its brute-force,
closed-form and C-vs-Python pins, and the library's host code (argument
checks, planning, FASTA / FASTQ ingest, fault injection) built with
host-only AddressSanitizer + UndefinedBehaviorSanitizer runs the CPU tests
that drive it.  Each runs in a child process with the sanitizer runtime
preloaded; any report fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def _runtime(compiler, name):
    out = subprocess.run([compiler, f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _child(env_extra, tests, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr


def test_oracle_under_asan_ubsan():
    import oracle
    asan, ubsan = _runtime("gcc", "libasan.so"), _runtime("gcc", "libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    oracle.build(force=True, sanitize=True)
    _child({"LD_PRELOAD": f"{asan}:{ubsan}", "DSA_ORACLE_SANITIZED": "1"},
           ["tests/test_oracle_brute.py", "tests/test_oracle_closed_forms.py", "tests/test_oracle_c_vs_py.py",
            "tests/test_golden.py", "tests/test_golden_topk.py"])


def test_host_runtime_under_asan_ubsan(tmp_path):
    from paper_1701_01575_amd import build, build_san
    lib = build_san.build(str(tmp_path))
    clang = os.path.join(os.path.dirname(build.HIPCC), "..", "llvm", "bin", "clang")
    asan = _runtime(clang, "libclang_rt.asan-x86_64.so") or _runtime(clang, "libclang_rt.asan.so")
    if not asan:
        pytest.skip("clang sanitizer runtime not found")
    _child({"LD_PRELOAD": asan, "DSA_LIBRARY": lib},
           ["tests/test_abi.py", "tests/test_ingest.py", "tests/test_faults.py"])
