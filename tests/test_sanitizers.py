"""The CPU parts of the project under sanitizers (no GPU needed):
  - the oracle library built with AddressSanitizer and UndefinedBehavior-
    Sanitizer (gcc), running its own pins (tests/test_oracle.py);
  - the library's host code (argument validation, per-view constants, the
    render server, the autotune cache) built with AddressSanitizer + UndefinedBehaviorSanitizer
    and, separately, ThreadSanitizer (clang), driven by
    tests/sanitize/serve_stress.cpp: validation of every one-view entry
    point, the server's scheduler in dry-run mode with concurrent
    submitters, pollers and statistics readers, drain and timed destroy,
    and the batch autotune cache's file handling and order classifier.
Any sanitizer report fails the run."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1908_02681_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
ROCM = "/opt/rocm"


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if not shutil.which("gcc") or not asan:
        pytest.skip("gcc with AddressSanitizer not available")
    lib = str(tmp_path / "librz_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                    "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "rz_oracle.c"), "-o", lib, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, RZ_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the instrumented library is the one loaded
    probe = subprocess.run(
        [sys.executable, "-c",
         "from oracle import oracle; oracle._load(); "
         "print(open('/proc/self/maps').read())"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert lib in probe.stdout and "libasan" in probe.stdout
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert run.returncode == 0, (run.stdout[-3000:], run.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr


def _build_driver(tmp_path, name, flags):
    if not os.path.exists(CLANG) or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("clang or the HIP runtime library not available")
    exe = str(tmp_path / name)
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
           "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", f"-I{CSRC}", f"-I{ROCM}/include",
           os.path.join(ROOT, "tests", "sanitize", "serve_stress.cpp"),
           os.path.join(CSRC, "rz_serve.cpp"), os.path.join(CSRC, "rz_api.cpp"),
           os.path.join(CSRC, "rz_tune.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib", "-lpthread", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = _build_driver(tmp_path, "serve_asan",
                        ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    for merge in ("4", "0"):   # merging; then chaining behind running requests
        run = subprocess.run([exe, merge], capture_output=True, text=True, timeout=300,
                             env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
        assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
        assert "served 600 requests, 0 errors" in run.stdout
        assert _count(run.stdout, "merged" if merge == "4" else "chained") > 0   # the path ran


def _count(out, what):
    line = [l for l in out.splitlines() if l.startswith(what + " ")][0]
    return int(line.split()[1])


def test_scheduler_under_tsan(tmp_path):
    exe = _build_driver(tmp_path, "serve_tsan", ["-fsanitize=thread"])
    for merge in ("4", "0"):
        run = subprocess.run([exe, merge], capture_output=True, text=True, timeout=300,
                             env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
        assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
        assert "ThreadSanitizer" not in run.stderr
        assert "served 600 requests, 0 errors" in run.stdout
