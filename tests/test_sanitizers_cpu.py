"""The oracle and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU code is instrumented),
each running its CPU tests in a child process with the sanitizer runtime
preloaded: the oracle's pins, and the device-less checks of the C ABI
(geometry, tables and option validation)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.slow

# errors abort the child; leaks of the interpreter itself are not ours
ENV = {"ASAN_OPTIONS": "detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _pytest(env, args, timeout):
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           "-m", "not gpu and not slow", *args],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


def _check(r):
    text = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, text
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, text


def test_oracle_pins_under_sanitizers(tmp_path):
    import oracle
    lib = oracle.build(force=True, out=str(tmp_path / "liboracle_san.so"),
                       extra=("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                              "-fno-sanitize-recover=all"))
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=asan, FCS_ORACLE_LIB=lib, **ENV)
    _check(_pytest(env, ["tests/test_oracle_pins.py"], 1200))


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2103_14737_amd import build
    lib = str(tmp_path / "libfcs_san.so")
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", flag]
    subprocess.check_call([HIPCC, *build.FLAGS, "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2103_14737_amd", "csrc"), build.SRC,
                           "-o", lib, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", *san])
    rt = subprocess.check_output(["/opt/rocm/llvm/bin/clang",
                                  "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=rt, FCS_TEST_LIB=lib, **ENV)
    _check(_pytest(env, ["tests/test_abi_cpu.py"], 900))
