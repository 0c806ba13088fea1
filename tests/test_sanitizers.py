"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle, built with gcc and both sanitizers, runs its pin tests in a
  child process with gcc's sanitizer runtime preloaded.
* The library, built with the host pass sanitized (device code is not),
  runs the C-ABI tests in a child process with clang's runtime preloaded:
  argument checks, parameter suggestion, plan set-up and its error path
  (without a GPU, set-up stops at its first device call), the allocation-free
  entry point's checks.

Both children must pass and print no sanitizer report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT_MARKS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "UndefinedBehaviorSanitizer")


def _child(env_extra, args, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    for m in REPORT_MARKS:
        assert m not in out, m


def _gcc_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_oracle_pins_under_sanitizers(tmp_path):
    rt = _gcc_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    from oracle import oracle as orc
    lib = orc.build(out=str(tmp_path / "liboracle_asan.so"),
                    extra_flags=("-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                 "-fno-omit-frame-pointer", "-g"))
    _child({"LD_PRELOAD": rt, "MPEWALD_ORACLE_LIB": lib},
           ["tests/test_oracle_pins.py", "tests/test_region_pins.py"])


def test_library_host_code_under_sanitizers(tmp_path):
    rt = _clang_runtime()
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    from paper_2408_03273_amd import build
    # host-pass options only: each one follows -Xarch_host
    host = ("-Xarch_host", "-fsanitize=address,undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer")
    lib = build.build(out=str(tmp_path / "libmpewald_asan.so"), objdir=str(tmp_path / "obj"), extra_flags=host)
    _child({"LD_PRELOAD": rt, "MPEWALD_LIB": lib}, ["tests/test_abi.py", "tests/test_params.py"])


def test_sanitizer_catches_a_planted_overflow(tmp_path):
    """The runtime in this environment reports what it should: a one-past-the-
    end read in a small C program built the same way stops it with a report."""
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\nint main(int c, char** v) {\n  (void)v;\n"
                   "  double* a = malloc(4 * sizeof(double));\n  for (int i = 0; i < 4; i++) a[i] = i;\n"
                   "  double s = a[3 + c];\n  free(a);\n  return s > 1e300;\n}\n")
    exe = tmp_path / "planted"
    subprocess.run(["gcc", "-O0", "-g", "-fsanitize=address,undefined", "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]
