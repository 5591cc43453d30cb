"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two instrumented builds, each driven by existing tests in a child process that
preloads its sanitizer runtime (Python itself is not instrumented):

- the HIP library with the sanitizers on its host side only (planning, layouts,
  workspace sizing, plan cache, argument checks); its device code is compiled
  at -O0 to keep the build short and is never run here.  Driven by the
  host-only ABI tests.
- the C oracle built by gcc.  Driven by the oracle's pin tests (generator,
  transforms, brute-force and structural checks of A_hat).

Every report is fatal (no recovery), so any out-of-bounds access, use after
free or undefined operation fails the child and this test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}

# a child process that points a module at the instrumented build, then runs pytest
RUNNER = """
import sys
sys.path.insert(0, {root!r})
import {module} as M
M.{attr} = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *{files!r}]))
"""


def _run_child(preload, module, attr, lib, files):
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload)
    code = RUNNER.format(root=ROOT, module=module, attr=attr, lib=lib, files=files)
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=900)
    out = res.stdout[-4000:] + res.stderr[-8000:]
    assert res.returncode == 0, out
    assert "passed" in res.stdout, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_library_host_code_under_asan_ubsan():
    rt = _clang_asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or the clang ASan runtime is not installed")
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libsketch_san.so")
    src = os.path.join(ROOT, "paper_2310_15419_amd", "csrc", "sk_lib.hip")
    cmd = [HIPCC, "-O0", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(src),
           "-Xarch_host", "-O1", "-Xarch_host", "-g",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-o", lib, src]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    _run_child(rt, "paper_2310_15419_amd.binding", "LIB_PATH", lib,
               [os.path.join(ROOT, "tests", "test_lib_abi.py")])


@pytest.mark.slow
def test_oracle_under_asan_ubsan():
    res = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    rt = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(rt):
        pytest.skip("gcc's ASan runtime is not installed")
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libskoracle_san.so")
    src = os.path.join(ROOT, "oracle", "sk_oracle.c")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", lib, src, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    _run_child(rt, "oracle", "_LIB_PATH", lib,
               [os.path.join(ROOT, "tests", f) for f in
                ("test_oracle_rng.py", "test_oracle_sketch.py")])


@pytest.mark.slow
def test_the_harness_reports_a_planted_overflow():
    """The same flags and preload catch a heap read one past the end (a CPU-only
    C function written for this check, not part of the library or the oracle)."""
    res = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    rt = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(rt):
        pytest.skip("gcc's ASan runtime is not installed")
    os.makedirs(OUT, exist_ok=True)
    src = os.path.join(OUT, "planted.c")
    lib = os.path.join(OUT, "libplanted.so")
    with open(src, "w") as f:
        f.write("#include <stdlib.h>\n"
                "int planted(int n) { int* p = malloc(n * sizeof(int));\n"
                "  for (int i = 0; i < n; ++i) p[i] = i;\n"
                "  int s = p[n]; free(p); return s; }\n")
    res = subprocess.run(["gcc", "-O0", "-g", "-fPIC", "-shared", "-fsanitize=address,undefined",
                          "-fno-sanitize-recover=all", "-o", lib, src],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=rt)
    code = f"import ctypes; print(ctypes.CDLL({lib!r}).planted(8))"
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120)
    assert res.returncode != 0
    assert "heap-buffer-overflow" in res.stderr
