"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU.

Two instrumented builds are made in a temporary folder and driven by the
existing CPU tests in a child process:
- oracle.c built with gcc -fsanitize=address,undefined, loaded in place of the
  oracle's library (ORACLE_LIBRARY) while the oracle pin tests run;
- the host side of libcorr (corr_host.cpp, prop_host.cpp: argument checks,
  planning, the C ABI) built with the sanitizers on the host pass only and
  linked with the ordinary kernel objects, loaded in place of the library
  (CORR_LIBRARY) while the C-ABI tests run.
A planted heap overflow in a throwaway program shows that the instrumentation
is live. No GPU is used: the ABI tests stop at argument checking.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1711_05075_amd")
BUILD = os.path.join(PKG, "_build")
HIPCC = "/opt/rocm/bin/hipcc"
# sanitizers on the host pass only; device code is built as usual
HOST_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined " \
           "-Xarch_host -fno-sanitize-recover=undefined".split()


def _gcc_rt(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_asan_rt():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def _env(**extra):
    env = dict(os.environ)
    env.update(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", **extra)
    return env


def _run(cmd, env=None, timeout=900):
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


@pytest.fixture(scope="module")
def gcc_san():
    asan, ubsan = _gcc_rt("libasan.so"), _gcc_rt("libubsan.so")
    if shutil.which("gcc") is None or asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    return asan + ":" + ubsan


def test_instrumentation_catches_a_planted_overflow(tmp_path, gcc_san):
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\n"
                   "int main(int c, char** v) { int* a = malloc(4 * sizeof(int)); (void)v;\n"
                   "  a[c + 3] = 1; int r = a[0]; free(a); return r; }\n")
    exe = tmp_path / "overflow"
    r = _run(["gcc", "-O0", "-g", "-fsanitize=address,undefined", str(src), "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=_env())
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


def test_oracle_pins_under_asan_ubsan(tmp_path, gcc_san):
    lib = tmp_path / "liboracle_san.so"
    r = _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
              "-o", str(lib), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    assert r.returncode == 0, r.stderr
    r = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
              "tests/test_oracle_pins.py", "tests/test_oracle_lift_pins.py", "tests/test_oracle_raster_pins.py",
              "tests/test_synth_cpu.py"],
             env=_env(ORACLE_LIBRARY=str(lib), LD_PRELOAD=gcc_san))
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail


def test_host_validation_under_asan_ubsan(tmp_path):
    rt = _clang_asan_rt()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or clang's ASan runtime not installed")
    kernels = [os.path.join(BUILD, f + ".o") for f in ("corr_kernels.hip", "raster_kernels.hip", "prop_kernels.hip")]
    if not all(os.path.exists(k) for k in kernels):
        import paper_1711_05075_amd.build as b
        b.build_library()
    objs = []
    for src in ("corr_host.cpp", "prop_host.cpp"):
        obj = str(tmp_path / (src + ".o"))
        r = _run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer",
                  "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
                  "-c", os.path.join(PKG, "csrc", src), "-o", obj])
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    lib = str(tmp_path / "libcorr_san.so")
    r = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, "-shared-libasan",
              "-o", lib, *kernels, *objs])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "tests/test_abi_cpu.py"],
             env=_env(CORR_LIBRARY=lib, LD_PRELOAD=rt))
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
