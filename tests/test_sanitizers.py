"""The FP64 oracle and the library's host code run clean under
AddressSanitizer and UndefinedBehaviorSanitizer on the CPU.

- The oracle (plain C, gcc) is rebuilt with -fsanitize=address,undefined and
  the oracle test modules run against it in a child process that preloads
  gcc's sanitizer runtimes (LWACM_ORACLE_LIB selects the library file).
- The library's host side (lwacm_api.hip: argument checks, omega
  coefficients, error strings, the no-context step's checks) is rebuilt with
  the host-only sanitizer flags of hipcc (the device code is untouched) and
  tests/test_abi.py runs against it with clang's ASan runtime preloaded
  (LWACM_LIBRARY selects the library file).  Device work needs a GPU and is not
  exercised here.
- A control plants a heap overflow in a throwaway C library, built and loaded
  the same way, and requires the sanitizer to report it: the harness can see
  an error.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))


def _gcc_runtimes():
    out = []
    for lib in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={lib}"], capture_output=True, text=True)
        out.append(p.stdout.strip())
    return ":".join(out)


def _env(**kw):
    env = dict(os.environ)
    env.update(ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4", PYTHONPATH=ROOT)
    env.update(kw)
    return env


def _clean(proc):
    text = proc.stdout + proc.stderr
    return proc.returncode == 0 and "AddressSanitizer" not in text and "runtime error" not in text


def test_harness_reports_a_planted_heap_overflow(tmp_path):
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\n"
                   "int bad(int n) { int *a = malloc(4 * n); a[n] = 1; int r = a[0]; free(a);"
                   " return r; }\n")
    lib = tmp_path / "libbad.so"
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fPIC", "-shared",
                    "-o", str(lib), str(src)], check=True)
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).bad(8)"
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       env=_env(LD_PRELOAD=_gcc_runtimes()))
    assert p.returncode != 0 and "heap-buffer-overflow" in p.stderr


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build
    lib = build.build(out=str(tmp_path / "liblwacm_oracle_san.so"), sanitize=True)
    tests = [os.path.join(ROOT, "tests", f) for f in (
        "test_oracle_pins.py", "test_oracle_omega_p.py", "test_oracle_interpolated_bb.py",
        "test_oracle_wall_force.py", "test_oracle_thermal.py", "test_oracle_forced.py")]
    tests.append(os.path.join(ROOT, "tests", "test_oracle_circular_couette.py") +
                 "::test_link_velocities_equal_to_the_table_give_the_table_step")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p",
                        "no:cacheprovider"] + tests, capture_output=True, text=True, cwd=ROOT,
                       env=_env(LD_PRELOAD=_gcc_runtimes(), LWACM_ORACLE_LIB=lib))
    assert _clean(p), (p.stdout[-3000:], p.stderr[-3000:])
    assert " passed" in p.stdout


@pytest.mark.skipif(not CLANG_RT or not os.path.exists(HIPCC), reason="needs ROCm's clang")
def test_host_api_runs_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1111_2142_amd import build as hb
    objs = [os.path.join(hb.BUILD, os.path.basename(s) + ".o")
            for s in sorted(glob.glob(os.path.join(hb.CSRC, "*.hip")))
            if not s.endswith("lwacm_api.hip")]
    if not all(os.path.exists(o) for o in objs):
        hb.build()
    api = str(tmp_path / "lwacm_api_san.o")
    # host-only sanitizers: -Xarch_host before each -fsanitize= flag
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = [f for f in hb.CFLAGS if f != "-O3"]
    subprocess.run([HIPCC] + flags + ["-O1", "-g"] + san +
                   ["-c", os.path.join(hb.CSRC, "lwacm_api.hip"), "-o", api], check=True,
                   capture_output=True)
    lib = str(tmp_path / "liblwacm_san.so")
    subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={hb.ARCH}"] + san[:4] +
                   ["-shared-libsan", "-o", lib, api] + objs, check=True, capture_output=True)
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], capture_output=True,
                       text=True, cwd=ROOT,
                       env=_env(LD_PRELOAD=CLANG_RT[-1], LWACM_LIBRARY=lib))
    assert _clean(p), (p.stdout[-3000:], p.stderr[-3000:])
    assert " passed" in p.stdout
