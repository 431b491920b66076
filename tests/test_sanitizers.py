"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU:

- the FP64 oracle (oracle/oracle.c) built with gcc's sanitizers and run on small seeded problems,
  degenerate ones included (tests/sanitize/oracle_driver.c);
- the library's argument validation and host-side sizing (every entry point of include/nnls.h
  called with invalid arguments, the batched sizing with valid ones), in a build whose host code
  carries clang's sanitizers (tests/sanitize/capi_driver.c).  Device code is built as usual; no
  call in the driver reaches the GPU.

Both drivers exit non-zero on a wrong return code, and the sanitizers abort them on any memory
error, undefined behaviour or leak."""
import os
import shlex
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1502_01645_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang"

# sanitizers for the host pass only (the device pass is built without them)
HOST_SAN = shlex.split("-Xarch_host -g -Xarch_host -fno-omit-frame-pointer "
                       "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                       "-Xarch_host -fno-sanitize-recover=all")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_driver.c"),
          "-lm", "-o", exe])
    res = _run([exe], env=dict(SAN_ENV, OMP_NUM_THREADS="4"), timeout=120)
    assert "all checks passed" in res.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not installed")
def test_c_abi_validation_under_address_and_ub_sanitizers(tmp_path):
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-c",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
              *HOST_SAN, os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libnnls_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", *HOST_SAN, *objs, "-o", lib])
    exe = str(tmp_path / "capi_driver")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(SAN, "capi_driver.c"), lib, f"-Wl,-rpath,{tmp_path}", "-o", exe])
    res = _run([exe, str(tmp_path)], env=SAN_ENV, timeout=120)
    assert "all checks passed" in res.stdout
