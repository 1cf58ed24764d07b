"""Address- and undefined-behaviour-sanitizer runs on the CPU.

1. The oracle (plain C) built with gcc -fsanitize=address,undefined and driven
   by oracle/sanitize_check.c through every exported routine at small sizes,
   with results checked against the oracle's own invariants.
2. The library's host code built with hipcc, sanitizers on the host pass only
   (-Xarch_host before each -fsanitize=), linked to
   paper_1307_6748_amd/csrc/validate_check.c, which calls every entry point of
   the C ABI with arguments that validation must reject, and the host-only
   size and layout queries.  No call reaches a GPU.

Both drivers abort on the first sanitizer report (-fno-sanitize-recover=all,
halt_on_error), so a zero exit status means a clean run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1307_6748_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _clang():
    p = "/opt/rocm/llvm/bin/clang"
    return p if os.path.exists(p) else shutil.which("clang")


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    """Start all compiles at once (the device pass of the library dominates)."""
    if shutil.which("gcc") is None or shutil.which("hipcc") is None or _clang() is None:
        pytest.skip("gcc, hipcc and clang are needed")
    d = tmp_path_factory.mktemp("san")
    orc_exe = str(d / "orc_san")
    procs = {
        "oracle": subprocess.Popen(
            ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp", *SAN, "-o", orc_exe,
             os.path.join(ROOT, "oracle", "sanitize_check.c"),
             os.path.join(ROOT, "oracle", "isis_oracle.c"), "-lm"],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True),
    }
    objs = []
    for src in ("isis_mg.hip", "unet.hip"):
        obj = str(d / (src + ".o"))
        objs.append(obj)
        procs[src] = subprocess.Popen(
            ["hipcc", "--offload-arch=gfx950", "-O1", "-Xarch_host", "-g", "-std=c++17", "-fPIC",
             "-c", *HOST_SAN, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-o", obj, os.path.join(CSRC, src)],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = {k: p.communicate(timeout=600)[0] for k, p in procs.items()}
    for k, p in procs.items():
        assert p.returncode == 0, f"{k} build failed:\n{out[k][-3000:]}"
    lib = str(d / "libisis_san.so")
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN,
                        "-o", lib, *objs], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    val_exe = str(d / "val_san")
    r = subprocess.run([_clang(), "-g", *SAN, "-I/opt/rocm/include", "-o", val_exe,
                        os.path.join(CSRC, "validate_check.c"), lib, f"-Wl,-rpath,{d}", "-lm"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return orc_exe, val_exe


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    assert "runtime error" not in text and "ERROR: AddressSanitizer" not in text, text[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(builds):
    assert "0 failures" in _run(builds[0])


def test_host_validation_under_sanitizers(builds):
    assert "0 failures" in _run(builds[1])
