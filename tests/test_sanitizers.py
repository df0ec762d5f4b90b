"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

Both are rebuilt with gcc's -fsanitize=address,undefined (the library's HIP
objects are linked in as built; only the host C/C++ is instrumented) into a
temporary directory, and the oracle pins, the host-structure comparison and
the ABI checks run against those builds in a child process that preloads the
sanitizer runtimes.  Any report (out-of-bounds access, use after free,
signed overflow, misaligned access, ...) aborts the child and fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1902_01829_amd", "csrc")
HOST_SOURCES = ["h2_structure.cpp", "h2_build.cpp", "h2_run.cpp", "h2_batch.cpp", "h2_transform.cpp", "h2_api.cpp"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _tool(name):
    path = shutil.which(name)
    if path is None:
        pytest.skip(f"{name} not available")
    return path


def _run(cmd, **kw):
    subprocess.run(cmd, check=True, capture_output=True, text=True, **kw)


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    gcc, gxx = _tool("gcc"), _tool("g++")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hip_objs = [os.path.join(ROOT, "_build", f + ".o") for f in
                ("h2_kernels.hip", "h2_mm.hip", "h2_orth.hip", "h2_comp.hip", "h2_noalloc.hip")]
    if not all(os.path.exists(o) for o in hip_objs):
        pytest.skip("the library's HIP objects are not built (python -m paper_1902_01829_amd.build)")
    d = tmp_path_factory.mktemp("san")
    oracle_so = str(d / "liboracle.so")
    _run([gcc, *SAN, "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", oracle_so,
          os.path.join(ROOT, "oracle", "h2oracle.c"), "-lm"])
    objs = []
    for src in HOST_SOURCES:
        obj = str(d / (src + ".o"))
        _run([gxx, *SAN, "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"),
              "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-ffp-contract=off", "-c",
              os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib_so = str(d / "libh2mv.so")
    _run([gxx, "-shared", "-fsanitize=address,undefined", "-o", lib_so, *objs, *hip_objs,
          "-L" + os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lamdhip64", "-lpthread"])
    runtimes = [subprocess.run([gcc, "-print-file-name=" + n], check=True, capture_output=True,
                               text=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    return oracle_so, lib_so, runtimes


def test_host_code_and_oracle_clean_under_sanitizers(sanitized):
    oracle_so, lib_so, runtimes = sanitized
    env = dict(os.environ)
    env.update({
        "H2_ORACLE_LIBRARY": oracle_so,
        "H2MV_LIBRARY": lib_so,
        "LD_PRELOAD": ":".join(runtimes),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "OMP_NUM_THREADS": "4",
    })
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_oracle.py", "test_structure.py", "test_abi.py")]
    # -s: a sanitizer report ends the process inside a test, so pytest's own
    # output capture would swallow it
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *tests], env=env, capture_output=True, text=True, cwd=ROOT, timeout=1200)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
