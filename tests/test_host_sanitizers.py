"""The host runtime built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code of the C++ runtime sources only, no GPU needed) and driven through
its validation and parsing paths by tests/sanitize/host_checks.cpp."""

import glob
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_02273_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp")
C_CALLER = os.path.join(ROOT, "tests", "sanitize", "c_caller.c")
OUT = os.path.join(ROOT, "_build", "sanitize")
# each -fsanitize= applies to the host side only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
       "-fno-sanitize-recover=all"]


def _tools():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clangxx = "/opt/rocm/llvm/bin/clang++"
    clang = "/opt/rocm/llvm/bin/clang"
    if not all(os.path.exists(t) for t in (hipcc, clangxx, clang)):
        pytest.skip("hipcc / ROCm clang not found")
    return hipcc, clangxx, clang


def _build():
    """The host runtime's C++ sources (and the harness, which includes the
    tuning-file code) compiled with the sanitizers; the HIP sources' objects
    (kernels and their launch wrappers, not instrumented) come from the
    library build."""
    hipcc, clangxx, clang = _tools()
    from paper_2402_02273_amd.build import BUILD, build, sources

    hip_objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in sources() if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in hip_objs):
        build()
    srcs = [s for s in sources() if s.endswith(".cpp") and os.path.basename(s) != "autotune.cpp"]
    digest = hashlib.sha256()
    for p in srcs + [HARNESS, C_CALLER] + hip_objs + glob.glob(os.path.join(CSRC, "*.hpp")) + [
            os.path.join(ROOT, "include", "expint.h")]:
        digest.update(open(p, "rb").read())
    exe = os.path.join(OUT, "host_checks_" + digest.hexdigest()[:16])
    if os.path.exists(exe):
        return exe
    os.makedirs(OUT, exist_ok=True)
    common = ["--cuda-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, "-I",
              os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for src in srcs + [HARNESS]:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        procs.append(subprocess.Popen([hipcc, *common, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT))
        objs.append(obj)
    cobj = os.path.join(OUT, "c_caller.c.o")
    procs.append(subprocess.Popen([clang, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                                   "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-c", C_CALLER,
                                   "-o", cobj], stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    objs.append(cobj)
    for p in procs:
        out = p.communicate()[0].decode()
        assert p.returncode == 0, out
    r = subprocess.run([clangxx, "-fsanitize=address,undefined", *objs, *hip_objs, "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx",
                        "-Wl,-rpath,/opt/rocm/lib", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    exe = _build()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.pop("EXPINT_TUNE_FILE", None)
    env.pop("EXPINT_MAX_BYTES", None)
    r = subprocess.run([exe], cwd=tmp_path, env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert "runtime error" not in out, out
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out
    assert r.returncode == 0, out
    assert "host checks: 0 failed" in out
