"""AddressSanitizer and UndefinedBehaviorSanitizer builds of host code (CPU
only): the FP64 oracle with a harness that calls each of its functions on a
small scene, and the C ABI's host side (argument checks, workspace layout)
with a harness of calls that all return before any kernel launch.  Device
code is not instrumented (no sanitizer for it on this platform)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert p.returncode == 0, "%s\n%s" % (" ".join(cmd), p.stdout[-4000:])
    return p.stdout


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_check.c"), "-o", exe, "-lm"])
    out = _run([exe], env=SAN_ENV)
    assert "oracle harness ok" in out


def test_abi_host_checks_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from paper_2412_04459_amd import build as B
    objs = [os.path.join(B.BUILD, s.replace(".hip", ".o")) for s in B.SOURCES if s != "svr_api.hip"]
    if not all(os.path.exists(o) for o in objs) or not shutil.which("g++"):
        pytest.skip("library objects not built (run the build first)")
    api = str(tmp_path / "svr_api_san.o")
    # the HIP source: sanitizers on the host pass only
    _run([B.hipcc()] + B.compile_flags() + ["-O1", "-g",
                                            "-Xarch_host", "-fsanitize=address",
                                            "-Xarch_host", "-fsanitize=undefined",
                                            "-Xarch_host", "-fno-sanitize-recover=all",
                                            "-c", os.path.join(B.CSRC, "svr_api.hip"), "-o", api])
    harness = str(tmp_path / "abi_check.o")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I", B.INCLUDE, "-c", os.path.join(HERE, "abi_check.cpp"),
          "-o", harness])
    exe = str(tmp_path / "abi_check")
    _run(["g++", "-fsanitize=address,undefined", harness, api] + objs +
         ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", exe])
    # the HIP runtime keeps allocations until exit: leaks are not checked here
    env = dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    out = _run([exe], env=env)
    assert "abi harness ok" in out
