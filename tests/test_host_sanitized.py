"""The library's host code under the address and undefined-behaviour sanitizers (no GPU needed).

Every HIP and C++ source of libph is compiled with the sanitizers on the host side only (the
device code is built as usual), linked with the checks in ``tests/host/host_checks.cpp``, and
run: argument validation, plan teardown after a failed create (no device on this machine),
the FP64 operator build, the own-cell integral, the plan-time octree and the list-range
clamp.  A sanitizer report or a failed check fails the test."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_10059_amd", "csrc")
OUT = os.path.join(ROOT, "tests", "host", "_build_sanitized")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
         "-Wno-unused-command-line-argument", "-Wno-pass-failed"]


def _compile(src, obj):
    lang = ["-x", "hip"]
    return subprocess.Popen([HIPCC] + FLAGS + SAN + lang + ["-c", src, "-o", obj],
                            stdout=subprocess.PIPE, stderr=subprocess.STDOUT)


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not installed")
def test_host_code_under_sanitizers():
    if os.path.isdir(OUT):
        shutil.rmtree(OUT)
    os.makedirs(OUT)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs.append(os.path.join(ROOT, "tests", "host", "host_checks.cpp"))
    objs, procs = [], []
    for s in srcs:
        o = os.path.join(OUT, os.path.basename(s) + ".o")
        objs.append(o)
        procs.append((s, _compile(s, o)))
    for s, p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, f"compile {s}:\n{out.decode(errors='replace')[-4000:]}"
    exe = os.path.join(OUT, "host_checks")
    link = subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", exe] + objs +
                          ["-L/opt/rocm/lib", "-lamdhip64", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"],
                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert link.returncode == 0, link.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    run = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    print(run.stdout[-6000:])
    assert run.returncode == 0, run.stdout[-6000:]
    assert "host checks passed" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stdout and "runtime error" not in run.stdout
