"""The host planner and the CPU oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The planner (``spinsum_plan.cpp``, ``spinsum_tune.cpp``) is compiled with g++
against ``tests/sanitize/hip_host_stub.cpp``, which serves the HIP runtime
calls it makes from host memory and can make any one device allocation fail;
``tests/sanitize/plan_driver.cpp`` plans every form (groups at any position,
index pairs, subgroups, batched, chains, FP32, re-tiling) host-only with the
ownership check, and again with each allocation failing in turn: every
failure must return ``SPINSUM_ERR_OUT_OF_MEMORY`` and leave no allocation
behind (LeakSanitizer checks the host side).  The oracle is compiled with
gcc and driven by ``tests/sanitize/oracle_driver.c``.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1705_06661_amd", "csrc")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="no host compiler")


def _compile(cmds, cwd):
    procs = [subprocess.Popen(c, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
             for c in cmds]
    for c, p in zip(cmds, procs):
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, f"{' '.join(c)}\n{out.decode(errors='replace')[-4000:]}"


def _run(exe, cwd):
    r = subprocess.run([exe], cwd=cwd, env=ENV, capture_output=True, text=True, timeout=900)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-6000:]
    assert "PASSED" in r.stdout and "ERROR: AddressSanitizer" not in text and \
        "runtime error" not in text, text[-6000:]
    return r.stdout


def test_planner_under_asan_ubsan(tmp_path):
    inc = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    srcs = [os.path.join(CSRC, "spinsum_plan.cpp"), os.path.join(CSRC, "spinsum_tune.cpp"),
            os.path.join(SAN, "hip_host_stub.cpp"), os.path.join(SAN, "plan_driver.cpp")]
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]
    _compile([["g++"] + inc + SAN_FLAGS + ["-c", s, "-o", o] for s, o in zip(srcs, objs)],
             str(tmp_path))
    exe = str(tmp_path / "plan_driver")
    _compile([["g++"] + SAN_FLAGS + objs + ["-o", exe]], str(tmp_path))
    out = _run(exe, str(tmp_path))
    assert out.count("ok ") >= 17


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _compile([["gcc", "-std=c11", "-fopenmp"] + SAN_FLAGS +
              [os.path.join(ROOT, "oracle", "spinsum_oracle.c"),
               os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe]], str(tmp_path))
    out = _run(exe, str(tmp_path))
    assert out.count("ok ") == 9
