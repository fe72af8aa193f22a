"""The library's host code (include/qoc.h calls as implemented in qoc_api.cpp) on the CPU, with the
HIP runtime and the kernel launchers replaced by a host-memory stand-in (tests/host_harness/):
system builds, single-context calls, batches of every size from one to five contexts with mixed
backward schedules and exactly sufficient capacities, per-context status, qoc_batch_gradient,
argument errors, and teardown without leaked device blocks.

Two builds: -O3 (the optimisation level of the library; it emits the 16-byte aligned stores of
the batch tables, so a misaligned staging section faults as it did on the GPU machine) and -O1
with AddressSanitizer and UBSan."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/llvm/bin/clang++"
HIP_INC = "/opt/rocm/include"


def build(tmp, flags):
    objs = []
    # a 256 KiB table capacity for the allocation-free call, so its over-capacity path is reached
    # with a few small contexts
    cap = ["-DQOC_NOALLOC_SCRATCH_BYTES=262144"]
    srcs = [(os.path.join(ROOT, "paper_2407_13950_amd", "csrc", "qoc_api.cpp"), ["-D__HIP_PLATFORM_AMD__", *cap]),
            (os.path.join(ROOT, "tests", "host_harness", "hip_standin.cpp"), ["-D__HIP_PLATFORM_AMD__", *cap]),
            (os.path.join(ROOT, "tests", "host_harness", "main.cpp"), [])]
    for src, extra in srcs:
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        subprocess.check_call([CXX, "-std=c++17", "-g", *flags, *extra, "-I", HIP_INC, "-I",
                               os.path.join(ROOT, "include"), "-c", src, "-o", obj])
        objs.append(obj)
    exe = os.path.join(tmp, "harness")
    subprocess.check_call([CXX, *flags, "-o", exe, *objs])
    return exe


@pytest.mark.skipif(not (os.path.exists(CXX) and os.path.isdir(HIP_INC)), reason="needs ROCm's clang++ and HIP headers")
@pytest.mark.parametrize("flags", [["-O3"], ["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                             "-fno-omit-frame-pointer"]], ids=["O3", "asan-ubsan"])
def test_host_code_on_the_stand_in(tmp_path, flags):
    exe = build(str(tmp_path), flags)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "HARNESS OK" in r.stdout
