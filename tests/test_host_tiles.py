"""The conv work lists under the host sanitizers (CPU only).

`tests/host/tiles_check.cpp` calls the plan's own builders of the
convolution's work lists (tiles, packed rows, tasks, partial-sum slots) over
a sweep of fault sizes, step sizes, cut-offs, learned-closure cuts, engines
and tile shapes, and checks every property that the conv kernels and the
mode stage rely on.  Here the plan's source and the check are compiled with
the address and undefined-behaviour sanitizers on the host side (the device
code is untouched), linked with the library's other objects, and run.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2107_03550_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
OTHERS = ("exec.cpp.o", "kernels.hip.o", "closure.hip.o", "kernel_eval.cpp.o")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.timeout(600)
def test_work_lists_hold_their_invariants_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("ROCm compilers not found")
    if not all(os.path.exists(os.path.join(BUILD, o)) for o in OTHERS):
        from paper_2107_03550_amd.build import build
        build()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-x", "hip",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             # host code only: the device code of these files is not instrumented
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]
    plan_o, check_o = str(tmp_path / "plan.o"), str(tmp_path / "check.o")
    _run([HIPCC] + flags + ["-c", os.path.join(CSRC, "plan.cpp"), "-o", plan_o])
    _run([HIPCC] + flags + ["-c", os.path.join(ROOT, "tests", "host", "tiles_check.cpp"),
                            "-o", check_o])
    exe = str(tmp_path / "tiles_check")
    # the link is a host-only step (no device source named on it)
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, check_o, plan_o]
         + [os.path.join(BUILD, o) for o in OTHERS]
         + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    last = r.stdout.strip().splitlines()[-1]
    assert last.endswith(" 0 failures") and int(last.split()[0]) > 1000, last
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
