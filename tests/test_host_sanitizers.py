"""The threaded host CSR builder under AddressSanitizer + UBSan and under
ThreadSanitizer (host code only: the harness makes no device call).  The
harness compares every built graph with a plain sort-and-unique
construction."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2311_10290_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = os.environ.get("CLANGXX", "/opt/rocm/llvm/bin/clang++")
BASE = ["-x", "hip", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC]


@pytest.mark.skipif(not os.path.exists(HIPCC) or not os.path.exists(CLANGXX), reason="hipcc or clang++ not found")
@pytest.mark.parametrize("san", [["address", "undefined"], ["thread"]])
def test_csr_builder_under_sanitizers(tmp_path, san):
    host = []
    for s in san:
        host += ["-Xarch_host", f"-fsanitize={s}"]
    objs = []
    for src in (os.path.join(HERE, "host", "csr_check.cpp"), os.path.join(CSRC, "graph.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call([HIPCC, *BASE, *host, "-c", src, "-o", obj])
        objs.append(obj)
    # host link of the two objects with the plain host compiler and the HIP
    # runtime (the harness makes no device call)
    exe = str(tmp_path / "csr_check")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    subprocess.check_call([CLANGXX, *[f"-fsanitize={s}" for s in san], *objs, "-o", exe, "-L", f"{rocm}/lib",
                           "-lamdhip64", f"-Wl,-rpath,{rocm}/lib", "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
