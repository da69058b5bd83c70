"""Host code under sanitizers (no device call anywhere):
  - the threaded host CSR builder under AddressSanitizer + UBSan and under
    ThreadSanitizer; the harness compares every built graph with a plain
    sort-and-unique construction;
  - the oracle's C sampler under AddressSanitizer + UBSan, every entry point
    with one thread and several."""
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


ORACLE = os.path.join(HERE, "..", "oracle", "sampler.c")


@pytest.mark.skipif(not os.path.exists("/usr/bin/gcc"), reason="gcc not found")
def test_oracle_sampler_under_address_and_ub_sanitizers(tmp_path):
    """The oracle's C sampler (every entry point, one thread and several)
    built with AddressSanitizer and UBSan; the harness checks tree shape and
    count invariants and equal results across thread counts."""
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", os.path.join(HERE, "host", "oracle_check.c"), ORACLE,
                           "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


@pytest.mark.skipif(not os.path.exists("/usr/bin/g++"), reason="g++ not found")
def test_serving_arena_policy(tmp_path):
    """The serving result arena's first-fit policy (host code, no device)
    under AddressSanitizer and UBSan, against a per-word occupancy map."""
    exe = str(tmp_path / "arena_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-I", CSRC, os.path.join(HERE, "host", "arena_check.cpp"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
