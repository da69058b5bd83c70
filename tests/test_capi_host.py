"""The C-ABI library loads, exports every symbol include/lap.h declares, and
rejects bad arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lap.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lap_[a-zA-Z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    from paper_2311_10290_amd import _capi
    assert _declared() == sorted(_capi.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2311_10290_amd import load_library
    lib = load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_nm_shows_c_linkage():
    from paper_2311_10290_amd import _capi
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", _capi.LIB_PATH], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for name in _declared():
        assert name in syms, name


def _build(n, src, dst, flags=0):
    from paper_2311_10290_amd import load_library
    lib = load_library()
    h = ctypes.c_void_p()
    s = np.ascontiguousarray(src, np.int32)
    d = np.ascontiguousarray(dst, np.int32)
    rc = lib.lap_build_csr(n, len(s), s.ctypes.data, d.ctypes.data, flags, None, ctypes.byref(h))
    return rc, lib.lap_last_error().decode()


def test_host_side_rejections():
    from paper_2311_10290_amd import _capi as C
    assert _build(4, [0, 2], [1, 3])[0] == C.LAP_ENOTCONN                 # two components, no LCC flag
    assert _build(3, [0, 1], [1, 5])[0] == C.LAP_EINVAL                   # id out of range
    assert _build(0, [], [])[0] == C.LAP_EINVAL                           # empty node set
    assert _build(3, [0, 1], [1, 2], flags=64)[0] == C.LAP_EINVAL         # unknown flag
    rc, msg = _build(4, [0, 2], [1, 3])
    assert "connected components" in msg


def test_degree_limit_rejected_before_device_work():
    """A star whose centre has 2^24 neighbours: the degree field of the
    adjacency record holds 24 bits, so the build stops with LAP_ERANGE."""
    from paper_2311_10290_amd import _capi as C
    d = 1 << 24
    rc, msg = _build(d + 1, np.zeros(d, np.int32), np.arange(1, d + 1, dtype=np.int32))
    assert rc == C.LAP_ERANGE and "2^24" in msg


def test_null_handle_rejections():
    from paper_2311_10290_amd import _capi as C, load_library
    lib = load_library()
    assert lib.lap_graph_info(None, None, None, None, None) == C.LAP_EINVAL
    a = C.SampleArgs(n_samples=1)
    c = C.Counts()
    assert lib.lap_sample_forests(None, ctypes.byref(a), ctypes.byref(c), None) == C.LAP_EINVAL
    assert lib.lap_prof_read(b"no_such_kernel", None, None) == C.LAP_EINVAL
    lib.lap_graph_free(None)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2311_10290_amd.api as api
    from paper_2311_10290_amd import _capi
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "liblap.so"))
    monkeypatch.setattr(api, "_lib", None)
    with pytest.raises(ImportError):
        api.load_library()


STRUCTS = {"SampleArgs": "lap_sample_args", "Counts": "lap_counts", "Estimates": "lap_estimates",
           "BatchJob": "lap_batch_job", "BatchTuning": "lap_batch_tuning", "BatchOut": "lap_batch_out",
           "Query": "lap_query", "QueryResult": "lap_query_result", "ServerConfig": "lap_server_config"}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror has the C struct's size and field offsets (the
    header compiled by the host C compiler)."""
    import subprocess
    from paper_2311_10290_amd import _capi
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lap.h"', 'int main(void) {']
    for py, c in STRUCTS.items():
        lines.append(f'printf("{py} size %zu\\n", sizeof({c}));')
        for f, _ in getattr(_capi, py)._fields_:
            lines.append(f'printf("{py} {f} %zu\\n", offsetof({c}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for py in STRUCTS:
        cls = getattr(_capi, py)
        assert got[(py, "size")] == ctypes.sizeof(cls), py
        for f, _ in cls._fields_:
            assert got[(py, f)] == getattr(cls, f).offset, (py, f)
