"""CPU-side checks of the C ABI: the library builds, loads and exports every
entry point that include/lds.h declares (no device calls here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lds.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(lds_[a-z0-9_]+)\s*\(", src))
    # typedef'd function pointer types are not symbols
    names -= set(re.findall(r"\(\*(lds_[a-z0-9_]+)\)", src))
    return sorted(names)


def test_header_declares_core_calls():
    names = declared_functions()
    for core in ("lds_create_graph", "lds_frank_wolfe", "lds_destroy_graph", "lds_last_error"):
        assert core in names


def test_library_exports_every_declared_symbol():
    import paper_2504_10937_amd as lds
    lib = lds.load()
    out = subprocess.run(["nm", "-D", "--defined-only", lds.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lds_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_pure_host_calls():
    import paper_2504_10937_amd as lds
    assert lds.lds_denominator(lds.LDS_EDGE, 0) == 2
    assert lds.lds_denominator(lds.LDS_EDGE, 100) == 101 * 102
    assert lds.lds_denominator(lds.LDS_TRIANGLE, 200) == 3 * 201 * 202
    assert lds.load().lds_last_error() == b""


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2504_10937_amd as lds
    monkeypatch.setattr(lds, "_lib", None)
    monkeypatch.setattr(lds, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        lds.load()


def test_topk_host_side_errors():
    import ctypes
    import paper_2504_10937_amd as lds
    L = lds.load()
    r = lds._Result()
    assert L.lds_topk(None, lds.LDS_EDGE, 3, 10, ctypes.byref(r), None) == 1
    assert r.count == 0 and not r.offsets
    L.lds_result_free(ctypes.byref(r))
    L.lds_result_free(None)
