"""CPU-side checks of the C ABI: the library loads and exports every symbol the
public header declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"\b(gwn_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ("gwn_build_mesh", "gwn_query_batch", "gwn_query_grid", "gwn_mesh_destroy", "gwn_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2605_01536_amd import gwn
    if not os.path.exists(gwn.LIB_PATH):
        pytest.fail("libgwn.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(gwn.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_status_strings_and_null_handle_errors():
    from paper_2605_01536_amd import gwn
    L = gwn.load()
    assert L.gwn_status_str(0) == b"ok"
    assert L.gwn_status_str(1) == b"invalid argument"
    # host-side validation runs before any device work
    assert L.gwn_mesh_info_get(None, None) == 1
    assert b"null" in L.gwn_last_error()
    assert L.gwn_mesh_destroy(None) == 0
    assert L.gwn_query_batch(None, None, None, None, 1, 10, 0, None, None, None) == 1
    out = ctypes.c_void_p(1)
    assert L.gwn_build_mesh(None, None, None, 1, -1, None, 0, None, ctypes.byref(out)) == 1
    assert out.value is None
    # build options are checked before any device work
    from paper_2605_01536_amd.gwn import BuildOpts
    opts = BuildOpts(0, 7)
    out = ctypes.c_void_p(1)
    assert L.gwn_build_mesh_opts(None, None, None, 1, 0, None, 0, ctypes.byref(opts), None, ctypes.byref(out)) == 1
    assert b"axis" in L.gwn_last_error()


def test_surrogate_checkpoint_validation_on_the_host(tmp_path):
    # gwn_surrogate_load checks the file before it touches the device
    from paper_2605_01536_amd import gwn
    L = gwn.load()
    gwn._load_mlp(L)
    h = ctypes.c_void_p(1)
    assert L.gwn_surrogate_load(str(tmp_path / "missing").encode(), ctypes.byref(h)) == 1
    assert h.value is None and b"cannot open" in L.gwn_last_error()
    p = tmp_path / "junk.gwns"
    p.write_bytes(b"GWNSURR1" + bytes(300))
    assert L.gwn_surrogate_load(str(p).encode(), ctypes.byref(h)) == 1
    assert b"not a version-2" in L.gwn_last_error()
    assert L.gwn_surrogate_save(None, str(p).encode()) == 1
    assert L.gwn_surrogate_train(None, None, None, None, None, 0, None, None, None) == 1
    assert L.gwn_surrogate_destroy(None) == 0
