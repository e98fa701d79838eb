"""The C-ABI library loads and exports every entry point include/wdlb.h
declares (no compute calls: this runs without a GPU)."""
import os
import re

from paper_1304_7880_amd import wdlb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wdlb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wdlb_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_symbols():
    assert sorted(wdlb.SYMBOLS) == _declared()


def test_library_exports_every_symbol():
    if not os.path.exists(wdlb.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    L = wdlb.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_invalid_arguments_rejected_without_device():
    L = wdlb.load()
    import ctypes as C
    n = C.c_size_t(0)
    bad = wdlb.make_desc(0, 4, 4)
    p = wdlb.make_params()
    assert L.wdlb_workspace_size(C.byref(bad), C.byref(p), C.byref(n)) == wdlb.E_INVAL
    good = wdlb.make_desc(8, 8, 8)
    for kw in (dict(tau=0.5), dict(eta=1.0), dict(sigma=0.5), dict(eta=0.0)):
        p = wdlb.make_params(**kw)
        assert L.wdlb_workspace_size(C.byref(good), C.byref(p), C.byref(n)) == wdlb.E_INVAL, kw
    p = wdlb.make_params()
    assert L.wdlb_workspace_size(C.byref(good), C.byref(p), C.byref(n)) == wdlb.OK
    assert n.value > 8 * 8 * 8 * 19 * 4 * 2
    # null context
    assert L.wdlb_step(None, 1) == wdlb.E_INVAL
