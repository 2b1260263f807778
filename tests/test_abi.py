"""The C ABI library loads and exports every symbol include/disco.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "disco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(disco_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_path():
    names = _declared()
    for must in ("disco_create", "disco_gauge_set", "disco_clover_setup", "disco_dirac_apply",
                 "disco_dirac_block_apply", "disco_solve_multi_rhs"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2609_37049_amd as d
    h = d.lib()
    missing = [n for n in _declared() if not hasattr(h, n)]
    assert not missing, missing
    # the binding knows every declared entry point
    assert set(_declared()) <= set(d.exported_symbols())


def test_errors_without_gpu_work():
    import paper_2609_37049_amd as d
    h = d.lib()
    assert h.disco_destroy(None) == 0
    assert h.disco_set_stream(None, None) == d.EINVAL
    assert h.disco_last_error(None) == b"null context"


def test_every_entry_point_rejects_null_handles():
    """Every entry point, called with a null context or handle and null
    pointers, returns a negative error code (the destroy functions accept NULL
    and return DISCO_OK), without touching a device or aborting."""
    import ctypes
    import paper_2609_37049_amd.binding as B
    h = B.lib()
    ints = (ctypes.c_int, ctypes.c_uint, ctypes.c_long, ctypes.c_longlong, ctypes.c_ulonglong)
    checked = 0
    for name, (args, _res) in B._SIGS.items():
        if name == "disco_last_error":
            continue
        vals = [0.0 if a is ctypes.c_double else (0 if a in ints else None) for a in args]
        r = getattr(h, name)(*vals)
        if name.endswith("_destroy"):
            assert r == 0, name
        else:
            assert r < 0, name
        checked += 1
    assert checked >= 40


def test_create_failure_keeps_its_message():
    """A failed disco_create leaves no context, so its message is kept for
    disco_last_error(NULL) on the same thread."""
    import ctypes
    import paper_2609_37049_amd as d
    h = d.lib()
    out = ctypes.c_void_p()
    bc = (ctypes.c_int * 4)(1, 1, 1, -1)
    assert h.disco_create((ctypes.c_int * 4)(4, 0, 4, 4), bc, 0, ctypes.byref(out)) == d.EINVAL
    assert out.value is None
    assert b"dims[1]" in h.disco_last_error(None)
    assert h.disco_create((ctypes.c_int * 4)(4, 4, 4, 4), (ctypes.c_int * 4)(1, 2, 1, -1), 0,
                          ctypes.byref(out)) == d.EINVAL
    assert b"bc[1]" in h.disco_last_error(None)
