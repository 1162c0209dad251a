"""The C-ABI library loads and exports every entry point of include/probetrace.h, and its
host-side argument checks fail cleanly before anything touches a GPU (no compute here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "probetrace.h")
LIB = os.path.join(ROOT, "paper_2507_14624_amd", "libprobetrace.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:pt_status|void|const char \*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("probe_grid_create", "probe_grid_destroy", "probe_trace", "probe_trace_rays",
                     "probe_trace_backward", "probe_autotune", "pt_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    import paper_2507_14624_amd as pt
    assert set(pt.EXPORTED) == set(_declared())


def test_host_side_argument_errors():
    import paper_2507_14624_amd as pt
    lib = pt.load_library()
    assert lib.probe_grid_create(None, None, None, None, None) == 1
    assert b"NULL" in lib.pt_last_error()
    d = pt.PtGridDesc()
    d.dims[:] = [0, 2, 2]  # no probes along x
    d.spacing[:] = [1, 1, 1]
    d.map_res = 64
    d.mip_levels = 4
    d.scene_max[:] = [1, 1, 1]
    out = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert lib.probe_grid_create(ctypes.byref(d), dummy, dummy, None, ctypes.byref(out)) == 1
    assert b"dims" in lib.pt_last_error() and not out.value
    d.dims[:] = [4, 2, 1]  # 8 probes must form a grid with 2 or more per axis
    assert lib.probe_grid_create(ctypes.byref(d), dummy, dummy, None, ctypes.byref(out)) == 1
    assert b"per axis" in lib.pt_last_error() and not out.value
    d.dims[:] = [2, 2, 2]
    d.map_res = 48  # not a power of two
    assert lib.probe_grid_create(ctypes.byref(d), dummy, dummy, None, ctypes.byref(out)) == 1
    assert b"map_res" in lib.pt_last_error()
    d.map_res = 64
    d.mip_levels = 7  # 64 >> 6 = 1 < 2
    assert lib.probe_grid_create(ctypes.byref(d), dummy, dummy, None, ctypes.byref(out)) == 1
    assert b"mip_levels" in lib.pt_last_error()
    assert lib.probe_trace(None, None, None, 0, None, None, None, None, None, None) == 1
    assert lib.probe_trace_backward(None, None, 0, None, None, None, None) == 1
    assert lib.probe_trace_rays(None, None, None, None, 0, None, None, None, None, None, None) == 1
    assert lib.probe_trace_noalloc(None, None, None, 0, None, None, None, None, None, None) == 1
    assert b"NULL" in lib.pt_last_error()
    o = pt.PtTraceOpts()
    lib.pt_trace_opts_default(ctypes.byref(o))
    assert o.max_probes_per_cell == 8 and o.tile_w * o.tile_h == 64 and o.start_level == -1
    # the optimizer step checks its arguments before any launch
    assert lib.pt_adam_step(None, None, None, None, None, 8, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0, None) == 1
    assert b"NULL" in lib.pt_last_error()
    for n, step, lr, b1, b2, eps in ((-1, 1, 1e-3, 0.9, 0.999, 1e-8), (8, 0, 1e-3, 0.9, 0.999, 1e-8),
                                     (8, 1, -1.0, 0.9, 0.999, 1e-8), (8, 1, 1e-3, 1.0, 0.999, 1e-8),
                                     (8, 1, 1e-3, 0.9, 1.5, 1e-8), (8, 1, 1e-3, 0.9, 0.999, float("inf"))):
        assert lib.pt_adam_step(dummy, dummy, dummy, dummy, None, n, step, lr, b1, b2, eps, 0.0, None) == 1
    lib.probe_grid_destroy(None)  # ignored


def test_binding_flags_match_the_header():
    # every PT_FLAG_* of the header has the same value in the Python binding, and no two
    # flags share a bit
    import paper_2507_14624_amd as pt
    flags = dict((k, int(v)) for k, v in re.findall(r"#define (PT_FLAG_\w+) (\d+)u", open(HEADER).read()))
    assert len(flags) >= 9
    for k, v in flags.items():
        assert getattr(pt, k) == v, k
        assert v & (v - 1) == 0, k
    assert len(set(flags.values())) == len(flags)
