"""The C-ABI library loads without a GPU and exports every function that
include/lbm.h declares; the host-side binding mirrors the header's structs."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(lbm_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_core_entry_points():
    names = declared_functions()
    for core in ("lbm_create", "lbm_init_tgv", "lbm_set_rotor", "lbm_step",
                 "lbm_get_fields", "lbm_rotor_loads"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2402_13171_amd import lbm
    if not os.path.exists(lbm.SO_PATH):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(lbm.SO_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(lbm.EXPORTS) == declared_functions()


def test_struct_sizes_match_header_layout():
    from paper_2402_13171_amd import lbm
    # lbm_config: 3 ints, pad, 10 doubles, 2 ints, double, 3 ints, pad, 6 doubles, int, pad, pointer
    assert ctypes.sizeof(lbm.Config) == 3 * 4 + 4 + 10 * 8 + 2 * 4 + 8 + 3 * 4 + 4 + 6 * 8 + 4 + 4 + 8 + 8
    assert ctypes.sizeof(lbm.Rotor) == 6 * 8 + 5 * 8 + 2 * 4 + 4 * 8 + 8 + 3 * 8 + 2 * 4
    # lbm_node: 6 ints, 31 doubles (pos, rot, axis, 5 motion values, disp, dir, normal, coef, pitch), 4 pointers
    assert ctypes.sizeof(lbm.Node) == 6 * 4 + 31 * 8 + 4 * 8
    # lbm_turbine: int + pad, pointer, int + pad, double, int + pad, double, int + pad, 3 pointers
    assert ctypes.sizeof(lbm.Turbine) == 8 + 8 + 8 + 8 + 8 + 8 + 8 + 3 * 8


def test_error_strings_without_gpu():
    from paper_2402_13171_amd import lbm
    L = lbm.lib()
    assert L.lbm_strerror(-4).decode().startswith("simulation unstable")
    assert L.lbm_strerror(0).decode() == "ok"
    # argument validation happens before any device work
    cfg = lbm.Config()
    cfg.nx = cfg.ny = cfg.nz = 1
    cfg.omega = 1.9
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == lbm.EINVAL
    cfg.nx = cfg.ny = cfg.nz = 8
    cfg.omega = 2.5
    assert L.lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == lbm.EINVAL
    cfg.omega = 1.9
    cfg.bc_z_lo = 2  # one periodic and one wall side is not allowed
    assert L.lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == lbm.EINVAL


def test_copy_probe_validates_before_any_device_work():
    from paper_2402_13171_amd import lbm
    L = lbm.lib()
    vp = ctypes.c_void_p
    assert L.lbm_copy_probe(None, vp(256), 4096, None) == lbm.EINVAL
    assert L.lbm_copy_probe(vp(256), None, 4096, None) == lbm.EINVAL
    assert L.lbm_copy_probe(vp(256), vp(512), 4100, None) == lbm.EINVAL   # not a multiple of 16 bytes
    assert L.lbm_copy_probe(vp(264), vp(512), 4096, None) == lbm.EINVAL   # source not 16-byte aligned
    assert L.lbm_copy_probe(vp(256), vp(520), 4096, None) == lbm.EINVAL   # destination not 16-byte aligned
    assert L.lbm_copy_probe(vp(256), vp(512), 0, None) == lbm.OK          # nothing to copy: no launch
