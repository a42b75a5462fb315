"""The C-ABI library loads on the CPU and exports every entry point declared
in include/hlbm.h; the pure host helpers validate their arguments."""
import ctypes as C
import os
import re

import pytest

from paper_2510_13726_amd import hlbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hlbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hlbm.lib()
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert sorted(n for n, _, _ in hlbm.SIGNATURES) == names


def test_struct_sizes_match_header_layout():
    # hlbm_desc: 8 int32 + 2 int64 + pointer; hlbm_params / hlbm_rotor as declared
    assert C.sizeof(hlbm.Desc) == 8 * 4 + 2 * 8 + 8
    assert C.sizeof(hlbm.Params) == 3 * 8 + 2 * 4 + 4 * 8 + 2 * 4 + 3 * 8 + 8 + 8 + 2 * 4 + 8
    assert C.sizeof(hlbm.Rotor) == 14 * 8 + 2 * 4 + 2 * 8


def test_host_size_helpers():
    L = hlbm.lib()
    d = hlbm.make_desc(256, 128, 128, hlbm.F32)
    pb = L.hlbm_population_bytes(C.byref(d))
    N = 256 * 128 * 128
    assert pb == 27 * N * 4  # blocks of 64 x cells: no padding when 64 divides nx
    d16 = hlbm.make_desc(256, 128, 128, hlbm.F16)
    assert L.hlbm_population_bytes(C.byref(d16)) == pb // 2
    # a ragged row is padded to whole blocks of 64 cells
    dr = hlbm.make_desc(100, 3, 2, hlbm.F64)
    assert L.hlbm_population_bytes(C.byref(dr)) == 27 * 128 * 3 * 2 * 8
    assert L.hlbm_workspace_bytes(C.byref(d)) > 0
    bad = hlbm.make_desc(1, 4, 4, hlbm.F32)
    assert L.hlbm_population_bytes(C.byref(bad)) == -1
    mixed = hlbm.make_desc(8, 8, 8, hlbm.F16, compute=hlbm.F64)
    assert L.hlbm_workspace_bytes(C.byref(mixed)) == -1


def test_rotor_bbox_cells():
    from paper_2510_13726_amd import workloads as W
    L = hlbm.lib()
    w = W.config2()
    d = hlbm.make_desc(w.nx, w.ny, w.nz, hlbm.F32, bc_x=w.bc_x)
    arr = hlbm._rotor_array(w.rotors)
    n = L.hlbm_rotor_bbox_cells(C.byref(d), arr, 1)
    # bounding box of a cylinder of radius ~40 and half-length ~4, plus the
    # widest band the workspace allows for (3 cells)
    assert 85 ** 2 * 10 < n < 95 ** 2 * 18
    w.rotors[0].center = (51.0, 10.0, 64.0)  # sticks out of the domain
    assert L.hlbm_rotor_bbox_cells(C.byref(d), hlbm._rotor_array(w.rotors), 1) == -1


def test_create_rejects_null_buffers():
    L = hlbm.lib()
    d = hlbm.make_desc(8, 8, 8, hlbm.F32)
    h = C.c_void_p()
    rc = L.hlbm_lattice_create(C.byref(d), None, None, None, C.byref(h))
    assert rc == hlbm.HLBM_ERR_INVALID and not h.value
    assert b"NULL" in L.hlbm_last_error(None)


def test_size_limits_of_the_descriptor():
    # tile and cell indices are 32-bit: the last accepted lattice has
    # 2^31 - 2^21 cells, one more z plane reaches 2^31 and is refused
    L = hlbm.lib()
    top = hlbm.make_desc(2048, 1024, 1023, hlbm.F16)
    assert L.hlbm_population_bytes(C.byref(top)) == 27 * 2048 * 1024 * 1023 * 2
    assert L.hlbm_workspace_bytes(C.byref(top)) > 0
    over = hlbm.make_desc(2048, 1024, 1024, hlbm.F16)
    assert L.hlbm_population_bytes(C.byref(over)) == -1
    assert L.hlbm_workspace_bytes(C.byref(over)) == -1
    # D3Q19 rows hold 19 runs per block of 64 cells; other velocity sets are refused
    q19 = hlbm.make_desc(100, 3, 2, hlbm.F32)
    q19.velocities = 19
    assert L.hlbm_population_bytes(C.byref(q19)) == 19 * 128 * 3 * 2 * 4
    q15 = hlbm.make_desc(100, 3, 2, hlbm.F32)
    q15.velocities = 15
    assert L.hlbm_population_bytes(C.byref(q15)) == -1
