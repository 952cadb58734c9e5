"""The C-ABI library loads on the CPU and exports every symbol that
include/cloversap.h declares; host-side argument checks work without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cloversap.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2112_00501_amd import cloversap
    return cloversap.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["cs_lattice_create", "cs_gauge_create", "cs_clover_create", "cs_apply_D",
                     "cs_apply_Ddag", "cs_sap_smooth", "cs_gcr_solve"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2112_00501_amd import cloversap
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(cloversap.EXPORTED) == declared_functions()


def test_geometry_validation_on_host(lib):
    h = C.c_void_p()
    I4 = C.c_int * 4
    assert lib.cs_lattice_create(I4(8, 8, 8, 6), I4(4, 4, 4, 4), 0, C.byref(h)) == -2
    assert b"multiple of 4" in lib.cs_last_error()
    assert lib.cs_lattice_create(I4(8, 8, 8, 8), I4(2, 4, 4, 4), 0, C.byref(h)) == -2
    assert lib.cs_lattice_create(None, I4(4, 4, 4, 4), 0, C.byref(h)) == -3
    assert lib.cs_lattice_create(I4(8, 4, 12, 16), I4(4, 4, 4, 4), 2, C.byref(h)) == -1
    assert b"flags" in lib.cs_last_error()
    assert lib.cs_lattice_create(I4(8, 4, 12, 16), I4(4, 4, 4, 4), 1, C.byref(h)) == 0
    assert lib.cs_lattice_destroy(h) == 0
    assert lib.cs_lattice_create(I4(8, 4, 12, 16), I4(4, 4, 4, 4), 0, C.byref(h)) == 0
    assert lib.cs_lattice_volume(h) == 8 * 4 * 12 * 16
    assert lib.cs_field_bytes(h, 0, 1) == 192 * 6144
    assert lib.cs_field_bytes(h, 1, 3) == 96 * 6144 * 3
    assert lib.cs_field_bytes(h, 2, 1) == 52 * 6144
    assert lib.cs_field_bytes(h, 9, 1) == 0
    assert lib.cs_lattice_destroy(h) == 0


def test_null_handles_rejected_on_host(lib):
    assert lib.cs_apply_D(None, None, 0, None, None, 1, None) == -3
    assert lib.cs_sap_smooth(None, None, 0, None, None, 2, 4, 1, 1, None) == -3
    assert lib.cs_gcr_solve(None, None, None, None, None, 1, None, None) == -3
    assert lib.cs_strerror(1) == b"not converged within max_iter"


def test_binding_refuses_undersized_buffers():
    """The C ABI takes raw device pointers and cannot see buffer sizes; the
    binding checks every field and coarse-vector buffer against the size the
    kernels will touch before any launch (no GPU needed to see the refusal)."""
    import torch

    from paper_2112_00501_amd import cloversap as cs
    lat = cs.Lattice((8, 8, 8, 8))
    one = torch.empty(lat.field_bytes(cs.F32, 1), dtype=torch.uint8)
    with pytest.raises(ValueError):
        lat.export_field(one, cs.F32, 8)
    with pytest.raises(ValueError):
        lat.import_field(torch.zeros((2, lat.volume, 4, 3), dtype=torch.complex128), cs.F32, out=one)
