"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/tmhop.h declares, and rejects bad geometry before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmhop.h")
LIB = os.path.join(ROOT, "paper_1311_4521_amd", "libtmhop.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tmh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ("tmh_hop_apply", "tmh_qtm_apply", "tmh_cg_solve", "tmh_hop_force",
                 "tmh_lattice_create", "tmh_scalar_prod_r"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1311_4521_amd import tmhop
    assert sorted(tmhop.EXPORTED) == declared_symbols()


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 5), (0, 4, 4, 4), (4, 1, 4, 4),
                                  (4, 4, -2, 4), (2048, 2048, 2048, 2)])
def test_bad_geometry_rejected(dims):
    from paper_1311_4521_amd import tmhop
    st, h = tmhop.raw_lattice_create(dims)
    assert st == tmhop.TMH_ERR_GEOMETRY
    assert not h.value


def test_status_strings():
    from paper_1311_4521_amd import tmhop
    for st in range(-8, 1):
        assert tmhop.status_string(st) not in ("", "unknown status")
    assert tmhop.status_string(-99) == "unknown status"


def test_null_handle_rejected():
    from paper_1311_4521_amd import tmhop
    lib = tmhop._lib
    assert lib.tmh_hop_apply(None, 0, None, None, None, 0.1, None, 0) == tmhop.TMH_ERR_ARG
    assert lib.tmh_hop_force(None, 0, None, None, None, None, 0.1, None, 1.0, 0) == tmhop.TMH_ERR_ARG
    assert lib.tmh_qtm_force(None, None, None, None, None, 0.1, 0.1, None, 1, 1.0, 0) == tmhop.TMH_ERR_ARG
    assert lib.tmh_spinor_bytes(None, 0) == 0
