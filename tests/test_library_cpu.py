"""The C-ABI library loads and exports every declared entry point (no GPU)."""
import ctypes
import os

import pytest

from paper_2305_15955_amd import cdwac


def test_header_declares_the_boundary():
    names = cdwac.header_functions()
    for n in ("cdwac_ctx_create", "cdwac_prepare", "cdwac_qp", "cdwac_solve", "cdwac_sigma",
              "cdwac_polarizability", "cdwac_pade_fit_eval", "cdwac_mlp_train"):
        assert n in names


def test_library_exports_every_header_symbol():
    if not os.path.exists(cdwac.LIB_PATH):
        pytest.fail("libcdwac.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(cdwac.LIB_PATH)
    for name in cdwac.header_functions():
        assert hasattr(lib, name), name
    # the binding declares a signature for every header function
    assert sorted(cdwac._SIGNATURES) == cdwac.header_functions()


def test_struct_layouts_match_header():
    # 4 int32, 1 pointer, 2 pointers, 2 pointers, 2 doubles
    assert ctypes.sizeof(cdwac.CdwacSystem) == 4 * 4 + 5 * 8 + 2 * 8
    assert ctypes.sizeof(cdwac.CdwacStateOut) == 5 * 8 + 2 * 4
