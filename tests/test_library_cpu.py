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


def test_params_layout_matches_header():
    # n_freq(+pad), freq, weight, n_ref_im(+pad), ref_im_idx, n_ref_re(+pad), ref_re, eta_ref, eta,
    # pade_tol, win_lo, win_hi, qp_tol, qp_maxit, prec, use_mlp_seed(+pad), mlp_accept, freq_rank_tol
    assert ctypes.sizeof(cdwac.CdwacParams) == 8 + 16 + 8 + 8 + 8 + 8 + 3 * 8 + 2 * 8 + 8 + 3 * 4 + 4 + 2 * 8


def test_freq_decomposition_interpolates_the_weights():
    """Host logic of the imaginary-axis frequency decomposition: every
    weight function c_f(D) = -2sD/(w_f^2 + D^2) is reproduced by the skeleton
    nodes to the requested tolerance at transition energies off the grid."""
    import numpy as np
    from paper_2305_15955_amd import grids
    w, _ = grids.gauss_legendre_imag(64)
    dmin, dmax = 0.2, 13.0
    rng = np.random.default_rng(0)
    d = np.sort(np.exp(rng.uniform(np.log(dmin), np.log(dmax), 20000)))
    c = lambda f: -4.0 * d / (w[f] ** 2 + d ** 2)
    sizes = []
    for tol in (1e-6, 1e-10, 1e-13):
        skel, rest, T = cdwac.freq_decomposition(w, dmin, dmax, tol)
        assert len(set(skel) | set(rest)) == 64 and not set(skel) & set(rest)
        sizes.append(len(skel))
        for r, f in enumerate(rest):
            approx = sum(T[r, j] * c(s) for j, s in enumerate(skel))
            err = np.max(np.abs(approx - c(f))) / np.max(np.abs(c(f)))
            assert err <= 3 * tol, (tol, f, err)
    assert sizes[0] < sizes[1] < sizes[2] < 64
    # a tolerance below what FP64 can certify keeps every node
    skel, rest, T = cdwac.freq_decomposition(w, dmin, dmax, 1e-17)
    assert len(skel) == 64 and len(rest) == 0
