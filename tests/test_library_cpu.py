"""The C-ABI library loads and exports every declared entry point (no GPU)."""
import ctypes
import os

import pytest

from paper_2305_15955_amd import cdwac


def test_header_declares_the_boundary():
    names = cdwac.header_functions()
    for n in ("cdwac_ctx_create", "cdwac_prepare", "cdwac_qp", "cdwac_solve", "cdwac_solve_batch", "cdwac_sigma",
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
    assert ctypes.sizeof(cdwac.CdwacStateOut) == 5 * 8 + 3 * 4 + 4      # tail padding to 8 bytes


def test_params_layout_matches_header():
    # n_freq(+pad), freq, weight, n_ref_im(+pad), ref_im_idx, n_ref_re(+pad), ref_re, eta_ref, eta,
    # pade_tol, win_lo, win_hi, qp_tol, qp_maxit, prec, use_mlp_seed(+pad), mlp_accept, freq_rank_tol,
    # fit_all, near_real_f64, quad_limit (+pad)
    assert ctypes.sizeof(cdwac.CdwacParams) == 8 + 16 + 8 + 8 + 8 + 8 + 3 * 8 + 2 * 8 + 8 + 3 * 4 + 4 + 2 * 8 + 16
    assert cdwac.CdwacParams.fit_all.offset == ctypes.sizeof(cdwac.CdwacParams) - 16
    assert cdwac.CdwacParams.near_real_f64.offset == ctypes.sizeof(cdwac.CdwacParams) - 12
    assert cdwac.CdwacParams.quad_limit.offset == ctypes.sizeof(cdwac.CdwacParams) - 8


def test_freq_decomposition_interpolates_w_family():
    """Host logic of the imaginary-node skeleton: every 1/(w_f^2 + O^2) is
    reproduced by the skeleton nodes to the requested tolerance (relative to its
    maximum) at excitation energies off the decomposition's grid, and so is a
    pole sum W(i w) = -sum_s p_s / (w^2 + O_s^2) with arbitrary p_s >= 0."""
    import numpy as np
    from paper_2305_15955_amd import grids
    w, _ = grids.gauss_legendre_imag(64)
    lo, hi = 0.2, 50.0
    rng = np.random.default_rng(0)
    om = np.sort(np.exp(rng.uniform(np.log(lo), np.log(hi), 20000)))
    h = lambda f: 1.0 / (w[f] ** 2 + om ** 2)
    sizes = []
    for tol in (1e-6, 1e-10, 1e-13):
        skel, rest, T = cdwac.freq_decomposition(w, lo, hi, tol)
        assert len(set(skel) | set(rest)) == 64 and not set(skel) & set(rest)
        assert 63 in skel and np.all(np.diff(skel) > 0)
        sizes.append(len(skel))
        for r, f in enumerate(rest):
            approx = sum(T[r, j] * h(s) for j, s in enumerate(skel))
            assert np.max(np.abs(approx - h(f))) <= 3 * tol * np.max(h(f)), (tol, f)
        # a pole sum with positive weights, as W^c_nm(i w) on the imaginary axis
        poles = np.exp(rng.uniform(np.log(lo), np.log(hi), 40))
        p = rng.uniform(0.0, 1.0, 40)
        W = lambda f: -np.sum(p / (w[f] ** 2 + poles ** 2))
        for r, f in enumerate(rest):
            approx = sum(T[r, j] * W(s) for j, s in enumerate(skel))
            assert abs(approx - W(f)) <= 3 * tol * np.sum(p) / (w[f] ** 2 + lo ** 2)
    assert sizes[0] < sizes[1] < sizes[2] < 64
    # a tolerance below what FP64 can certify keeps every node
    skel, rest, T = cdwac.freq_decomposition(w, lo, hi, 1e-17)
    assert len(skel) == 64 and len(rest) == 0


def test_skeleton_tolerance_table_covers_every_mode():
    """cdwac.SKELETON_TOL has an entry for every precision mode: 0 (every node)
    for the FP64 path, and a tolerance no looser for the split modes than for
    the one-product modes (the splits leave less W error to hide it under)."""
    from paper_2305_15955_amd import cdwac
    assert set(cdwac.SKELETON_TOL) == set(cdwac.PREC)
    assert cdwac.SKELETON_TOL["p64"] == 0.0
    for k, v in cdwac.SKELETON_TOL.items():
        assert 0.0 <= v < 1.0, k
    assert cdwac.SKELETON_TOL["f16x3"] <= cdwac.SKELETON_TOL["f16"]
    assert cdwac.SKELETON_TOL["b16x3"] <= cdwac.SKELETON_TOL["b16"]
