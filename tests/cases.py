"""Seeded test cases shared by the parity tests (inputs only)."""
import dataclasses

import numpy as np

from paper_2305_15955_amd import grids, synth


@dataclasses.dataclass
class Case:
    name: str
    system: object
    freq: np.ndarray
    weight: np.ndarray
    ref_im: np.ndarray
    ref_re: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    eta: float = 1e-3
    eta_ref: float = 1e-3
    pade_tol: float = 1e-9


def build(system, n_freq, n_im, n_re, window_ev, name="case", pade_tol=1e-9):
    freq, wts = grids.gauss_legendre_imag(n_freq)
    lo, hi = grids.windows(system.eps, system.state_idx, window_ev)
    ref_im = grids.imag_ref_indices(n_freq, n_im)
    ref_re = grids.generic_refs(system.eps, system.n_occ, lo, n_re)
    return Case(name, system, freq, wts, ref_im, ref_re, lo, hi, pade_tol=pade_tol)


def ragged(seed=21, n_pade=24):
    """Several matrix-core tiles and a ragged tail in every padded dimension.

    48 imaginary nodes; n_pade/2 imaginary and n_pade/2 near-real Pade points.
    With 12 points this system's CD-WAC result is ~60 meV from full CD, with
    32 within 0.14 meV.  FP64 parity at 1e-9 uses 24: with 32 the Thiele
    interpolant amplifies last-digit differences of W to ~5e-7 in Sigma, so
    the two sides agree only to the conditioning of the fit, not to rounding.
    """
    s = synth.make_system(90, 15, 300, 3, 0.04, kappa=0.2, seed=seed)
    return build(s, 48, n_pade // 2, n_pade - n_pade // 2, 30.0, name=f"ragged_naux300_m{n_pade}")


def workload(name):
    spec = synth.WORKLOADS[name]
    s = synth.make_workload(name)
    nim = spec["n_pade"] // 2
    return build(s, spec["n_freq"], nim, spec["n_pade"] - nim, spec["window_ev"], name=name)


def one_transition():
    eps = np.array([-10.0, 20.0 / synth.HARTREE_EV - 10.0])
    s = synth.System(eps=eps, n_occ=1, o_ia=np.array([[0.3]]), o_nm=np.array([[[0.4, 0.3]]]),
                     state_idx=np.array([0], np.int32))
    return build(s, 32, 4, 4, 30.0, name="one_transition")


def oracle(case, **kw):
    from oracle import cdwac_ref as R
    return R.CdwacOracle(case.system, case.freq, case.weight, case.ref_im, case.ref_re, case.lo,
                         case.hi, eta=case.eta, eta_ref=case.eta_ref, pade_tol=case.pade_tol, **kw)
