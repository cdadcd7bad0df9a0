"""Frequency grids and reference-point sets handed to the library as inputs.

* The imaginary-axis quadrature for the integral term of the contour
  deformation (Sec. 4, a modified Gauss-Legendre grid): Gauss-Legendre nodes
  x in (-1, 1) mapped to (0, inf) by omega = omega0 (1 + x) / (1 - x), with
  weights w' = 2 omega0 w / (1 - x)^2.  The paper does not print the mapping;
  this is the usual rational map and the grid is an input of every call.
* The Pade reference set F_wac (Sec. 3.3): the imaginary nodes that are
  re-used, plus points just above the real axis.  ``generic_refs`` spreads the
  near-real points evenly over every residue |eps_m - omega| that can occur up
  to the Fermi level (the generic core setting); ``refined_refs`` places
  N_core points around a core residue and N_valence points around the
  residue at the Fermi level (the refined setting, CD-WAC(N_core, N_valence,
  N_Im)).
"""
from __future__ import annotations

import numpy as np

from .synth import HARTREE_EV


def gauss_legendre_imag(n: int, omega0: float = 1.0):
    """Imaginary-axis nodes omega_k > 0 (ascending) and weights for int_0^inf."""
    x, w = np.polynomial.legendre.leggauss(n)
    omega = omega0 * (1.0 + x) / (1.0 - x)
    weight = 2.0 * omega0 * w / (1.0 - x) ** 2
    return omega.astype(np.float64), weight.astype(np.float64)


def midgap(eps: np.ndarray, n_occ: int) -> float:
    """Fermi level of a closed-shell molecule: midway between HOMO and LUMO."""
    return 0.5 * (float(eps[n_occ - 1]) + float(eps[n_occ]))


def windows(eps: np.ndarray, state_idx, window_ev):
    """QP search windows [lo, hi] per state (Hartree).

    ``window_ev`` is either a fixed (lo, hi) pair in eV or a half-width in eV
    around each state's own energy.
    """
    e = np.asarray(eps)[np.asarray(state_idx)]
    if isinstance(window_ev, (tuple, list)):
        lo = np.full(e.shape, window_ev[0] / HARTREE_EV)
        hi = np.full(e.shape, window_ev[1] / HARTREE_EV)
    else:
        lo = e - float(window_ev) / HARTREE_EV
        hi = e + float(window_ev) / HARTREE_EV
    return lo.astype(np.float64), hi.astype(np.float64)


def imag_ref_indices(n_freq: int, n_im: int) -> np.ndarray:
    """Evenly strided indices into the imaginary grid (both ends included)."""
    if n_im <= 0:
        return np.zeros(0, dtype=np.int32)
    if n_im == 1:
        return np.array([0], dtype=np.int32)
    idx = np.rint(np.arange(n_im) * (n_freq - 1) / (n_im - 1)).astype(np.int32)
    if len(np.unique(idx)) != n_im:
        raise ValueError("more imaginary reference points than grid nodes")
    return idx


def generic_refs(eps: np.ndarray, n_occ: int, win_lo, n_re: int):
    """Real parts of the generic near-real reference points.

    n_re points evenly spaced on [0, x_max], x_max = eps_F - min(win_lo): the
    largest residue |eps_m - omega| of an occupied state m above a QP
    candidate omega in any window.
    """
    if n_re <= 0:
        return np.zeros(0, dtype=np.float64)
    x_max = midgap(eps, n_occ) - float(np.min(win_lo))
    if n_re == 1:
        return np.array([x_max], dtype=np.float64)
    return (np.arange(n_re) * x_max / (n_re - 1)).astype(np.float64)


def refined_refs(eps: np.ndarray, n_occ: int, state_idx, win_lo, win_hi, n_core: int,
                 n_val: int, delta_c: float = 10.0 / HARTREE_EV, delta_v: float = 30.0 / HARTREE_EV):
    """Real parts of the refined reference points, omega_C then omega_V (Sec. 3.3).

    The paper centres one neighbourhood on a typical core residue
    |eps_c - omega| and one on the residue at the Fermi level |eps_F - omega|,
    with radii delta_c and delta_v, but prints neither the centres' omega nor
    the radii.  Reading: omega is the mean centre of the QP windows and eps_c
    the mean energy of the computed core states, so the core neighbourhood
    holds the residues of the core band itself (near 0) and the valence one
    the residues of the valence band seen from the core window.  Each region
    gets its points evenly over [max(0, centre - delta), centre + delta]
    (one point sits at the centre).  Defaults: delta_c = 10 eV,
    delta_v = 30 eV.
    """
    lo = np.asarray(win_lo, np.float64)
    hi = np.asarray(win_hi, np.float64)
    omega = 0.5 * (float(np.mean(lo)) + float(np.mean(hi)))
    ec = float(np.mean(np.asarray(eps)[np.asarray(state_idx)]))
    ef = midgap(eps, n_occ)
    out = []
    for centre, n, d in ((abs(ec - omega), n_core, delta_c), (abs(ef - omega), n_val, delta_v)):
        if n < 0 or not d > 0:
            raise ValueError("need n >= 0 and delta > 0")
        if n == 0:
            continue
        if n == 1:
            out.append(np.array([centre]))
        else:
            out.append(np.linspace(max(0.0, centre - d), centre + d, n))
    if not out:
        return np.zeros(0, dtype=np.float64)
    return np.concatenate(out).astype(np.float64)


def cdwac_setting(eps: np.ndarray, n_occ: int, state_idx, win_lo, win_hi, n_core: int,
                  n_val: int, n_im: int, n_freq: int, **deltas):
    """Reference set of CD-WAC(N_core, N_valence, N_Im) (Sec. 3.3): N_Im evenly
    strided imaginary nodes (all of them when N_Im = n_freq) and the refined
    near-real points.  M = N_core + N_valence + N_Im."""
    return (imag_ref_indices(n_freq, n_im),
            refined_refs(eps, n_occ, state_idx, win_lo, win_hi, n_core, n_val, **deltas))
