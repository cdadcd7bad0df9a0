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


def refined_refs(eps: np.ndarray, n_occ: int, omega_core: float, n_core: int,
                 n_val: int, delta_c: float, delta_v: float, core_eps=None):
    """Real parts of the refined reference points (omega_C and omega_V).

    ``omega_core`` is a typical QP energy of the core state; the core region is
    centred on a typical core residue |eps_c - omega| (``core_eps`` defaults
    to the lowest orbital), the valence region on |eps_F - omega|.  Points are
    spaced evenly over [centre - delta, centre + delta], clipped at 0.
    """
    ef = midgap(eps, n_occ)
    ec = float(eps[0]) if core_eps is None else float(core_eps)
    out = []
    for centre, n, d in ((abs(ec - omega_core), n_core, delta_c),
                         (abs(ef - omega_core), n_val, delta_v)):
        if n <= 0:
            continue
        if n == 1:
            pts = np.array([centre])
        else:
            pts = np.linspace(centre - d, centre + d, n)
        out.append(np.clip(pts, 0.0, None))
    if not out:
        return np.zeros(0, dtype=np.float64)
    return np.concatenate(out).astype(np.float64)
