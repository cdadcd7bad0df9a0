"""FP64 CPU oracle for the CD-WAC core-level self-energy (test infrastructure).

Follows Panades-Barrueta & Golze, "Accelerating core-level GW calculations by
combining the contour deformation approach with the analytic continuation of
W" (JCTC 2023).  Units: Hartree.  Orbitals are real, so O^{mn}_P = O^{nm}_P.

Readings of passages the paper leaves open:

* spin: closed shell, the spin sum of the Adler-Wiser expression (Eq. aw)
  becomes a factor ``spin`` = 2 in Pi;
* Fermi level: midway between HOMO and LUMO;
* the broadening of Eq. (piriv) is carried by the complex argument z itself:
  Pi(z) = spin * sum_ia O^ia O^ia [1/(z - D_ia) - 1/(z + D_ia)], which at
  z = i omega is real and negative semidefinite;
* Lambda of Eq. (bigLambda) is evaluated as (I - Pi)^{-1} Pi, which equals
  (I - Pi)^{-1} - I exactly and avoids the cancellation at large omega;
* the integral term of Eq. (In_term) is taken in the limit eta -> 0 and folded
  over +-omega' (W^c(i omega') is real and even):  I_n(omega) =
  (1/pi) sum_m sum_k w_k W_nm(i omega_k) a_m / (a_m^2 + omega_k^2),
  a_m = omega - eps_m;  the a_m = 0 term vanishes (principal value);
* the Heaviside steps of Eq. (ffact) take theta(0) = 1/2;
* the Pade model of Eq. (pade) is built in u = z^2 by the recursion of
  Eqs. (pre_rec, rec_eq); the greedy order of Sec. 3.2 starts at the largest
  |W| and then adds the point where the current convergent has the largest
  L1 error |Re(W - T)| + |Im(W - T)| (lowest index on ties); it stops once
  that largest error is <= ``tol`` * max|W| or no point is left;
* the residue term evaluates the model at u = (|eps_m - omega| + i eta)^2 and
  keeps the real part;
* the QP equation (Eq. qp_eq) is solved by secant from omega_0 = eps_n and one
  fixed-point step; if an iterate leaves the window, the iteration does not
  converge or Z is outside (0, 1], the window is scanned, every upward sign
  change with |f| < 0.1 Ha on both sides is bisected to 1e-12 Ha, candidates
  with |f| > 1e-8 Ha at the final midpoint (a jump across a pole, not a zero)
  are dropped, and the root with the largest Z (then the one nearest eps_n)
  is kept;
* optionally (``quad_limit``) the integral term takes the a_m -> 0 limit
  analytically: W_nm(i w') = w0 g(w') + [W_nm(i w') - w0 g(w')] with
  g = Gamma^2 / (Gamma^2 + w'^2), w0 the residue term's own W at a_m = 0; the
  first part is integrated in closed form, the remainder by the quadrature.

Test infrastructure only: the tests, the package's smoke check and the
benchmark's CPU baseline use it; the GPU path never does.  Every function is
pinned by tests/test_oracle_pins.py or tests/test_oracle_mlp.py except one
result, whose parity is unpinned: the G_dH W0 root with the plain quadrature
(``solve_hedin`` without ``quad_limit``), which sits next to the state's own
shifted G pole where the quadrature steps (with the limit it is pinned
against the pole form).
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np

QP_SCAN_STEP = 0.01       # Ha, fallback scan spacing
QP_SCAN_FMAX = 0.1        # Ha, |f| bound on both sides of an accepted sign change
QP_BISECT_TOL = 1e-12     # Ha
QP_Z_STEP = 1e-4          # Ha, central difference for Z
QP_F_TOL = 1e-9           # Ha, |f| bound for secant convergence
QP_ROOT_FTOL = 1e-8       # Ha, |f| bound at a bisected fallback root
QUAD_GAMMA = 1.0          # Ha, width of the subtracted Lorentzian of the a_m -> 0 limit

FLAG_NOROOT = 1
FLAG_FALLBACK = 2
FLAG_MLP_ACCEPTED = 4


# ---------------------------------------------------------------------------
# Mean-field quantities
# ---------------------------------------------------------------------------

def fermi_level(eps: np.ndarray, n_occ: int) -> float:
    """Fermi level of a closed-shell molecule (Sec. 2.1, Eq. gnot): midgap."""
    return 0.5 * (float(eps[n_occ - 1]) + float(eps[n_occ]))


def transition_energies(eps: np.ndarray, n_occ: int) -> np.ndarray:
    """D_ia = eps_a - eps_i for every occupied i and virtual a, a fastest."""
    return (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)


def exchange(o_n: np.ndarray, n_occ: int) -> float:
    """Sigma^x_n = -sum_i^occ (ni|in) with the RI-V factorisation.

    Eq. (exs) projected on state n gives -sum_i (ni|in); Eq. (workriv) writes
    (ni|in) = sum_P O^{ni}_P O^{in}_P.  ``o_n`` is O^{nm}_P as [n_aux, n_mo].
    Pin: a four-index brute force over (nm|kl) on tiny inputs.
    """
    occ = o_n[:, :n_occ]
    return -float(np.sum(occ * occ))


# ---------------------------------------------------------------------------
# Screened interaction (Sec. 2.3, Eqs. wriv, bigLambda, piriv)
# ---------------------------------------------------------------------------

def polarizability(o_ia: np.ndarray, eps: np.ndarray, n_occ: int, z: complex,
                   spin: float = 2.0) -> np.ndarray:
    """Pi_PQ(z) of Eq. (piriv), the RI form of the Adler-Wiser sum (Eq. aw).

    Returns a real array when z is purely imaginary (Pi is then real), else a
    complex one.  Pins: brute-force double loop on tiny inputs, Pi(i w) <= 0,
    Pi(-z) = Pi(z), Pi(conj z) = conj Pi(z), single-transition closed form.
    """
    delta = transition_energies(eps, n_occ)
    z = complex(z)
    d = spin * (1.0 / (z - delta) - 1.0 / (z + delta))
    if z.real == 0.0:
        return (o_ia * d.real[None, :]) @ o_ia.T
    # o_ia is real: the real and imaginary parts of the sum are each a real
    # product (no complex copy of o_ia)
    return (o_ia * d.real[None, :]) @ o_ia.T + 1j * ((o_ia * d.imag[None, :]) @ o_ia.T)


def polarizability_entries(o_ia: np.ndarray, eps: np.ndarray, n_occ: int, z: complex,
                           spin: float, pairs) -> np.ndarray:
    """Selected elements Pi_PQ(z) of Eq. (piriv), one dot product each.

    For sampled checks at sizes where the full matrix is out of reach.  Pin:
    equals ``polarizability`` element by element on small inputs.
    """
    delta = transition_energies(eps, n_occ)
    z = complex(z)
    d = spin * (1.0 / (z - delta) - 1.0 / (z + delta))
    return np.array([np.dot(o_ia[p] * d, o_ia[q]) for p, q in pairs])


def lambda_matrix(pi: np.ndarray) -> np.ndarray:
    """Lambda = [I - Pi]^{-1} - I of Eq. (bigLambda), as (I - Pi)^{-1} Pi."""
    n = pi.shape[0]
    return np.linalg.solve(np.eye(n, dtype=pi.dtype) - pi, pi)


def w_elements(o_n: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """W^c_nm = sum_PQ O^{nm}_P Lambda_PQ O^{mn}_Q for every m (Eq. wriv)."""
    return np.sum(o_n * (lam @ o_n), axis=0)


def w_table(system, zs) -> np.ndarray:
    """W^c_nm(z) for every core state n, orbital m and argument z.

    Returns [n_states, n_mo, len(zs)]; complex unless every z is imaginary.
    This is the ``wmatrix`` procedure of Sec. 3.4 applied to a set of points.
    """
    zs = [complex(z) for z in zs]
    all_imag = all(z.real == 0.0 for z in zs)
    dtype = np.float64 if all_imag else np.complex128
    out = np.empty((system.n_states, system.n_mo, len(zs)), dtype=dtype)
    for k, z in enumerate(zs):
        lam = lambda_matrix(polarizability(system.o_ia, system.eps, system.n_occ, z,
                                           system.spin))
        for s in range(system.n_states):
            out[s, :, k] = w_elements(system.o_nm[s], lam)
    return out


# ---------------------------------------------------------------------------
# Greedy Thiele-Pade model of W (Sec. 2.4 Eqs. pade, pre_rec, rec_eq; Sec. 3.2)
# ---------------------------------------------------------------------------

def thiele_eval(coef, nodes, u):
    """Continued fraction of Eq. (pade) in u = z^2, evaluated from the bottom.

    T = a_1 / (1 + a_2 (u - u_1) / (1 + ... / (1 + a_p (u - u_{p-1})))).
    ``coef`` = [a_1..a_p], ``nodes`` = [u_1..u_p] (the last node is not used).
    """
    u = np.asarray(u, dtype=np.complex128)
    p = len(coef)
    if p == 0:
        return np.zeros_like(u)
    t = np.ones_like(u)
    for q in range(p - 1, 0, -1):
        t = 1.0 + coef[q] * (u - nodes[q - 1]) / t
    return coef[0] / t


def thiele_greedy(u, w, tol: float = 0.0):
    """Greedy Vidberg-Serene fit of the points (u_j, w_j), u_j = z_j^2.

    a_p = g_p(u_p) (Eq. pre_rec) with g_1 = W and
    g_p(u_i) = [g_{p-1}(u_{p-1}) - g_{p-1}(u_i)] / [(u_i - u_{p-1}) g_{p-1}(u_i)]
    (Eq. rec_eq).  The order of the points is chosen greedily (Sec. 3.2):
    first the largest |W|, then the point with the largest L1 error of the
    current convergent.  Returns (coef, nodes) as complex arrays.
    """
    u = np.asarray(u, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    m = len(u)
    if m == 0:
        return np.zeros(0, np.complex128), np.zeros(0, np.complex128)
    scale = float(np.max(np.abs(w)))
    g = w.copy()
    remaining = list(range(m))
    coef, nodes = [], []
    j = int(np.argmax(np.abs(w)))
    while True:
        a = g[j]
        if not np.isfinite(a):
            break
        coef.append(a)
        nodes.append(u[j])
        remaining.remove(j)
        if not remaining:
            break
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            for i in remaining:
                g[i] = (a - g[i]) / ((u[i] - u[j]) * g[i])
            t = thiele_eval(coef, nodes, u[remaining])
        r = w[remaining] - t
        err = np.abs(r.real) + np.abs(r.imag)
        if np.any(np.isnan(err)):
            break
        k = int(np.argmax(err))        # first maximum = lowest index
        if not err[k] > tol * scale:
            break
        j = remaining[k]
    return np.array(coef, np.complex128), np.array(nodes, np.complex128)


# ---------------------------------------------------------------------------
# Self-energy by contour deformation (Sec. 2.3, Eqs. cdmain ... cdselfe)
# ---------------------------------------------------------------------------

def occupation_factor(eps_m: np.ndarray, eps_f: float, omega: float) -> np.ndarray:
    """f_m of Eq. (ffact) with theta(0) = 1/2."""
    def theta(x):
        return np.where(x > 0, 1.0, np.where(x < 0, 0.0, 0.5))
    return -theta(eps_f - eps_m) * theta(eps_m - omega) + \
        theta(eps_m - eps_f) * theta(omega - eps_m)


def integral_term(omega: float, eps: np.ndarray, w_imag: np.ndarray,
                  freq: np.ndarray, weight: np.ndarray, w0=None,
                  gamma: float = QUAD_GAMMA) -> float:
    """I_n(omega) of Eq. (In_term) by quadrature on the imaginary grid.

    ``w_imag`` is W^c_nm(i omega_k) as [n_mo, n_freq].  The integrand is
    folded over +-omega' (W even and real there) and eta -> 0.

    With ``w0`` ([n_mo], the value W_nm takes at a_m = 0 in the residue term)
    the a_m -> 0 limit is taken analytically: the Lorentzian a/(a^2 + w'^2)
    concentrates at w' = 0 as a_m -> 0, below the grid's smallest node, and
    the exact integral jumps by W_nm(0) there (the jump the residue term's
    occupation factor makes in the other direction, Eq. ffact).  The part
    w0 g(w'), g = gamma^2 / (gamma^2 + w'^2), is integrated in closed form,
    int_0^inf g a / (a^2 + w'^2) dw' = (pi/2) sgn(a) gamma / (|a| + gamma),
    and only the remainder, which vanishes at w' = 0, by quadrature.
    """
    a = omega - eps
    kern = a[:, None] / (a[:, None] ** 2 + freq[None, :] ** 2)
    if w0 is None:
        return float(np.sum(weight[None, :] * w_imag * kern) / math.pi)
    w0 = np.asarray(w0, np.float64)
    g = gamma * gamma / (gamma * gamma + freq * freq)
    smooth = np.sum(weight[None, :] * (w_imag - w0[:, None] * g[None, :]) * kern) / math.pi
    limit = np.sum(w0 * 0.5 * np.sign(a) * gamma / (np.abs(a) + gamma))
    return float(smooth + limit)


def residue_term_complex(omega: float, eps: np.ndarray, eps_f: float, eta: float,
                         w_at: Callable[[int, complex], complex]) -> complex:
    """R_n(omega) of Eq. (Rn_term): sum_m f_m W^c_nm(|eps_m - omega| + i eta).

    ``w_at(m, z)`` returns W^c_nm(z) (a Pade model for CD-WAC, a direct
    evaluation for full CD).  Its real part enters the QP equation; its
    imaginary part is the imaginary part of Sigma_n (the integral term is real
    with eta -> 0), which the spectral function needs.
    """
    f = occupation_factor(eps, eps_f, omega)
    total = 0j
    for m in np.nonzero(f)[0]:
        z = abs(float(eps[m]) - omega) + 1j * eta
        total += f[m] * complex(w_at(int(m), z))
    return complex(total)


def residue_term(omega: float, eps: np.ndarray, eps_f: float, eta: float,
                 w_at: Callable[[int, complex], complex]) -> float:
    """Re R_n(omega) of Eq. (Rn_term)."""
    return float(residue_term_complex(omega, eps, eps_f, eta, w_at).real)


def spectral_function(omega: float, eps_n: float, sigma: complex, vxc: float) -> float:
    """A_nn(omega) = (1/pi) |Im[(omega - eps_n - Sigma_n(omega) + v^xc_n)^-1]|
    (the diagonal spectral function the paper discusses in Sec. 5.5, normalised
    like a Lorentzian)."""
    return abs((1.0 / (omega - eps_n - sigma + vxc)).imag) / math.pi


def fit_range(eps: np.ndarray, n_occ: int, lo: float, hi: float):
    """Orbitals m whose f_m can be non-zero for some omega in [lo, hi].

    Occupied m need eps_m >= lo, virtual m need eps_m <= hi (Eq. ffact); the
    two groups are contiguous, so the set is the range [m0, m1).  Callers
    widen the window by the Z-factor step so that every evaluation of the QP
    solver finds a model.
    """
    n_mo = len(eps)
    m0 = int(np.searchsorted(eps[:n_occ], lo, side="left"))
    m1 = n_occ + int(np.searchsorted(eps[n_occ:], hi, side="right"))
    return m0, min(m1, n_mo)


# ---------------------------------------------------------------------------
# Quasiparticle equation (Eq. qp_eq)
# ---------------------------------------------------------------------------

def qp_solve(f: Callable[[float], float], e_n: float, lo: float, hi: float,
             tol: float = 1e-10, maxit: int = 100):
    """Root of f(omega) = omega - eps_n - Re Sigma_n(omega) + v^xc_n in [lo, hi].

    Returns (qp, z, n_evals, flags).  Secant first (omega_0 = eps_n plus one
    fixed-point step), then the scan-and-bisect fallback described in the
    module docstring.
    """
    n_eval = 0

    def fe(x):
        nonlocal n_eval
        n_eval += 1
        return float(f(x))

    def z_factor(x):
        fp = fe(x + QP_Z_STEP)
        fm = fe(x - QP_Z_STEP)
        return 2.0 * QP_Z_STEP / (fp - fm)

    # secant
    w0 = e_n
    f0 = fe(w0)
    w1 = w0 - f0
    ok = False
    if lo <= w1 <= hi:
        f1 = fe(w1)
        for _ in range(maxit):
            if f1 == f0:
                break
            w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
            if not (lo <= w2 <= hi):
                break
            w0, f0 = w1, f1
            w1 = w2
            f1 = fe(w1)
            if abs(w1 - w0) < tol and abs(f1) < QP_F_TOL:
                ok = True
                break
    if ok:
        z = z_factor(w1)
        if 0.0 < z <= 1.0:
            return w1, z, n_eval, 0

    # fallback: scan, bisect every admissible upward sign change, pick max Z
    n = int(math.ceil((hi - lo) / QP_SCAN_STEP))
    xs = [lo + (hi - lo) * j / n for j in range(n + 1)]
    fs = [fe(x) for x in xs]
    best = None
    for j in range(n):
        fa, fb = fs[j], fs[j + 1]
        if not (fa <= 0.0 < fb):
            continue
        if abs(fa) >= QP_SCAN_FMAX or abs(fb) >= QP_SCAN_FMAX:
            continue
        a, b = xs[j], xs[j + 1]
        while b - a > QP_BISECT_TOL:
            c = 0.5 * (a + b)
            if fe(c) <= 0.0:
                a = c
            else:
                b = c
        root = 0.5 * (a + b)
        if not abs(fe(root)) <= QP_ROOT_FTOL:
            continue      # a jump across a (near-)pole, not a zero of f
        z = z_factor(root)
        key = (z, -abs(root - e_n))
        if best is None or key > best[0]:
            best = (key, root, z)
    if best is None:
        return float("nan"), float("nan"), n_eval, FLAG_NOROOT | FLAG_FALLBACK
    return best[1], best[2], n_eval, FLAG_FALLBACK


# ---------------------------------------------------------------------------
# The whole path (Sec. 3.4): wmatrix -> AC -> QP iteration
# ---------------------------------------------------------------------------

class CdwacOracle:
    """CD-WAC for the core states of one system (Sec. 3.4, CD-WAC branch).

    ``freq``/``weight``: imaginary quadrature grid.  ``ref_im_idx``: indices
    of the grid nodes re-used as Pade reference points; ``ref_re``: real parts
    of the near-real reference points x_j + i ``eta_ref``.  ``vxc=None`` sets
    v^xc_n = Sigma^x_n.
    """

    def __init__(self, system, freq, weight, ref_im_idx, ref_re, win_lo, win_hi,
                 eta: float = 1e-3, eta_ref: float = 1e-3, pade_tol: float = 1e-9,
                 vxc=None, eps_fermi: Optional[float] = None, fit_all: bool = False,
                 eps_qp=None, quad_limit: bool = False):
        self.sys = system
        self.quad_limit = quad_limit
        self.eps = np.asarray(system.eps, np.float64)
        # energies of G in the self-energy (set_g_energies replaces them) and
        # eps_n of the QP equation (the KS energies)
        self.eps_g = self.eps
        self.eps_qp = self.eps if eps_qp is None else np.asarray(eps_qp, np.float64)
        self.fit_all = fit_all
        self.freq = np.asarray(freq, np.float64)
        self.weight = np.asarray(weight, np.float64)
        self.ref_im_idx = np.asarray(ref_im_idx, np.int64)
        self.ref_re = np.asarray(ref_re, np.float64)
        self.win_lo = np.asarray(win_lo, np.float64)
        self.win_hi = np.asarray(win_hi, np.float64)
        self.eta = float(eta)
        self.eta_ref = float(eta_ref)
        self.pade_tol = float(pade_tol)
        self.eps_f = fermi_level(self.eps, system.n_occ) if eps_fermi is None else eps_fermi
        self.sigma_x = np.array([exchange(system.o_nm[s], system.n_occ)
                                 for s in range(system.n_states)])
        self.vxc = self.sigma_x.copy() if vxc is None else np.asarray(vxc, np.float64)
        # wmatrix(F_im)
        self.w_im = w_table(system, [1j * w for w in self.freq])
        # wmatrix(F_real), fits over F_wac
        self.z_re = self.ref_re + 1j * self.eta_ref
        self.w_re = w_table(system, list(self.z_re)) if len(self.z_re) else \
            np.zeros((system.n_states, system.n_mo, 0), np.complex128)
        self.fits = []
        for s in range(system.n_states):
            m0, m1 = (0, system.n_mo) if fit_all else fit_range(
                self.eps, system.n_occ, self.win_lo[s] - QP_Z_STEP, self.win_hi[s] + QP_Z_STEP)
            models = {}
            for m in range(m0, m1):
                u, w = self.reference_data(s, m)
                models[m] = thiele_greedy(u, w, self.pade_tol)
            self.fits.append(models)
        self.w0 = self.limit_values() if quad_limit else None

    def limit_values(self):
        """W^c_nm at a_m = 0 as the residue term takes it, Re T_nm((i eta)^2),
        for every m with a model (0 for the others, whose residue cannot
        reach the window): [n_states, n_mo]."""
        w0 = np.zeros((self.sys.n_states, self.sys.n_mo))
        for s in range(self.sys.n_states):
            for m in self.fits[s]:
                w0[s, m] = self.w_model(s, m, 1j * self.eta).real
        return w0

    def i_term(self, s: int, omega: float, eps_g) -> float:
        return integral_term(omega, eps_g, self.w_im[s], self.freq, self.weight,
                             None if self.w0 is None else self.w0[s])

    def set_g_energies(self, eps_g, eps_fermi: Optional[float] = None):
        """Orbital energies of G in I_n, R_n and Eq. (ffact); W and its models
        stay (the G of the eigenvalue-self-consistent schemes, Sec. 4).  Every
        m needs a model, so the oracle must be built with fit_all."""
        if not self.fit_all:
            raise ValueError("set_g_energies needs an oracle built with fit_all=True")
        self.eps_g = np.asarray(eps_g, np.float64)
        self.eps_f = fermi_level(self.eps_g, self.sys.n_occ) if eps_fermi is None else eps_fermi

    def reference_data(self, s: int, m: int):
        """(u_j, W_j) over F_wac = re-used imaginary nodes + near-real points."""
        z_im = 1j * self.freq[self.ref_im_idx]
        u = np.concatenate([z_im ** 2, self.z_re ** 2])
        w = np.concatenate([self.w_im[s, m, self.ref_im_idx].astype(np.complex128),
                            self.w_re[s, m, :]])
        return u, w

    def w_model(self, s: int, m: int, z: complex) -> complex:
        coef, nodes = self.fits[s][m]
        return complex(thiele_eval(coef, nodes, np.array([z * z]))[0])

    def w_residue(self, s: int, m: int, z: complex) -> complex:
        """W^c_nm at a residue point of Eq. (Rn_term): the Pade model."""
        return self.w_model(s, m, z)

    def sigma(self, s: int, omega: float) -> float:
        """Re Sigma_n(omega) = Sigma^x + Re R - I (Eq. cdselfe), CD-WAC."""
        i_term = self.i_term(s, omega, self.eps_g)
        r_term = residue_term(omega, self.eps_g, self.eps_f, self.eta,
                              lambda m, z: self.w_model(s, m, z))
        return self.sigma_x[s] + r_term - i_term

    def sigma_c(self, s: int, omega: float) -> float:
        return self.sigma(s, omega) - self.sigma_x[s]

    def sigma_complex(self, s: int, omega: float) -> complex:
        """Sigma^x + R - I with the complex residue term."""
        i_term = self.i_term(s, omega, self.eps_g)
        r_term = residue_term_complex(omega, self.eps_g, self.eps_f, self.eta,
                                      lambda m, z: self.w_model(s, m, z))
        return self.sigma_x[s] + r_term - i_term

    def spectral(self, s: int, omega: float, vxc: Optional[float] = None) -> float:
        n = int(self.sys.state_idx[s])
        v = float(self.vxc[s]) if vxc is None else vxc
        return spectral_function(omega, float(self.eps_qp[n]), self.sigma_complex(s, omega), v)

    def solve(self, s: int, tol: float = 1e-10, maxit: int = 100):
        n = int(self.sys.state_idx[s])
        e_n = float(self.eps_qp[n])
        vxc = float(self.vxc[s])
        return qp_solve(lambda x: x - e_n - self.sigma(s, x) + vxc, e_n,
                        float(self.win_lo[s]), float(self.win_hi[s]), tol, maxit)

    def solve_all(self, tol: float = 1e-10, maxit: int = 100):
        return [self.solve(s, tol, maxit) for s in range(self.sys.n_states)]

    # -- G_{Delta H} W_0 (Sec. 4) ------------------------------------------
    def sigma_g_shifted(self, s: int, omega: float, dh: float) -> float:
        """Re Sigma_n(omega) with a shift dh in the denominator of G: every
        energy of G and the Fermi level moved by dh (W and its models stay)."""
        eps_g = self.eps_g + dh
        ef = self.eps_f + dh
        i_term = self.i_term(s, omega, eps_g)
        r_term = residue_term(omega, eps_g, ef, self.eta, lambda m, z: self.w_residue(s, m, z))
        return self.sigma_x[s] + r_term - i_term

    def hedin_shift(self, s: int) -> float:
        """Delta H_n, fixed before the QP iteration: the first-order G0W0
        correction at the Kohn-Sham energy, Re Sigma_n(eps_n) - v^xc_n (the
        paper names the shift and where it enters, not its recipe; this
        moves G's pole of state n to the linearised G0W0 energy)."""
        n = int(self.sys.state_idx[s])
        return self.sigma(s, float(self.eps_qp[n])) - float(self.vxc[s])

    def solve_hedin(self, s: int, tol: float = 1e-10, maxit: int = 100):
        """QP root of Eq. (qp_eq) with the self-energy of the shifted G.
        Every model m must exist, so the oracle must be built with fit_all
        (the shifted residues |eps_m + dh - omega| reach beyond the window's
        fit range).  Returns (qp, z, n_evals, flags, dh)."""
        if not self.fit_all and not isinstance(self, FullCdOracle):
            raise ValueError("solve_hedin needs an oracle built with fit_all=True")
        dh = self.hedin_shift(s)
        n = int(self.sys.state_idx[s])
        e_n = float(self.eps_qp[n])
        vxc = float(self.vxc[s])
        r = qp_solve(lambda x: x - e_n - self.sigma_g_shifted(s, x, dh) + vxc, e_n,
                     float(self.win_lo[s]), float(self.win_hi[s]), tol, maxit)
        return (*r, dh)


class FullCdOracle(CdwacOracle):
    """Full contour deformation (Sec. 3.4, CD branch): W at every residue.

    The residue term calls ``wmatrix`` at z = |eps_m - omega| + i eta for every
    m with f_m != 0, i.e. one complex polarizability per residue.  This is the
    O(N^5) reference CD-WAC approximates.  Results are cached per z.
    """

    def __init__(self, system, freq, weight, win_lo, win_hi, eta: float = 1e-3,
                 vxc=None, eps_fermi: Optional[float] = None, eps_qp=None,
                 quad_limit: bool = False):
        super().__init__(system, freq, weight, np.zeros(0, np.int64), np.zeros(0),
                         win_lo, win_hi, eta=eta, eta_ref=eta, pade_tol=0.0,
                         vxc=vxc, eps_fermi=eps_fermi, fit_all=True, eps_qp=eps_qp)
        self._cache = {}
        self.quad_limit = quad_limit
        # W^c_nm at the residue point of a_m = 0, i eta, evaluated directly
        self.w0 = w_table(system, [1j * eta]).real[:, :, 0] if quad_limit else None

    def w_residue(self, s: int, m: int, z: complex) -> complex:
        """W^c_nm at a residue point: evaluated directly (full CD)."""
        return self.w_direct(s, m, z)

    def w_direct(self, s: int, m: int, z: complex) -> complex:
        key = (s, complex(z))
        if key not in self._cache:
            lam = lambda_matrix(polarizability(self.sys.o_ia, self.eps, self.sys.n_occ, z,
                                               self.sys.spin))
            self._cache[key] = w_elements(self.sys.o_nm[s], lam)
        return complex(self._cache[key][m])

    def sigma(self, s: int, omega: float) -> float:
        i_term = self.i_term(s, omega, self.eps_g)
        r_term = residue_term(omega, self.eps_g, self.eps_f, self.eta,
                              lambda m, z: self.w_direct(s, m, z))
        return self.sigma_x[s] + r_term - i_term


# ---------------------------------------------------------------------------
# Eigenvalue self-consistency (Sec. 4: evGW0 and evGW)
# ---------------------------------------------------------------------------

def evgw(system, make, mode: str, max_iter: int = 20, tol: float = 1e-8):
    """Iterates the QP equations with the QP energies fed back.

    ``make(system_w, eps_qp)`` builds a self-energy object (an oracle with
    fit_all) whose W comes from ``system_w.eps`` and whose QP equation uses
    ``eps_qp`` (the KS energies).  evGW0 builds it once from the KS energies
    and replaces only the energies of G; evGW rebuilds it (Pi, Lambda, W, the
    fits) from the current energies every iteration.  The energies of the
    computed states are replaced after each solve (a state without a root
    keeps its energy); the others keep their input values.  Stops once no
    energy moves by more than ``tol`` or after ``max_iter`` solves.
    Returns (energies, solves, results of the last solve).
    """
    import dataclasses
    ks = np.asarray(system.eps, np.float64).copy()
    cur = ks.copy()
    o = None
    it = 0
    res = None
    for it in range(1, max_iter + 1):
        if mode == "evgw" or o is None:
            sys_w = dataclasses.replace(system, eps=cur.copy()) if mode == "evgw" else system
            o = make(sys_w, ks)
        o.set_g_energies(cur)
        res = o.solve_all()
        nxt = cur.copy()
        for j, r in enumerate(res):
            if not r[3] & FLAG_NOROOT:
                nxt[int(system.state_idx[j])] = r[0]
        delta = float(np.max(np.abs(nxt - cur)))
        cur = nxt
        if delta < tol:
            break
    return cur, it, res


# ---------------------------------------------------------------------------
# Closed-form pole sum (Eq. sigma_pole) for tiny inputs
# ---------------------------------------------------------------------------

def rpa_poles(system):
    """Neutral excitations Omega_s and couplings of the RI-RPA problem.

    With A = O^{ia} diag(sqrt(2 spin D_ia)) and C = D^2 + A^T A = V Omega^2 V^T,
    Woodbury on Eq. (bigLambda) gives Lambda(z) = sum_s (A v_s)(A v_s)^T /
    (z^2 - Omega_s^2), so W^c_nm(z) = sum_s c_nms / (z^2 - Omega_s^2) with
    c_nms = (O^{nm}^T A v_s)^2.  Returns (Omega [K], c [n_states, n_mo, K]).
    """
    delta = transition_energies(system.eps, system.n_occ)
    a = system.o_ia * np.sqrt(2.0 * system.spin * delta)[None, :]
    c_mat = np.diag(delta ** 2) + a.T @ a
    om2, v = np.linalg.eigh(c_mat)
    omega = np.sqrt(om2)
    av = a @ v                                            # [n_aux, K]
    coup = np.einsum("spm,pk->smk", system.o_nm, av) ** 2
    return omega, coup


def w_poles(omega, coup, z: complex) -> np.ndarray:
    """W^c_nm(z) from the pole form, [n_states, n_mo]."""
    return np.sum(coup / (z * z - omega[None, None, :] ** 2), axis=-1)


def sigma_c_poles(system, s: int, omega_eval: float, poles=None,
                  eps_fermi: Optional[float] = None) -> float:
    """Sigma^c_n(omega) of Eq. (sigma_pole) with eta -> 0.

    Each pole of W^c_nm, c/(z^2 - Omega^2) = (c / 2 Omega)[1/(z - Omega) -
    1/(z + Omega)], contributes P_s = c / (2 Omega_s) over
    omega - eps_m + Omega_s sgn(eps_F - eps_m).
    """
    om, coup = rpa_poles(system) if poles is None else poles
    ef = fermi_level(system.eps, system.n_occ) if eps_fermi is None else eps_fermi
    eps = system.eps
    sgn = np.where(ef - eps > 0, 1.0, -1.0)
    p = coup[s] / (2.0 * om[None, :])                      # [n_mo, K]
    den = omega_eval - eps[:, None] + om[None, :] * sgn[:, None]
    return float(np.sum(p / den))
