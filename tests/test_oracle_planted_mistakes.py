"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in the oracle for the duration of the test (a
flipped sign, a dropped term, a transposed or shifted index, a wrong factor
or order) through ``monkeypatch``, runs the pins of tests/test_oracle_pins.py
and tests/test_oracle_mlp.py that should see it, and requires that at least
one of them fails with an AssertionError.  Nothing under oracle/ is changed
on disk; the unmutated oracle passes the same pins (the first case).
"""
import math

import numpy as np
import pytest

import test_oracle_mlp as PM
import test_oracle_pins as P
from oracle import cdwac_ref as R
from oracle import mlp_ref as M

_pi = R.polarizability
_delta = R.transition_energies
_integral = R.integral_term
_occ = R.occupation_factor
_residue = R.residue_term_complex
_qp = R.qp_solve
_hedin = R.CdwacOracle.hedin_shift
_forward = M.forward


def pi_plus(o_ia, eps, n_occ, z, spin=2.0):
    """The two fractions of Eq. (piriv) added instead of subtracted."""
    delta = R.transition_energies(eps, n_occ)
    z = complex(z)
    d = spin * (1.0 / (z - delta) + 1.0 / (z + delta))
    if z.real == 0.0:
        d = d.real
    return (o_ia * d[None, :]) @ o_ia.T


def pi_real_part_only(o_ia, eps, n_occ, z, spin=2.0):
    """Pi at complex z with the imaginary part of the weights dropped."""
    out = _pi(o_ia, eps, n_occ, z, spin)
    return out.real if np.iscomplexobj(out) else out


def delta_occ_fastest(eps, n_occ):
    """D_ia flattened with i fastest, while O^{ia} has a fastest."""
    return (eps[None, n_occ:] - eps[:n_occ, None]).T.reshape(-1)


def lambda_without_minus_identity(pi):
    """(I - Pi)^{-1} returned for Lambda, the - I of Eq. (bigLambda) dropped."""
    return np.linalg.inv(np.eye(pi.shape[0], dtype=pi.dtype) - pi)


def w_diagonal_lambda_only(o_n, lam):
    """W with only the diagonal of Lambda (the P != Q coupling dropped)."""
    return np.sum(o_n * o_n * np.diag(lam)[:, None], axis=0)


def integral_sign_flipped(omega, eps, w_imag, freq, weight, w0=None, gamma=R.QUAD_GAMMA):
    """a_m = eps_m - omega in place of omega - eps_m (the whole term flips)."""
    return -_integral(omega, eps, w_imag, freq, weight, w0, gamma)


def integral_limit_factor_one(omega, eps, w_imag, freq, weight, w0=None, gamma=R.QUAD_GAMMA):
    """The closed-form part of the a_m -> 0 limit with pi instead of pi/2."""
    v = _integral(omega, eps, w_imag, freq, weight, w0, gamma)
    if w0 is None:
        return v
    a = omega - eps
    return v + float(np.sum(np.asarray(w0) * 0.5 * np.sign(a) * gamma / (np.abs(a) + gamma)))


def theta_zero_is_one(eps_m, eps_f, omega):
    """theta(0) = 1 instead of 1/2 in Eq. (ffact)."""
    th = lambda x: np.where(x >= 0, 1.0, 0.0)
    return -th(eps_f - eps_m) * th(eps_m - omega) + th(eps_m - eps_f) * th(omega - eps_m)


def occupation_swapped(eps_m, eps_f, omega):
    """The signs of the occupied and virtual residues exchanged."""
    return -_occ(eps_m, eps_f, omega)


def residue_parts_swapped(omega, eps, eps_f, eta, w_at):
    """The imaginary part of the residue sum taken for its real part (and the
    other way round)."""
    v = _residue(omega, eps, eps_f, eta, w_at)
    return complex(v.imag, v.real)


def greedy_smallest_error(u, w, tol=0.0):
    """The greedy order of Sec. 3.2 with the best-fitted point added next."""
    u = np.asarray(u, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    scale = float(np.max(np.abs(w)))
    g = w.copy()
    remaining = list(range(len(u)))
    coef, nodes = [], []
    j = int(np.argmax(np.abs(w)))
    while True:
        a = g[j]
        coef.append(a)
        nodes.append(u[j])
        remaining.remove(j)
        if not remaining:
            break
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            for i in remaining:
                g[i] = (a - g[i]) / ((u[i] - u[j]) * g[i])
            t = R.thiele_eval(coef, nodes, u[remaining])
        r = w[remaining] - t
        err = np.abs(r.real) + np.abs(r.imag)
        k = int(np.argmin(err))
        if not np.max(err) > tol * scale:
            break
        j = remaining[k]
    return np.array(coef, np.complex128), np.array(nodes, np.complex128)


def thiele_eval_shifted_nodes(coef, nodes, u):
    """The continued fraction with each coefficient paired with its own node
    (u - u_q) instead of the previous one (u - u_{q-1})."""
    u = np.asarray(u, dtype=np.complex128)
    p = len(coef)
    if p == 0:
        return np.zeros_like(u)
    t = np.ones_like(u)
    for q in range(p - 1, 0, -1):
        t = 1.0 + coef[q] * (u - nodes[q]) / t
    return coef[0] / t


def exchange_over_virtuals(o_n, n_occ):
    """Sigma^x summed over the virtual orbitals."""
    return -float(np.sum(o_n[:, n_occ:] ** 2))


def spectral_without_one_over_pi(omega, eps_n, sigma, vxc):
    return abs((1.0 / (omega - eps_n - sigma + vxc)).imag)


def qp_z_wrong_sign(*a, **k):
    r = _qp(*a, **k)
    return (r[0], -r[1]) + tuple(r[2:])


def hedin_shift_negated(self, s):
    return -_hedin(self, s)


def forward_without_second_tanh(theta, x):
    p = M.unpack(theta)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = h1 @ p["W2"].T + p["b2"]
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], (h1, h2)


# (what is planted, [(module, attribute, replacement)], pins that should see it)
CASES = [
    ("nothing (control)", [], [P.test_polarizability_bruteforce_two_fractions, P.test_w_matches_pole_form]),
    ("Pi: fractions added", [(R, "polarizability", pi_plus)],
     [P.test_polarizability_bruteforce_two_fractions, P.test_polarizability_invariants]),
    ("Pi: imaginary part dropped at complex z", [(R, "polarizability", pi_real_part_only)],
     [P.test_polarizability_bruteforce_two_fractions]),
    ("transition energies in the wrong order", [(R, "transition_energies", delta_occ_fastest)],
     [P.test_polarizability_bruteforce_two_fractions]),
    ("Lambda without - I", [(R, "lambda_matrix", lambda_without_minus_identity)],
     [P.test_dielectric_and_w_invariants, P.test_w_matches_pole_form]),
    ("W from the diagonal of Lambda only", [(R, "w_elements", w_diagonal_lambda_only)],
     [P.test_w_matches_pole_form]),
    ("integral term with a_m of the wrong sign", [(R, "integral_term", integral_sign_flipped)],
     [P.test_single_transition_cd_equals_pole_sum]),
    ("a_m -> 0 limit with pi instead of pi/2", [(R, "integral_term", integral_limit_factor_one)],
     [P.test_integral_term_limit_single_pole_closed_form, P.test_full_cd_with_limit_is_continuous_and_equals_pole_sum]),
    ("theta(0) = 1", [(R, "occupation_factor", theta_zero_is_one)], [P.test_occupation_factor_cases]),
    ("occupied and virtual residues swapped", [(R, "occupation_factor", occupation_swapped)],
     [P.test_single_transition_cd_equals_pole_sum]),
    ("residue term: real and imaginary parts exchanged", [(R, "residue_term_complex", residue_parts_swapped)],
     [P.test_single_transition_cd_equals_pole_sum]),
    ("greedy Thiele: best-fitted point next", [(R, "thiele_greedy", greedy_smallest_error)],
     [P.test_thiele_greedy_order_by_hand]),
    ("Thiele evaluation with shifted nodes", [(R, "thiele_eval", thiele_eval_shifted_nodes)],
     [P.test_thiele_interpolates_used_nodes, P.test_thiele_exact_on_single_and_double_pole]),
    ("exchange over the virtual orbitals", [(R, "exchange", exchange_over_virtuals)],
     [P.test_exchange_equals_real_space_exchange_operator, P.test_full_cd_sigma_with_exchange_and_given_vxc]),
    ("spectral function without 1/pi", [(R, "spectral_function", spectral_without_one_over_pi)],
     [P.test_spectral_function_constant_sigma_is_a_unit_lorentzian]),
    ("Z with the wrong sign", [(R, "qp_solve", qp_z_wrong_sign)], [P.test_qp_solver_fallback_and_noroot]),
    ("Hedin shift with the wrong sign", [(R.CdwacOracle, "hedin_shift", hedin_shift_negated)],
     [P.test_hedin_shifted_g_full_cd_equals_pole_sum]),
    ("MLP: second tanh dropped", [(M, "forward", forward_without_second_tanh)], [PM.test_forward_hand_evaluated_network]),
]


@pytest.mark.parametrize("what, patches, pins", CASES, ids=[c[0] for c in CASES])
def test_pins_catch_a_planted_mistake(monkeypatch, what, patches, pins):
    for obj, name, repl in patches:
        monkeypatch.setattr(obj, name, repl)
    failed = []
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    if not patches:
        assert not failed, failed
    else:
        print(f"{what}: caught by {failed}")
        assert failed, f"no pin caught: {what}"
