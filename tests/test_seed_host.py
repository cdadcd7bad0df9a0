"""Host side of the learned seed (no GPU): the base estimates that the
training script computes from the four self-energy samples, against roots
known in closed form."""
import numpy as np

from paper_2305_15955_amd import seed_train


def sig4_for(f, eps_n, vxc):
    """Sigma at the four sample points such that f(eps_n + d) = f(d)."""
    d = seed_train.OFFSETS
    return (d - f(d) + vxc)[None, :]


def test_cubic_estimate_recovers_the_zero_of_a_cubic():
    """f a cubic with a simple zero at d = 0.07 (outside the samples' inner
    pair, inside their span) and one far away: the estimate is eps_n + 0.07
    to rounding, also when the line estimate starts on the other side."""
    r = 0.07
    f = lambda d: 1.2 * (d - r) + 0.5 * (d - r) ** 2 - 2.0 * (d - r) ** 3
    eps_n, vxc = np.array([-10.0]), np.array([-0.4])
    sig4 = sig4_for(f, eps_n, vxc)
    lo, hi = eps_n - 1.0, eps_n + 1.0
    wl = seed_train.line_estimate(eps_n, vxc, sig4, lo, hi)
    assert abs(wl[0] - (eps_n[0] + r)) > 5e-4          # the line alone misses it by ~19 meV
    wc = seed_train.cubic_estimate(eps_n, vxc, sig4, lo, hi, wl)
    assert abs(wc[0] - (eps_n[0] + r)) < 1e-13
    wc = seed_train.cubic_estimate(eps_n, vxc, sig4, lo, hi, eps_n - 0.02)
    assert abs(wc[0] - (eps_n[0] + r)) < 1e-13


def test_cubic_estimate_extrapolates_a_quadratic_exactly():
    """A quadratic f (the cubic's leading coefficient vanishes) with its zero
    at d = 0.25, beyond the samples: recovered to rounding."""
    f = lambda d: 0.9 * (d - 0.25) + 0.3 * (d - 0.25) ** 2
    eps_n, vxc = np.array([-5.0]), np.array([0.1])
    sig4 = sig4_for(f, eps_n, vxc)
    lo, hi = eps_n - 1.0, eps_n + 1.0
    wc = seed_train.cubic_estimate(eps_n, vxc, sig4, lo, hi, seed_train.line_estimate(eps_n, vxc, sig4, lo, hi))
    assert abs(wc[0] - (eps_n[0] + 0.25)) < 1e-12


def test_cubic_estimate_falls_back_to_the_line():
    """A zero outside the window, and a cubic whose slope at the start is
    negative, both give the line estimate back."""
    eps_n, vxc = np.array([-5.0]), np.array([0.0])
    f = lambda d: d - 0.6
    sig4 = sig4_for(f, eps_n, vxc)
    lo, hi = eps_n - 0.5, eps_n + 0.5
    wl = seed_train.line_estimate(eps_n, vxc, sig4, lo, hi)
    assert wl[0] == hi[0]
    assert seed_train.cubic_estimate(eps_n, vxc, sig4, lo, hi, wl)[0] == wl[0]
    g = lambda d: -d + 0.01
    sig4 = sig4_for(g, eps_n, vxc)
    start = np.array([-4.9])
    assert seed_train.cubic_estimate(eps_n, vxc, sig4, lo, hi, start)[0] == start[0]
