"""The allocation-free fit entry point (cdwac_pade_fit_eval_noalloc) against
the allocating one (cdwac_pade_fit_eval), through the C ABI: the same greedy
Thiele fits (Sec. 3.2; Eqs. pade, rec_eq) and values, term counts identical,
on two calls in a row (the second smaller, so it runs over what the first
left in the fixed scratch), and the size limit rejected before any launch."""
import numpy as np
import pytest

from oracle import cdwac_ref as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2305_15955_amd import cdwac
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = cdwac.Cdwac(0)
    yield c
    c.close()


def fit_sets(n_fit, n_pts, seed):
    """Pole sums in u = z^2 sampled on imaginary and near-real points, the
    shape of the W^c_nm data the fits take."""
    rng = np.random.default_rng(seed)
    n_im = n_pts // 2
    z = np.concatenate([1j * np.geomspace(0.05, 40.0, n_im), np.linspace(0.0, 12.0, n_pts - n_im) + 1e-3j])
    u = np.broadcast_to(z * z, (n_fit, n_pts)).copy()
    om = rng.uniform(0.5, 15.0, (n_fit, 3))
    c = rng.uniform(0.01, 0.3, (n_fit, 3))
    w = np.sum(-c[:, None, :] * om[:, None, :] / (om[:, None, :] ** 2 - u[:, :, None]), axis=-1)
    x = (np.linspace(0.1, 11.0, 17)[None, :] + 1e-3j) ** 2 * np.ones((n_fit, 1))
    return u, w, x


def test_noalloc_matches_allocating_entry_point(lib):
    for n_fit, n_pts, seed in ((3000, 24, 1), (700, 16, 2)):
        u, w, x = fit_sets(n_fit, n_pts, seed)
        print(f"no-alloc fits: n_fit={n_fit}, n_pts={n_pts}, seed={seed}", flush=True)
        ref, nt_ref = lib.cdwac_pade_fit_eval(u, w, 1e-9, x)
        got, nt = lib.cdwac_pade_fit_eval_noalloc(u, w, 1e-9, x)
        np.testing.assert_array_equal(nt, nt_ref)
        np.testing.assert_array_equal(got, ref)            # same kernels: bit for bit
        # and against the oracle's fits of the first few sets
        for f in range(5):
            coef, nodes = R.thiele_greedy(u[f], w[f], 1e-9)
            assert len(coef) == nt[f]
            np.testing.assert_allclose(got[f], R.thiele_eval(coef, nodes, x[f]), rtol=1e-8, atol=1e-12)


def test_noalloc_rejects_sizes_beyond_the_scratch(lib):
    from paper_2305_15955_amd import cdwac
    n_pts = 256
    n_fit = (1 << 19) // n_pts + 1
    u = np.zeros((n_fit, n_pts), complex)
    with pytest.raises(cdwac.CdwacError) as e:
        lib.cdwac_pade_fit_eval_noalloc(u, u, 1e-9, np.zeros((n_fit, 1), complex))
    assert e.value.code == cdwac.CDWAC_EINVAL
