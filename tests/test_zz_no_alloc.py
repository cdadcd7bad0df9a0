"""The allocation-free fit entry point (cdwac_pade_fit_eval_noalloc) against
the allocating one (cdwac_pade_fit_eval), through the C ABI: the same greedy
Thiele fits (Sec. 3.2; Eqs. pade, rec_eq) and values, term counts identical,
on two calls in a row (the second smaller, so it runs over what the first
left in the fixed scratch), the size limit rejected before any launch, and
the call recorded into a HIP graph and replayed."""
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


def test_noalloc_under_graph_capture():
    """Recorded into a HIP graph on its context's stream and replayed four
    times over two input sets copied into the same device buffers between
    the replays: every replay equals the allocating entry point's eager
    result for that set bit for bit, with eager work on the same context
    between the replays."""
    import ctypes

    import torch
    from paper_2305_15955_amd import cdwac
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = torch.cuda.Stream()
    lib = cdwac.Cdwac(0, stream=s)
    try:
        n_fit, n_pts = 600, 24
        sets = [fit_sets(n_fit, n_pts, seed) for seed in (5, 6)]
        refs = [lib.cdwac_pade_fit_eval(u, w, 1e-9, x) for u, w, x in sets]
        assert not np.array_equal(refs[0][0], refs[1][0])

        def c2(a):
            a = np.asarray(a, np.complex128)
            return torch.from_numpy(np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1)))

        host = [[c2(a) for a in st] for st in sets]
        nx = sets[0][2].shape[1]
        dev = [t.to("cuda:0") for t in host[0]]
        out = torch.empty((n_fit, nx, 2), dtype=torch.float64, device="cuda:0")
        nt = torch.empty(n_fit, dtype=torch.int32, device="cuda:0")
        p = lambda t: ctypes.c_void_p(t.data_ptr())

        def call():
            return lib.lib.cdwac_pade_fit_eval_noalloc(lib.ctx, n_fit, n_pts, p(dev[0]), p(dev[1]), 1e-9, nx,
                                                       p(dev[2]), p(out), p(nt))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            assert call() == 0                      # eager, outside the capture
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        out.zero_()
        torch.cuda.synchronize()
        print("capturing the allocation-free fit call", flush=True)
        with torch.cuda.graph(g, stream=s):
            rc = call()
        assert rc == 0, rc
        for k in (0, 1, 0, 1):
            print(f"replay with input set {k}", flush=True)
            with torch.cuda.stream(s):
                for d, h in zip(dev, host[k]):
                    d.copy_(h.to("cuda:0"))
                out.zero_()
                nt.zero_()
            s.synchronize()
            g.replay()
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            np.testing.assert_array_equal(nt.cpu().numpy(), refs[k][1])
            np.testing.assert_array_equal(o[..., 0] + 1j * o[..., 1], refs[k][0])
            # eager work on the same context between the replays
            again = lib.cdwac_pade_fit_eval(*sets[1 - k][:2], 1e-9, sets[1 - k][2])
            np.testing.assert_array_equal(again[0], refs[1 - k][0])
        del g
    finally:
        lib.close()
