"""The learned QP seed: hand-written FP32 kernels against the FP64 reference,
and what the trained network changes in the root search."""
import os

import numpy as np
import pytest

import cases
from oracle import mlp_ref as M
from paper_2305_15955_amd import synth

pytestmark = pytest.mark.gpu
MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2305_15955_amd",
                     "seed_model.npz")


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2305_15955_amd import cdwac
    assert torch.cuda.is_available()
    c = cdwac.Cdwac(0)
    yield c
    c.close()


def data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 8))
    t = np.sin(x[:, 0]) + 0.3 * x[:, 1] * x[:, 2] - 0.2 * x[:, 5]
    return x, t


def test_forward_matches_reference(lib):
    x, _ = data(1000, 1)
    theta = M.init_params(3)
    theta[-1] = 0.2
    y32 = lib.cdwac_mlp_forward(theta, x)
    y64, _ = M.forward(theta.astype(np.float64), x.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(y32, y64, rtol=1e-5, atol=1e-5)


def gradient_scale(theta, x, t):
    """Per parameter, the sum over samples of the moduli of its chain-rule
    terms, with the output residual |y - t| widened by the scale of the
    output's own computation (|W3| |h2| + |b3| + |W3| (|W2| |h1| + |b2| +
    |W2| (|W1| |x| + |b1|))), which bounds how far FP32 rounding of the
    forward pass can move y.  FP32 rounding of the whole gradient stays
    within a small multiple of u_32 times this scale, element by element."""
    p = M.unpack(theta)
    n = len(x)
    y, (h1, h2) = M.forward(theta, x)
    a1 = np.abs(x) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    a2 = np.abs(h1) @ np.abs(p["W2"]).T + np.abs(p["b2"]) + a1 @ np.abs(p["W2"]).T
    ys = (np.abs(h2) + a2) @ np.abs(p["W3"][0]) + abs(p["b3"][0])
    ady = (2.0 / n) * (np.abs(y - t) + ys)[:, None]
    dz2 = (ady @ np.abs(p["W3"])) * np.abs(1.0 - h2 * h2)
    dz1 = (dz2 @ np.abs(p["W2"])) * np.abs(1.0 - h1 * h1)
    return np.concatenate([(dz1.T @ np.abs(x)).ravel(), dz1.sum(0), (dz2.T @ np.abs(h1)).ravel(), dz2.sum(0),
                           (ady.T @ np.abs(h2)).ravel(), ady.sum(0)])


@pytest.mark.parametrize("n", [1, 31, 32, 1000, 5003])
def test_gradient_matches_reference(lib, n):
    """Element by element: |g - g_ref| <= 64 u_32 times the gradient's own
    scale (gradient_scale).  Each chain-rule term carries a few FP32
    roundings (an 8- or 64-term dot product, tanhf, the sample sum); an
    FP32 emulation of the same backpropagation stays within 0.32 u_32 of
    the scale here."""
    x, t = data(n, 2)
    theta = M.init_params(4).astype(np.float32).astype(np.float64)
    xf = x.astype(np.float32).astype(np.float64)
    tf = t.astype(np.float32).astype(np.float64)
    loss, g = lib.cdwac_mlp_grad(theta, xf, tf)
    loss_ref, g_ref = M.loss_and_grad(theta, xf, tf)
    assert loss == pytest.approx(loss_ref, rel=1e-5)
    bound = 64.0 * 2.0 ** -24 * gradient_scale(theta, xf, tf)
    over = np.abs(g - g_ref) / bound
    print(f"n={n}: largest |g - g_ref| / (u_32 scale) = {64.0 * over.max():.3f} (parameter {int(over.argmax())})")
    assert np.all(over <= 1.0), (int(over.argmax()), float(over.max()))


def test_adam_step_matches_reference(lib):
    import torch
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(4801)
    grad = rng.standard_normal(4801)
    m = rng.standard_normal(4801) * 0.1
    v = np.abs(rng.standard_normal(4801)) * 0.1
    dev = torch.device("cuda", 0)
    td, gd, md, vd = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (theta, grad, m, v))
    lib.cdwac_mlp_adam(td, gd, md, vd, 7, 1e-3)
    th, mm, vv = theta.copy(), m.copy(), v.copy()
    M.adam_step(th, grad, mm, vv, 7, 1e-3)
    np.testing.assert_allclose(td.cpu().numpy(), th, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(md.cpu().numpy(), mm, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(vd.cpu().numpy(), vv, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(lib):
    x, t = data(4096, 6)
    theta0 = M.init_params(7).astype(np.float32)
    loss0, _ = M.loss_and_grad(theta0.astype(np.float64), x, t)
    theta, curve = lib.cdwac_mlp_train(theta0, x, t, epochs=40, batch=128, lr=3e-3, seed=1)
    loss1, _ = M.loss_and_grad(theta.astype(np.float64), x.astype(np.float32).astype(np.float64), t)
    assert curve[-1] < 0.2 * curve[0]
    assert loss1 < 0.1 * loss0


def test_seed_saves_rounds_when_accepted(lib):
    """The seed takes one pass over the tables (Sigma at four points around
    eps_n); an accepted seed (|f| <= 1 meV, Z in (0, 1]) ends the search
    after one more (f at the seed and its Z pair): 2 passes, against 6-7 for
    the plain secant.  Held-out 60-orbital system, v^xc shifted over +-0.3
    Ha: fewer passes in total, the same roots within 1 meV."""
    mdl = np.load(MODEL)
    lib.cdwac_mlp_set_model(mdl["theta"], mdl["mu"], mdl["sd"], float(mdl["out_mu"]), float(mdl["out_sd"]))
    case = cases.workload("fp64_1core_nmo60")
    s = case.system
    sysc, keep = lib.make_system(s)
    tot = {}
    for mlp in (False, True):
        prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                    prec="p64", use_mlp_seed=mlp, mlp_accept=1.0e-3 / synth.HARTREE_EV)
        lib.cdwac_prepare(sysc, prm)
        _, _, sx, _ = lib.cdwac_w_table(s.n_states, s.n_mo, len(case.freq), len(case.ref_re))
        rows = []
        for sh in (-0.3, -0.2, -0.12, -0.06, 0.0, 0.06, 0.12, 0.2, 0.3):
            out = lib.cdwac_qp(s.n_states, vxc=sx + sh)
            rows.append([(o["qp"], o["n_rounds"], o["flags"]) for o in out])
        tot[mlp] = rows
    plain = sum(r[1] for row in tot[False] for r in row)
    seeded = sum(r[1] for row in tot[True] for r in row)
    accepted = sum(bool(r[2] & 4) for row in tot[True] for r in row)
    print(f"passes plain {plain}, seeded {seeded}, seed accepted {accepted} of {len(tot[True])}")
    for row0, row1 in zip(tot[False], tot[True]):
        for (q0, n0, f0), (q1, n1, f1) in zip(row0, row1):
            assert abs(q1 - q0) <= 1.0e-3 / synth.HARTREE_EV
            assert not f1 & 4 or n1 in (2, 3)
    assert accepted >= 1 and seeded < plain


def test_seed_on_held_out_systems_of_the_training_recipe(lib):
    """Systems of the training recipe with seeds training never used: every
    seeded root within 1 meV of the plain one and none lost (a failed seeded
    search falls back to the plain one), and fewer passes over the tables
    than the plain full-tolerance secant and than three network-free early
    stops with the same 1 meV tolerance, each charged its most favourable
    count: the plain search stopped at omega_2, the line estimate w_N of the
    same four samples followed by the seed's Newton step, omega_2 followed
    by that Newton step, and the seed's own base estimate w_C (the zero of
    the cubic through the four samples) followed by that Newton step, i.e.
    the seed without its network."""
    from paper_2305_15955_amd import seed_train
    rows = seed_train.held_out_evaluations(lib, dict(np.load(MODEL)), n_systems=12, max_mo=300)
    tot = rows.sum(axis=0)
    print(f"{len(rows)} states: passes plain {tot[0]:.0f}, seeded {tot[1]:.0f} "
          f"(accepted {rows[:, 2].mean():.2f}), early stop at omega_2 {tot[4]:.0f}, "
          f"line estimate + Newton {tot[5]:.0f}, omega_2 + Newton {tot[6]:.0f}, cubic + Newton {tot[7]:.0f}")
    assert np.all(np.isfinite(rows[:, 3])) and rows[:, 3].max() <= 1.0e-3 / synth.HARTREE_EV
    assert tot[1] < min(tot[0], tot[4], tot[5], tot[6], tot[7])


def test_trained_seed_gain_on_held_out_system(lib):
    """Same QP energies (<= 1 meV) with and without the seed on the
    600-orbital workload; report the passes."""
    assert os.path.exists(MODEL), "seed_model.npz missing (python -m paper_2305_15955_amd.seed_train)"
    mdl = np.load(MODEL)
    lib.cdwac_mlp_set_model(mdl["theta"], mdl["mu"], mdl["sd"], float(mdl["out_mu"]), float(mdl["out_sd"]))
    case = cases.workload("acene_nmo600")
    s = case.system
    sysc, keep = lib.make_system(s)
    res = {}
    for mlp in (False, True):
        prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                    prec="p64", use_mlp_seed=mlp, mlp_accept=1.0e-3 / synth.HARTREE_EV)
        lib.cdwac_prepare(sysc, prm)
        res[mlp] = lib.cdwac_qp(s.n_states)
    d = [abs(a["qp"] - b["qp"]) * synth.HARTREE_EV * 1e3 for a, b in zip(res[False], res[True])]
    r0 = np.mean([o["n_rounds"] for o in res[False]])
    r1 = np.mean([o["n_rounds"] for o in res[True]])
    acc = np.mean([(o["flags"] & 4) != 0 for o in res[True]])
    print(f"seed: mean passes {r0:.1f} -> {r1:.1f}, accepted {acc:.2f}, max |dQP| {max(d):.4f} meV")
    assert max(d) <= 1.0


def test_zero_network_seed_changes_nothing(lib):
    """With every weight of the network zero the seed is the cubic estimate
    w_C of the four samples (out_mu = 0, out_sd = 1); with mlp_accept = 0 it
    is never accepted, and the secant continued from it reaches the roots of
    the plain search (1e-9 relative), with the same flags and no state
    flagged as seeded.  Ragged case, three states."""
    from paper_2305_15955_amd import cdwac
    case = cases.ragged()
    s = case.system
    sysc, keep = lib.make_system(s)
    lib.cdwac_mlp_set_model(np.zeros(cdwac.MLP_NPARAM), np.zeros(8), np.ones(8), 0.0, 1.0)
    res = {}
    for mlp in (False, True):
        prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                    prec="p64", use_mlp_seed=mlp, mlp_accept=0.0)
        res[mlp] = lib.cdwac_solve(sysc, prm)
    for a, b in zip(res[False], res[True]):
        assert abs(a["qp"] - b["qp"]) <= 1e-9 * abs(a["qp"]) and abs(a["z"] - b["z"]) <= 1e-6
        assert not b["flags"] & cdwac.FLAG_MLP_ACCEPTED and a["flags"] == b["flags"]


def test_zero_network_seed_is_the_cubic_estimate(lib):
    """The device's base estimate against the host's: with every weight zero
    (out_mu = 0) and an acceptance bound no f can exceed, every state whose
    Z at w_C is physical returns w_C itself after two passes; it agrees with
    seed_train.cubic_estimate from the same four self-energy samples to
    1e-12 relative.  Ragged case and the 60-orbital case, v^xc shifted."""
    from paper_2305_15955_amd import cdwac, seed_train
    lib.cdwac_mlp_set_model(np.zeros(cdwac.MLP_NPARAM), np.zeros(8), np.ones(8), 0.0, 1.0)
    n_checked = 0
    for case in (cases.ragged(), cases.workload("fp64_1core_nmo60")):
        s = case.system
        sysc, keep = lib.make_system(s)
        prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                    prec="p64", use_mlp_seed=True, mlp_accept=1.0e6)
        lib.cdwac_prepare(sysc, prm)
        _, _, sx, _ = lib.cdwac_w_table(s.n_states, s.n_mo, len(case.freq), len(case.ref_re))
        eps_n = s.eps[s.state_idx]
        sig4 = seed_train.samples(lib, eps_n)
        for sh in (-0.2, 0.0, 0.15):
            vxc = sx + sh
            wl = seed_train.line_estimate(eps_n, vxc, sig4, case.lo, case.hi)
            wc = seed_train.cubic_estimate(eps_n, vxc, sig4, case.lo, case.hi, wl)
            for n, o in enumerate(lib.cdwac_qp(s.n_states, vxc=vxc)):
                if o["flags"] & cdwac.FLAG_MLP_ACCEPTED and o["n_rounds"] == 2:
                    assert abs(o["qp"] - wc[n]) <= 1e-12 * abs(wc[n]), (n, sh, o["qp"], wc[n], wl[n])
                    n_checked += 1
    print(f"{n_checked} states compared")
    assert n_checked >= 6
