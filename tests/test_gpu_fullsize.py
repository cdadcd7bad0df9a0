"""Parity at the full workload sizes, in the launch configuration bench.py times.

* 600-orbital workload (N_aux = 2000): the FP64 path against stored oracle
  results (tests/golden/acene_nmo600_oracle.json, written by
  tests/golden/make_golden.py from the oracle alone): QP energies to 1e-9
  relative, sampled W^c_nm and Sigma values; the fp16-split path to 1 meV.
* N_aux = 5000 workload (the benchmark): the FP64 path against stored
  oracle results (tests/golden/precision_naux5000_oracle.json) and the
  benchmark's configuration within 1 meV of them; sampled polarizability
  entries against the oracle's one-by-one definition, and properties that
  hold at any size (W^c(i w) <= 0 and non-decreasing in w, bounded by
  -|O^nm|^2, QP residual, Z in (0, 1]); the fp16-split QP energies within
  1 meV of the FP64 GPU path.
"""
import json
import os

import numpy as np
import pytest

import cases
from oracle import cdwac_ref as R
from paper_2305_15955_amd import synth
from paper_2305_15955_amd.cdwac import SKELETON_TOL

pytestmark = pytest.mark.gpu
MEV = 1e-3 / synth.HARTREE_EV
# The greedy Pade fit takes discrete decisions (argmax, stop test) on W values
# that the two sides compute to ~1e-13 relative; with 600 fits of 24 points a
# few decisions near the stop threshold can differ, which moves Sigma by up to
# ~3e-7 and one QP energy by ~4e-9 relative.  The small cases meet 1e-9.
QP_RTOL = 1e-8
SIGMA_RTOL = 1e-6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "acene_nmo600_oracle.json")


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2305_15955_amd import cdwac
    assert torch.cuda.is_available()
    c = cdwac.Cdwac(0)
    yield c
    c.close()


def prepare(lib, case, prec, sysc, freq_rank_tol=0.0):
    prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                pade_tol=1e-9, prec=prec, freq_rank_tol=freq_rank_tol)
    lib.cdwac_prepare(sysc, prm)
    return arrs


def test_acene_nmo600_against_stored_oracle(lib):
    g = json.load(open(GOLDEN))
    case = cases.workload("acene_nmo600")
    s = case.system
    sysc, keep = lib.make_system(s)
    prepare(lib, case, "p64", sysc)
    out = lib.cdwac_qp(s.n_states)
    w_im, w_re, sx, (m0, m1) = lib.cdwac_w_table(s.n_states, s.n_mo, len(case.freq), len(case.ref_re))
    for n, m, k, v in g["w_im"]:
        assert abs(w_im[n, m, k] - v) <= 1e-10 * np.max(np.abs(w_im[n, m])), (n, m, k)
    off = np.concatenate([[0], np.cumsum(m1 - m0)])
    for n, m, j, vr, vi in g["w_re"]:
        assert m0[n] <= m < m1[n]
        got = w_re[off[n] + m - m0[n], j]
        assert abs(got - (vr + 1j * vi)) <= 1e-10 * np.max(np.abs(w_re[off[n] + m - m0[n]]))
    for n in range(s.n_states):
        assert out[n]["flags"] == g["flags"][n]
        print(n, out[n]["qp"], g["qp"][n], (out[n]["qp"] - g["qp"][n]) / abs(g["qp"][n]))
        assert abs(out[n]["qp"] - g["qp"][n]) <= QP_RTOL * abs(g["qp"][n]), n
        assert out[n]["sigma_x"] == pytest.approx(g["sigma_x"][n], rel=1e-12)
    oms = np.full((s.n_states, 3), np.nan)
    want = np.full((s.n_states, 3), np.nan)
    cnt = [0] * s.n_states
    for n, om, v in g["sigma"]:
        oms[n, cnt[n]] = om
        want[n, cnt[n]] = v
        cnt[n] += 1
    got = lib.cdwac_sigma(oms)
    np.testing.assert_allclose(got, want, rtol=SIGMA_RTOL)
    # reduced precision against the stored FP64 oracle, with every imaginary
    # node contracted and with the skeleton-node decomposition
    for prec, rank_tol in (("b16x3", 0.0), ("f16x3", 0.0), ("f16x3", 1e-10), ("f16", 1e-10),
                           ("f16", SKELETON_TOL["f16"])):
        prepare(lib, case, prec, sysc, rank_tol)
        out = lib.cdwac_qp(s.n_states)
        d = [(out[n]["qp"] - g["qp"][n]) / MEV for n in range(s.n_states)]
        print(prec, "rank_tol", rank_tol, "vs oracle (meV)", np.round(d, 4))
        assert max(abs(x) for x in d) <= 1.0, (prec, rank_tol, d)


FULLCD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "acene_nmo600_fullcd_oracle.json")


@pytest.mark.timeout(900)
def test_acene_nmo600_full_cd(lib):
    """The full-CD reference of the 600-orbital workload (Sec. 3.4, CD
    branch): cdwac_sigma_cd evaluates W directly at every residue
    |eps_m - omega| + i eta (about 100 per evaluation here).  Its
    self-energy at each state's CD-WAC root matches the oracle's stored
    full-CD value (tests/golden/acene_nmo600_fullcd_oracle.json, written by
    make_fullcd_golden.py from the oracle alone) to 1e-9 of |Sigma^x| +
    |Sigma|; the full-CD root, found by the secant rule of the library's
    root search over cdwac_sigma_cd (started at the CD-WAC root and 1 meV
    above it), lies within 5 meV of CD-WAC for every state, the agreement the
    paper's convergence study asks of CD-WAC (Sec. 5.1)."""
    if not os.path.exists(FULLCD):
        pytest.skip("stored full-CD oracle values not written yet")
    g = json.load(open(FULLCD))
    gw = json.load(open(GOLDEN))
    case = cases.workload("acene_nmo600")
    s = case.system
    sysc, keep = lib.make_system(s)
    prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                eta=g["eta"], prec="p64")
    for row in g["states"]:
        n = row["state"]
        sig, r_term, i_term, n_res = lib.cdwac_sigma_cd(sysc, prm, n, row["omega"])
        scale = abs(row["sigma_x"]) + abs(row["sigma"])
        print(f"state {n}: full-CD Sigma {sig:.12f} (oracle {row['sigma']:.12f}), {n_res} residues, "
              f"rel. diff {abs(sig - row['sigma']) / scale:.2e}", flush=True)
        assert n_res == row["n_residues"]
        assert abs(sig - row["sigma"]) <= 1e-9 * scale
        assert abs(r_term - row["r_term"]) <= 1e-9 * scale and abs(i_term - row["i_term"]) <= 1e-9 * scale
    errs = []
    for n in range(s.n_states):
        e_n = float(s.eps[s.state_idx[n]])
        sx = g["states"][n]["sigma_x"]
        f = lambda w: w - e_n - lib.cdwac_sigma_cd(sysc, prm, n, w)[0] + sx
        w0, w1 = gw["qp"][n], gw["qp"][n] + MEV
        f0, f1 = f(w0), f(w1)
        for _ in range(20):
            w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
            w0, f0, w1 = w1, f1, w2
            f1 = f(w1)
            if abs(w1 - w0) < 1e-10 and abs(f1) < 1e-9:
                break
        assert abs(f1) < 1e-9, (n, f1)
        errs.append((gw["qp"][n] - w1) / MEV)
        print(f"state {n}: full-CD root {w1 * synth.HARTREE_EV:.6f} eV, CD-WAC - full CD = {errs[-1]:.4f} meV",
              flush=True)
    assert max(abs(e) for e in errs) <= 5.0, errs


GOLDEN5000 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision_naux5000_oracle.json")


@pytest.mark.timeout(600)
def test_naux5000_against_stored_oracle(lib):
    """The benchmark's workload (N_aux = 5000, 16 core states) against stored
    oracle results (tests/golden/precision_naux5000_oracle.json, written by
    tests/golden/make_golden.py from the oracle alone): the FP64 path's
    sampled W to 1e-10, QP energies to 1e-8 relative and Sigma samples; the
    benchmark's stated configuration (bf16 split at every imaginary node,
    with and without the learned seed) and the faster variants within 1 meV
    of the oracle for every state."""
    if not os.path.exists(GOLDEN5000):
        pytest.skip("stored oracle values for precision_naux5000 not written yet (tests/golden/make_golden.py)")
    import torch
    g = json.load(open(GOLDEN5000))
    case = cases.workload("precision_naux5000")
    s = case.system
    dev = torch.device("cuda", 0)
    o_ia = torch.from_numpy(s.o_ia).to(dev)
    o_nm = torch.from_numpy(s.o_nm).to(dev)
    sysc, keep = lib.make_system(s, o_ia_dev=o_ia, o_nm_dev=o_nm)
    print("workload on the device", flush=True)
    prepare(lib, case, "p64", sysc)
    out = lib.cdwac_qp(s.n_states)
    w_im, w_re, sx, (m0, m1) = lib.cdwac_w_table(s.n_states, s.n_mo, len(case.freq), len(case.ref_re))
    for n, m, k, v in g["w_im"]:
        assert abs(w_im[n, m, k] - v) <= 1e-10 * np.max(np.abs(w_im[n, m])), (n, m, k)
    off = np.concatenate([[0], np.cumsum(m1 - m0)])
    for n, m, j, vr, vi in g["w_re"]:
        if m0[n] <= m < m1[n]:
            got = w_re[off[n] + m - m0[n], j]
            assert abs(got - (vr + 1j * vi)) <= 1e-10 * np.max(np.abs(w_re[off[n] + m - m0[n]])), (n, m, j)
    for n in range(s.n_states):
        assert out[n]["flags"] == g["flags"][n]
        assert abs(out[n]["qp"] - g["qp"][n]) <= QP_RTOL * abs(g["qp"][n]), (n, out[n]["qp"], g["qp"][n])
        assert out[n]["sigma_x"] == pytest.approx(g["sigma_x"][n], rel=1e-12)
    oms = np.full((s.n_states, 3), np.nan)
    want = np.full((s.n_states, 3), np.nan)
    cnt = [0] * s.n_states
    for n, om, v in g["sigma"]:
        oms[n, cnt[n]] = om
        want[n, cnt[n]] = v
        cnt[n] += 1
    np.testing.assert_allclose(lib.cdwac_sigma(oms), want, rtol=SIGMA_RTOL)
    print("FP64 path agrees with the stored oracle", flush=True)
    mdl = np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                               "paper_2305_15955_amd", "seed_model.npz"))
    lib.cdwac_mlp_set_model(mdl["theta"], mdl["mu"], mdl["sd"], float(mdl["out_mu"]), float(mdl["out_sd"]))
    # the benchmark accepts a seed at |f| <= 0.1 meV; 1 meV (the bar) is shown too
    for key, prec, rank_tol, accept in (("b16x3 (stated configuration)", "b16x3", 0.0, None),
                                        ("b16x3 + learned seed (benchmark)", "b16x3", 0.0, 0.1 * MEV),
                                        ("b16x3 + learned seed accepted at 1 meV", "b16x3", 0.0, MEV),
                                        ("f16 every node", "f16", 0.0, None),
                                        ("f16 skeleton nodes", "f16", SKELETON_TOL["f16"], None)):
        prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                    pade_tol=1e-9, prec=prec, freq_rank_tol=rank_tol,
                                    use_mlp_seed=accept is not None, mlp_accept=accept or 0.0)
        lib.cdwac_prepare(sysc, prm)
        out = lib.cdwac_qp(s.n_states)
        d = np.array([(out[n]["qp"] - g["qp"][n]) / MEV for n in range(s.n_states)])
        print(f"{key}: vs oracle max {np.max(np.abs(d)):.4f} meV, mean {np.mean(np.abs(d)):.4f} meV", flush=True)
        assert np.max(np.abs(d)) <= 1.0, (key, d)


def test_naux5000_sampled_pi_and_properties(lib):
    import torch
    case = cases.workload("precision_naux5000")
    s = case.system
    dev = torch.device("cuda", 0)
    o_ia = torch.from_numpy(s.o_ia).to(dev)
    o_nm = torch.from_numpy(s.o_nm).to(dev)
    sysc, keep = lib.make_system(s, o_ia_dev=o_ia, o_nm_dev=o_nm)
    rng = np.random.default_rng(3)
    pairs = [(int(p), int(q)) for p, q in zip(rng.integers(0, s.n_aux, 12), rng.integers(0, s.n_aux, 12))]
    pairs += [(0, 0), (s.n_aux - 1, s.n_aux - 1), (s.n_aux - 1, 0)]
    zs = [1j * case.freq[5], case.ref_re[4] + 1e-3j]
    # fp16 split: products exact to ~2^-22, but FP32 accumulation over
    # K / 16 = 19 532 matrix-core steps gives ~sqrt(19 532) * 2^-24 = 8e-6
    # relative to the largest partial sums
    for prec, tol in (("p64", 1e-12), ("f16x3", 3e-5), ("f16", 3e-5)):
        pis = lib.cdwac_polarizability(sysc, zs, prec=prec)
        for j, z in enumerate(zs):
            ref = R.polarizability_entries(s.o_ia, s.eps, s.n_occ, z, s.spin, pairs)
            got = np.array([pis[j][p, q] for p, q in pairs])
            scale = np.max(np.abs(np.diagonal(pis[j])))
            print(prec, j, "max |dPi| / max|diag|", np.max(np.abs(got - ref)) / scale)
            assert np.max(np.abs(got - ref)) <= tol * scale, (prec, j)
        del pis
    qp = {}
    evals = {}
    # r: skeleton nodes at 1e-10; s: at the mode's own tolerance (the benchmark's setting)
    runs = (("f16x3", "f16x3", 0.0), ("f16x3r", "f16x3", 1e-10), ("f16r", "f16", 1e-10),
            ("f16s", "f16", SKELETON_TOL["f16"]), ("p64", "p64", 0.0))
    for key, p, rank_tol in runs:
        prepare(lib, case, p, sysc, rank_tol)
        out = lib.cdwac_qp(s.n_states)
        qp[key] = np.array([o["qp"] for o in out])
        evals[key] = [o["n_rounds"] for o in out]
        prec = key
        for n, o in enumerate(out):
            # a root whose Z falls outside (0, 1] is re-found by the scan (flag 2)
            assert not o["flags"] & 1 and o["z"] > 0.5 and abs(o["residual"]) < 1e-8, (prec, n, o)
        if prec == "p64":
            w_im, _, _, _ = lib.cdwac_w_table(s.n_states, s.n_mo, len(case.freq), len(case.ref_re))
            norm2 = np.einsum("spm,spm->sm", s.o_nm, s.o_nm)
            assert np.all(w_im <= 1e-15)
            assert np.all(w_im >= -norm2[:, :, None] * (1 + 1e-9))
            assert np.all(np.diff(w_im, axis=2) >= -1e-13)
    for key in ("f16x3", "f16x3r", "f16r", "f16s"):
        err = np.abs(qp[key] - qp["p64"]) / MEV
        print(key, "vs p64 (meV):", np.round(err, 4))
        assert np.max(err) <= 1.0
    # the learned seed on the same workload
    mdl = np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                               "paper_2305_15955_amd", "seed_model.npz"))
    lib.cdwac_mlp_set_model(mdl["theta"], mdl["mu"], mdl["sd"], float(mdl["out_mu"]), float(mdl["out_sd"]))
    prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                pade_tol=1e-9, prec="f16x3", use_mlp_seed=True, mlp_accept=MEV)
    lib.cdwac_prepare(sysc, prm)
    out = lib.cdwac_qp(s.n_states)
    ev = [o["n_rounds"] for o in out]
    d = np.abs(np.array([o["qp"] for o in out]) - qp["f16x3"]) / MEV
    print("passes plain", evals["f16x3"], "seeded", ev, "max |dQP| meV", np.round(d, 4))
    for n, o in enumerate(out):
        if o["flags"] & R.FLAG_MLP_ACCEPTED:
            # accepted seed: |f(seed)| <= 1 meV, so within ~1 meV / Z of the root
            assert abs(o["residual"]) <= MEV and d[n] <= 1.1, (n, o)
        else:
            # rejected seed: the secant from it reaches the plain path's root
            assert d[n] <= 1e-8 * abs(qp["f16x3"][n]) / MEV, (n, o)


def test_deploy_naux6600_learned_seed(lib):
    """The learned seed at its deployment size (N_mo = 2000, N_aux = 6600, 24
    core states; O^{ia} is 29 GB): the benchmark mode (Pi in one fp16
    product, W in the fp16 split, skeleton nodes) with and without the seed,
    against the fp16 split (FP32-level Pi) without it.  Every root has Z in
    (0.5, 1] and |f| <= 1e-8 Ha, or <= 1 meV where the seed is accepted (the
    secant is the fallback and decides); all states within 1 meV of the
    reference; an accepted seed ends the search after 2 passes over the
    tables (3 where the Newton step from it is accepted).  Sampled Pi entries against the oracle's one-by-one definition."""
    import torch
    case = cases.workload("mlp_deploy_naux6600")
    s = case.system
    print("deploy workload drawn", flush=True)
    dev = torch.device("cuda", 0)
    o_ia = torch.from_numpy(s.o_ia).to(dev)
    o_nm = torch.from_numpy(s.o_nm).to(dev)
    sysc, keep = lib.make_system(s, o_ia_dev=o_ia, o_nm_dev=o_nm)
    rng = np.random.default_rng(6)
    pairs = [(int(p), int(q)) for p, q in zip(rng.integers(0, s.n_aux, 8), rng.integers(0, s.n_aux, 8))]
    pairs += [(0, 0), (s.n_aux - 1, s.n_aux - 1)]
    zs = [1j * case.freq[9]]
    for prec, tol in (("p64", 1e-12), ("f16", 3e-5)):
        pis = lib.cdwac_polarizability(sysc, zs, prec=prec)
        ref = R.polarizability_entries(s.o_ia, s.eps, s.n_occ, zs[0], s.spin, pairs)
        got = np.array([pis[0][p, q] for p, q in pairs])
        scale = np.max(np.abs(np.diagonal(pis[0])))
        print(prec, "max |dPi| / max|diag|", np.max(np.abs(got - ref)) / scale, flush=True)
        assert np.max(np.abs(got - ref)) <= tol * scale, prec
        del pis
    mdl = np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                               "paper_2305_15955_amd", "seed_model.npz"))
    lib.cdwac_mlp_set_model(mdl["theta"], mdl["mu"], mdl["sd"], float(mdl["out_mu"]), float(mdl["out_sd"]))
    res = {}
    for key, prec, mlp in (("ref", "f16x3", False), ("plain", "f16", False), ("seeded", "f16", True)):
        prm, arrs = lib.make_params(case.freq, case.weight, case.ref_im, case.ref_re, case.lo, case.hi,
                                    pade_tol=1e-9, prec=prec, use_mlp_seed=mlp, mlp_accept=MEV,
                                    freq_rank_tol=1e-10)
        lib.cdwac_prepare(sysc, prm)
        res[key] = lib.cdwac_qp(s.n_states)
        print(key, "passes", [o["n_rounds"] for o in res[key]], flush=True)
    qref = np.array([o["qp"] for o in res["ref"]])
    for key in ("plain", "seeded"):
        for n, o in enumerate(res[key]):
            accepted = bool(o["flags"] & R.FLAG_MLP_ACCEPTED)
            assert not o["flags"] & R.FLAG_NOROOT and 0.5 < o["z"] <= 1.0, (key, n, o)
            assert abs(o["residual"]) <= (MEV if accepted else 1e-8), (key, n, o)
            assert abs(o["qp"] - qref[n]) <= MEV, (key, n, o["qp"], qref[n])
    n_acc = sum(bool(o["flags"] & R.FLAG_MLP_ACCEPTED) for o in res["seeded"])
    mean_plain = np.mean([o["n_rounds"] for o in res["plain"]])
    mean_seeded = np.mean([o["n_rounds"] for o in res["seeded"]])
    print(f"seed accepted for {n_acc} of {s.n_states}; mean passes {mean_plain:.2f} -> {mean_seeded:.2f}")
    for o1 in res["seeded"]:
        if o1["flags"] & R.FLAG_MLP_ACCEPTED:
            assert o1["n_rounds"] in (2, 3)
