"""The uneven batch through cdwac_solve_batch: many independent systems of
different sizes, the greedy fits of all (n, m) pairs of all systems in one
launch and the QP roots of all states in one launch.

* A small FP64 batch: every QP energy equals the one-system path bit for bit
  (same kernels on the same data) and the oracle to 1e-9 relative.
* The 48-system batch (N_mo uniform in [100, 1200], N_aux = 3.3 N_mo, 1-12
  core states, 48 imaginary nodes, 24 Pade points): the fp16-split path
  (FP32-level Pi and W) at every imaginary node, with the near-real planes
  of Pi on the FP64 path; the smallest and the largest system against the
  one-system path bit for bit, every state's residual and Z, and the five
  smallest systems against the oracle within 1 meV.

The Pade set has 24 points (12 near-real, 12 imaginary).  With 16 the
continuation of some of these systems is not converged: the greedy fit uses
every point without meeting its tolerance, and a 1e-7 relative perturbation
of W (the rounding the 16-bit W contraction leaves) moves the oracle's own
roots by up to 3.9 meV (158-orbital system); with 24 points by at most
0.29 meV.  16-bit Pi at the near-real points leaves W there good to only
~1e-4 (RPA poles of ~10 Ha within eta_ref = 1e-3 of the points); with those
planes on the FP64 path, W keeps <= 2e-7 of the state's largest value.
"""
import json
import math
import os

import numpy as np
import pytest

import cases
from oracle import cdwac_ref as R
from paper_2305_15955_amd import grids, synth

pytestmark = pytest.mark.gpu
MEV = 1e-3 / synth.HARTREE_EV


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2305_15955_amd import cdwac
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = cdwac.Cdwac(0)
    yield c
    c.close()


def batch_cases(specs, n_freq=48, n_pade=24):
    out = []
    for sp in specs:
        s = synth.make_system(sp["n_mo"], sp["n_occ"], sp["n_aux"], sp["n_core"], sp["sigma"], seed=sp["seed"])
        out.append(cases.build(s, n_freq, n_pade // 2, n_pade - n_pade // 2, 30.0, name=f"batch_nmo{sp['n_mo']}"))
    return out


def descriptors(lib, cs, prec, **kw):
    systems, params, keep = [], [], []
    for c in cs:
        sysc, k1 = lib.make_system(c.system)
        prm, k2 = lib.make_params(c.freq, c.weight, c.ref_im, c.ref_re, c.lo, c.hi, eta=c.eta,
                                  eta_ref=c.eta_ref, pade_tol=c.pade_tol, prec=prec, **kw)
        systems.append(sysc)
        params.append(prm)
        keep.append((k1, k2))
    return systems, params, keep


def same_result(a, b):
    for x, y in zip(a, b):
        for key in ("qp", "z", "residual", "sigma_c"):
            if not (x[key] == y[key] or (math.isnan(x[key]) and math.isnan(y[key]))):
                return False
        if x["flags"] != y["flags"] or x["n_evals"] != y["n_evals"]:
            return False
    return True


def test_small_batch_fp64(lib):
    specs = [dict(n_mo=n, n_occ=max(2, round(n / 6)), n_aux=round(3.3 * n), n_core=c,
                  sigma=math.sqrt(synth.SCREENING / (round(n / 6) * (n - round(n / 6)))), seed=700 + j)
             for j, (n, c) in enumerate(((40, 2), (75, 1), (52, 4), (90, 3), (61, 2)))]
    cs = batch_cases(specs, n_freq=32)
    systems, params, keep = descriptors(lib, cs, "p64", fit_all=True)
    res = lib.cdwac_solve_batch(systems, params)
    assert [len(r) for r in res] == [c.system.n_states for c in cs]
    for j, c in enumerate(cs):
        one = lib.cdwac_solve(systems[j], params[j])
        assert same_result(res[j], one), j
        for n, r in enumerate(cases.oracle(c).solve_all()):
            assert res[j][n]["flags"] == r[3], (j, n)
            if not r[3] & R.FLAG_NOROOT:
                assert abs(res[j][n]["qp"] - r[0]) <= 1e-9 * abs(r[0]), (j, n, res[j][n]["qp"], r[0])


def test_batch_rejects_mixed_pade_sizes(lib):
    from paper_2305_15955_amd import cdwac
    specs = [dict(n_mo=40, n_occ=7, n_aux=132, n_core=2, sigma=0.03, seed=1),
             dict(n_mo=50, n_occ=8, n_aux=165, n_core=1, sigma=0.03, seed=2)]
    cs = batch_cases(specs, n_freq=32)
    cs[1].ref_re = cs[1].ref_re[:-1]
    systems, params, keep = descriptors(lib, cs, "p64")
    with pytest.raises(cdwac.CdwacError) as e:
        lib.cdwac_solve_batch(systems, params)
    assert e.value.code == cdwac.CDWAC_EINVAL


def test_small_batch_fp64_quad_limit(lib):
    """The analytic a_m -> 0 limit in a batch, switched on for every other
    system: each system bit-identical to its own cdwac_solve with the same
    parameters, and the limit's systems within 1e-9 of the oracle with the
    limit."""
    specs = [dict(n_mo=n, n_occ=max(2, round(n / 6)), n_aux=round(3.3 * n), n_core=c,
                  sigma=math.sqrt(synth.SCREENING / (round(n / 6) * (n - round(n / 6)))), seed=700 + j)
             for j, (n, c) in enumerate(((40, 2), (75, 1), (52, 4), (90, 3), (61, 2)))]
    cs = batch_cases(specs, n_freq=32)
    systems, params, keep = [], [], []
    for j, c in enumerate(cs):
        sy, pr, kp = descriptors(lib, [c], "p64", fit_all=True, quad_limit=(j % 2 == 0))
        systems += sy
        params += pr
        keep += kp
    res = lib.cdwac_solve_batch(systems, params)
    for j, c in enumerate(cs):
        assert same_result(res[j], lib.cdwac_solve(systems[j], params[j])), j
        if j % 2 == 0:
            for n, r in enumerate(cases.oracle(c, fit_all=True, quad_limit=True).solve_all()):
                assert res[j][n]["flags"] == r[3], (j, n)
                if not r[3] & R.FLAG_NOROOT:
                    assert abs(res[j][n]["qp"] - r[0]) <= 1e-9 * abs(r[0]), (j, n, res[j][n]["qp"], r[0])


def test_uneven_batch_48_systems(lib):
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.batch_specs()
    order = np.argsort([sp["n_mo"] for sp in specs])
    small = set(int(j) for j in order[:5])
    # 72 GB of O^{ia} in all: drawn on 8 threads (one generator per system),
    # moved to the device system by system; only the oracle's three keep a
    # host copy
    systems, params, keep, cs = [], [], [], []
    with ThreadPoolExecutor(8) as ex:
        for j, c in enumerate(ex.map(lambda sp: batch_cases([sp])[0], specs)):
            sy, pr, kp = descriptors(lib, [c], "f16x3", fit_all=True, near_real_f64=True)
            systems += sy
            params += pr
            keep += kp
            if j not in small:
                c.system.o_ia = None
                c.system.o_nm = None
            cs.append(c)
    print("batch staged on the device", flush=True)
    import time
    t = time.perf_counter()
    res = lib.cdwac_solve_batch(systems, params)
    print(f"cdwac_solve_batch: 48 systems in {time.perf_counter() - t:.2f} s", flush=True)
    n_states = sum(c.system.n_states for c in cs)
    assert sum(len(r) for r in res) == n_states == sum(sp["n_core"] for sp in specs)
    noroot = [(j, n) for j, r in enumerate(res) for n, x in enumerate(r) if x["flags"] & R.FLAG_NOROOT]
    print("states", n_states, "no root:", noroot, flush=True)
    # system 37 (202 orbitals, 10 cores within 0.82 eV): the roots of states 6
    # and 8 would lie inside the 1 eV core band, next to other cores' Kohn-Sham
    # levels; there the residue term switches W_nm off (Eq. ffact) and f jumps
    # across zero, which the root search rejects as a step, not a root (the
    # oracle agrees, below)
    assert noroot == [(37, 6), (37, 8)]
    for j, r in enumerate(res):
        for n, x in enumerate(r):
            if x["flags"] & R.FLAG_NOROOT:
                continue
            assert abs(x["residual"]) < 1e-8 and 0.0 < x["z"] <= 1.0, (j, n, x)
            assert cs[j].lo[n] <= x["qp"] <= cs[j].hi[n]
    # what the root search met where it found no root: f on the scan grid
    for j, n in noroot:
        lib.cdwac_prepare(systems[j], params[j])
        xs = np.arange(cs[j].lo[n], cs[j].hi[n], 0.01)
        om = np.full((cs[j].system.n_states, len(xs)), np.nan)
        om[:, :] = [np.clip(xs, cs[j].lo[k], cs[j].hi[k]) for k in range(cs[j].system.n_states)]
        sig = lib.cdwac_sigma(om)[n]
        one = lib.cdwac_qp(cs[j].system.n_states)[n]
        e_n = float(cs[j].system.eps[cs[j].system.state_idx[n]])
        f = xs - e_n - sig + one["sigma_x"]
        ups = [k for k in range(len(xs) - 1) if f[k] <= 0 < f[k + 1]]
        print(f"no root: system {j} (N_mo {cs[j].system.n_mo}, {cs[j].system.n_states} cores) state {n}: "
              f"upward sign changes of f at {[round(xs[k] * synth.HARTREE_EV, 3) for k in ups]} eV with "
              f"|f| {[(round(abs(f[k]), 4), round(abs(f[k + 1]), 4)) for k in ups]} Ha; "
              f"core KS levels {np.round(cs[j].system.eps[:cs[j].system.n_states] * synth.HARTREE_EV, 3).tolist()} eV",
              flush=True)
    for j in (order[0], order[-1]):
        assert same_result(res[j], lib.cdwac_solve(systems[j], params[j])), j
    # with the analytic limit of the integral term (quad_limit) the step at the
    # other cores' levels is gone: system 37 again, in a batch with the two
    # smallest systems, has a root for every state, within 1 meV of the
    # oracle with the same limit
    sub = [37, int(order[0]), int(order[1])]
    sy, pr, kp = descriptors(lib, [cs[j] for j in sub], "f16x3", fit_all=True, near_real_f64=True, quad_limit=True)
    res_l = lib.cdwac_solve_batch(sy, pr)
    o37 = cases.oracle(cs[37], fit_all=True, quad_limit=True)
    for n, x in enumerate(res_l[0]):
        r = o37.solve(n)
        print(f"system 37 state {n} with the limit: {x['qp'] * synth.HARTREE_EV:.4f} eV, Z {x['z']:.3f}, "
              f"{abs(x['qp'] - r[0]) / MEV:.4f} meV from the oracle", flush=True)
        assert not x["flags"] & R.FLAG_NOROOT and r[3] == 0 and 0.9 < x["z"] <= 1.0, (n, x, r)
        assert abs(x["qp"] - r[0]) <= MEV, (n, x["qp"], r[0])
    del sy, pr, kp
    # every system whose oracle QP energies are stored (tests/golden/batch48_oracle.json,
    # written by tests/golden/make_batch_golden.py from the smallest system up)
    stored = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch48_oracle.json")
    if os.path.exists(stored):
        g = json.load(open(stored))
        worst, n_cmp = 0.0, 0
        for key, sy in g["systems"].items():
            j = int(key)
            assert sy["n_mo"] == specs[j]["n_mo"] and len(sy["qp"]) == len(res[j]), j
            for n, x in enumerate(res[j]):
                assert bool(x["flags"] & R.FLAG_NOROOT) == bool(sy["flags"][n] & R.FLAG_NOROOT), (j, n)
                if not sy["flags"][n] & R.FLAG_NOROOT:
                    err = abs(x["qp"] - sy["qp"][n])
                    worst = max(worst, err)
                    n_cmp += 1
                    assert err <= MEV, (j, n, x["qp"], sy["qp"][n], err / MEV)
        print(f"stored oracle values: {len(g['systems'])} systems, {n_cmp} states within "
              f"{worst / MEV:.4f} meV", flush=True)
    for j in order[:5]:
        o = cases.oracle(cs[j])
        for n, r in enumerate(o.solve_all()):
            assert res[j][n]["flags"] & R.FLAG_NOROOT == r[3] & R.FLAG_NOROOT, (j, n)
            if not r[3] & R.FLAG_NOROOT:
                err = abs(res[j][n]["qp"] - r[0])
                print(f"system {j} (N_mo {cs[j].system.n_mo}) state {n}: {err / MEV:.4f} meV from the oracle",
                      flush=True)
                assert err <= MEV, (j, n, res[j][n]["qp"], r[0])
