"""Trains the learned QP-root seed on solves the method itself produces.

Data: many seeded systems (60-700 orbitals, log-uniform, N_aux = 3.3 N_mo,
1-8 core states, 32 or 64 imaginary nodes, 16 or 24 Pade points, the
screening and core-coupling recipe of ``synth``).  Each
system is prepared once on the GPU (FP64 contractions); the QP root is solved
for a range of v^xc shifts, which re-uses the prepared tables.  Only roots
found by the plain secant (no fallback) are kept as targets.

The seed starts where the root search starts: f(omega) = omega - eps_n -
Sigma(omega) + v^xc at omega_0 = eps_n and at omega_1 = omega_0 - f(omega_0),
and the secant step omega_2 they give.  Features (the library's order):
eps_n, eps_F, Sigma^x - v^xc, Re Sigma^c(omega_0), Re Sigma^c(omega_1),
omega_1 - omega_0, f(omega_1), omega_2 - omega_1; target omega* - omega_2.
The seed thus costs no self-energy evaluation beyond those two.  Training
runs on the GPU through cdwac_mlp_train (the library's forward, backward and
Adam kernels).

Usage:  python -m paper_2305_15955_amd.seed_train --out seed_model.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2305_15955_amd import cdwac, grids, synth  # noqa: E402

SHIFT = 0.3     # Ha, largest v^xc shift of the training solves


def first_steps(eps_n, vxc, sig0, sig1_fn):
    """omega_1, f(omega_0), f(omega_1), omega_2 of the root search."""
    f0 = eps_n - eps_n - sig0 + vxc
    w1 = eps_n - f0
    sig1 = sig1_fn(w1)
    f1 = w1 - eps_n - sig1 + vxc
    w2 = np.where(f1 != f0, w1 - f1 * (w1 - eps_n) / np.where(f1 != f0, f1 - f0, 1.0), w1)
    return w1, f0, f1, sig1, w2


def features(eps_n, eps_f, sx, vxc, sig0, sig1, w1, f1, w2):
    return np.array([eps_n, eps_f, sx - vxc, sig0 - sx, sig1 - sx, w1 - eps_n, f1, w2 - w1])


def sample_setting(rng, system_seed, max_mo=700):
    """One system of the training recipe and its frequency setting."""
    n_mo = int(round(math.exp(rng.uniform(math.log(60), math.log(max_mo)))))
    n_occ = max(3, int(round(n_mo / 6)))
    n_core = int(rng.integers(1, 9))
    n_core = min(n_core, n_occ - 1)
    n_aux = int(round(3.3 * n_mo))
    k = n_occ * (n_mo - n_occ)
    sigma = math.sqrt(synth.SCREENING / k)
    kappa = float(rng.uniform(0.12, 0.3))
    s = synth.make_system(n_mo, n_occ, n_aux, n_core, sigma, kappa=kappa, seed=system_seed)
    n_freq = int(rng.choice([32, 64]))
    n_half = int(rng.choice([8, 12]))
    freq, wts = grids.gauss_legendre_imag(n_freq)
    lo, hi = grids.windows(s.eps, s.state_idx, 30.0)
    ref_im = grids.imag_ref_indices(n_freq, n_half)
    ref_re = grids.generic_refs(s.eps, s.n_occ, lo, n_half)
    return s, freq, wts, ref_im, ref_re, lo, hi


def generate(lib, n_systems, shifts_per_system, seed, log=print):
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    t0 = time.time()
    for j in range(n_systems):
        s, freq, wts, ref_im, ref_re, lo, hi = sample_setting(rng, 10_000 + seed + j)
        n_freq = len(freq)
        sysc, keep = lib.make_system(s)
        prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64")
        lib.cdwac_prepare(sysc, prm)
        eps_n = s.eps[s.state_idx]
        eps_f = grids.midgap(s.eps, s.n_occ)
        sig0 = lib.cdwac_sigma(eps_n[:, None])[:, 0]
        _, _, sx, _ = lib.cdwac_w_table(s.n_states, s.n_mo, n_freq, len(ref_re))
        for q in range(shifts_per_system):
            shift = 0.0 if q == 0 else float(rng.uniform(-SHIFT, SHIFT))
            vxc = sx + shift
            w1, f0, f1, sig1, w2 = first_steps(eps_n, vxc, sig0, lambda w: lib.cdwac_sigma(w[:, None])[:, 0])
            out = lib.cdwac_qp(s.n_states, vxc=vxc)
            for n, o in enumerate(out):
                if o["flags"] != 0 or not np.isfinite(o["qp"]) or not (lo[n] <= w1[n] <= hi[n]):
                    continue
                xs.append(features(eps_n[n], eps_f, sx[n], vxc[n], sig0[n], sig1[n], w1[n], f1[n], w2[n]))
                ys.append(o["qp"] - w2[n])
        if (j + 1) % 50 == 0:
            log(f"systems {j + 1}/{n_systems}: {len(ys)} samples ({time.time() - t0:.0f} s)")
    return np.array(xs), np.array(ys)


def held_out_evaluations(lib, model, n_systems=24, shifts=(-0.2, 0.0, 0.2), seed=900_000, max_mo=400,
                         accept=1.0e-3 / synth.HARTREE_EV):
    """Self-energy evaluations of the root search with and without the seed on
    systems of the training recipe that training never saw (other seeds).

    Returns per-state rows (plain evals, seeded evals, seed accepted, |dQP|,
    evals of the plain search that also stops at omega_2 when |f(omega_2)|
    is within the same tolerance) over the states whose plain search needed
    no fallback.  The last column is the network-free version of the early
    stop: what the seed gains is measured against it as well."""
    lib.cdwac_mlp_set_model(model["theta"], model["mu"], model["sd"], float(model["out_mu"]),
                            float(model["out_sd"]))
    rng = np.random.default_rng(seed)
    rows = []
    for j in range(n_systems):
        s, freq, wts, ref_im, ref_re, lo, hi = sample_setting(rng, seed + j, max_mo)
        sysc, keep = lib.make_system(s)
        res = {}
        for mlp in (False, True):
            prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64", use_mlp_seed=mlp,
                                        mlp_accept=accept)
            lib.cdwac_prepare(sysc, prm)
            _, _, sx, _ = lib.cdwac_w_table(s.n_states, s.n_mo, len(freq), len(ref_re))
            res[mlp] = [lib.cdwac_qp(s.n_states, vxc=sx + sh) for sh in shifts]
        eps_n = s.eps[s.state_idx]
        sig0 = lib.cdwac_sigma(eps_n[:, None])[:, 0]
        for q, (q0, q1) in enumerate(zip(res[False], res[True])):
            vxc = sx + shifts[q]
            _, _, _, _, w2 = first_steps(eps_n, vxc, sig0, lambda w: lib.cdwac_sigma(w[:, None])[:, 0])
            f2 = w2 - eps_n - lib.cdwac_sigma(w2[:, None])[:, 0] + vxc
            for n, (o0, o1) in enumerate(zip(q0, q1)):
                if o0["flags"] != 0:
                    continue
                stop2 = 5 if abs(f2[n]) <= accept else o0["n_evals"]
                rows.append((o0["n_evals"], o1["n_evals"], bool(o1["flags"] & 4), abs(o1["qp"] - o0["qp"]), stop2))
    return np.array(rows, dtype=np.float64).reshape(-1, 5)


def init_params(rng):
    parts = []
    for shape in ((64, 8), (64,), (64, 64), (64,), (1, 64), (1,)):
        if len(shape) == 2:
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--systems", type=int, default=700)
    ap.add_argument("--shifts", type=int, default=12)
    ap.add_argument("--epochs", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="seed_model.npz")
    args = ap.parse_args()

    lib = cdwac.Cdwac(0)
    x, y = generate(lib, args.systems, args.shifts, args.seed, log=lambda m: print(m, flush=True))
    rng = np.random.default_rng(args.seed)
    perm = rng.permutation(len(y))
    n_val = max(1, len(y) // 10)
    val, tr = perm[:n_val], perm[n_val:]
    mu = x[tr].mean(axis=0)
    sd = x[tr].std(axis=0)
    sd[sd < 1e-12] = 1.0
    out_mu, out_sd = float(y[tr].mean()), float(y[tr].std())
    xn = ((x - mu) / sd).astype(np.float32)
    yn = ((y - out_mu) / out_sd).astype(np.float32)
    theta0 = init_params(rng)
    t0 = time.time()
    theta, curve = lib.cdwac_mlp_train(theta0, xn[tr], yn[tr], args.epochs, args.batch, args.lr, seed=args.seed)
    t_train = time.time() - t0
    pred = lib.cdwac_mlp_forward(theta, xn[val]).astype(np.float64) * out_sd + out_mu
    err_mev = np.abs(pred - y[val]) * synth.HARTREE_EV * 1e3
    report = dict(samples=int(len(y)), train=int(len(tr)), val=int(len(val)), epochs=args.epochs,
                  train_s=t_train, loss_first=float(curve[0]), loss_last=float(curve[-1]),
                  val_mae_mev=float(err_mev.mean()), val_p90_mev=float(np.percentile(err_mev, 90)),
                  val_within_1mev=float(np.mean(err_mev <= 1.0)))
    model = dict(theta=theta.astype(np.float32), mu=mu.astype(np.float32), sd=sd.astype(np.float32),
                 out_mu=np.float32(out_mu), out_sd=np.float32(out_sd))
    rows = held_out_evaluations(lib, model)
    report.update(held_out_states=int(len(rows)), held_out_evals_plain=int(rows[:, 0].sum()),
                  held_out_evals_seeded=int(rows[:, 1].sum()), held_out_evals_stop_at_omega2=int(rows[:, 4].sum()),
                  held_out_accepted=float(rows[:, 2].mean()),
                  held_out_max_dqp_mev=float(rows[:, 3].max() * synth.HARTREE_EV * 1e3))
    print(json.dumps(report), flush=True)
    np.savez(args.out, theta=theta.astype(np.float32), mu=mu.astype(np.float32), sd=sd.astype(np.float32),
             out_mu=np.float32(out_mu), out_sd=np.float32(out_sd), curve=curve,
             report=json.dumps(report))
    lib.close()


if __name__ == "__main__":
    main()
