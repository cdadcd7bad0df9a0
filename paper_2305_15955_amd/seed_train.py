"""Trains the learned QP-root seed on solves the method itself produces.

Data: many seeded systems (60-700 orbitals, log-uniform, N_aux = 3.3 N_mo,
1-8 core states, 32 or 64 imaginary nodes, 16 or 24 Pade points, the
screening and core-coupling recipe of ``synth``).  Each
system is prepared once on the GPU (FP64 contractions); the QP root is solved
for a range of v^xc shifts, which re-uses the prepared tables.  Only roots
found by the plain secant (no fallback) are kept as targets.

The seed costs one pass over the tables: f(omega) = omega - eps_n -
Sigma(omega) + v^xc at the four points w_j = eps_n + d_j, d = (-0.1, -0.05,
0.05, 0.1) Ha, evaluated together.  The least-squares line through
(d_j, f(w_j)) gives w_N (its zero; eps_n - mean f if the slope is not
positive; clamped to the window).  Features (the library's order): eps_n,
eps_F, Sigma^x - v^xc, Re Sigma^c(w_0..w_3), w_N - eps_n; target w* - w_N.
A second pass evaluates f at the seed and at seed +- 1e-4 Ha, which gives
the acceptance test and Z together.  Training runs on the GPU through
cdwac_mlp_train (the library's forward, backward and Adam kernels).

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
OFFSETS = np.array([-0.1, -0.05, 0.05, 0.1])   # Ha, the seed's sample points around eps_n


def first_steps(eps_n, vxc, sig0, sig1_fn):
    """omega_1, f(omega_0), f(omega_1), omega_2 of the plain root search."""
    f0 = eps_n - eps_n - sig0 + vxc
    w1 = eps_n - f0
    sig1 = sig1_fn(w1)
    f1 = w1 - eps_n - sig1 + vxc
    w2 = np.where(f1 != f0, w1 - f1 * (w1 - eps_n) / np.where(f1 != f0, f1 - f0, 1.0), w1)
    return w1, f0, f1, sig1, w2


def samples(lib, eps_n):
    """Sigma at the four sample points of every state: [n_states, 4]."""
    return lib.cdwac_sigma(eps_n[:, None] + OFFSETS[None, :])


def line_estimate(eps_n, vxc, sig4, lo, hi):
    """w_N: the zero of the least-squares line through (d_j, f(eps_n + d_j))."""
    f = (eps_n[:, None] + OFFSETS[None, :]) - eps_n[:, None] - sig4 + vxc[:, None]
    slope = (f * OFFSETS[None, :]).sum(axis=1) / np.sum(OFFSETS ** 2)
    mean = f.mean(axis=1)
    wn = np.where(slope > 0.0, eps_n - mean / np.where(slope > 0.0, slope, 1.0), eps_n - mean)
    return np.clip(wn, lo, hi)


def features(eps_n, eps_f, sx, vxc, sig4, wn):
    return np.array([eps_n, eps_f, sx - vxc, *(sig4 - sx), wn - eps_n])


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
        sig4 = samples(lib, eps_n)
        _, _, sx, _ = lib.cdwac_w_table(s.n_states, s.n_mo, n_freq, len(ref_re))
        for q in range(shifts_per_system):
            shift = 0.0 if q == 0 else float(rng.uniform(-SHIFT, SHIFT))
            vxc = sx + shift
            wn = line_estimate(eps_n, vxc, sig4, lo, hi)
            out = lib.cdwac_qp(s.n_states, vxc=vxc)
            for n, o in enumerate(out):
                if o["flags"] != 0 or not np.isfinite(o["qp"]):
                    continue
                xs.append(features(eps_n[n], eps_f, sx[n], vxc[n], sig4[n], wn[n]))
                ys.append(o["qp"] - wn[n])
        if (j + 1) % 50 == 0:
            log(f"systems {j + 1}/{n_systems}: {len(ys)} samples ({time.time() - t0:.0f} s)")
    return np.array(xs), np.array(ys)


def held_out_evaluations(lib, model, n_systems=24, shifts=(-0.2, 0.0, 0.2), seed=900_000, max_mo=400,
                         accept=1.0e-3 / synth.HARTREE_EV):
    """Passes over the tables (rounds of self-energy evaluations) of the root
    search with and without the seed, on systems of the training recipe that
    training never saw (other seeds).

    Returns per-state rows over the states whose plain search needed no
    fallback: plain rounds, seeded rounds, seed accepted, |dQP| (seeded -
    plain), and two network-free early stops with the same tolerance: the
    plain search stopped at omega_2 (3 rounds: f(omega_0), f(omega_1), then
    f(omega_2) with its Z pair in one pass) and the line estimate w_N of the
    same four samples the network sees (2 rounds: the samples, then f(w_N)
    with its Z pair); when a stop's test fails it is charged the plain
    search's rounds (the most favourable charge for it)."""
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
        sig4 = samples(lib, eps_n)
        for q, (q0, q1) in enumerate(zip(res[False], res[True])):
            vxc = sx + shifts[q]
            _, _, _, _, w2 = first_steps(eps_n, vxc, sig0, lambda w: lib.cdwac_sigma(w[:, None])[:, 0])
            f2 = w2 - eps_n - lib.cdwac_sigma(w2[:, None])[:, 0] + vxc
            wn = line_estimate(eps_n, vxc, sig4, lo, hi)
            fn = wn - eps_n - lib.cdwac_sigma(wn[:, None])[:, 0] + vxc
            for n, (o0, o1) in enumerate(zip(q0, q1)):
                if o0["flags"] != 0:
                    continue
                stop2 = 3 if abs(f2[n]) <= accept else o0["n_rounds"]
                line = 2 if abs(fn[n]) <= accept else o0["n_rounds"]
                rows.append((o0["n_rounds"], o1["n_rounds"], bool(o1["flags"] & 4), abs(o1["qp"] - o0["qp"]), stop2,
                             line))
    return np.array(rows, dtype=np.float64).reshape(-1, 6)


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
    ap.add_argument("--systems", type=int, default=400)
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
    report.update(held_out_states=int(len(rows)), held_out_rounds_plain=int(rows[:, 0].sum()),
                  held_out_rounds_seeded=int(rows[:, 1].sum()), held_out_rounds_stop_at_omega2=int(rows[:, 4].sum()),
                  held_out_rounds_line_estimate=int(rows[:, 5].sum()),
                  held_out_accepted=float(rows[:, 2].mean()),
                  held_out_max_dqp_mev=float(rows[:, 3].max() * synth.HARTREE_EV * 1e3))
    print(json.dumps(report), flush=True)
    np.savez(args.out, theta=theta.astype(np.float32), mu=mu.astype(np.float32), sd=sd.astype(np.float32),
             out_mu=np.float32(out_mu), out_sd=np.float32(out_sd), curve=curve,
             report=json.dumps(report))
    lib.close()


if __name__ == "__main__":
    main()
