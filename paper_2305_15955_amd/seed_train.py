"""Trains the learned QP-root seed on solves the method itself produces.

Data: many small seeded systems (60-300 orbitals, N_aux = 3.3 N_mo, 1-6
core states, the screening and core-coupling recipe of ``synth``).  Each
system is prepared once on the GPU (FP64 contractions); the self-energy is
sampled at eps_n + {-3, -1, 1, 3}/16 Ha and the QP root is solved for a range
of v^xc shifts, which re-uses the prepared tables.  Only roots found by the
plain secant (no fallback) are kept as targets.

Features (the library's order): eps_n, eps_F, Sigma^x - v^xc, the four
Re Sigma^c samples, and Sigma^x - v^xc + (central samples)/2; target
eps^QP - eps_n.  Training runs on the GPU through cdwac_mlp_train (the
library's forward, backward and Adam kernels).

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

OFFSETS = np.array([-3.0, -1.0, 1.0, 3.0]) / 16.0


def features(eps_n, eps_f, d0, sc):
    return np.array([eps_n, eps_f, d0, sc[0], sc[1], sc[2], sc[3], d0 + 0.5 * (sc[1] + sc[2])])


def generate(lib, n_systems, shifts_per_system, seed, log=print):
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    t0 = time.time()
    for j in range(n_systems):
        n_mo = int(rng.integers(60, 301))
        n_occ = max(3, int(round(n_mo / 6)))
        n_core = int(rng.integers(1, 7))
        n_core = min(n_core, n_occ - 1)
        n_aux = int(round(3.3 * n_mo))
        k = n_occ * (n_mo - n_occ)
        sigma = math.sqrt(synth.SCREENING / k)
        kappa = float(rng.uniform(0.12, 0.3))
        s = synth.make_system(n_mo, n_occ, n_aux, n_core, sigma, kappa=kappa, seed=10_000 + seed + j)
        n_freq = 32
        freq, wts = grids.gauss_legendre_imag(n_freq)
        lo, hi = grids.windows(s.eps, s.state_idx, 30.0)
        ref_im = grids.imag_ref_indices(n_freq, 8)
        ref_re = grids.generic_refs(s.eps, s.n_occ, lo, 8)
        sysc, keep = lib.make_system(s)
        prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64")
        lib.cdwac_prepare(sysc, prm)
        eps_n = s.eps[s.state_idx]
        eps_f = grids.midgap(s.eps, s.n_occ)
        oms = eps_n[:, None] + OFFSETS[None, :]
        sig = lib.cdwac_sigma(oms)
        _, _, sx, _ = lib.cdwac_w_table(s.n_states, s.n_mo, n_freq, len(ref_re))
        sc = sig - sx[:, None]
        for q in range(shifts_per_system):
            shift = 0.0 if q == 0 else float(rng.uniform(-0.12, 0.12))
            vxc = sx + shift
            out = lib.cdwac_qp(s.n_states, vxc=vxc)
            for n, o in enumerate(out):
                if o["flags"] != 0 or not np.isfinite(o["qp"]):
                    continue
                xs.append(features(eps_n[n], eps_f, sx[n] - vxc[n], sc[n]))
                ys.append(o["qp"] - eps_n[n])
        if (j + 1) % 50 == 0:
            log(f"systems {j + 1}/{n_systems}: {len(ys)} samples ({time.time() - t0:.0f} s)")
    return np.array(xs), np.array(ys)


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
    ap.add_argument("--systems", type=int, default=600)
    ap.add_argument("--shifts", type=int, default=12)
    ap.add_argument("--epochs", type=int, default=300)
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
    print(json.dumps(report), flush=True)
    np.savez(args.out, theta=theta.astype(np.float32), mu=mu.astype(np.float32), sd=sd.astype(np.float32),
             out_mu=np.float32(out_mu), out_sd=np.float32(out_sd), curve=curve,
             report=json.dumps(report))
    lib.close()


if __name__ == "__main__":
    main()
