#!/usr/bin/env python
"""Throughput of the CD-WAC core-level G0W0 path on one MI355X.

One step = one full solve through the C ABI (cdwac_solve): polarizability on
the imaginary grid and at the near-real Pade references, dielectric
inversion, W contraction, exchange, greedy Thiele fits and the QP root of
every core state.  Inputs (KS energies, RI coefficients) are seeded synthetic
arrays already resident in HBM when the timed region starts.

Prints one JSON line.  value = core QP energies per second of the whole job
at the stated configuration: Pi and W contracted on the matrix cores in the
bf16 hi/lo split (three products, FP32 accumulation), the dielectric
inversion, Pade fits, self-energy and root search in FP64, Pi, eps^-1 and W
at every one of the 64 imaginary Gauss-Legendre nodes and at every near-real
Pade reference, and the learned seed if a model is installed.
Also reported: the plain FP64 GPU path (warm, timed over several steps), the
per-state error of the reduced path against it in meV, per-stage times from
HIP events on the library's stream, the roofline of the polarizability
kernel, faster variants of the method under their own key (never as value),
and the FP64 oracle timed on a bounded sample of the same workload on the
host CPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f16": 2.5e15, "f16x3": 2.5e15, "b16x3": 2.5e15, "b16": 2.5e15, "p64": 78.6e12}   # dense MFMA, FLOP/s
PRODUCTS = {"f16": 1, "f16x3": 3, "b16x3": 3, "b16": 1, "p64": 1}      # matrix-core products per MAC of Pi
DTYPE = {"f16": "f16 (Pi, one product) + f16x3 (W) + f64",
         "f16x3": "f16x3 (fp16 hi/lo split, in place of FP32) + f64",
         "b16x3": "bf16x3 (bf16 hi/lo split, FP32 accumulation) + f64",
         "b16": "bf16 + f64", "p64": "f64"}
MODEL_PATH = os.path.join(ROOT, "paper_2305_15955_amd", "seed_model.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(prec, workload, launches, planes):
    """HBM bytes per k_pi_gemm launch from the committed rocprofv3 counter
    summary of this precision mode and workload (FETCH_SIZE + WRITE_SIZE,
    calibrated on a 1 GiB copy), or None if there is none, or if it is for
    another kernel source, launch count or plane count."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_pi_gemm_{prec}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "k_dense_sha256_16",
                                                  "launches_per_step", "contracted_planes"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    src = os.path.join(ROOT, "paper_2305_15955_amd", "csrc", "k_dense.hip")
    if vals.get("k_dense_sha256_16") != hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]:
        return None
    if vals.get("launches_per_step") != str(launches) or vals.get("contracted_planes") != str(planes):
        return None
    return float(vals["traffic_bytes_per_launch"])


def full_cd_qp(lib, sysc, prm, system, state, sigma_x):
    """Full-CD QP energy of one state: the secant of the library's root search
    (omega_0 = eps_n, one fixed-point step, |d omega| < 1e-10 Ha) over
    cdwac_sigma_cd, which evaluates W directly at every residue; v^xc = Sigma^x."""
    e_n = float(system.eps[system.state_idx[state]])
    f = lambda w: w - e_n - lib.cdwac_sigma_cd(sysc, prm, state, w)[0] + sigma_x
    w0, f0 = e_n, f(e_n)
    w1 = w0 - f0
    f1 = f(w1)
    for _ in range(50):
        if f1 == f0:
            break
        w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
        w0, f0, w1 = w1, f1, w2
        f1 = f(w1)
        if abs(w1 - w0) < 1e-10:
            break
    return w1


def heatmap(n_systems, cores, vals, n_im, n_freq, mo_range=(90, 150)):
    """CD-WAC against full CD as the refined reference set grows (Sec. 3.3,
    the study behind the recommended CD-WAC(20, 20, 200)): mean absolute error
    in meV of the core QP energies over seeded synthetic systems, for every
    CD-WAC(N_core, N_valence, N_Im) on an n_freq-node imaginary grid, FP64 path
    on both sides."""
    from paper_2305_15955_amd import cdwac, grids, synth
    lib = cdwac.Cdwac(0)
    freq, wts = grids.gauss_legendre_imag(n_freq)
    err = np.full((len(cores), len(vals)), 0.0)
    worst = np.full((len(cores), len(vals)), 0.0)
    lost = np.zeros((len(cores), len(vals)), np.int64)
    n_states = 0
    sizes = []
    for j in range(n_systems):
        rng = np.random.default_rng(700 + j)
        n_mo = int(rng.integers(mo_range[0], mo_range[1] + 1))
        n_occ = max(3, round(n_mo / 6))
        n_core = int(rng.integers(1, 4))
        n_aux = round(3.3 * n_mo)
        k = n_occ * (n_mo - n_occ)
        s = synth.make_system(n_mo, n_occ, n_aux, n_core, math.sqrt(synth.SCREENING / k), kappa=0.2, seed=700 + j)
        sizes.append([n_mo, n_aux, n_core])
        lo, hi = grids.windows(s.eps, s.state_idx, 30.0)
        sysc, keep = lib.make_system(s)
        ref_im, ref_re = grids.cdwac_setting(s.eps, s.n_occ, s.state_idx, lo, hi, 20, 20, n_im, n_freq)
        prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64")
        out = lib.cdwac_solve(sysc, prm)
        cd = [full_cd_qp(lib, sysc, prm, s, n, float(out[n]["sigma_x"])) for n in range(s.n_states)]
        for a, nc in enumerate(cores):
            for b, nv in enumerate(vals):
                ref_im, ref_re = grids.cdwac_setting(s.eps, s.n_occ, s.state_idx, lo, hi, nc, nv, n_im, n_freq)
                prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64")
                out = lib.cdwac_solve(sysc, prm)
                for n in range(s.n_states):
                    d = abs(out[n]["qp"] - cd[n]) * synth.HARTREE_EV * 1e3
                    if not np.isfinite(d):
                        lost[a, b] += 1
                        continue
                    err[a, b] += d
                    worst[a, b] = max(worst[a, b], d)
        n_states += s.n_states
        log(f"heatmap system {j + 1}/{n_systems}: N_mo={n_mo}, {s.n_states} core states")
        del keep
    lib.close()
    counted = n_states - lost
    return {"metric": "MAE of CD-WAC(N_core, N_valence, N_Im) against full CD, core QP energies",
            "unit": "meV", "n_im": n_im, "n_freq": n_freq, "n_core": list(cores), "n_valence": list(vals),
            "systems": sizes, "states": n_states,
            "mae_mev": (err / np.maximum(counted, 1)).tolist(), "max_mev": worst.tolist(),
            "states_without_root": lost.tolist(),
            "data": "synthetic (seeded Gaussian RI coefficients, no molecule)"}


def build_inputs(name):
    from paper_2305_15955_amd import grids, synth
    spec = synth.WORKLOADS[name]
    s = synth.make_workload(name)
    freq, wts = grids.gauss_legendre_imag(spec["n_freq"])
    lo, hi = grids.windows(s.eps, s.state_idx, spec["window_ev"])
    nim = spec["n_pade"] // 2
    ref_im = grids.imag_ref_indices(len(freq), nim)
    ref_re = grids.generic_refs(s.eps, s.n_occ, lo, spec["n_pade"] - nim)
    return spec, s, freq, wts, ref_im, ref_re, lo, hi


def cpu_baseline(s, freq, ref_re, n_states):
    """The oracle's wmatrix (Pi, Lambda, W of every state) at full size, timed
    at one imaginary node and at one near-real reference point; scaled to QP
    energies per second: the oracle's preparation runs n_freq real and n_re
    complex such evaluations, and its fits and QP loop are negligible next to
    them (timed on the 60-orbital case: well under a second)."""
    from oracle import cdwac_ref as R
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [os.cpu_count() or 1])
    except Exception:
        threads = os.cpu_count() or 1

    def one(z):
        t0 = time.perf_counter()
        pi = R.polarizability(s.o_ia, s.eps, s.n_occ, z, s.spin)
        lam = R.lambda_matrix(pi)
        del pi
        for st in range(n_states):
            R.w_elements(s.o_nm[st], lam)
        return time.perf_counter() - t0
    t_re = one(1j * float(freq[len(freq) // 2]))
    log(f"cpu baseline: real node {t_re:.1f} s")
    t_cx = one(complex(float(ref_re[len(ref_re) // 2]), 1e-3))
    log(f"cpu baseline: complex node {t_cx:.1f} s")
    t_job = t_re * len(freq) + t_cx * len(ref_re)
    return {"value": n_states / t_job, "unit": "core QP energies/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"oracle wmatrix (Pi, Lambda, W for {n_states} states) at full size, timed at one of "
                       f"{len(freq)} imaginary nodes ({t_re:.1f} s) and one of {len(ref_re)} near-real "
                       f"points ({t_cx:.1f} s); job time {len(freq)} x {t_re:.1f} + {len(ref_re)} x "
                       f"{t_cx:.1f} = {t_job:.0f} s")}


def scaling(sizes, cd_qp_max):
    """Full CD against CD-WAC on one GPU as the system grows (Sec. 5,
    scaling): N_mo in `sizes`, N_occ = N_mo / 6, N_aux = 3.3 N_mo, one core
    state, 64 imaginary nodes, 24 Pade points, FP64 path on both sides.
    CD-WAC: one cdwac_solve.  Full CD: cdwac_sigma_cd evaluates W directly at
    every residue of one omega; its cost per QP solve is the imaginary-axis
    part once plus the residue part per self-energy evaluation (as many as the
    CD-WAC solve used).  Up to N_mo = cd_qp_max the full-CD QP energy is also
    solved on the GPU (secant over cdwac_sigma_cd, each evaluation computing
    the imaginary-axis part again), timed, to give CD-WAC's error."""
    import torch
    from paper_2305_15955_amd import cdwac, grids, synth
    lib = cdwac.Cdwac(0)
    rows = []
    for n_mo in sizes:
        n_occ = max(2, round(n_mo / 6))
        n_aux = round(3.3 * n_mo)
        k = n_occ * (n_mo - n_occ)
        s = synth.make_system(n_mo, n_occ, n_aux, 1, math.sqrt(synth.SCREENING / k), seed=900 + n_mo)
        freq, wts = grids.gauss_legendre_imag(64)
        lo, hi = grids.windows(s.eps, s.state_idx, 30.0)
        ref_im = grids.imag_ref_indices(64, 12)
        ref_re = grids.generic_refs(s.eps, s.n_occ, lo, 12)
        sysc, keep = lib.make_system(s)
        prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64")
        one, ones = grids.gauss_legendre_imag(1)
        prm1, arrs1 = lib.make_params(one, ones, [0], ref_re, lo, hi, prec="p64")
        lib.cdwac_solve(sysc, prm)                       # warm-up (allocations)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = lib.cdwac_solve(sysc, prm)[0]
        t_wac = time.perf_counter() - t
        qp = out["qp"]
        lib.cdwac_sigma_cd(sysc, prm1, 0, qp)
        t = time.perf_counter()
        _, _, _, n_res = lib.cdwac_sigma_cd(sysc, prm, 0, qp)
        t_call = time.perf_counter() - t
        t = time.perf_counter()
        lib.cdwac_sigma_cd(sysc, prm1, 0, qp)
        t_res = time.perf_counter() - t
        # the spectral function on 1000 points of the window from the prepared
        # tables (Sec. 5.5): per point against one full-CD self-energy
        lib.cdwac_solve(sysc, prm)
        om_sp = (s.eps[0] + np.linspace(-25.0, 25.0, 1000) / synth.HARTREE_EV)[None, :]
        lib.cdwac_spectral(om_sp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lib.cdwac_spectral(om_sp)
        torch.cuda.synchronize()
        t_spec = time.perf_counter() - t
        row = {"n_mo": n_mo, "n_aux": n_aux, "n_occ": n_occ, "K": k, "cdwac_s": t_wac,
               "sigma_evals": out["n_evals"], "cd_residues": n_res, "cd_residue_part_s": t_res,
               "cd_imag_part_s": max(t_call - t_res, 0.0),
               "cd_qp_estimate_s": max(t_call - t_res, 0.0) + out["n_evals"] * t_res}
        row["cd_over_cdwac"] = row["cd_qp_estimate_s"] / t_wac
        row["spectral_1000pts_s"] = t_spec
        row["spectral_speedup_per_point"] = t_call / (t_spec / 1000.0)
        if n_mo <= cd_qp_max:
            e_n = float(s.eps[0])
            n_cd = [0]

            def f(w):
                n_cd[0] += 1
                v = w - e_n - lib.cdwac_sigma_cd(sysc, prm, 0, w)[0] + float(out["sigma_x"])
                log(f"  N_mo={n_mo} full-CD evaluation {n_cd[0]}: f = {v:.3e} Ha")
                return v
            t = time.perf_counter()
            w0, f0 = e_n, f(e_n)
            w1 = w0 - f0
            f1 = f(w1)
            for _ in range(50):
                w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
                w0, f0, w1 = w1, f1, w2
                f1 = f(w1)
                if abs(w1 - w0) < 1e-10:
                    break
            row["cd_qp_solve_s"] = time.perf_counter() - t
            row["cd_qp_solve_evals"] = n_cd[0]
            row["cd_qp_ev"] = w1 * synth.HARTREE_EV
            row["cdwac_minus_cd_mev"] = (qp - w1) * synth.HARTREE_EV * 1e3
        log(f"scaling N_mo={n_mo}: CD-WAC {t_wac:.3f} s, CD residue part {t_res:.3f} s x {out['n_evals']} "
            f"evals ({n_res} residues)")
        rows.append(row)
        del keep
    lib.close()

    def slope(key):
        big = rows[-3:]
        x = np.log([r["n_mo"] for r in big])
        y = np.log([r[key] for r in big])
        return float(np.polyfit(x, y, 1)[0])
    solved = all("cd_qp_solve_s" in r for r in rows[-3:])
    return {"metric": "full CD vs CD-WAC cost per core QP energy on one GPU (FP64 path)",
            "unit": "s", "rows": rows,
            "exponent_cdwac": slope("cdwac_s"), "exponent_cd": slope("cd_qp_estimate_s"),
            "exponent_cd_solved": slope("cd_qp_solve_s") if solved else None,
            "exponent_cd_per_eval": slope("cd_residue_part_s"),
            "data": "synthetic (seeded Gaussian RI coefficients, no molecule)"}


def literal_screening(sigma=0.02):
    """The 600-orbital workload with the coefficients drawn at N(0, sigma^2)
    for every size (sigma = 0.02: screening strength K sigma^2 = 20, against
    1.25 for sigma = sqrt(1.25 / K) of the workload recipe), the rest of the
    recipe unchanged.  Per core state: the CD-WAC root of the FP64 path and of
    the bf16 split (flags, Z), and the full-CD root (secant over
    cdwac_sigma_cd from the CD-WAC root) where CD-WAC found one.  One JSON
    line."""
    from paper_2305_15955_amd import cdwac, grids, synth
    spec = synth.WORKLOADS["acene_nmo600"]
    s = synth.make_system(spec["n_mo"], spec["n_occ"], spec["n_aux"], spec["n_core"], sigma, kappa=0.2,
                          seed=spec["seed"])
    freq, wts = grids.gauss_legendre_imag(spec["n_freq"])
    lo, hi = grids.windows(s.eps, s.state_idx, spec["window_ev"])
    nim = spec["n_pade"] // 2
    ref_im = grids.imag_ref_indices(len(freq), nim)
    ref_re = grids.generic_refs(s.eps, s.n_occ, lo, spec["n_pade"] - nim)
    lib = cdwac.Cdwac(0)
    sysc, keep = lib.make_system(s)
    res = {}
    for prec in ("p64", "b16x3"):
        prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec=prec)
        res[prec] = lib.cdwac_solve(sysc, prm)
    prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec="p64")
    rows = []
    for n in range(s.n_states):
        a, b = res["p64"][n], res["b16x3"][n]
        row = {"state": n, "ks_ev": float(s.eps[n] * synth.HARTREE_EV), "flags_p64": a["flags"],
               "flags_b16x3": b["flags"], "qp_ev": a["qp"] * synth.HARTREE_EV, "z": a["z"],
               "b16x3_minus_p64_mev": (b["qp"] - a["qp"]) * synth.HARTREE_EV * 1e3}
        if math.isfinite(a["qp"]):
            e_n = float(s.eps[n])
            f = lambda w: w - e_n - lib.cdwac_sigma_cd(sysc, prm, n, w)[0] + a["sigma_x"]
            w0, w1 = a["qp"], a["qp"] + 1e-3 / synth.HARTREE_EV
            f0, f1 = f(w0), f(w1)
            for _ in range(20):
                if f1 == f0:
                    break
                w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
                w0, f0, w1 = w1, f1, w2
                f1 = f(w1)
                if abs(w1 - w0) < 1e-10:
                    break
            row["full_cd_qp_ev"] = w1 * synth.HARTREE_EV
            row["cdwac_minus_full_cd_mev"] = (a["qp"] - w1) * synth.HARTREE_EV * 1e3
            row["full_cd_residual_ha"] = f1
        rows.append(row)
        log(f"literal screening: state {n} done")
    lib.close()
    return {"metric": "core QP roots of the 600-orbital workload with O ~ N(0, sigma^2) at every size",
            "sigma": sigma, "screening_k_sigma2": s.n_occ * s.n_virt * sigma ** 2, "states": rows,
            "roots_found_p64": sum(math.isfinite(r["qp_ev"]) for r in rows),
            "data": "synthetic (seeded Gaussian RI coefficients, no molecule)"}


def self_consistency(name="precision_naux5000", prec="b16x3", tol=1e-7):
    """The eigenvalue-self-consistent flavours and G_dH W0 (Sec. 4) on a
    full-size workload, with the analytic a_m -> 0 limit of the integral term
    (with the plain quadrature a core state's own G pole makes the loops
    wander) and every (n, m) fitted, which moved G energies need.  Per flavour:
    the QP solves to convergence (no energy moving by more than tol Ha), the
    wall time, the QP energies and Z of the computed states and their shift
    from G0W0.  One JSON line."""
    import torch
    from paper_2305_15955_amd import cdwac, synth
    spec, s, freq, wts, ref_im, ref_re, lo, hi = build_inputs(name)
    lib = cdwac.Cdwac(0)
    dev = torch.device("cuda", 0)
    o_ia = torch.from_numpy(s.o_ia).to(dev)
    o_nm = torch.from_numpy(s.o_nm).to(dev)
    sysc, keep = lib.make_system(s, o_ia_dev=o_ia, o_nm_dev=o_nm)
    prm, arrs = lib.make_params(freq, wts, ref_im, ref_re, lo, hi, pade_tol=1e-9, prec=prec, fit_all=True,
                                quad_limit=True)
    ev = synth.HARTREE_EV
    summary = lambda qp, z, flags: {"qp_ev": [q * ev for q in qp], "z": list(z), "flags": list(flags),
                                    "z_min": float(np.min(z)), "roots": int(sum(math.isfinite(q) for q in qp))}
    res = {}
    lib.cdwac_solve(sysc, prm)                                # warm-up (allocations)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g0 = lib.cdwac_solve(sysc, prm)
    torch.cuda.synchronize()
    res["g0w0"] = dict(summary([o["qp"] for o in g0], [o["z"] for o in g0], [o["flags"] for o in g0]),
                       s=time.perf_counter() - t)
    qp0 = np.array([o["qp"] for o in g0])
    t = time.perf_counter()
    hed, dh = lib.cdwac_qp_hedin(s.n_states)
    res["g_dh_w0"] = dict(summary([o["qp"] for o in hed], [o["z"] for o in hed], [o["flags"] for o in hed]),
                          s=time.perf_counter() - t, shift_dh_ev=[x * ev for x in dh],
                          mean_shift_from_g0w0_ev=float(np.mean([o["qp"] for o in hed] - qp0) * ev))
    log(f"self-consistency: G0W0 and G_dH W0 done")
    for mode in ("evgw0", "evgw"):
        t = time.perf_counter()
        e, it, out = lib.cdwac_evgw(sysc, prm, mode, max_iter=30, tol=tol)
        torch.cuda.synchronize()
        qp = np.array([o["qp"] for o in out])
        res[mode] = dict(summary(qp, [o["z"] for o in out], [o["flags"] for o in out]), solves=it,
                         converged=it < 30, s=time.perf_counter() - t,
                         mean_shift_from_g0w0_ev=float(np.mean(qp - qp0) * ev))
        log(f"self-consistency: {mode} {it} solves, {res[mode]['s']:.1f} s")
    lib.close()
    return {"metric": "eigenvalue self-consistency and G_dH W0 at full size (solves to convergence, wall time)",
            "workload": name, "precision": prec, "tol_ha": tol, "quad_limit": True, "fit_all": True,
            "n_states": s.n_states, **res, "data": "synthetic (seeded Gaussian RI coefficients, no molecule)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision_naux5000")
    ap.add_argument("--prec", default="b16x3", choices=["f16", "f16x3", "b16x3", "b16", "p64"])
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed steps of the FP64 GPU path")
    ap.add_argument("--fp64-warmup", type=int, default=1, help="untimed steps of the FP64 GPU path")
    ap.add_argument("--rank-tol", type=float, default=0.0,
                    help="imaginary-node decomposition tolerance of the 16-bit path (0, the default: Pi, "
                         "eps^-1 and W at every node)")
    ap.add_argument("--variant-steps", type=int, default=3,
                    help="timed steps of each faster variant reported under 'variants' (0: none)")
    ap.add_argument("--near-real-f64", action="store_true",
                    help="16-bit modes: Pi at the near-real reference points on the FP64 path")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--scaling", action="store_true",
                    help="instead of the benchmark: full CD against CD-WAC as N_mo grows (one JSON line)")
    ap.add_argument("--literal-screening", action="store_true",
                    help="instead of the benchmark: the 600-orbital workload at sigma = 0.02 (one JSON line)")
    ap.add_argument("--self-consistency", action="store_true",
                    help="instead of the benchmark: evGW0, evGW and G_dH W0 on the workload (one JSON line)")
    ap.add_argument("--heatmap", action="store_true",
                    help="instead of the benchmark: CD-WAC against full CD over (N_core, N_valence) (one JSON line)")
    args = ap.parse_args()
    if args.scaling:
        print(json.dumps(scaling([60, 120, 240, 480, 960], 960)), flush=True)
        return
    if args.literal_screening:
        print(json.dumps(literal_screening()), flush=True)
        return
    if args.self_consistency:
        print(json.dumps(self_consistency(args.workload, args.prec)), flush=True)
        return
    if args.heatmap:
        grid = [0, 2, 4, 8, 12, 16, 20]
        print(json.dumps(heatmap(6, grid, grid, 16, 64, (200, 400))), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU mode", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_15955_amd import cdwac, synth

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    spec, s, freq, wts, ref_im, ref_re, lo, hi = build_inputs(args.workload)
    log(f"inputs {args.workload}: n_aux={s.n_aux} n_mo={s.n_mo} K={s.o_ia.shape[1]} "
        f"states={s.n_states} ({time.perf_counter() - t0:.1f} s)")
    lib = cdwac.Cdwac(0)
    o_ia = torch.from_numpy(s.o_ia).to(dev)
    o_nm = torch.from_numpy(s.o_nm).to(dev)
    torch.cuda.synchronize()

    use_mlp = (not args.no_mlp) and os.path.exists(MODEL_PATH)
    if use_mlp:
        m = np.load(MODEL_PATH)
        lib.cdwac_mlp_set_model(m["theta"], m["mu"], m["sd"], float(m["out_mu"]), float(m["out_sd"]))

    def params(prec, mlp, rank_tol=None):
        rank_tol = args.rank_tol if rank_tol is None else rank_tol
        return lib.make_params(freq, wts, ref_im, ref_re, lo, hi, prec=prec,
                               pade_tol=1e-9, use_mlp_seed=mlp, mlp_accept=1e-4 / synth.HARTREE_EV,
                               freq_rank_tol=rank_tol if prec != "p64" else 0.0,
                               near_real_f64=args.near_real_f64 and prec != "p64")

    sysc, keep = lib.make_system(s, o_ia_dev=o_ia, o_nm_dev=o_nm)
    lib.cdwac_set_timing(True)

    def run_steps(prec, mlp, warmup, steps, rank_tol=None):
        prm, arrs = params(prec, mlp, rank_tol)
        for i in range(warmup):
            lib.cdwac_solve(sysc, prm)
            log(f"warmup {prec} {i + 1}/{warmup} done")
        stage_sum = {k: 0.0 for k in lib.STAGES}
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = None
        for i in range(steps):
            out = lib.cdwac_solve(sysc, prm)
            for k, v in lib.cdwac_get_timing().items():
                stage_sum[k] += v
            log(f"step {prec} {i + 1}/{steps} done")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / max(steps, 1)
        launches = lib.cdwac_get_timing_segments()
        launches["planes"] = lib.cdwac_plane_counts()
        return out, dt, {k: v / max(steps, 1) for k, v in stage_sum.items()}, launches

    out, dt, stages, launches = run_steps(args.prec, use_mlp, args.warmup, args.steps)
    qps = s.n_states / dt
    res = {"metric": "core QP energies/sec at N_aux=5000 (mixed+MLP vs FP64), meV err, MFMA util",
           "value": qps, "unit": "core QP energies/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.prec],
           "data": "synthetic (seeded Gaussian RI coefficients, no molecule)",
           "config": {"workload": args.workload, "n_aux": s.n_aux, "n_mo": s.n_mo, "n_occ": s.n_occ,
                      "n_states": s.n_states, "n_freq": len(freq), "n_pade": len(ref_im) + len(ref_re),
                      "contraction_precision": args.prec, "mlp_seed": use_mlp,
                      "freq_rank_tol": args.rank_tol if args.prec != "p64" else 0.0,
                      "near_real_f64": bool(args.near_real_f64 and args.prec != "p64")}}

    # roofline of the dominant kernel: the polarizability contraction, one
    # launch per batch of frequency planes; achieved = algorithmic flops of
    # one launch / its average duration (HIP events on the library's stream)
    n_im_planes, n_f = launches["planes"]         # planes the contraction computes
    res["config"]["imaginary_planes"] = n_im_planes
    res["config"]["contracted_planes"] = n_f
    k_dim = s.o_ia.shape[1]
    n_launch = max(int(launches["polarizability"]), 1)
    flops = float(n_f) * s.n_aux * (s.n_aux + 1) * k_dim / n_launch   # lower-triangle SYRK, 2 flop/MAC
    launch_s = stages["polarizability"] * 1e-3 / n_launch
    achieved = flops / launch_s / 1e12
    peak = PEAK[args.prec] / 1e12
    nb = int(math.ceil(s.n_aux / 256.0))
    kpad = int(math.ceil(k_dim / 32.0) * 32)
    if args.prec == "p64":
        nt = nb * 2
        tile_elems = nt * (nt + 1) // 2 * 128 * 128         # lower-triangle 128 x 128 FP64 tiles
    else:
        tile_elems = nb * (nb + 1) // 2 * 256 * 256        # lower-triangle 256 x 256 tiles
    issued = float(n_f) / n_launch * tile_elems * kpad * 2.0 * PRODUCTS[args.prec]
    traffic = measured_traffic(args.prec, args.workload, n_launch, n_f)
    res["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                       "frac": achieved / peak, "traffic": traffic,
                       "kernel": "k_pi_gemm" if args.prec != "p64" else "k_pi_f64",
                       "launches": n_launch, "algorithmic_flop_per_launch": flops,
                       "launch_ms": launch_s * 1e3,
                       "mfma_issued_frac": issued / launch_s / PEAK[args.prec]}
    if res["config"]["near_real_f64"]:
        # the polarizability stage then mixes the 16-bit and the FP64 kernel:
        # no single-kernel roofline
        res["roofline"] = None
    res["stages_ms"] = stages
    # the W contraction stage against the same peak: the quadratic form
    # o^T Lambda o of a symmetric Lambda takes N_aux (N_aux + 1) / 2 products
    # per column (its lower triangle), N_aux (N_aux + 1) flop, for every (n, m)
    # column at the imaginary planes and the fitted ones at the near-real
    # planes (the stage also holds the small transposes of B, so this is a
    # lower bound for its kernel)
    _, _, _, (m0, m1) = lib.cdwac_w_table(s.n_states, s.n_mo, len(freq), len(ref_re))
    n_fit = int(np.sum(m1 - m0))
    flops_w = s.n_aux * (s.n_aux + 1.0) * (n_im_planes * s.n_states * s.n_mo + (n_f - n_im_planes) * n_fit)
    w_s = stages["w_contraction"] * 1e-3
    res["roofline_w"] = {"bound": "mfma", "achieved": flops_w / w_s / 1e12, "peak": peak, "unit": "TFLOP/s",
                         "frac": flops_w / w_s / 1e12 / peak, "kernel": "k_w_gemm (the whole W stage)",
                         "algorithmic_flop_per_step": flops_w, "stage_ms": w_s * 1e3}
    # spectral function (Sec. 5.5) on 5000 points per state over a 50 eV range,
    # from the prepared tables of the last step
    om = np.stack([s.eps[s.state_idx[n]] + np.linspace(-25.0, 25.0, 5000) / synth.HARTREE_EV
                   for n in range(s.n_states)])
    lib.cdwac_spectral(om)
    torch.cuda.synchronize()
    t_sp = time.perf_counter()
    spec = lib.cdwac_spectral(om)
    res["spectral_5000pts_ms"] = (time.perf_counter() - t_sp) * 1e3
    res["spectral_peak_ev"] = [float(om[n, int(np.argmax(spec[n]))] * synth.HARTREE_EV) for n in range(s.n_states)]
    res["qp_ev"] = [o["qp"] * synth.HARTREE_EV for o in out]
    res["n_evals_mean"] = float(np.mean([o["n_evals"] for o in out]))
    res["n_rounds_mean"] = float(np.mean([o["n_rounds"] for o in out]))
    res["seed_accepted"] = int(sum(bool(o["flags"] & cdwac.FLAG_MLP_ACCEPTED) for o in out))
    # per-state error against the oracle's QP energies where they are stored
    # for this workload (tests/golden, written by the oracle alone)
    stored = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.json")
    res["mev_err_vs_oracle"] = None
    if os.path.exists(stored):
        g = json.load(open(stored))
        if g.get("workload") == args.workload and len(g["qp"]) == len(out):
            e = [abs(o["qp"] - q) * synth.HARTREE_EV * 1e3 for o, q in zip(out, g["qp"])]
            res["mev_err_vs_oracle"] = {"max": max(e), "mean": float(np.mean(e)), "per_state": e,
                                        "stored": os.path.relpath(stored, ROOT)}

    res["inversion_residual"] = lib.cdwac_inversion_residual()[0]

    out64 = None
    if args.fp64_steps > 0 and args.prec != "p64":
        out64, dt64, st64, _ = run_steps("p64", False, args.fp64_warmup, args.fp64_steps)
        err = [abs(a["qp"] - b["qp"]) * synth.HARTREE_EV * 1e3 for a, b in zip(out, out64)]
        pi64_s = st64["polarizability"] * 1e-3            # one k_pi_f64 launch over every plane
        flops64 = float(n_f) * s.n_aux * (s.n_aux + 1) * k_dim
        res["fp64_path"] = {"value": s.n_states / dt64, "ms_per_step": dt64 * 1e3, "steps": args.fp64_steps,
                            "warmup": args.fp64_warmup, "stages_ms": st64,
                            "roofline": {"bound": "mfma", "kernel": "k_pi_f64", "achieved": flops64 / pi64_s / 1e12,
                                         "peak": PEAK["p64"] / 1e12, "unit": "TFLOP/s",
                                         "frac": flops64 / pi64_s / PEAK["p64"], "launch_ms": pi64_s * 1e3},
                            "n_evals_mean": float(np.mean([o["n_evals"] for o in out64])),
                            "n_rounds_mean": float(np.mean([o["n_rounds"] for o in out64]))}
        res["mev_err_vs_fp64"] = {"max": max(err), "mean": float(np.mean(err)), "per_state": err}
        res["speedup_vs_fp64_path"] = dt64 / dt

    # faster variants of the method, reported beside the stated configuration
    # and never as its value: the one-product fp16 Pi (W in the fp16 split)
    # at every node, and the same with Pi, eps^-1 and W only at a skeleton of
    # the imaginary nodes (W interpolated at the others: an addition to the
    # method, not in the paper)
    if args.variant_steps > 0 and args.prec != "p64":
        variants = {}
        for name, prec, tol in (("f16_every_node", "f16", 0.0),
                                ("f16_skeleton_nodes", "f16", cdwac.SKELETON_TOL["f16"])):
            o_v, dt_v, st_v, l_v = run_steps(prec, use_mlp, 1, args.variant_steps, tol)
            v = {"value": s.n_states / dt_v, "ms_per_step": dt_v * 1e3, "dtype": DTYPE[prec],
                 "freq_rank_tol": tol, "imaginary_planes": l_v["planes"][0], "contracted_planes": l_v["planes"][1],
                 "stages_ms": st_v}
            if out64 is not None:
                e = [abs(a["qp"] - b["qp"]) * synth.HARTREE_EV * 1e3 for a, b in zip(o_v, out64)]
                v["mev_err_vs_fp64"] = {"max": max(e), "mean": float(np.mean(e))}
            variants[name] = v
        res["variants"] = variants

    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = 2 * a.numel() * 8

    del o_ia, o_nm
    lib.close()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        res["cpu_baseline"] = cpu_baseline(s, freq, ref_re, s.n_states)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
