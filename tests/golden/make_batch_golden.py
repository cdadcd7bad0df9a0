"""Writes the stored oracle QP energies of the 48-system uneven batch.

The batch of synth.batch_specs() (N_mo uniform in [100, 1200], N_aux = 3.3
N_mo, 1-12 core states) with 48 imaginary Gauss-Legendre nodes and 24 Pade
points (12 imaginary, 12 near-real), the settings of the GPU batch test.
Calls only the FP64 oracle (``oracle/``) on the seeded synthetic inputs; the
systems go from the smallest to the largest, and the file is rewritten
after each one ("complete" is set once all are there); a run started on an
existing file with the same settings keeps its systems and adds the rest.  About 8 h on 8 host
cores (the largest systems take 20-40 min each).  Run from the repository root:
    python tests/golden/make_batch_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cdwac_ref as R  # noqa: E402
from paper_2305_15955_amd import grids, synth  # noqa: E402

N_FREQ, N_IM, N_RE, WINDOW_EV = 48, 12, 12, 30.0


def main():
    specs = synth.batch_specs()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch48_oracle.json")
    out = dict(n_systems=len(specs), seed=400, n_freq=N_FREQ, n_pade=N_IM + N_RE, window_ev=WINDOW_EV,
               complete=False, systems={})
    if os.path.exists(path):
        # resume: the systems already written for the same settings are kept
        # (each system's result depends on its own seeded input only)
        old = json.load(open(path))
        if all(old.get(k) == out[k] for k in ("n_systems", "seed", "n_freq", "n_pade", "window_ev")):
            out["systems"] = old["systems"]
    freq, wts = grids.gauss_legendre_imag(N_FREQ)
    for j in np.argsort([sp["n_mo"] for sp in specs], kind="stable"):
        j = int(j)
        sp = specs[j]
        if str(j) in out["systems"]:
            continue
        t = time.time()
        s = synth.make_system(sp["n_mo"], sp["n_occ"], sp["n_aux"], sp["n_core"], sp["sigma"], seed=sp["seed"])
        lo, hi = grids.windows(s.eps, s.state_idx, WINDOW_EV)
        ref_im = grids.imag_ref_indices(N_FREQ, N_IM)
        ref_re = grids.generic_refs(s.eps, s.n_occ, lo, N_RE)
        o = R.CdwacOracle(s, freq, wts, ref_im, ref_re, lo, hi)
        res = o.solve_all()
        out["systems"][str(j)] = dict(n_mo=sp["n_mo"], n_aux=sp["n_aux"], qp=[r[0] for r in res],
                                      z=[r[1] for r in res], flags=[r[3] for r in res])
        out["complete"] = len(out["systems"]) == len(specs)
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)          # readers never see a partial file
        print(f"system {j} (N_mo {sp['n_mo']}, {sp['n_core']} states): {time.time() - t:.0f} s, "
              f"{len(out['systems'])}/{len(specs)} written", flush=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
