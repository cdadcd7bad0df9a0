"""Writes the stored oracle results of a synthetic workload: QP energies,
sampled W and sampled Sigma.

Calls only the FP64 oracle (``oracle/``) on the seeded synthetic input; the
GPU tests compare against the JSON this writes.  Run from the repository
root:
    python tests/golden/make_golden.py                      (acene_nmo600, ~12 min on 8 cores)
    python tests/golden/make_golden.py precision_naux5000   (~1.5 h on 8 cores, ~26 GB of memory)
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

def main(name="acene_nmo600"):
    spec = synth.WORKLOADS[name]
    s = synth.make_workload(name)
    freq, wts = grids.gauss_legendre_imag(spec["n_freq"])
    lo, hi = grids.windows(s.eps, s.state_idx, spec["window_ev"])
    nim = spec["n_pade"] // 2
    ref_im = grids.imag_ref_indices(len(freq), nim)
    ref_re = grids.generic_refs(s.eps, s.n_occ, lo, spec["n_pade"] - nim)
    t0 = time.time()
    o = R.CdwacOracle(s, freq, wts, ref_im, ref_re, lo, hi)
    t_prep = time.time() - t0
    res = o.solve_all()
    rng = np.random.default_rng(7)
    w_im = [(int(n), int(m), int(k), float(o.w_im[n, m, k]))
            for n, m, k in zip(rng.integers(0, s.n_states, 40), rng.integers(0, s.n_mo, 40),
                               rng.integers(0, len(freq), 40))]
    w_re = [(int(n), int(m), int(j), float(o.w_re[n, m, j].real), float(o.w_re[n, m, j].imag))
            for n, m, j in zip(rng.integers(0, s.n_states, 40), rng.integers(0, s.n_occ, 40),
                               rng.integers(0, len(ref_re), 40))]
    sig = []
    for n in range(s.n_states):
        for d in (-0.2, 0.1, 0.3):
            om = float(s.eps[n] + d)
            sig.append((n, om, o.sigma(n, om)))
    out = dict(workload=name, seed=spec["seed"], oracle_prepare_s=t_prep,
               qp=[r[0] for r in res], z=[r[1] for r in res], n_evals=[r[2] for r in res],
               flags=[r[3] for r in res], sigma_x=[float(x) for x in o.sigma_x],
               w_im=w_im, w_re=w_re, sigma=sig)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "qp (eV):", [q * synth.HARTREE_EV for q in out["qp"]])


if __name__ == "__main__":
    main(*sys.argv[1:2])
