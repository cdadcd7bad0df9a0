"""Writes stored full-CD self-energies of the 600-orbital workload.

Full contour deformation (Sec. 3.4, CD branch; Eqs. In_term, Rn_term, ffact,
cdselfe) evaluates W directly at every residue |eps_m - omega| + i eta of the
residue term, one complex polarizability and inversion per residue.  For each
core state this script evaluates Sigma_n(omega) that way at one omega, the
state's CD-WAC quasiparticle energy stored by ``make_golden.py`` (so both
files come from the oracle alone).  The GPU tests compare the library's
full-CD self-energy against these values and solve the full-CD root next to
the CD-WAC one.

Calls only the FP64 oracle (``oracle/``) on the seeded synthetic input.  About
1.5 hours on 8 host cores.  Run from the repository root:
python tests/golden/make_fullcd_golden.py
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

NAME = "acene_nmo600"
HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    spec = synth.WORKLOADS[NAME]
    s = synth.make_workload(NAME)
    freq, wts = grids.gauss_legendre_imag(spec["n_freq"])
    lo, hi = grids.windows(s.eps, s.state_idx, spec["window_ev"])
    with open(os.path.join(HERE, f"{NAME}_oracle.json")) as f:
        wac = json.load(f)
    t0 = time.time()
    fc = R.FullCdOracle(s, freq, wts, lo, hi)
    t_prep = time.time() - t0
    rows = []
    for n in range(s.n_states):
        om = float(wac["qp"][n])
        t = time.time()
        i_term = R.integral_term(om, fc.eps_g, fc.w_im[n], fc.freq, fc.weight)
        r_term = R.residue_term(om, fc.eps_g, fc.eps_f, fc.eta, lambda m, z: fc.w_direct(n, m, z))
        n_res = int(np.count_nonzero(R.occupation_factor(fc.eps_g, fc.eps_f, om)))
        sig = float(fc.sigma_x[n] + r_term - i_term)
        rows.append(dict(state=n, omega=om, sigma=sig, r_term=float(r_term), i_term=float(i_term),
                         sigma_x=float(fc.sigma_x[n]), n_residues=n_res, seconds=time.time() - t))
        fc._cache.clear()
        print(f"state {n}: omega = {om * synth.HARTREE_EV:.6f} eV, Sigma = {sig:.15e} Ha, "
              f"{n_res} residues, {time.time() - t:.0f} s", flush=True)
    out = dict(workload=NAME, seed=spec["seed"], eta=fc.eta, oracle_imag_axis_s=t_prep, states=rows)
    path = os.path.join(HERE, f"{NAME}_fullcd_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
