"""Seeded synthetic inputs for the core-level G0W0 self-energy.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic.  The arrays it returns are what the caller of the
library supplies in a real calculation: Kohn-Sham orbital energies (the
eigenvalues entering the non-interacting Green's function, Sec. 2.1) and the
RI-V three-centre coefficients O^{nm}_P (Sec. 2.2, the transformed
three-centre quantities).  Molecules, basis sets and DFT are outside the
library, so the coefficients are Gaussian draws with the shapes of a real run.

Energies are in Hartree.  Recipe (one ``numpy.random.default_rng(seed)`` per
system, fixed draw order):

1. core energies: one core at exactly -290 eV, or ``n_core`` cores drawn
   uniformly in [-290.5, -289.5] eV (a 1 eV band of chemical shifts) and
   sorted;
2. valence energies uniform in [-30, -5] eV, sorted;
3. virtual energies uniform in [0.5, 50] eV, sorted;
4. O^{ia}_P ~ N(0, sigma^2) for every occupied i and virtual a, laid out as
   ``o_ia[P, i * n_virt + a]``;
5. the core x occupied block O^{ni}_P ~ N(0, sigma^2), symmetric in (n, i)
   inside the core x core block;
6. core localisation: every O^{nm}_P with n a core state and m != n is
   multiplied by ``kappa``; the diagonal O^{nn}_P is left as drawn.

Step 6 is a modelling choice for synthetic data: with uncorrelated
coefficients of equal size the core state has no distinct quasiparticle peak,
while the damped coupling gives a single root with Z close to 0.9.

The 1 eV core band keeps every quasiparticle energy (about 3 eV below its
Kohn-Sham level) clear of the other cores' Kohn-Sham levels.  At omega = eps_m
of an occupied m the residue term switches W^c_nm off (Eq. ffact) while the
quadrature of the integral term, which has no node at zero, cannot follow:
Sigma jumps by ~|W^c_nm(0)| there, and a root that would sit inside the jump
does not exist (a 4 eV band put one of 16 cores there).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

#: Hartree in eV (CODATA 2018).
HARTREE_EV = 27.211386245988


@dataclasses.dataclass
class System:
    """One synthetic molecule: energies and RI coefficients (Hartree units).

    ``o_ia``  : [n_aux, n_occ * n_virt] float64, O^{ia}_P with a fastest.
    ``o_nm``  : [n_states, n_aux, n_mo] float64, O^{nm}_P for each core state n.
    ``state_idx`` : orbital index of each core state (the cores are the lowest
    orbitals, so ``state_idx[j] == j``).
    """

    eps: np.ndarray
    n_occ: int
    o_ia: np.ndarray
    o_nm: np.ndarray
    state_idx: np.ndarray
    spin: float = 2.0

    @property
    def n_mo(self) -> int:
        return int(self.eps.shape[0])

    @property
    def n_virt(self) -> int:
        return self.n_mo - self.n_occ

    @property
    def n_aux(self) -> int:
        return int(self.o_ia.shape[0])

    @property
    def n_states(self) -> int:
        return int(self.state_idx.shape[0])


def make_system(n_mo: int, n_occ: int, n_aux: int, n_core: int, sigma: float,
                kappa: float = 0.2, seed: int = 0,
                single_core_ev: float = -290.0) -> System:
    """Draw one synthetic system following the recipe in the module docstring."""
    if not (1 <= n_core <= n_occ < n_mo):
        raise ValueError("need 1 <= n_core <= n_occ < n_mo")
    rng = np.random.default_rng(seed)
    n_virt = n_mo - n_occ
    if n_core == 1:
        core = np.array([single_core_ev])
    else:
        core = np.sort(rng.uniform(-290.5, -289.5, n_core))
    val = np.sort(rng.uniform(-30.0, -5.0, n_occ - n_core))
    virt = np.sort(rng.uniform(0.5, 50.0, n_virt))
    eps = np.concatenate([core, val, virt]) / HARTREE_EV

    k = n_occ * n_virt
    o_ia = np.empty((n_aux, k), dtype=np.float64)
    rows_per_chunk = max(1, (1 << 26) // max(k, 1))
    for r0 in range(0, n_aux, rows_per_chunk):
        r1 = min(n_aux, r0 + rows_per_chunk)
        rng.standard_normal(out=o_ia[r0:r1])
    o_ia *= sigma

    c = rng.standard_normal((n_aux, n_core, n_occ)) * sigma
    cc = c[:, :, :n_core]
    upper = np.triu(np.ones((n_core, n_core), dtype=bool), 1)
    cc_sym = np.where(upper[None], cc, np.transpose(cc, (0, 2, 1)))
    c[:, :, :n_core] = cc_sym

    # core localisation (step 6)
    o3 = o_ia.reshape(n_aux, n_occ, n_virt)
    o3[:, :n_core, :] *= kappa
    offdiag = np.ones((n_core, n_occ))
    offdiag[np.arange(n_core), np.arange(n_core)] = 0.0
    c *= np.where(offdiag > 0, kappa, 1.0)[None]

    o_nm = np.empty((n_core, n_aux, n_mo), dtype=np.float64)
    for n in range(n_core):
        o_nm[n, :, :n_occ] = c[:, n, :]
        o_nm[n, :, n_occ:] = o3[:, n, :]
    return System(eps=eps, n_occ=n_occ, o_ia=o_ia, o_nm=o_nm,
                  state_idx=np.arange(n_core, dtype=np.int32))


#: Workload shapes (energies in the recipe above).  ``sigma=None`` means
#: sigma = sqrt(1.25 / K) with K = n_occ * n_virt: the screening strength
#: K sigma^2 of the 60-orbital case is kept at every size.  With it the
#: largest RPA excitation stays near 70 eV; at K sigma^2 = 20 it rises to
#: ~250 eV and valence-hole + plasmon satellites fall inside the core window,
#: leaving several core states without a distinct quasiparticle root.  The
#: same rule keeps the core coupling n_mo * n_aux * sigma^2 * kappa^2 fixed,
#: since n_mo * n_aux / K is 24 for every workload below.
WORKLOADS = {
    "fp64_1core_nmo60": dict(n_mo=60, n_occ=10, n_aux=200, n_core=1, sigma=0.05,
                             n_freq=32, n_pade=16, window_ev=(-320.0, -260.0), seed=1),
    "acene_nmo600": dict(n_mo=600, n_occ=100, n_aux=2000, n_core=6, sigma=None,
                         n_freq=64, n_pade=24, window_ev=30.0, seed=2),
    "precision_naux5000": dict(n_mo=1500, n_occ=250, n_aux=5000, n_core=16, sigma=None,
                               n_freq=64, n_pade=24, window_ev=30.0, seed=3),
    "mlp_deploy_naux6600": dict(n_mo=2000, n_occ=333, n_aux=6600, n_core=24, sigma=None,
                                n_freq=64, n_pade=24, window_ev=30.0, seed=5),
}


SCREENING = 1.25   # K sigma^2 of the 60-orbital workload


def workload_sigma(spec: dict) -> float:
    if spec.get("sigma") is not None:
        return float(spec["sigma"])
    k = spec["n_occ"] * (spec["n_mo"] - spec["n_occ"])
    return math.sqrt(SCREENING / k)


def make_workload(name: str, seed: Optional[int] = None, kappa: float = 0.2) -> System:
    spec = WORKLOADS[name]
    return make_system(spec["n_mo"], spec["n_occ"], spec["n_aux"], spec["n_core"],
                       workload_sigma(spec), kappa=kappa,
                       seed=spec["seed"] if seed is None else seed)


def batch_specs(n_sys: int = 48, seed: int = 400):
    """Shapes of the uneven batch: N_mo ~ U{100..1200}, N_occ = round(N_mo/6),
    N_aux = round(3.3 N_mo), 1..12 core states; one seed per system."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_sys):
        n_mo = int(rng.integers(100, 1201))
        n_occ = max(2, int(round(n_mo / 6)))
        n_core = int(rng.integers(1, 13))
        n_core = min(n_core, n_occ - 1)
        n_aux = int(round(3.3 * n_mo))
        k = n_occ * (n_mo - n_occ)
        out.append(dict(n_mo=n_mo, n_occ=n_occ, n_aux=n_aux, n_core=n_core,
                        sigma=math.sqrt(SCREENING / k), seed=seed + j))
    return out
