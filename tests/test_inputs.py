"""Host logic: synthetic generator and frequency grids (no GPU)."""
import numpy as np
import pytest

from paper_2305_15955_amd import grids, synth


def test_generator_shapes_and_symmetry():
    s = synth.make_system(40, 8, 30, 3, 0.05, kappa=0.2, seed=4)
    assert s.eps.shape == (40,) and np.all(np.diff(s.eps) > 0)
    assert s.o_ia.shape == (30, 8 * 32) and s.o_nm.shape == (3, 30, 40)
    ev = s.eps * synth.HARTREE_EV
    assert np.all((ev[:3] > -290.5) & (ev[:3] < -289.5))
    assert np.all((ev[3:8] > -30) & (ev[3:8] < -5))
    assert np.all((ev[8:] > 0.5) & (ev[8:] < 50))
    # O^{nm} consistent with O^{ia} for the virtual block, symmetric core block
    for n in range(3):
        np.testing.assert_array_equal(s.o_nm[n, :, 8:], s.o_ia.reshape(30, 8, 32)[:, n, :])
        for m in range(3):
            np.testing.assert_array_equal(s.o_nm[n, :, m], s.o_nm[m, :, n])
    # seeded: identical on a second draw, different for another seed
    s2 = synth.make_system(40, 8, 30, 3, 0.05, kappa=0.2, seed=4)
    np.testing.assert_array_equal(s.o_ia, s2.o_ia)
    s3 = synth.make_system(40, 8, 30, 3, 0.05, kappa=0.2, seed=5)
    assert not np.array_equal(s.o_ia, s3.o_ia)


def test_single_core_at_minus_290():
    s = synth.make_workload("fp64_1core_nmo60")
    assert s.eps[0] * synth.HARTREE_EV == pytest.approx(-290.0, abs=1e-9)
    assert s.n_aux == 200 and s.n_mo == 60 and s.n_occ == 10


def test_grids():
    f, w = grids.gauss_legendre_imag(32)
    assert np.all(f > 0) and np.all(np.diff(f) > 0) and np.all(w > 0)
    idx = grids.imag_ref_indices(32, 8)
    assert idx[0] == 0 and idx[-1] == 31 and len(np.unique(idx)) == 8
    eps = np.array([-10.0, -1.0, -0.5, 0.2, 1.0])
    lo, hi = grids.windows(eps, [0], 27.211386245988)
    assert lo[0] == pytest.approx(-11.0) and hi[0] == pytest.approx(-9.0)
    x = grids.generic_refs(eps, 3, lo, 5)
    assert x[0] == 0.0 and x[-1] == pytest.approx(grids.midgap(eps, 3) + 11.0)
    r = grids.refined_refs(eps, 3, [0], lo, hi, 4, 3, 0.5, 0.2)
    assert len(r) == 7 and np.all(r >= 0)


def test_batch_specs():
    specs = synth.batch_specs()
    assert len(specs) == 48
    for sp in specs:
        assert 100 <= sp["n_mo"] <= 1200 and 1 <= sp["n_core"] <= 12
        assert sp["n_aux"] == round(3.3 * sp["n_mo"])


def test_refined_reference_points():
    """CD-WAC(N_core, N_valence, N_Im) reference sets (Sec. 3.3)."""
    s = synth.make_workload("acene_nmo600")
    lo, hi = grids.windows(s.eps, s.state_idx, 30.0)
    ev = 1.0 / synth.HARTREE_EV
    ri, rr = grids.cdwac_setting(s.eps, s.n_occ, s.state_idx, lo, hi, 20, 20, 200, 200)
    assert len(ri) == 200 and np.array_equal(ri, np.arange(200)) and len(rr) == 40
    core, val = rr[:20], rr[20:]
    omega = 0.5 * (lo.mean() + hi.mean())
    cc = abs(s.eps[s.state_idx].mean() - omega)
    cv = abs(grids.midgap(s.eps, s.n_occ) - omega)
    # the core neighbourhood starts at 0 (centre < delta_c), ends at centre + 10 eV
    assert core[0] == 0.0 and core[-1] == pytest.approx(cc + 10 * ev)
    assert val[0] == pytest.approx(cv - 30 * ev) and val[-1] == pytest.approx(cv + 30 * ev)
    for part in (core, val):
        assert np.all(np.diff(part) > 0) and np.allclose(np.diff(part), np.diff(part)[0])
    # every valence residue seen from the core energies lies in the valence neighbourhood
    occ_val = s.eps[s.n_states:s.n_occ]          # the cores are the lowest orbitals
    res = np.abs(occ_val[:, None] - s.eps[s.state_idx][None, :])
    assert res.min() >= val[0] and res.max() <= val[-1]
    # one point sits at the centre; N = 0 drops the region
    one = grids.refined_refs(s.eps, s.n_occ, s.state_idx, lo, hi, 1, 0)
    assert one.shape == (1,) and one[0] == pytest.approx(cc)
    assert len(grids.refined_refs(s.eps, s.n_occ, s.state_idx, lo, hi, 0, 0)) == 0
    with pytest.raises(ValueError):
        grids.refined_refs(s.eps, s.n_occ, s.state_idx, lo, hi, 2, 2, delta_c=0.0)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message before touching a GPU."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
