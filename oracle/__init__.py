"""Plain, slow FP64 CPU oracle for the CD-WAC core-level G0W0 self-energy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; both sides take
the same seeded inputs and nothing else.

Modules
-------
``cdwac_ref`` : the self-energy path of Panades-Barrueta & Golze (JCTC 2023),
    step by step (Secs. 2.3, 2.4, 3.2, 3.4): polarizability, dielectric
    inversion, W^c_nm, greedy Thiele-Pade fits, Sigma_n(omega) = Sigma^x +
    R - I and the quasiparticle root.  Also the two references the method
    approximates: full contour deformation (W evaluated directly at every
    residue) and the closed-form pole sum.
``mlp_ref``   : the small learned root seed (8 -> 64 -> 64 -> 1, tanh), its
    gradients by hand and the Adam update.  Not part of the paper.

Every public function cites the passage it follows.  Parity is pinned by the
CPU tests (closed forms, invariants, brute force on tiny inputs); see each
function's docstring for the pin.
"""
