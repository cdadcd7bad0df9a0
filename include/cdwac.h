/*
 * cdwac.h - C ABI of the MI355X (gfx950) CD-WAC core-level G0W0 library.
 *
 * Computes core quasiparticle energies from Kohn-Sham orbital energies and
 * RI-V three-centre coefficients by contour deformation with the screened
 * interaction analytically continued from the imaginary axis (CD-WAC),
 * after Panades-Barrueta & Golze, JCTC 2023:
 *
 *   Pi_PQ(z)   = spin sum_ia O^ia_P O^ia_Q [1/(z - D_ia) - 1/(z + D_ia)]   Eq. (piriv)
 *   Lambda(z)  = [I - Pi(z)]^-1 - I                                        Eq. (bigLambda)
 *   W^c_nm(z)  = sum_PQ O^nm_P Lambda_PQ(z) O^mn_Q                         Eq. (wriv)
 *   T_nm(z)    = greedy Thiele continued fraction in z^2                   Eqs. (pade, rec_eq), Sec. 3.2
 *   Sigma_n(w) = Sigma^x_n + R_n(w) - I_n(w)                               Eqs. (In_term, Rn_term, cdselfe)
 *   eps^QP_n   = eps_n + Re Sigma_n(eps^QP_n) - v^xc_n                     Eq. (qp_eq)
 *
 * Conventions
 *   - Energies in Hartree.  Arrays are row-major (last index fastest).
 *   - "host" pointers are read during the call only; "device" pointers are
 *     HIP device memory on the context's device.  The caller owns every
 *     buffer it passes; the library never frees caller memory.
 *   - Every function returns a cdwac_status.  Arguments are validated before
 *     any kernel is launched; on an error nothing is written to outputs and
 *     cdwac_last_error() describes the problem.  Device-side failures (a
 *     singular pivot in the dielectric inversion, an inverse that fails its
 *     residual check) are reported after the call has synchronised its
 *     stream.
 *   - All work is queued on the context's stream; every call returns after
 *     that stream has been synchronised.  One context per host thread.
 *   - Calls that overlap on one context are not allowed.
 */
#ifndef CDWAC_H
#define CDWAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cdwac_ctx cdwac_ctx;

typedef enum {
    CDWAC_OK = 0,
    CDWAC_EINVAL = -1,   /* invalid argument (shape, ordering, NaN, NULL)            */
    CDWAC_ENOMEM = -2,   /* device allocation failed or caller workspace too small   */
    CDWAC_EHIP = -3,     /* a HIP runtime call failed                                */
    CDWAC_ENOTPD = -4,   /* zero or non-finite pivot while inverting eps = I - Pi    */
    CDWAC_ESTATE = -5,   /* cdwac_qp / cdwac_sigma / cdwac_w_table before prepare    */
    CDWAC_EFACT = -6,    /* an inverse of eps failed its residual check (element
                            growth in the unpivoted sweep of the complex-symmetric,
                            indefinite eps(x + i eta) at a near-real point)          */
    CDWAC_WNOROOT = 1    /* warning: at least one state has no root (qp = NaN)       */
} cdwac_status;

/* Arithmetic of the two dense contractions (Pi and W).  The dielectric
 * inversion, the Pade recursion, the self-energy and the root search are
 * always FP64. */
typedef enum {
    CDWAC_P64 = 0,       /* FP64 matrix cores                                        */
    CDWAC_B16X3 = 1,     /* bf16 hi/lo split (16-bit significands), 3 products       */
    CDWAC_B16 = 2,       /* plain bf16, one product (accuracy ablation only)         */
    CDWAC_F16X3 = 3,     /* fp16 hi/lo split of power-of-two-scaled operands (22-bit
                            significands), 3 products; same matrix-core rate as bf16 */
    CDWAC_F16 = 4        /* Pi: plain fp16 of the scaled operands, one product (its
                            K-term sums average the operand rounding out); W: the
                            fp16 split of CDWAC_F16X3                                */
} cdwac_prec;
/* Every 16-bit mode accumulates in FP32 in the matrix cores over the whole
 * contraction; the sums are converted to FP64 at the end. */

/* Per-state outcome flags. */
enum {
    CDWAC_FLAG_NOROOT = 1,       /* no admissible root in the window: qp = NaN       */
    CDWAC_FLAG_FALLBACK = 2,     /* secant failed, scan + bisection was used          */
    CDWAC_FLAG_MLP_ACCEPTED = 4  /* learned seed, or one Newton step from it, accepted */
};

/* The molecule: mean-field energies and RI-V coefficients (Sec. 2.1-2.2). */
typedef struct {
    int32_t n_mo;              /* number of orbitals                                       */
    int32_t n_occ;             /* occupied orbitals, 1 <= n_occ < n_mo                     */
    int32_t n_aux;             /* auxiliary (RI) functions                                 */
    int32_t n_states;          /* core states to solve, >= 1                               */
    const int32_t *state_idx;  /* host [n_states]: orbital index of each state, < n_occ   */
    const double *eps;         /* host [n_mo]: KS energies, strictly ascending             */
    const double *vxc;         /* host [n_states]: <n|v_xc|n>; NULL means v^xc = Sigma^x   */
    const double *o_ia;        /* device [n_aux][n_occ*(n_mo-n_occ)]: O^{ia}_P, a fastest  */
    const double *o_nm;        /* device [n_states][n_aux][n_mo]: O^{nm}_P of each state   */
    double spin;               /* spin factor of Pi; 2 for a closed shell                  */
    double eps_fermi;          /* Fermi level; NaN selects (HOMO + LUMO) / 2               */
} cdwac_system;

/* Frequencies, Pade reference set and solver settings (Secs. 3.3, 3.4, 4). */
typedef struct {
    int32_t n_freq;            /* imaginary quadrature nodes, >= 1                         */
    const double *freq;        /* host [n_freq]: omega_k > 0                               */
    const double *weight;      /* host [n_freq]: quadrature weights for int_0^inf          */
    int32_t n_ref_im;          /* imaginary nodes re-used as Pade references               */
    const int32_t *ref_im_idx; /* host [n_ref_im]: distinct indices into freq              */
    int32_t n_ref_re;          /* near-real Pade references x_j + i*eta_ref;
                                  1 <= n_ref_im + n_ref_re <= 256 (M of the paper's
                                  CD-WAC(N_core, N_valence, N_Im) is at most 240)         */
    const double *ref_re;      /* host [n_ref_re]: x_j >= 0                                */
    double eta_ref;            /* imaginary part of the near-real references (> 0)         */
    double eta;                /* broadening of the residue term, W(|eps_m - w| + i eta)   */
    double pade_tol;           /* greedy stop: max remaining L1 error <= tol * max|W|      */
    const double *win_lo;      /* host [n_states]: QP search window; must contain the
                                  state's own eps_n, where the root search starts        */
    const double *win_hi;      /* host [n_states]                                          */
    double qp_tol;             /* secant step tolerance (Ha), e.g. 1e-10                   */
    int32_t qp_maxit;          /* secant iterations, e.g. 100                              */
    int32_t prec;              /* cdwac_prec                                               */
    int32_t use_mlp_seed;      /* 1: start the root search at the learned seed             */
    double mlp_accept;         /* |f(seed)| (Ha) below which the seed is the answer        */
    double freq_rank_tol;      /* 16-bit modes: > 0 runs Pi, the inversion and the W
                                  contraction only at a skeleton of the imaginary nodes and
                                  interpolates W^c_nm at the others (decomposition of the
                                  family 1/(w^2 + Omega^2) over the RPA excitation range,
                                  sup-norm error <= tol relative to each function's
                                  maximum; falls back to every node if the range check
                                  fails); 0 uses every node.  Ignored by CDWAC_P64.  [0, 1).
                                  A tolerance at the mode's own imaginary-axis W error adds
                                  no visible error: about 1e-6 for CDWAC_F16, 1e-8 for the
                                  splits (measured at N_aux = 5000). */
    int32_t fit_all;           /* 1: fit W^c_nm of every m (all (n, m) pairs); 0: only the
                                  m whose residue can enter the window (Eq. ffact).  The
                                  QP results are the same; 1 is the heavier fit load.     */
    int32_t near_real_f64;     /* 16-bit modes: 1 computes Pi at the near-real reference
                                  points on the FP64 path (the imaginary nodes stay 16-bit).
                                  There W sits within eta_ref of RPA poles Omega_s of up to
                                  ~10 Ha (core excitations); a relative error d of Pi moves
                                  them by ~d*Omega, i.e. by d*Omega/eta_ref of the pole
                                  width, so 16-bit Pi leaves W good to only ~1e-4..1e-2
                                  there.  Costs FP64 matrix-core time for 2*n_ref_re planes
                                  and an FP64 copy of O^{ia}.                              */
    int32_t quad_limit;        /* 1: the integral term I_n takes the a_m = omega - eps_m -> 0
                                  limit analytically: W_nm(i w') is split into
                                  w0 g(w') + [W_nm(i w') - w0 g(w')], g = 1 / (1 + w'^2 / Ha^2),
                                  w0 = Re of the residue term's own W at a_m = 0 (the Pade
                                  model at i eta), the first part integrated in closed form
                                  and only the remainder by quadrature.  Without it a
                                  Lorentzian narrower than the grid's smallest node is
                                  missed and Sigma_n steps by ~W_nm(0) at omega = eps_m:
                                  the evGW0 and G_dH W0 roots sit at such a point for the
                                  state's own m.  Applies to the orbitals with a model (the
                                  fit range, or every m with fit_all).  0: the plain
                                  quadrature.  May differ between the systems of a
                                  batch.                                                   */
} cdwac_params;

/* Result for one state (host, written by cdwac_qp / cdwac_solve). */
typedef struct {
    double qp;                 /* quasiparticle energy, NaN if no root                     */
    double z;                  /* renormalisation factor 1 / (1 - dSigma/dw) at qp         */
    double sigma_x;            /* exchange self-energy Sigma^x_n                           */
    double sigma_c;            /* Re Sigma^c_n(qp) = R_n(qp) - I_n(qp)                      */
    double residual;           /* f(qp) = qp - eps_n - Re Sigma_n(qp) + v^xc_n             */
    int32_t n_evals;           /* self-energy evaluations used                             */
    int32_t flags;             /* CDWAC_FLAG_*                                             */
    int32_t n_rounds;          /* passes over the W tables and fits those evaluations took;
                                  points evaluated together (the Z pair, the learned seed's
                                  samples) count once                                      */
} cdwac_state_out;

/* Context: binds a device and a stream.  hip_stream NULL = the null stream. */
int cdwac_ctx_create(cdwac_ctx **out, int device, void *hip_stream);
void cdwac_ctx_destroy(cdwac_ctx *ctx);
const char *cdwac_last_error(const cdwac_ctx *ctx);

/* Device workspace needed by cdwac_prepare for this system and settings. */
size_t cdwac_workspace_bytes(const cdwac_system *sys, const cdwac_params *prm);

/* Hands the context a caller-owned device workspace (e.g. a torch tensor).
 * Without one, cdwac_prepare allocates (and the context frees) its own. */
int cdwac_set_workspace(cdwac_ctx *ctx, void *dev_ptr, size_t bytes);

/* Stages (a) Pi, (b) eps = I - Pi and Lambda, (c) W^c_nm at every imaginary
 * node and near-real reference, Sigma^x, and (d) the greedy Thiele fits of
 * every (n, m) whose residue can enter a window (Sec. 3.4, everything before
 * the QP iteration).  The results stay in the workspace for the calls below;
 * the input arrays may be freed afterwards.
 * Every inverse eps^-1 (Eq. bigLambda) is checked on 4 sampled columns eps_j
 * of eps: CDWAC_EFACT if max|eps^-1 eps_j - e_j| exceeds 1e-8 of
 * max(|eps^-1| |eps_j|) (cdwac_inversion_residual gives the value).
 * CDWAC_ENOTPD for a zero or non-finite pivot. */
int cdwac_prepare(cdwac_ctx *ctx, const cdwac_system *sys, const cdwac_params *prm);

/* Stage (e): Sigma_n(omega) and the QP root for every state, using the
 * prepared W tables and fits.  vxc: host [n_states] or NULL (the value given
 * to prepare).  out: host [n_states]. */
int cdwac_qp(cdwac_ctx *ctx, const double *vxc, cdwac_state_out *out);

/* cdwac_prepare followed by cdwac_qp. */
int cdwac_solve(cdwac_ctx *ctx, const cdwac_system *sys, const cdwac_params *prm,
                cdwac_state_out *out);

/* A batch of independent systems of uneven size (Sec. 3.4 for each): Pi,
 * eps^-1 and W of every system in turn (each a full-width launch of its own
 * shape), then the greedy Thiele fits of all systems in ONE launch and the QP
 * roots of all states of all systems in ONE launch.
 * sys, prm: host arrays [n_sys]; every prm[j] must have the same
 * n_ref_im + n_ref_re and pade_tol (the fits share one launch).
 * out: host [sum of sys[j].n_states], the states of system 0 first.
 * The batch's W tables, fits and QP inputs live in device memory the context
 * allocates (kept for reuse, freed by cdwac_ctx_destroy); the per-system work
 * uses the workspace as cdwac_prepare does.  The context is left unprepared
 * (cdwac_qp/cdwac_sigma need a new cdwac_prepare).  Every argument is checked
 * before any launch; returns CDWAC_WNOROOT if a state has no root. */
int cdwac_solve_batch(cdwac_ctx *ctx, int32_t n_sys, const cdwac_system *sys, const cdwac_params *prm,
                      cdwac_state_out *out);

/* Re Sigma_n(omega) = Sigma^x + Re R_n - I_n (Eq. cdselfe) at n_omega
 * frequencies per state.  omega, sigma: device [n_states][n_omega].
 * Also writes I_n and R_n when i_term / r_term are non-NULL (same shape).
 * Unless the preparation had fit_all = 1, every omega of state j must lie in
 * its window [win_lo[j], win_hi[j]] widened by 1e-4 Ha: only the orbitals whose
 * residue can enter that window have Pade models, so CDWAC_EINVAL otherwise. */
int cdwac_sigma(cdwac_ctx *ctx, int32_t n_omega, const double *omega, double *sigma,
                double *i_term, double *r_term);

/* Replaces the orbital energies of G in the self-energy (I_n and R_n of
 * Eqs. In_term, Rn_term, the occupation factors of Eq. ffact and the Fermi
 * level) while W and its continuation stay as prepared: the G of the
 * eigenvalue-self-consistent schemes of Sec. 4.  The QP equation keeps the KS
 * eps_n and v^xc_n.  eps_g: host [n_mo] (Ha).  eps_fermi: NaN selects the
 * midpoint of eps_g[n_occ - 1] and eps_g[n_occ].  Needs a preparation with
 * fit_all = 1 (moved energies can put any m's residue in the window).
 * Holds until the next cdwac_prepare. */
int cdwac_set_g_energies(cdwac_ctx *ctx, const double *eps_g, double eps_fermi);

/* Eigenvalue self-consistency (Sec. 4, the evGW0 and evGW flavours):
 * mode 0 (evGW0) prepares W once from the KS energies and iterates the QP
 * equations with the QP energies in G; mode 1 (evGW) also rebuilds Pi, eps^-1,
 * W and the fits from the QP energies every iteration.  The energies of the
 * computed states (sys->state_idx) are updated after every iteration, the
 * others keep their input values; a state without a root keeps its energy.
 * Stops when no energy moves by more than tol (Ha) or after max_iter QP
 * solves.  prm is used with fit_all = 1 and without the learned seed.
 * eps_out: host [n_mo], the final energies; n_iter: host, the QP solves done;
 * out: host [n_states], the last solve's results.  Returns CDWAC_WNOROOT if a
 * state of the last solve has no root. */
int cdwac_evgw(cdwac_ctx *ctx, const cdwac_system *sys, const cdwac_params *prm, int32_t mode,
               int32_t max_iter, double tol, double *eps_out, int32_t *n_iter, cdwac_state_out *out);

/* G_dH W0 (Sec. 4, the Hedin-shift flavour): a shift dH_n in the denominator
 * of G, i.e. every energy of G and the Fermi level moved by dH_n in the
 * self-energy of state n, W and its continuation kept as prepared.  dH_n is
 * fixed before the QP iteration; the paper gives its place, not its recipe,
 * and it is taken here as the first-order G0W0 correction at the state's
 * own energy, dH_n = Re Sigma_n(eps_n) - v^xc_n (prepared G).  Then Eq. (qp_eq)
 * is solved with Sigma_n of the shifted G (which equals the unshifted
 * Sigma_n at omega - dH_n).  Needs a preparation with fit_all = 1 (the shifted
 * residues reach every m).  vxc: host [n_states] or NULL (the value in use);
 * out: host [n_states]; shift: host [n_states], the dH_n used, or NULL.
 * Returns CDWAC_WNOROOT if a state has no root. */
int cdwac_qp_hedin(cdwac_ctx *ctx, const double *vxc, cdwac_state_out *out, double *shift);

/* Sigma_n(omega) by full contour deformation (Sec. 2.3, Eqs. Rn_term,
 * In_term, cdselfe): W^c_nm evaluated directly at every residue
 * |eps_m - omega| + i*eta with f_m(omega) != 0 (Eq. ffact), i.e. one complex
 * polarizability, inversion and contraction per residue -- the O(N^5) method
 * CD-WAC replaces.  state: index into sys->state_idx; the imaginary grid and
 * the precision come from prm (its Pade reference set is not used).
 * out: host [3] = {Sigma_n, R_n, I_n} (Ha).  n_res: host, the residue count
 * (may be NULL).  The residues go through in chunks of at most 255 near-real
 * planes per preparation (the imaginary-axis part is recomputed for each
 * chunk).  Leaves the context unprepared.  Synchronous. */
int cdwac_sigma_cd(cdwac_ctx *ctx, const cdwac_system *sys, const cdwac_params *prm, int32_t state,
                   double omega, double *out, int32_t *n_res);

/* Diagonal spectral function (Sec. 5.5): with the complex self-energy
 * Sigma_n = Sigma^x + R_n - I_n (the imaginary part comes from the residue
 * term, i.e. from the Pade models at |eps_m - w| + i eta),
 *   A_n(w) = (1/pi) |Im[1 / (w - eps_n - Sigma_n(w) + v^xc_n)]|.
 * omega, spectral: device [n_states][n_omega] (Ha, 1/Ha); sigma_re, sigma_im:
 * device, same shape, or NULL.  vxc: host [n_states] or NULL (the value in
 * use; a non-NULL vxc replaces it, as in cdwac_qp).  n_omega <= 65535 per call.
 * The window condition of cdwac_sigma applies. */
int cdwac_spectral(cdwac_ctx *ctx, int32_t n_omega, const double *omega, const double *vxc, double *spectral,
                   double *sigma_re, double *sigma_im);

/* Copies of the prepared tables (device outputs):
 * w_im [n_states][n_mo][n_freq]  W^c_nm(i omega_k), real;
 * w_re [n_fit][n_ref_re][2]      W^c_nm(x_j + i eta_ref) for the fitted (n, m),
 *                                 in the order of cdwac_fit_ranges;
 * sigma_x [n_states].  Any pointer may be NULL. */
int cdwac_w_table(cdwac_ctx *ctx, double *w_im, double *w_re, double *sigma_x);

/* Fitted orbital range [m0, m1) of each state (host [n_states] each). */
int cdwac_fit_ranges(cdwac_ctx *ctx, int32_t *m0, int32_t *m1, int32_t *n_fit_total);

/* Stage (a) alone: Pi(z) for n_z complex arguments z = z_re + i z_im (host).
 * pi_re, pi_im: device [n_z][n_aux][n_aux], full symmetric; pi_im may be NULL
 * when every z_re is 0 (Pi is then real). */
int cdwac_polarizability(cdwac_ctx *ctx, const cdwac_system *sys, int32_t prec, int32_t n_z,
                         const double *z_re, const double *z_im, double *pi_re, double *pi_im);

/* Stage (d) alone: greedy Thiele fits of n_fit independent data sets and
 * their values at n_x points each.  u, w: device [n_fit][n_pts][2] (complex
 * u_j = z_j^2 and W_j); x: device [n_fit][n_x][2] (complex z^2 at which to
 * evaluate); out: device [n_fit][n_x][2]; n_terms: device [n_fit] or NULL.
 * n_pts <= 256. */
int cdwac_pade_fit_eval(cdwac_ctx *ctx, int32_t n_fit, int32_t n_pts, const double *u,
                        const double *w, double tol, int32_t n_x, const double *x,
                        double *out, int32_t *n_terms);

/* Largest sampled residual of the inversions of the last preparation,
 * max|eps^-1 eps_j - e_j| / max(|eps^-1| |eps_j|) over 4 columns j of every
 * eps(z) (Eq. bigLambda), also after CDWAC_EFACT; matrix: its index (imaginary
 * planes first, then one per near-real reference), -1 if none was checked.
 * Host outputs; either may be NULL. */
int cdwac_inversion_residual(const cdwac_ctx *ctx, double *worst, int32_t *matrix);

/* cdwac_pade_fit_eval without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results; the coefficients,
 * nodes and term counts live in a fixed scratch array of the library (one per
 * device, about 18 MiB, held until the process ends) instead of a per-call
 * allocation.  Limit: n_fit * n_pts <= 524288 (CDWAC_EINVAL beyond, checked
 * before any launch).  Every call on a device uses that device's one scratch
 * array: calls that overlap on one device (several contexts or host threads)
 * race and must be serialised by the caller.  Synchronous, except while the
 * context's stream is being captured into a HIP graph: then the kernels and
 * the copy of n_terms are recorded into the caller's graph and the call
 * returns at once; the results appear when the graph runs (each replay reads
 * u, w and x afresh and rewrites the scratch, out and n_terms). */
int cdwac_pade_fit_eval_noalloc(cdwac_ctx *ctx, int32_t n_fit, int32_t n_pts, const double *u,
                                const double *w, double tol, int32_t n_x, const double *x,
                                double *out, int32_t *n_terms);

/* Per-stage timing with HIP events recorded on the context's stream around
 * the kernels of each stage (0 = off, the default). */
int cdwac_set_timing(cdwac_ctx *ctx, int on);

/* Milliseconds of the stages of the last cdwac_prepare / cdwac_qp with timing
 * on: [0] staging (weights, operand split), [1] polarizability contraction
 * kernels only, [2] sweep inversion, [3] Lambda finalisation, [4] W
 * contraction and reduction, [5] exchange and Pade fits, [6] QP kernel,
 * [7] prescaling of the polarizability operand (16-bit modes).  Writes
 * min(n, 8) values; stages not run are 0. */
#define CDWAC_N_STAGES 8
int cdwac_get_timing(const cdwac_ctx *ctx, double *ms, int32_t n);

/* Number of timed segments behind each stage of cdwac_get_timing (same
 * order).  Stage 1 times each polarizability launch as one segment, so
 * ms[1] / count[1] is the average duration of one contraction launch. */
int cdwac_get_timing_segments(const cdwac_ctx *ctx, int32_t *count, int32_t n);

/* Planes of the last cdwac_prepare: imaginary nodes that went through Pi,
 * the inversion and W (all n_freq, or the skeleton), and all planes
 * (imaginary + 2 per near-real reference). */
int cdwac_plane_counts(const cdwac_ctx *ctx, int32_t *n_imag, int32_t *n_planes);

/* Host-only: the decomposition that freq_rank_tol selects.  For imaginary
 * nodes freq [n_freq] (> 0) and excitation energies in [omega_lo, omega_hi]
 * (Ha), writes the skeleton node indices skel [*n_skel] (ascending, always
 * including the largest node), the other indices rest [n_freq - *n_skel] and
 * T [n_freq - *n_skel][*n_skel] with
 * 1/(w_rest[r]^2 + O^2) ~= sum_s T[r][s] / (w_skel[s]^2 + O^2).  If no rank
 * below n_freq meets tol, *n_skel = n_freq and skel = 0 .. n_freq-1.  Output
 * arrays must hold n_freq (skel, rest) and n_freq^2 (T) entries.  tol in (0, 1). */
int cdwac_freq_decomposition(int32_t n_freq, const double *freq, double omega_lo, double omega_hi, double tol,
                             int32_t *n_skel, int32_t *skel, int32_t *rest, double *T);

/* ---- Learned QP seed: MLP 8 -> 64 -> 64 -> 1 (tanh), FP32 ----------------
 * Parameter vector (CDWAC_MLP_NPARAM floats): W1[64][8], b1[64], W2[64][64],
 * b2[64], W3[1][64], b3[1].  With use_mlp_seed the root search first
 * evaluates, in one pass over the tables, f(w) = w - eps_n - Sigma_n(w) +
 * v^xc_n at the four points w_j = eps_n + d_j, d = (-0.1, -0.05, 0.05, 0.1)
 * Ha (all four must lie in the window, else the plain search runs).  The
 * least-squares line through (d_j, f(w_j)) gives w_N = eps_n - mean(f) /
 * slope (eps_n - mean(f) if the slope is not positive), clamped to the
 * window.  Newton's method on the cubic interpolating the four values of f
 * (divided differences), started from w_N, 40 steps or until the cubic's
 * slope is not positive, gives w_C (w_N if that point is outside the window
 * or not finite).  Features (Ha): eps_n, eps_F, Sigma^x - v^xc,
 * Re Sigma^c(w_0..w_3), w_C - eps_n; the network predicts w* - w_C.  Inputs are
 * standardised with (mu, sd) and the output is y * out_sd + out_mu.  A
 * second pass evaluates f at the seed and at seed +- 1e-4 Ha: the seed is
 * the root if |f| <= mlp_accept and its Z is in (0, 1] (flag
 * CDWAC_FLAG_MLP_ACCEPTED, two passes in all).  Otherwise, if that Z is in
 * (0, 1], a third pass evaluates f at the Newton step w_1 = seed - f Z and at
 * w_1 +- 1e-4 Ha, and w_1 is the root under the same test (the same flag,
 * three passes); if it fails the secant continues from the seed and w_1.
 * With an unphysical Z at the seed the secant continues from the sample
 * nearest the seed and the seed.  If that secant has not converged after 12
 * steps (or qp_maxit, if smaller) the plain search from eps_n runs.  An accepted root is good to mlp_accept in f, not to qp_tol. */
#define CDWAC_MLP_NIN 8
#define CDWAC_MLP_NPARAM 4801

/* Installs the seed model used by cdwac_qp when use_mlp_seed = 1 (copied;
 * the caller keeps its arrays).  theta: host [4801]; mu, sd: host [8];
 * out_mu, out_sd: scalars.  CDWAC_EINVAL for NULL arrays, sd <= 0, out_sd <= 0
 * or non-finite mu, out_mu, out_sd. */
int cdwac_mlp_set_model(cdwac_ctx *ctx, const float *theta, const float *mu, const float *sd,
                        float out_mu, float out_sd);

/* Forward pass on n standardised samples: x device [n][8] -> y device [n]. */
int cdwac_mlp_forward(cdwac_ctx *ctx, const float *theta, int32_t n, const float *x, float *y);

/* Mean squared error loss and its gradient: x device [n][8], t device [n],
 * grad device [4801], loss device [1]. */
int cdwac_mlp_grad(cdwac_ctx *ctx, const float *theta, int32_t n, const float *x,
                   const float *t, float *grad, float *loss);

/* One Adam step (Kingma & Ba) in place on device theta, m, v [4801];
 * step >= 1. */
int cdwac_mlp_adam(cdwac_ctx *ctx, float *theta, const float *grad, float *m, float *v,
                   int32_t step, float lr, float beta1, float beta2, float adam_eps);

/* Minibatch training: epochs over n samples in a seeded shuffled order,
 * batch size <= 1024.  theta, m, v: device [4801], updated in place;
 * loss_curve: host [epochs] (mean loss per epoch) or NULL. */
int cdwac_mlp_train(cdwac_ctx *ctx, float *theta, float *m, float *v, int32_t n,
                    const float *x, const float *t, int32_t epochs, int32_t batch, float lr,
                    uint64_t seed, float *loss_curve);

#ifdef __cplusplus
}
#endif
#endif /* CDWAC_H */
