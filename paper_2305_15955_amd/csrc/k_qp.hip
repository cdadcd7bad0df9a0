// Self-energy and quasiparticle root on the GPU, FP64 (Sec. 2.3 Eqs.
// In_term, Rn_term, ffact, cdselfe; Eq. qp_eq; Sec. 3.4).
//
//   I_n(w) = (1/pi) sum_m sum_k w_k W^c_nm(i w_k) a_m / (a_m^2 + w_k^2),  a_m = w - eps_m
//            (the imaginary-axis integral folded over +-w', W^c even and real there)
//   R_n(w) = sum_m f_m Re T_nm(|a_m| + i eta),  f_m of Eq. (ffact) with theta(0) = 1/2
//   Sigma_n(w) = Sigma^x_n + R_n(w) - I_n(w)
//
// One workgroup per state; every thread runs the same root-search control
// flow on block-reduced values.  Root search: secant from eps_n (or from the
// learned seed) and one fixed-point step; fallback: scan the window at 0.01 Ha,
// bisect every upward sign change with |f| < 0.1 Ha on both sides, drop a
// candidate whose |f| at the final midpoint exceeds 1e-8 Ha (a jump across a
// pole), and keep the root of largest Z (then the one nearest eps_n).
#include "common.h"
#include "kernels.h"

namespace cdwac {

constexpr double kScanStep = 0.01, kScanFmax = 0.1, kBisectTol = 1e-12, kZStep = 1e-4, kFTol = 1e-9,
                 kRootFTol = 1e-8;
constexpr int kQpThreads = 256, kMaxFreq = 512;
// Secant steps allowed after a rejected learned seed before the plain search
// from eps_n takes over (a seed in the wrong basin must not cost qp_maxit).
constexpr int kSeedSecantIt = 12;
// Newton iterations on the seed samples' interpolating cubic.
constexpr int kCubicIt = 40;
// Offsets from eps_n (Ha) of the learned seed's four self-energy samples
// (symmetric: they sum to zero).
__constant__ const double kSeedOffset[4] = {-0.1, -0.05, 0.05, 0.1};
constexpr double kPi = 3.14159265358979323846;

__device__ inline double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kQpThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double theta(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? 0.0 : 0.5); }

// Width (Ha) of the Lorentzian g(w') = 1 / (1 + w'^2 / gamma^2) split off in the
// analytic a_m -> 0 limit of the integral term.
constexpr double kQuadGamma = 1.0;

struct Shared {
    double red[kQpThreads];
    double freq[kMaxFreq];
    double weight[kMaxFreq];
    double glor[kMaxFreq];   // g(w_k) of the analytic limit
    float h1[64];
    float h2[64];
};

// I_n and R_n of state s at K frequencies in one pass over the tables: every
// W^c_nm(i w_k) and Pade model is read once and used for all K points, and the
// K sums are reduced together (one "round" of the root search).  The
// arithmetic of each point is that of a single evaluation.  A shift dH of
// every energy of G and of the Fermi level (G_dH W0) enters only through
// omega - eps_m and eps_F - eps_m, so it is applied as omega - dH.
template <int K, bool RES = true>
__device__ void sigma_multi(const QpArgs& A, int s, const double (&omega_in)[K], Shared& sh, double (&I)[K],
                            double (&R)[K], double* Ri = nullptr) {
    const double dh = A.g_shift ? A.g_shift[s] : 0.0;
    double omega[K];
#pragma unroll
    for (int j = 0; j < K; ++j) omega[j] = A.g_shift ? omega_in[j] - dh : omega_in[j];
    const int nf = A.n_freq;
    const double* W = A.w_im + (int64_t)s * A.n_mo * nf;
    double isum[K], rsum[K], risum[K];
#pragma unroll
    for (int j = 0; j < K; ++j) isum[j] = rsum[j] = risum[j] = 0.0;
    const int m0 = A.m0[s], m1 = A.m1[s], foff = A.fit_off[s];
    for (int m = threadIdx.x; m < A.n_mo; m += kQpThreads) {
        const double em = A.eps[m];
        double am[K], am2[K], acc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            am[j] = omega[j] - em;
            am2[j] = am[j] * am[j];
            acc[j] = 0.0;
        }
        const double* wm = W + (int64_t)m * nf;
        // the analytic a_m -> 0 limit: w0 g(w') integrated in closed form,
        // the remainder (zero at w' = 0) by quadrature
        const double w0 = (A.w0 && m >= m0 && m < m1) ? A.w0[foff + (m - m0)] : 0.0;
        if (w0 != 0.0) {
            for (int k = 0; k < nf; ++k) {
                const double wk = sh.weight[k] * (wm[k] - w0 * sh.glor[k]), f2 = sh.freq[k] * sh.freq[k];
#pragma unroll
                for (int j = 0; j < K; ++j) acc[j] += wk * (am[j] / (am2[j] + f2));
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double sg = am[j] > 0.0 ? 1.0 : (am[j] < 0.0 ? -1.0 : 0.0);
                acc[j] += w0 * (0.5 * kPi) * sg * kQuadGamma / (fabs(am[j]) + kQuadGamma);
            }
        } else {
            for (int k = 0; k < nf; ++k) {
                const double wk = sh.weight[k] * wm[k], f2 = sh.freq[k] * sh.freq[k];
#pragma unroll
                for (int j = 0; j < K; ++j) acc[j] += wk * (am[j] / (am2[j] + f2));
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) isum[j] += acc[j];
    }
    for (int m = m0 + threadIdx.x; RES && m < m1; m += kQpThreads) {
        const double em = A.eps[m];
        const int f = foff + (m - m0);
        const double* a = A.coef + (int64_t)f * A.n_pts * 2;
        const double* nd = A.node + (int64_t)f * A.n_pts * 2;
        const int p = A.nterm[f];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double fm =
                -theta(A.eps_f - em) * theta(em - omega[j]) + theta(em - A.eps_f) * theta(omega[j] - em);
            if (fm == 0.0) continue;
            const cplx z = cmk(fabs(em - omega[j]), A.eta);
            const cplx u = z * z;
            cplx val = cmk(0.0, 0.0);
            if (p > 0) {
                cplx t = cmk(1.0, 0.0);
                for (int q = p - 1; q >= 1; --q)
                    t = cmk(1.0, 0.0) + (cmk(a[2 * q], a[2 * q + 1]) * (u - cmk(nd[2 * q - 2], nd[2 * q - 1]))) / t;
                val = cmk(a[0], a[1]) / t;
            }
            rsum[j] += fm * val.re;
            risum[j] += fm * val.im;
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        I[j] = block_sum(isum[j], sh.red) / kPi;
        R[j] = block_sum(rsum[j], sh.red);
        if (Ri) Ri[j] = block_sum(risum[j], sh.red);
    }
}

// I_n(omega) and R_n(omega) for state s (Im R_n into *Ri when given).
__device__ inline void sigma_terms(const QpArgs& A, int s, double omega, Shared& sh, double& I, double& R,
                                   double* Ri = nullptr) {
    const double om[1] = {omega};
    double i1[1], r1[1];
    sigma_multi<1>(A, s, om, sh, i1, r1, Ri);
    I = i1[0];
    R = r1[0];
}

// The integral term alone (full CD adds the directly evaluated residues).
__device__ inline double integral_only(const QpArgs& A, int s, double omega, Shared& sh) {
    const double om[1] = {omega};
    double i1[1], r1[1];
    sigma_multi<1, false>(A, s, om, sh, i1, r1);
    return i1[0];
}

__device__ inline double sigma_total(const QpArgs& A, int s, double omega, Shared& sh) {
    double I, R;
    sigma_terms(A, s, omega, sh, I, R);
    return A.sigx[s] + R - I;
}

// Single-sample MLP 8 -> 64 -> 64 -> 1 (tanh) on standardised features.
__device__ float mlp_one(const float* __restrict__ th, const float* x, Shared& sh) {
    const float* W1 = th;
    const float* b1 = W1 + 64 * 8;
    const float* W2 = b1 + 64;
    const float* b2 = W2 + 64 * 64;
    const float* W3 = b2 + 64;
    const float* b3 = W3 + 64;
    if (threadIdx.x < 64) {
        float a = b1[threadIdx.x];
        for (int i = 0; i < 8; ++i) a += W1[threadIdx.x * 8 + i] * x[i];
        sh.h1[threadIdx.x] = tanhf(a);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        float a = b2[threadIdx.x];
        for (int i = 0; i < 64; ++i) a += W2[threadIdx.x * 64 + i] * sh.h1[i];
        sh.h2[threadIdx.x] = tanhf(a);
    }
    __syncthreads();
    float y = b3[0];
    for (int i = 0; i < 64; ++i) y += W3[i] * sh.h2[i];
    __syncthreads();
    return y;
}

// Root of the QP equation for state s of the system A, written to *dst by
// thread 0 (the whole workgroup evaluates Sigma together).
// Zero of the cubic interpolating (d_j, f_j), j = 0..3, in Newton's divided-
// difference form, by Newton's method on the cubic started from the line
// estimate wl (absolute energies: d = w - e_n).  An iteration stops where the
// cubic's slope is not positive; a result outside [lo, hi] or not finite
// gives wl back.
__device__ inline double cubic_root(const double* d, const double* f, double e_n, double wl, double lo,
                                    double hi) {
    double a[4] = {f[0], f[1], f[2], f[3]};
    for (int k = 1; k < 4; ++k)
        for (int j = 3; j >= k; --j) a[j] = (a[j] - a[j - 1]) / (d[j] - d[j - k]);
    double x = wl - e_n;
    for (int it = 0; it < kCubicIt; ++it) {
        double p = a[3], dp = 0.0;
        for (int k = 2; k >= 0; --k) {
            dp = dp * (x - d[k]) + p;
            p = p * (x - d[k]) + a[k];
        }
        if (!(dp > 0.0)) break;
        x -= p / dp;
    }
    const double w = e_n + x;
    return (isfinite(w) && lo <= w && w <= hi) ? w : wl;
}

__device__ void qp_state(const QpArgs& A, int s, Shared& sh, QpOut* dst) {
    for (int k = threadIdx.x; k < A.n_freq; k += kQpThreads) {
        sh.freq[k] = A.freq[k];
        sh.weight[k] = A.weight[k];
        sh.glor[k] = kQuadGamma * kQuadGamma / (kQuadGamma * kQuadGamma + A.freq[k] * A.freq[k]);
    }
    __syncthreads();
    const double e_n = A.eps_n[A.state_idx[s]];
    const double vxc = A.vxc[s];
    const double sx = A.sigx[s];
    const double lo = A.win_lo[s], hi = A.win_hi[s];
    // n_eval counts self-energy evaluations, n_round the passes over the
    // tables they took (points evaluated together count once)
    int n_eval = 0, n_round = 0, flags = 0;
    auto f = [&](double x) {
        ++n_eval;
        ++n_round;
        return x - e_n - sigma_total(A, s, x, sh) + vxc;
    };
    // f at K points in one pass
    auto f_multi = [&](auto& xs, auto& fs) {
        constexpr int K = sizeof(xs) / sizeof(double);
        double I[K], R[K];
        sigma_multi<K>(A, s, xs, sh, I, R);
#pragma unroll
        for (int j = 0; j < K; ++j) fs[j] = xs[j] - e_n - (sx + R[j] - I[j]) + vxc;
        n_eval += K;
        ++n_round;
    };
    auto z_factor = [&](double x) {
        const double xs[2] = {x + kZStep, x - kZStep};
        double fs[2];
        f_multi(xs, fs);
        return 2.0 * kZStep / (fs[0] - fs[1]);
    };

    double root = 0.0, zf = 0.0;
    bool done = false;
    // secant iteration from the pair (xa, fa), (xb, fb); on convergence with a
    // physical Z factor the root and Z are taken
    auto secant = [&](double xa, double fa, double xb, double fb, int maxit) {
        bool ok = false;
        for (int it = 0; it < maxit; ++it) {
            if (fb == fa) break;
            const double xc = xb - fb * (xb - xa) / (fb - fa);
            if (!(lo <= xc && xc <= hi)) break;
            xa = xb;
            fa = fb;
            xb = xc;
            fb = f(xb);
            if (fabs(xb - xa) < A.qp_tol && fabs(fb) < kFTol) {
                ok = true;
                break;
            }
        }
        if (!ok) return false;
        const double z = z_factor(xb);
        if (!(0.0 < z && z <= 1.0)) return false;
        root = xb;
        zf = z;
        return true;
    };
    if (A.use_mlp && lo <= e_n + kSeedOffset[0] && e_n + kSeedOffset[3] <= hi) {
        // learned seed: pass 1 evaluates Sigma^c at four fixed offsets from
        // eps_n; the zero w_C of the cubic through the four values of f is
        // the base estimate, and the network predicts the remaining
        // correction w* - w_C from eps_n, eps_F, Sigma^x - v^xc, the four
        // Sigma^c values and w_C - eps_n.  Pass 2 evaluates f at the seed and at seed +- h:
        // the seed is the root if |f| <= mlp_accept and Z is in (0, 1].  Else,
        // with a physical Z, pass 3 takes one Newton step with that slope and
        // applies the same test to its point.
        double xs[4], fs[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xs[j] = e_n + kSeedOffset[j];
        f_multi(xs, fs);
        double sdd = 0.0, sdf = 0.0, sf = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sdd += kSeedOffset[j] * kSeedOffset[j];
            sdf += kSeedOffset[j] * fs[j];
            sf += fs[j];
        }
        const double slope = sdf / sdd, mean = 0.25 * sf;      // the offsets sum to zero
        double wn = slope > 0.0 ? e_n - mean / slope : e_n - mean;
        wn = fmin(fmax(wn, lo), hi);
        const double wc = cubic_root(kSeedOffset, fs, e_n, wn, lo, hi);
        double raw[8] = {e_n, A.eps_f, sx - vxc, 0.0, 0.0, 0.0, 0.0, wc - e_n};
#pragma unroll
        for (int j = 0; j < 4; ++j) raw[3 + j] = xs[j] - e_n + vxc - fs[j] - sx;   // Sigma^c(x_j)
        float feat[8];
        for (int i = 0; i < 8; ++i) feat[i] = (float)((raw[i] - A.mlp_mu[i]) / A.mlp_sd[i]);
        const float y = mlp_one(A.mlp_theta, feat, sh);
        const double seed = wc + (double)y * A.mlp_out_sd + A.mlp_out_mu;
        if (seed - kZStep >= lo && seed + kZStep <= hi) {
            const double ps[3] = {seed, seed + kZStep, seed - kZStep};
            double pf[3];
            f_multi(ps, pf);
            const double z = 2.0 * kZStep / (pf[1] - pf[2]);
            const bool phys = 0.0 < z && z <= 1.0;
            if (fabs(pf[0]) <= A.mlp_accept && phys) {
                root = seed;
                zf = z;
                flags |= CDWAC_FLAG_MLP_ACCEPTED_DEV;
                done = true;
            } else if (phys && seed - pf[0] * z - kZStep >= lo && seed - pf[0] * z + kZStep <= hi) {
                // Newton step from the seed (f' = 1 / Z)
                const double x1 = seed - pf[0] * z;
                const double qs[3] = {x1, x1 + kZStep, x1 - kZStep};
                double qf[3];
                f_multi(qs, qf);
                const double z1 = 2.0 * kZStep / (qf[1] - qf[2]);
                if (fabs(qf[0]) <= A.mlp_accept && 0.0 < z1 && z1 <= 1.0) {
                    root = x1;
                    zf = z1;
                    flags |= CDWAC_FLAG_MLP_ACCEPTED_DEV;
                    done = true;
                } else {
                    done = secant(seed, pf[0], x1, qf[0], min(A.qp_maxit, kSeedSecantIt));
                }
            } else {
                // the secant continues from the sample nearest the seed and the seed
                int jn = 0;
#pragma unroll
                for (int j = 1; j < 4; ++j)
                    if (fabs(xs[j] - seed) < fabs(xs[jn] - seed)) jn = j;
                done = secant(xs[jn], fs[jn], seed, pf[0], min(A.qp_maxit, kSeedSecantIt));
            }
        }
    }
    // the plain search from omega_0 = eps_n and omega_1 = omega_0 - f(omega_0)
    // (also where a seeded search failed)
    if (!done) {
        const double w0 = e_n, f0 = f(w0), w1 = w0 - f0;
        if (lo <= w1 && w1 <= hi) done = secant(w0, f0, w1, f(w1), A.qp_maxit);
    }
    if (!done) {
        flags |= CDWAC_FLAG_FALLBACK_DEV;
        const int n = (int)ceil((hi - lo) / kScanStep);
        bool have = false;
        double best_z = 0.0, best_d = 0.0, best_r = 0.0;
        double xa = lo, fa = f(xa);
        for (int j = 0; j < n; ++j) {
            double xb = lo + (hi - lo) * (j + 1) / n;
            double fb = f(xb);
            if (fa <= 0.0 && 0.0 < fb && fabs(fa) < kScanFmax && fabs(fb) < kScanFmax) {
                double a = xa, b = xb;
                while (b - a > kBisectTol) {
                    double c = 0.5 * (a + b);
                    if (f(c) <= 0.0) a = c;
                    else b = c;
                }
                double r = 0.5 * (a + b);
                if (fabs(f(r)) <= kRootFTol) {   // else a jump across a (near-)pole
                    double z = z_factor(r);
                    double d = -fabs(r - e_n);
                    if (!have || z > best_z || (z == best_z && d > best_d)) {
                        have = true;
                        best_z = z;
                        best_d = d;
                        best_r = r;
                    }
                }
            }
            xa = xb;
            fa = fb;
        }
        if (have) {
            root = best_r;
            zf = best_z;
        } else {
            root = nan("");
            zf = nan("");
            flags |= CDWAC_FLAG_NOROOT_DEV;
        }
    }
    double I = 0.0, R = 0.0;
    if (!(flags & CDWAC_FLAG_NOROOT_DEV)) sigma_terms(A, s, root, sh, I, R);
    if (threadIdx.x == 0) {
        QpOut o;
        o.qp = root;
        o.z = zf;
        o.sigma_x = A.sigx[s];
        o.sigma_c = (flags & CDWAC_FLAG_NOROOT_DEV) ? nan("") : R - I;
        o.residual = (flags & CDWAC_FLAG_NOROOT_DEV) ? nan("") : root - e_n - (A.sigx[s] + R - I) + vxc;
        o.n_evals = n_eval;
        o.flags = flags;
        o.n_rounds = n_round;
        *dst = o;
    }
}

__global__ __launch_bounds__(kQpThreads) void k_qp_solve(QpArgs A, QpOut* __restrict__ out) {
    __shared__ Shared sh;
    qp_state(A, blockIdx.x, sh, out + blockIdx.x);
}

// One workgroup per (system, state) of a batch: map[b] = {system, state}.
__global__ __launch_bounds__(kQpThreads) void k_qp_solve_batch(const QpArgs* __restrict__ args,
                                                               const int2* __restrict__ map,
                                                               QpOut* __restrict__ out) {
    __shared__ Shared sh;
    const int2 m = map[blockIdx.x];
    qp_state(args[m.x], m.y, sh, out + blockIdx.x);
}

// sigma[s][k] = Re Sigma_n(omega[s][k]) (+ I and R terms).
__global__ __launch_bounds__(kQpThreads) void k_sigma_eval(QpArgs A, int n_omega, const double* __restrict__ omega,
                                                           double* __restrict__ sigma, double* __restrict__ iterm,
                                                           double* __restrict__ rterm) {
    __shared__ Shared sh;
    const int k = blockIdx.x, s = blockIdx.y;
    for (int q = threadIdx.x; q < A.n_freq; q += kQpThreads) {
        sh.freq[q] = A.freq[q];
        sh.weight[q] = A.weight[q];
        sh.glor[q] = kQuadGamma * kQuadGamma / (kQuadGamma * kQuadGamma + A.freq[q] * A.freq[q]);
    }
    __syncthreads();
    const int64_t o = (int64_t)s * n_omega + k;
    double I, R;
    sigma_terms(A, s, omega[o], sh, I, R);
    if (threadIdx.x == 0) {
        sigma[o] = A.sigx[s] + R - I;
        if (iterm) iterm[o] = I;
        if (rterm) rterm[o] = R;
    }
}

// Diagonal spectral function (Sec. 5.5): with Sigma_n = Sigma^x + R_n - I_n
// complex (Im from the residue term; the integral term is real for eta -> 0),
// A_n(w) = (1/pi) |Im[1 / (w - eps_n - Sigma_n(w) + v^xc_n)]|.
__global__ __launch_bounds__(kQpThreads) void k_spectral_eval(QpArgs A, int n_omega,
                                                              const double* __restrict__ omega,
                                                              double* __restrict__ spec,
                                                              double* __restrict__ sre,
                                                              double* __restrict__ sim) {
    __shared__ Shared sh;
    const int k = blockIdx.x, s = blockIdx.y;
    for (int q = threadIdx.x; q < A.n_freq; q += kQpThreads) {
        sh.freq[q] = A.freq[q];
        sh.weight[q] = A.weight[q];
        sh.glor[q] = kQuadGamma * kQuadGamma / (kQuadGamma * kQuadGamma + A.freq[q] * A.freq[q]);
    }
    __syncthreads();
    const int64_t o = (int64_t)s * n_omega + k;
    const double w = omega[o];
    double I, R, Ri;
    sigma_terms(A, s, w, sh, I, R, &Ri);
    if (threadIdx.x == 0) {
        const double re = A.sigx[s] + R - I;
        const double dr = w - A.eps_n[A.state_idx[s]] - re + A.vxc[s], di = -Ri;
        spec[o] = fabs(di) / (dr * dr + di * di) / kPi;
        if (sre) sre[o] = re;
        if (sim) sim[o] = Ri;
    }
}

// Full contour deformation (Sec. 2.3, Eqs. Rn_term, In_term, cdselfe) for
// state 0 of A at one omega: W evaluated directly at every residue.  Residue
// j is orbital rm[j] with occupation factor rf[j]; its W^c_nm(|eps_m - omega|
// + i eta) is column fit rm[j] (every m fitted) at near-real point j of w_re.
// out = {Sigma, R_n, I_n}.
__global__ __launch_bounds__(kQpThreads) void k_sigma_direct(QpArgs A, double omega, const double* __restrict__ w_re,
                                                             int stride, int n_res, const int* __restrict__ rm,
                                                             const double* __restrict__ rf, double* __restrict__ out) {
    __shared__ Shared sh;
    for (int k = threadIdx.x; k < A.n_freq; k += kQpThreads) {
        sh.freq[k] = A.freq[k];
        sh.weight[k] = A.weight[k];
        sh.glor[k] = kQuadGamma * kQuadGamma / (kQuadGamma * kQuadGamma + A.freq[k] * A.freq[k]);
    }
    __syncthreads();
    const double I = integral_only(A, 0, omega, sh);
    double rsum = 0.0;
    for (int j = threadIdx.x; j < n_res; j += kQpThreads) {
        const int f = A.fit_off[0] + (rm[j] - A.m0[0]);
        rsum += rf[j] * w_re[((int64_t)f * stride + j) * 2];
    }
    const double R = block_sum(rsum, sh.red);
    if (threadIdx.x == 0) {
        out[0] = A.sigx[0] + R - I;
        out[1] = R;
        out[2] = I;
    }
}

void launch_sigma_direct(hipStream_t s, const QpArgs& a, double omega, const double* w_re, int stride, int n_res,
                         const int* rm, const double* rf, double* out) {
    hipLaunchKernelGGL(k_sigma_direct, dim3(1), dim3(kQpThreads), 0, s, a, omega, w_re, stride, n_res, rm, rf, out);
}

int qp_max_freq() { return kMaxFreq; }

void launch_spectral(hipStream_t s, const QpArgs& a, int n_omega, const double* omega, double* spec, double* sre,
                     double* sim) {
    if (n_omega <= 0) return;
    hipLaunchKernelGGL(k_spectral_eval, dim3(n_omega, a.n_states), dim3(kQpThreads), 0, s, a, n_omega, omega, spec,
                       sre, sim);
}

void launch_qp(hipStream_t s, const QpArgs& a, QpOut* out) {
    hipLaunchKernelGGL(k_qp_solve, dim3(a.n_states), dim3(kQpThreads), 0, s, a, out);
}

void launch_qp_batch(hipStream_t s, int n_blocks, const QpArgs* args, const int2* map, QpOut* out) {
    if (n_blocks <= 0) return;
    hipLaunchKernelGGL(k_qp_solve_batch, dim3(n_blocks), dim3(kQpThreads), 0, s, args, map, out);
}

void launch_sigma(hipStream_t s, const QpArgs& a, int n_omega, const double* omega, double* sigma,
                  double* iterm, double* rterm) {
    if (n_omega <= 0) return;
    hipLaunchKernelGGL(k_sigma_eval, dim3(n_omega, a.n_states), dim3(kQpThreads), 0, s, a, n_omega, omega,
                       sigma, iterm, rterm);
}

}  // namespace cdwac
