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

struct Shared {
    double red[kQpThreads];
    double freq[kMaxFreq];
    double weight[kMaxFreq];
    float h1[64];
    float h2[64];
};

// Partial sum of I_n(omega) (Eq. In_term, times pi) over this thread's m.
__device__ inline double integral_partial(const QpArgs& A, int s, double omega, const Shared& sh) {
    const int nf = A.n_freq;
    const double* W = A.w_im + (int64_t)s * A.n_mo * nf;
    double isum = 0.0;
    for (int m = threadIdx.x; m < A.n_mo; m += kQpThreads) {
        double am = omega - A.eps[m];
        double am2 = am * am;
        const double* wm = W + (int64_t)m * nf;
        double acc = 0.0;
        for (int k = 0; k < nf; ++k) acc += sh.weight[k] * wm[k] * (am / (am2 + sh.freq[k] * sh.freq[k]));
        isum += acc;
    }
    return isum;
}

// I_n(omega) and R_n(omega) for state s (Im R_n into *Ri when given).  A
// shift dH of every energy of G and of the Fermi level (G_dH W0) enters only
// through omega - eps_m and eps_F - eps_m, so it is applied as omega - dH.
__device__ void sigma_terms(const QpArgs& A, int s, double omega_in, Shared& sh, double& I, double& R,
                            double* Ri = nullptr) {
    const double omega = A.g_shift ? omega_in - A.g_shift[s] : omega_in;
    const double isum = integral_partial(A, s, omega, sh);
    double rsum = 0.0, risum = 0.0;
    const int m0 = A.m0[s], m1 = A.m1[s], foff = A.fit_off[s];
    for (int m = m0 + threadIdx.x; m < m1; m += kQpThreads) {
        double em = A.eps[m];
        double fm = -theta(A.eps_f - em) * theta(em - omega) + theta(em - A.eps_f) * theta(omega - em);
        if (fm == 0.0) continue;
        const int f = foff + (m - m0);
        const double* a = A.coef + (int64_t)f * A.n_pts * 2;
        const double* nd = A.node + (int64_t)f * A.n_pts * 2;
        const int p = A.nterm[f];
        cplx z = cmk(fabs(em - omega), A.eta);
        cplx u = z * z;
        cplx val = cmk(0.0, 0.0);
        if (p > 0) {
            cplx t = cmk(1.0, 0.0);
            for (int q = p - 1; q >= 1; --q)
                t = cmk(1.0, 0.0) + (cmk(a[2 * q], a[2 * q + 1]) * (u - cmk(nd[2 * q - 2], nd[2 * q - 1]))) / t;
            val = cmk(a[0], a[1]) / t;
        }
        rsum += fm * val.re;
        risum += fm * val.im;
    }
    I = block_sum(isum, sh.red) / kPi;
    R = block_sum(rsum, sh.red);
    if (Ri) *Ri = block_sum(risum, sh.red);
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
__device__ void qp_state(const QpArgs& A, int s, Shared& sh, QpOut* dst) {
    for (int k = threadIdx.x; k < A.n_freq; k += kQpThreads) {
        sh.freq[k] = A.freq[k];
        sh.weight[k] = A.weight[k];
    }
    __syncthreads();
    const double e_n = A.eps_n[A.state_idx[s]];
    const double vxc = A.vxc[s];
    const double lo = A.win_lo[s], hi = A.win_hi[s];
    int n_eval = 0, flags = 0;
    auto f = [&](double x) {
        ++n_eval;
        return x - e_n - sigma_total(A, s, x, sh) + vxc;
    };
    auto z_factor = [&](double x) {
        double fp = f(x + kZStep);
        double fm = f(x - kZStep);
        return 2.0 * kZStep / (fp - fm);
    };

    double root = 0.0, zf = 0.0;
    bool done = false;
    // secant from omega_0 = eps_n and one fixed-point step
    double w0 = e_n, f0 = f(w0), w1 = w0 - f0, f1 = 0.0;
    bool in1 = lo <= w1 && w1 <= hi, have_f1 = false;
    if (in1) {
        f1 = f(w1);
        have_f1 = true;
    }
    // secant iteration from the pair (xa, fa), (xb, fb); on convergence with a
    // physical Z factor the root and Z are taken
    auto secant = [&](double xa, double fa, double xb, double fb) {
        bool ok = false;
        for (int it = 0; it < A.qp_maxit; ++it) {
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
    if (A.use_mlp && in1) {
        // learned seed: from the two evaluations above (Sigma^c at eps_n and at
        // omega_1) and the secant step they give, the network predicts the
        // remaining correction omega* - omega_2
        const double sx = A.sigx[s];
        const double sc0 = w0 - e_n + vxc - f0 - sx, sc1 = w1 - e_n + vxc - f1 - sx;
        const double w2 = f1 != f0 ? w1 - f1 * (w1 - w0) / (f1 - f0) : w1;
        const double raw[8] = {e_n, A.eps_f, sx - vxc, sc0, sc1, w1 - w0, f1, w2 - w1};
        float feat[8];
        for (int i = 0; i < 8; ++i) feat[i] = (float)((raw[i] - A.mlp_mu[i]) / A.mlp_sd[i]);
        const float y = mlp_one(A.mlp_theta, feat, sh);
        const double seed = w2 + (double)y * A.mlp_out_sd + A.mlp_out_mu;
        if (seed >= lo && seed <= hi) {
            const double fs = f(seed);
            if (fabs(fs) <= A.mlp_accept) {
                // the same physical-Z test as a secant root: a seed on an
                // unphysical crossing falls through to the plain search
                const double z = z_factor(seed);
                if (0.0 < z && z <= 1.0) {
                    root = seed;
                    zf = z;
                    flags |= CDWAC_FLAG_MLP_ACCEPTED_DEV;
                    done = true;
                }
            } else {
                // the secant continues from omega_1 and the seed
                done = secant(w1, f1, seed, fs);
            }
        }
    }
    // the plain search from omega_0 and omega_1 (also where a seeded search failed)
    if (!done && have_f1) done = secant(w0, f0, w1, f1);
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

// Diagonal spectral function (Sec. 4): with Sigma_n = Sigma^x + R_n - I_n
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
                                                             int n_re, const int* __restrict__ rm,
                                                             const double* __restrict__ rf, double* __restrict__ out) {
    __shared__ Shared sh;
    for (int k = threadIdx.x; k < A.n_freq; k += kQpThreads) {
        sh.freq[k] = A.freq[k];
        sh.weight[k] = A.weight[k];
    }
    __syncthreads();
    const double I = block_sum(integral_partial(A, 0, omega, sh), sh.red) / kPi;
    double rsum = 0.0;
    for (int j = threadIdx.x; j < n_re; j += kQpThreads) {
        const int f = A.fit_off[0] + (rm[j] - A.m0[0]);
        rsum += rf[j] * w_re[((int64_t)f * n_re + j) * 2];
    }
    const double R = block_sum(rsum, sh.red);
    if (threadIdx.x == 0) {
        out[0] = A.sigx[0] + R - I;
        out[1] = R;
        out[2] = I;
    }
}

void launch_sigma_direct(hipStream_t s, const QpArgs& a, double omega, const double* w_re, int n_re, const int* rm,
                         const double* rf, double* out) {
    hipLaunchKernelGGL(k_sigma_direct, dim3(1), dim3(kQpThreads), 0, s, a, omega, w_re, n_re, rm, rf, out);
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
