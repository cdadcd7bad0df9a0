// Greedy Thiele-Pade fits of W^c_nm (Sec. 2.4, Eqs. pade, pre_rec, rec_eq;
// Sec. 3.2), FP64 complex.  One wave per fit, one lane per reference point
// (at most 64).  Lane j keeps u_j = z_j^2, W_j and its current reciprocal
// difference g(u_j); lane q also keeps the q-th chosen coefficient a_q and
// node u_q, so evaluating the convergent at every remaining point is a loop
// of lane broadcasts.
//
// Order (greedy): the first point is the largest |W_j|; afterwards the point
// where the current convergent has the largest L1 error |Re(W-T)| + |Im(W-T)|
// is added (lowest index on ties).  The fit stops when that error is
// <= tol * max|W|, when no point is left, when a coefficient is not finite or
// when an error is NaN.
#include "common.h"
#include "kernels.h"

namespace cdwac {

__device__ inline double shfl_d(double v, int src) { return __shfl(v, src, 64); }

// Wave arg-max with the lowest index on ties; returns the winning lane.
__device__ inline int wave_argmax(double v, int idx, double& best) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off, 64);
        int oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    best = v;
    return idx;
}

// Convergent with p terms held by lanes 0..p-1, evaluated at u (per lane).
__device__ inline cplx eval_lanes(cplx u, double a_re, double a_im, double n_re, double n_im, int p) {
    cplx t = cmk(1.0, 0.0);
    for (int q = p - 1; q >= 1; --q) {
        cplx aq = cmk(shfl_d(a_re, q), shfl_d(a_im, q));
        cplx nq = cmk(shfl_d(n_re, q - 1), shfl_d(n_im, q - 1));
        t = cmk(1.0, 0.0) + (aq * (u - nq)) / t;
    }
    cplx a0 = cmk(shfl_d(a_re, 0), shfl_d(a_im, 0));
    return a0 / t;
}

__global__ __launch_bounds__(256) void k_thiele_fit(int n_fit, int n_pts, const double* __restrict__ u,
                                                    const double* __restrict__ w, double tol,
                                                    double* __restrict__ coef, double* __restrict__ node,
                                                    int* __restrict__ nterm) {
    const int fit = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (fit >= n_fit) return;                       // whole wave leaves together
    const bool valid = lane < n_pts;
    const int64_t base = ((int64_t)fit * n_pts + (valid ? lane : 0)) * 2;
    cplx uj = valid ? cmk(u[base], u[base + 1]) : cmk(0.0, 0.0);
    cplx wj = valid ? cmk(w[base], w[base + 1]) : cmk(0.0, 0.0);
    cplx g = wj;
    bool alive = valid;
    double a_re = 0.0, a_im = 0.0, n_re = 0.0, n_im = 0.0;   // lane q: q-th term
    double absw = valid ? sqrt(wj.re * wj.re + wj.im * wj.im) : -1.0;
    double scale;
    int jsel = wave_argmax(absw, lane, scale);
    int p = 0;
    while (true) {
        cplx a = cmk(shfl_d(g.re, jsel), shfl_d(g.im, jsel));
        if (!cfinite(a)) break;
        cplx un = cmk(shfl_d(uj.re, jsel), shfl_d(uj.im, jsel));
        if (lane == p) {
            a_re = a.re; a_im = a.im; n_re = un.re; n_im = un.im;
        }
        ++p;
        if (lane == jsel) alive = false;
        if (__ballot(alive) == 0) break;
        double err = -1.0;
        bool bad = false;
        if (alive) {
            g = (a - g) / ((uj - un) * g);
        }
        cplx t = eval_lanes(uj, a_re, a_im, n_re, n_im, p);
        if (alive) {
            cplx r = wj - t;
            err = fabs(r.re) + fabs(r.im);
            bad = isnan(err);
        }
        if (__ballot(bad) != 0) break;
        double emax;
        jsel = wave_argmax(alive ? err : -1.0, lane, emax);
        if (!(emax > tol * scale)) break;
    }
    const int64_t ob = ((int64_t)fit * n_pts + (valid ? lane : 0)) * 2;
    if (valid) {
        bool used = lane < p;
        coef[ob] = used ? a_re : 0.0;
        coef[ob + 1] = used ? a_im : 0.0;
        node[ob] = used ? n_re : 0.0;
        node[ob + 1] = used ? n_im : 0.0;
    }
    if (lane == 0 && nterm) nterm[fit] = p;
}

// out[f][i] = T_f(x[f][i]) for the fits above.
__global__ void k_thiele_eval(int n_fit, int n_pts, const double* __restrict__ coef,
                              const double* __restrict__ node, const int* __restrict__ nterm, int n_x,
                              const double* __restrict__ x, double* __restrict__ out) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_fit * n_x) return;
    int f = (int)(t / n_x);
    cplx u = cmk(x[2 * t], x[2 * t + 1]);
    int p = nterm[f];
    const double* a = coef + (int64_t)f * n_pts * 2;
    const double* nd = node + (int64_t)f * n_pts * 2;
    cplx r = cmk(0.0, 0.0);
    if (p > 0) {
        cplx tt = cmk(1.0, 0.0);
        for (int q = p - 1; q >= 1; --q)
            tt = cmk(1.0, 0.0) + (cmk(a[2 * q], a[2 * q + 1]) * (u - cmk(nd[2 * q - 2], nd[2 * q - 1]))) / tt;
        r = cmk(a[0], a[1]) / tt;
    }
    out[2 * t] = r.re;
    out[2 * t + 1] = r.im;
}

// Reference data of every fit: imaginary nodes first (u = -omega^2, W real),
// then the near-real points (u = (x + i eta_ref)^2, W complex).
__global__ void k_gather_refs(int n_fit, const int* __restrict__ fit_s, const int* __restrict__ fit_m,
                              int n_mo, int n_freq, const double* __restrict__ w_im,
                              const double* __restrict__ w_re, const double* __restrict__ freq,
                              const int* __restrict__ ref_im_idx, int n_im, const double* __restrict__ ref_re,
                              int n_re, double eta_ref, double* __restrict__ u, double* __restrict__ w) {
    const int n_pts = n_im + n_re;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_fit * n_pts) return;
    int f = (int)(t / n_pts), j = (int)(t % n_pts);
    int s = fit_s[f], m = fit_m[f];
    cplx uu, ww;
    if (j < n_im) {
        int k = ref_im_idx[j];
        double om = freq[k];
        uu = cmk(-om * om, 0.0);          // (i omega)^2
        ww = cmk(w_im[((int64_t)s * n_mo + m) * n_freq + k], 0.0);
    } else {
        int jj = j - n_im;
        cplx z = cmk(ref_re[jj], eta_ref);
        uu = z * z;
        ww = cmk(w_re[((int64_t)f * n_re + jj) * 2], w_re[((int64_t)f * n_re + jj) * 2 + 1]);
    }
    u[2 * t] = uu.re;
    u[2 * t + 1] = uu.im;
    w[2 * t] = ww.re;
    w[2 * t + 1] = ww.im;
}

void launch_thiele_fit(hipStream_t s, int n_fit, int n_pts, const double* u, const double* w, double tol,
                       double* coef, double* node, int* nterm) {
    if (n_fit <= 0) return;
    hipLaunchKernelGGL(k_thiele_fit, dim3((n_fit + 3) / 4), dim3(256), 0, s, n_fit, n_pts, u, w, tol, coef,
                       node, nterm);
}

void launch_thiele_eval(hipStream_t s, int n_fit, int n_pts, const double* coef, const double* node,
                        const int* nterm, int n_x, const double* x, double* out) {
    int64_t n = (int64_t)n_fit * n_x;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_thiele_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_fit, n_pts, coef,
                       node, nterm, n_x, x, out);
}

void launch_gather_refs(hipStream_t s, int n_fit, const int* fit_s, const int* fit_m, int n_mo, int n_freq,
                        const double* w_im, const double* w_re, const double* freq, const int* ref_im_idx,
                        int n_im, const double* ref_re, int n_re, double eta_ref, double* u, double* w) {
    int64_t n = (int64_t)n_fit * (n_im + n_re);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_refs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_fit, fit_s, fit_m,
                       n_mo, n_freq, w_im, w_re, freq, ref_im_idx, n_im, ref_re, n_re, eta_ref, u, w);
}

}  // namespace cdwac
