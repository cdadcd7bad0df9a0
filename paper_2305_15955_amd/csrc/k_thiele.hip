// Greedy Thiele-Pade fits of W^c_nm (Sec. 2.4, Eqs. pade, pre_rec, rec_eq;
// Sec. 3.2), FP64 complex.  One wave per fit; reference point j lives in lane
// j % 64, slot j / 64 (up to 4 slots, so at most 256 points, enough for the
// paper's default CD-WAC(20, 20, 200)).  Each point keeps u_j = z_j^2, W_j
// and its current reciprocal difference g(u_j).  The chosen coefficients a_q
// and nodes u_q go to the wave's LDS slice, from where every lane reads them
// (broadcast) to evaluate the convergent at its remaining points.
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

// Wave arg-max with the lowest index on ties; returns the winning index.
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

// Per-lane arg-max over the lane's slots (ascending index, so a strict '>'
// keeps the lowest index), then across the wave.
template <int P>
__device__ inline int points_argmax(const double (&v)[P], int lane, double& best) {
    double bv = v[0];
    int bi = lane;
#pragma unroll
    for (int s = 1; s < P; ++s)
        if (v[s] > bv) {
            bv = v[s];
            bi = lane + 64 * s;
        }
    return wave_argmax(bv, bi, best);
}

// Value of slot `slot` (wave-uniform) of lane `src`.
template <int P>
__device__ inline cplx pick(const cplx (&v)[P], int slot, int src) {
    cplx x = v[0];
#pragma unroll
    for (int s = 1; s < P; ++s)
        if (slot == s) x = v[s];
    return cmk(shfl_d(x.re, src), shfl_d(x.im, src));
}

// Convergent with p terms (coefficients a[], nodes nd[] in LDS) at u.
__device__ inline cplx eval_terms(cplx u, const cplx* a, const cplx* nd, int p) {
    cplx t = cmk(1.0, 0.0);
    for (int q = p - 1; q >= 1; --q) t = cmk(1.0, 0.0) + (a[q] * (u - nd[q - 1])) / t;
    return a[0] / t;
}

template <int P>
__global__ __launch_bounds__(256) void k_thiele_fit(int n_fit, int n_pts, const double* __restrict__ u,
                                                    const double* __restrict__ w, double tol,
                                                    double* __restrict__ coef, double* __restrict__ node,
                                                    int* __restrict__ nterm) {
    __shared__ cplx s_a[4][64 * P];
    __shared__ cplx s_n[4][64 * P];
    const int wv = threadIdx.x >> 6;
    const int fit = blockIdx.x * 4 + wv;
    const int lane = threadIdx.x & 63;
    if (fit >= n_fit) return;                       // whole wave leaves together
    cplx* a_l = s_a[wv];
    cplx* n_l = s_n[wv];
    cplx uj[P], wj[P], g[P];
    bool alive[P];
    double absw[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
        const int j = lane + 64 * s;
        const bool valid = j < n_pts;
        const int64_t base = ((int64_t)fit * n_pts + (valid ? j : 0)) * 2;
        uj[s] = valid ? cmk(u[base], u[base + 1]) : cmk(0.0, 0.0);
        wj[s] = valid ? cmk(w[base], w[base + 1]) : cmk(0.0, 0.0);
        g[s] = wj[s];
        alive[s] = valid;
        absw[s] = valid ? sqrt(wj[s].re * wj[s].re + wj[s].im * wj[s].im) : -1.0;
    }
    double scale;
    int jsel = points_argmax<P>(absw, lane, scale);
    int p = 0;
    while (true) {
        const cplx a = pick<P>(g, jsel >> 6, jsel & 63);
        if (!cfinite(a)) break;
        const cplx un = pick<P>(uj, jsel >> 6, jsel & 63);
        a_l[p] = a;                                 // every lane stores the same value
        n_l[p] = un;
        ++p;
        bool any = false;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            if (lane + 64 * s == jsel) alive[s] = false;
            any = any || alive[s];
        }
        if (__ballot(any) == 0) break;
        double err[P];
        bool bad = false;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            err[s] = -1.0;
            if (alive[s]) {
                g[s] = (a - g[s]) / ((uj[s] - un) * g[s]);
                const cplx r = wj[s] - eval_terms(uj[s], a_l, n_l, p);
                err[s] = fabs(r.re) + fabs(r.im);
                bad = bad || isnan(err[s]);
            }
        }
        if (__ballot(bad) != 0) break;
        double emax;
        jsel = points_argmax<P>(err, lane, emax);
        if (!(emax > tol * scale)) break;
    }
#pragma unroll
    for (int s = 0; s < P; ++s) {
        const int j = lane + 64 * s;
        if (j < n_pts) {
            const int64_t ob = ((int64_t)fit * n_pts + j) * 2;
            const bool used = j < p;
            const cplx av = used ? a_l[j] : cmk(0.0, 0.0);
            const cplx nv = used ? n_l[j] : cmk(0.0, 0.0);
            coef[ob] = av.re;
            coef[ob + 1] = av.im;
            node[ob] = nv.re;
            node[ob + 1] = nv.im;
        }
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

// w0[f] = Re T_f(u) at u = (i eta)^2 = -eta^2: the value the residue term
// takes for a_m = 0, which the integral term's analytic limit needs.
__global__ void k_w0_from_fits(int n_fit, int n_pts, const double* __restrict__ coef,
                               const double* __restrict__ node, const int* __restrict__ nterm, double eta,
                               double* __restrict__ w0) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_fit) return;
    const cplx u = cmk(-eta * eta, 0.0);
    const double* a = coef + (int64_t)f * n_pts * 2;
    const double* nd = node + (int64_t)f * n_pts * 2;
    const int p = nterm[f];
    cplx r = cmk(0.0, 0.0);
    if (p > 0) {
        cplx t = cmk(1.0, 0.0);
        for (int q = p - 1; q >= 1; --q)
            t = cmk(1.0, 0.0) + (cmk(a[2 * q], a[2 * q + 1]) * (u - cmk(nd[2 * q - 2], nd[2 * q - 1]))) / t;
        r = cmk(a[0], a[1]) / t;
    }
    w0[f] = r.re;
}

__global__ void k_w0_from_points(int n_fit, const double* __restrict__ w_re, int stride, int j,
                                 double* __restrict__ w0) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < n_fit) w0[f] = w_re[((int64_t)f * stride + j) * 2];
}

void launch_w0_from_fits(hipStream_t s, int n_fit, int n_pts, const double* coef, const double* node, const int* nterm,
                         double eta, double* w0) {
    if (n_fit > 0)
        hipLaunchKernelGGL(k_w0_from_fits, dim3((n_fit + 255) / 256), dim3(256), 0, s, n_fit, n_pts, coef, node, nterm,
                           eta, w0);
}

void launch_w0_from_points(hipStream_t s, int n_fit, const double* w_re, int stride, int j, double* w0) {
    if (n_fit > 0)
        hipLaunchKernelGGL(k_w0_from_points, dim3((n_fit + 255) / 256), dim3(256), 0, s, n_fit, w_re, stride, j, w0);
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
    const dim3 grid((n_fit + 3) / 4), block(256);
    if (n_pts <= 64)
        hipLaunchKernelGGL(k_thiele_fit<1>, grid, block, 0, s, n_fit, n_pts, u, w, tol, coef, node, nterm);
    else if (n_pts <= 128)
        hipLaunchKernelGGL(k_thiele_fit<2>, grid, block, 0, s, n_fit, n_pts, u, w, tol, coef, node, nterm);
    else
        hipLaunchKernelGGL(k_thiele_fit<4>, grid, block, 0, s, n_fit, n_pts, u, w, tol, coef, node, nterm);
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
