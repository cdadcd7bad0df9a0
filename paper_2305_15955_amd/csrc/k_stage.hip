// Staging kernels of the CD-WAC path: polarizability weights, operand
// scaling and hi/lo splitting, transposition of the RI rows, exchange,
// Lambda finalisation and the reductions of the W contraction.
//
// Split operands.  A value v is stored as two 16-bit numbers hi = rn(v s),
// lo = rn(v s - hi) with a power-of-two scale s chosen on the device from
// max|v| so that max|v s| lies in (2^13, 2^14]: the fp16 split then keeps
// 22 significant bits without overflow, the bf16 split 16 bits.  Scales are
// exact powers of two and are divided out in FP64 after the product.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace cdwac {

// 2^e with amax * 2^e in (2^13, 2^14]; 1 when amax is 0.
__device__ inline double pow2_for(double amax) {
    if (!(amax > 0.0)) return 1.0;
    int e;
    frexp(amax, &e);   // amax = m 2^e, m in [0.5, 1)
    return ldexp(1.0, 14 - e);
}

__device__ inline void atomic_absmax(uint32_t* slot, double v) {
    float f = (float)fabs(v);
    // round up so the stored bound is never below the true maximum
    if ((double)f < fabs(v)) f = nextafterf(f, INFINITY);
    atomicMax(slot, __float_as_uint(f));
}

__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// max |src| over rows x cols (leading dim lds) into *amax; non-finite -> err |= 2.
__global__ void k_absmax(const double* __restrict__ src, int64_t lds, int rows, int64_t cols,
                         uint32_t* __restrict__ amax, int* __restrict__ err) {
    double m = 0.0;
    bool bad = false;
    const int64_t tot = (int64_t)rows * cols;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = t / cols, c = t % cols;
        double v = src[r * lds + c];
        bad |= !isfinite(v);
        m = fmax(m, fabs(v));
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomic_absmax(amax, m);
    if (bad) atomicOr(err, 2);
}

// Weights c_f[k] of the polarizability for every real weight vector f:
// d(z) = spin (1/(z - D_k) - 1/(z + D_k)), D_k = eps_a - eps_i (k = i*nv + a),
// evaluated at z_f = zr[f] + i zi[f]; c_f = Re d (part[f] = 0) or Im d (1).
// Writes FP64 and/or FP32 tables and max|c_f| per f.
__global__ void k_weights(const double* __restrict__ eps, int n_occ, int n_virt, double spin,
                          const double* __restrict__ zr, const double* __restrict__ zi,
                          const int* __restrict__ part, int64_t kpad, double* __restrict__ cw64,
                          float* __restrict__ cw32, uint32_t* __restrict__ cmax) {
    const int f = blockIdx.y;
    const int64_t K = (int64_t)n_occ * n_virt;
    const cplx z = cmk(zr[f], zi[f]);
    const bool im_part = part[f] != 0;
    double m = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < kpad;
         k += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (k < K) {
            int i = (int)(k / n_virt), a = (int)(k % n_virt);
            double d = eps[n_occ + a] - eps[i];
            cplx one = cmk(1.0, 0.0);
            cplx t = (one / (z - cmk(d, 0.0))) - (one / (z + cmk(d, 0.0)));
            v = spin * (im_part ? t.im : t.re);
        }
        if (cw64) cw64[(int64_t)f * kpad + k] = v;
        if (cw32) cw32[(int64_t)f * kpad + k] = (float)v;
        m = fmax(m, fabs(v));
    }
    m = wave_max(m);
    if (cmax && (threadIdx.x & 63) == 0) atomic_absmax(cmax + f, m);
}

// Scales of the Pi contraction: sf[0] = x scale, sf[1] = B scale,
// cfac[f] = multiplier of the weight table, pi_unscale[f] = 1 / (x scale * y scale).
__global__ void k_scales_pi(const uint32_t* __restrict__ amax, int n_f, double* __restrict__ sf) {
    const double xmax = __uint_as_float(amax[0]);
    const double xs = pow2_for(xmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sf[0] = xs;
        sf[1] = pow2_for(__uint_as_float(amax[1]));
    }
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n_f; f += gridDim.x * blockDim.x) {
        double ys = pow2_for((double)__uint_as_float(amax[2 + f]) * xmax);
        sf[2 + f] = ys / xs;                   // cfac
        sf[2 + n_f + f] = 1.0 / (xs * ys);     // pi_unscale
    }
}

__global__ void k_scale_weights(float* __restrict__ cw32, int64_t kpad, const double* __restrict__ cfac) {
    const int f = blockIdx.y;
    const float c = (float)cfac[f];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < kpad;
         k += (int64_t)gridDim.x * blockDim.x)
        cw32[(int64_t)f * kpad + k] *= c;
}

// Scales of the W contraction: lam_scale[f], w_unscale[f] = 1 / (lam_scale * B scale).
__global__ void k_scales_w(const uint32_t* __restrict__ lmax, int n_f, double* __restrict__ sf_b,
                           double* __restrict__ lam_scale, double* __restrict__ w_unscale) {
    const double bs = sf_b[1];
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n_f; f += gridDim.x * blockDim.x) {
        double ls = pow2_for(__uint_as_float(lmax[f]));
        lam_scale[f] = ls;
        w_unscale[f] = 1.0 / (ls * bs);
    }
}

template <int ET>
__device__ inline void split_store(double v, uint16_t* hi, uint16_t* lo, int64_t o) {
    float x = (float)v;
    uint16_t h = Elem<ET>::bits(x);
    hi[o] = h;
    lo[o] = Elem<ET>::bits((float)(v - (double)Elem<ET>::val(h)));
}

// src [rows][cols] (leading dim lds) -> hi, lo planes of src * scale [rpad][cpad]
// (zero padded) and/or an FP64 padded copy.
template <int ET>
__global__ void k_split_pad(const double* __restrict__ src, int64_t lds, int rows, int64_t cols,
                            const double* __restrict__ scale, uint16_t* __restrict__ hi,
                            uint16_t* __restrict__ lo, double* __restrict__ f64, int rpad, int64_t cpad) {
    const int r = blockIdx.y;
    const double s = scale ? *scale : 1.0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cpad;
         c += (int64_t)gridDim.x * blockDim.x) {
        double v = (r < rows && c < cols) ? src[(int64_t)r * lds + c] : 0.0;
        int64_t o = (int64_t)r * cpad + c;
        if (hi) split_store<ET>(v * s, hi, lo, o);
        if (f64) f64[o] = v;
    }
}

// o_nm [S][N][n_mo] -> B^T rows c = s*n_mo + m: f64 [cpad][npad] (+ hi/lo planes of
// B * scale), LDS-tiled transpose, zero padded.  With rowsel, output row c takes
// source column rowsel[c].  Records max|B| into *bmax when given.
template <int ET>
__global__ void k_transpose_b(const double* __restrict__ onm, int S, int N, int n_mo,
                              const int* __restrict__ rowsel, int nrows, const double* __restrict__ scale,
                              double* __restrict__ bt64, uint16_t* __restrict__ bh,
                              uint16_t* __restrict__ bl, int cpad, int npad, uint32_t* __restrict__ bmax,
                              int* __restrict__ err) {
    __shared__ double tile[32][33];
    const int c0 = blockIdx.x * 32, p0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    double m = 0.0;
    for (int yy = ty; yy < 32; yy += 8) {
        int p = p0 + yy, c = c0 + tx;
        double v = 0.0;
        if (p < N && c < nrows) {
            int src = rowsel ? rowsel[c] : c;
            int s = src / n_mo, mm = src % n_mo;
            v = onm[((int64_t)s * N + p) * n_mo + mm];
            if (!isfinite(v)) atomicOr(err, 2);
        }
        tile[yy][tx] = v;
        m = fmax(m, fabs(v));
    }
    if (bmax) {
        m = wave_max(m);
        if ((threadIdx.x & 63) == 0) atomic_absmax(bmax, m);
    }
    __syncthreads();
    const double s = scale ? *scale : 1.0;
    for (int yy = ty; yy < 32; yy += 8) {
        int c = c0 + yy, p = p0 + tx;
        if (c < cpad && p < npad) {
            double v = tile[tx][yy];
            int64_t o = (int64_t)c * npad + p;
            if (bt64) bt64[o] = v;
            if (bh) split_store<ET>(v * s, bh, bl, o);
        }
    }
}

// Sigma^x_n = -sum_{i < n_occ} sum_P (O^{ni}_P)^2  (Eq. exs with RI-V).
__global__ void k_exchange(const double* __restrict__ onm, int N, int n_mo, int n_occ,
                           double* __restrict__ sx) {
    __shared__ double red[256];
    const int s = blockIdx.x;
    double acc = 0.0;
    const int64_t tot = (int64_t)N * n_occ;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
        int p = (int)(t / n_occ), i = (int)(t % n_occ);
        double v = onm[((int64_t)s * N + p) * n_mo + i];
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sx[s] = -red[0];
}

__device__ inline void lower_tile32(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// Lambda = -E - delta_f I after the sweep (E holds -eps^{-1} in its lower
// triangle; delta_f = 0 for the imaginary plane of a complex eps), mirrored in
// place to a full symmetric FP64 matrix; max|Lambda_f| into lmax[f] if given.
__global__ void k_finalize_lambda(double* __restrict__ E, int npad, const int* __restrict__ idflag,
                                  uint32_t* __restrict__ lmax) {
    __shared__ double tile[32][33];
    const int nt = npad / 32, T = nt * (nt + 1) / 2;
    const int f = blockIdx.x / T;
    int I, J;
    lower_tile32(blockIdx.x % T, I, J);
    double* Ef = E + (int64_t)f * npad * npad;
    const double id = idflag[f] ? 1.0 : 0.0;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double m = 0.0;
    for (int yy = ty; yy < 32; yy += 8) {
        int P = I * 32 + yy, Q = J * 32 + tx;
        double v = (I == J && Q > P) ? 0.0 : Ef[(int64_t)P * npad + Q];
        double l = -v - (P == Q ? id : 0.0);
        tile[yy][tx] = l;
        m = fmax(m, fabs(l));
    }
    __syncthreads();
    if (I == J) {
        for (int yy = ty; yy < 32; yy += 8)
            if (tx > yy) tile[yy][tx] = tile[tx][yy];
        __syncthreads();
    }
    for (int yy = ty; yy < 32; yy += 8) {
        Ef[(int64_t)(I * 32 + yy) * npad + J * 32 + tx] = tile[yy][tx];
        if (I != J) Ef[(int64_t)(J * 32 + yy) * npad + I * 32 + tx] = tile[tx][yy];
    }
    if (lmax) {
        m = wave_max(m);
        if ((threadIdx.x & 63) == 0) atomic_absmax(lmax + f, m);
    }
}

// Full FP64 Lambda_f -> hi/lo planes of Lambda_f * lam_scale[f].
template <int ET>
__global__ void k_split_lambda(const double* __restrict__ lam, int64_t n2, const double* __restrict__ lam_scale,
                               uint16_t* __restrict__ lh, uint16_t* __restrict__ ll) {
    const int f = blockIdx.y;
    const double s = lam_scale[f];
    const double* src = lam + (int64_t)f * n2;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n2; t += (int64_t)gridDim.x * blockDim.x)
        split_store<ET>(src[t] * s, lh + (int64_t)f * n2, ll + (int64_t)f * n2, t);
}

// W_im[s][m][f] = sum_I partial[f][I][s*n_mo + m]
__global__ void k_reduce_w_im(const double* __restrict__ partial, int ni, int cpad, int n_im, int ncols,
                              double* __restrict__ w_im) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)ncols * n_im) return;
    int c = (int)(t / n_im), f = (int)(t % n_im);
    double s = 0.0;
    for (int i = 0; i < ni; ++i) s += partial[((int64_t)f * ni + i) * cpad + c];
    w_im[(int64_t)c * n_im + f] = s;
}

// W_re[fit][j] = (sum partial[2j], sum partial[2j+1]) of fit column.
__global__ void k_reduce_w_re(const double* __restrict__ partial, int ni, int cpad, int n_re, int nfit,
                              double* __restrict__ w_re) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)nfit * n_re) return;
    int c = (int)(t / n_re), j = (int)(t % n_re);
    double sr = 0.0, si = 0.0;
    int fr = 2 * j, fi = fr + 1;
    for (int i = 0; i < ni; ++i) {
        sr += partial[((int64_t)fr * ni + i) * cpad + c];
        si += partial[((int64_t)fi * ni + i) * cpad + c];
    }
    w_re[((int64_t)c * n_re + j) * 2] = sr;
    w_re[((int64_t)c * n_re + j) * 2 + 1] = si;
}

// out[j][P][Q] = -E[2j+q][max(P,Q)][min(P,Q)] for P, Q < n (E = -Pi on the lower tiles).
__global__ void k_extract_pi(const double* __restrict__ E, int npad, int n, int n_z, int q,
                             double* __restrict__ out) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t tot = (int64_t)n_z * n * n;
    if (t >= tot) return;
    int j = (int)(t / ((int64_t)n * n));
    int64_t r = t % ((int64_t)n * n);
    int P = (int)(r / n), Q = (int)(r % n);
    int a = P > Q ? P : Q, b = P > Q ? Q : P;
    out[t] = -E[(int64_t)(2 * j + q) * npad * npad + (int64_t)a * npad + b];
}

// ============================================================================
// Host launchers
// ============================================================================
static unsigned grid1(int64_t n, int cap = 8192) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap)); }

void launch_absmax(hipStream_t s, const double* src, int64_t lds, int rows, int64_t cols, uint32_t* amax, int* err) {
    hipLaunchKernelGGL(k_absmax, dim3(grid1((int64_t)rows * cols)), dim3(256), 0, s, src, lds, rows, cols, amax, err);
}

void launch_weights(hipStream_t s, const double* eps, int n_occ, int n_virt, double spin, const double* zr,
                    const double* zi, const int* part, int n_f, int64_t kpad, double* cw64, float* cw32,
                    uint32_t* cmax) {
    dim3 grid(grid1(kpad, 4096), n_f);
    hipLaunchKernelGGL(k_weights, grid, dim3(256), 0, s, eps, n_occ, n_virt, spin, zr, zi, part, kpad, cw64, cw32,
                       cmax);
}

void launch_scales_pi(hipStream_t s, const uint32_t* amax, int n_f, double* sf) {
    hipLaunchKernelGGL(k_scales_pi, dim3(1), dim3(256), 0, s, amax, n_f, sf);
}

void launch_scale_weights(hipStream_t s, float* cw32, int64_t kpad, int n_f, const double* cfac) {
    hipLaunchKernelGGL(k_scale_weights, dim3(grid1(kpad, 4096), n_f), dim3(256), 0, s, cw32, kpad, cfac);
}

void launch_scales_w(hipStream_t s, const uint32_t* lmax, int n_f, double* sf, double* lam_scale, double* w_unscale) {
    hipLaunchKernelGGL(k_scales_w, dim3(1), dim3(256), 0, s, lmax, n_f, sf, lam_scale, w_unscale);
}

void launch_split_pad(hipStream_t s, int et, const double* src, int64_t lds, int rows, int64_t cols,
                      const double* scale, uint16_t* hi, uint16_t* lo, double* f64, int rpad, int64_t cpad) {
    dim3 grid(grid1(cpad, 2048), rpad);
    if (et == 1)
        hipLaunchKernelGGL(k_split_pad<1>, grid, dim3(256), 0, s, src, lds, rows, cols, scale, hi, lo, f64, rpad, cpad);
    else
        hipLaunchKernelGGL(k_split_pad<0>, grid, dim3(256), 0, s, src, lds, rows, cols, scale, hi, lo, f64, rpad, cpad);
}

void launch_transpose_b(hipStream_t s, int et, const double* onm, int S, int N, int n_mo, const int* rowsel,
                        int nrows, const double* scale, double* bt64, uint16_t* bh, uint16_t* bl, int cpad,
                        int npad, uint32_t* bmax, int* err) {
    dim3 grid(cpad / 32, npad / 32);
    if (et == 1)
        hipLaunchKernelGGL(k_transpose_b<1>, grid, dim3(256), 0, s, onm, S, N, n_mo, rowsel, nrows, scale, bt64, bh,
                           bl, cpad, npad, bmax, err);
    else
        hipLaunchKernelGGL(k_transpose_b<0>, grid, dim3(256), 0, s, onm, S, N, n_mo, rowsel, nrows, scale, bt64, bh,
                           bl, cpad, npad, bmax, err);
}

void launch_exchange(hipStream_t s, const double* onm, int S, int N, int n_mo, int n_occ, double* sx) {
    hipLaunchKernelGGL(k_exchange, dim3(S), dim3(256), 0, s, onm, N, n_mo, n_occ, sx);
}

void launch_finalize_lambda(hipStream_t s, double* E, int npad, int n_f, const int* idflag, uint32_t* lmax) {
    int nt = npad / 32, T = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_finalize_lambda, dim3(T * n_f), dim3(256), 0, s, E, npad, idflag, lmax);
}

void launch_split_lambda(hipStream_t s, int et, const double* lam, int npad, int n_f, const double* lam_scale,
                         uint16_t* lh, uint16_t* ll) {
    int64_t n2 = (int64_t)npad * npad;
    dim3 grid(grid1(n2, 4096), n_f);
    if (et == 1)
        hipLaunchKernelGGL(k_split_lambda<1>, grid, dim3(256), 0, s, lam, n2, lam_scale, lh, ll);
    else
        hipLaunchKernelGGL(k_split_lambda<0>, grid, dim3(256), 0, s, lam, n2, lam_scale, lh, ll);
}

void launch_extract_pi(hipStream_t s, const double* E, int npad, int n, int n_z, int q, double* out) {
    int64_t tot = (int64_t)n_z * n * n;
    hipLaunchKernelGGL(k_extract_pi, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, E, npad, n, n_z, q, out);
}

void launch_reduce_w(hipStream_t s, const double* partial_im, const double* partial_re, int ni, int cpad, int cfpad,
                     int n_im, int n_re, int ncols, int nfit, double* w_im, double* w_re) {
    int64_t n1 = (int64_t)ncols * n_im;
    if (n1 > 0)
        hipLaunchKernelGGL(k_reduce_w_im, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, partial_im, ni, cpad,
                           n_im, ncols, w_im);
    int64_t n2 = (int64_t)nfit * n_re;
    if (n2 > 0)
        hipLaunchKernelGGL(k_reduce_w_re, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, partial_re, ni, cfpad,
                           n_re, nfit, w_re);
}

}  // namespace cdwac
