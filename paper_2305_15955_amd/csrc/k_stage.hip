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
// ys[f] = scale of the prescaled operand X diag(c_f), pi_unscale[f] = 1 / (x scale * ys[f]).
__global__ void k_scales_pi(const uint32_t* __restrict__ amax, int n_f, double* __restrict__ sf) {
    const double xmax = __uint_as_float(amax[0]);
    const double xs = pow2_for(xmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sf[0] = xs;
        sf[1] = pow2_for(__uint_as_float(amax[1]));
    }
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n_f; f += gridDim.x * blockDim.x) {
        double ys = pow2_for((double)__uint_as_float(amax[2 + f]) * xmax);
        sf[2 + f] = ys;
        sf[2 + n_f + f] = 1.0 / (xs * ys);
    }
}

// Y_f = split(X diag(c_f) * ys[f]) for the weight vectors f = fmap[0 .. nfb) as
// hi/lo panel planes [fb][npad][kpad] (layout of panel_off), from the FP32
// row-major copy of X (zero padded).  One lane per row and 32-element k span:
// it reads one 128-byte line of X once and, for every plane of the batch, the
// matching line of c_f and four 16-byte words per output plane; the 64 lanes
// of a wave write 1 KiB runs.  yl == nullptr skips the lo planes (one-product
// modes).
template <int ET>
__global__ void k_prescale(const float* __restrict__ x32, int npad, int64_t kpad, const float* __restrict__ cw32,
                           const double* __restrict__ ys, const int* __restrict__ fmap, int nfb,
                           uint16_t* __restrict__ yh, uint16_t* __restrict__ yl) {
    const int lane = threadIdx.x & 63;
    const int64_t ks = kpad / 32, kw = kpad / 8;
    const int64_t nspan = (int64_t)(npad / 64) * ks;
    const int64_t plane = (int64_t)npad * kpad;
    const int64_t wstride = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; w < nspan; w += wstride) {
        const int64_t rb = w / ks, sp = w % ks;
        const float4* xr = reinterpret_cast<const float4*>(x32 + (rb * 64 + lane) * kpad + sp * 32);
        float4 x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = xr[q];
        for (int fb = 0; fb < nfb; ++fb) {
            const int f = fmap[fb];
            const float s = (float)ys[f];
            const float4* cr = reinterpret_cast<const float4*>(cw32 + (int64_t)f * kpad + sp * 32);
            uint4* oh = reinterpret_cast<uint4*>(yh + fb * plane);
            uint4* ol = yl ? reinterpret_cast<uint4*>(yl + fb * plane) : nullptr;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float4 x0 = x[2 * g], x1 = x[2 * g + 1], c0 = cr[2 * g], c1 = cr[2 * g + 1];
                const float y[8] = {x0.x * c0.x * s, x0.y * c0.y * s, x0.z * c0.z * s, x0.w * c0.w * s,
                                    x1.x * c1.x * s, x1.y * c1.y * s, x1.z * c1.z * s, x1.w * c1.w * s};
                uint32_t h[4], l[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint16_t h0 = Elem<ET>::bits(y[2 * e]), h1 = Elem<ET>::bits(y[2 * e + 1]);
                    const uint16_t l0 = Elem<ET>::bits(y[2 * e] - Elem<ET>::val(h0));
                    const uint16_t l1 = Elem<ET>::bits(y[2 * e + 1] - Elem<ET>::val(h1));
                    h[e] = h0 | ((uint32_t)h1 << 16);
                    l[e] = l0 | ((uint32_t)l1 << 16);
                }
                // streaming stores: the planes are far larger than the caches and
                // are next read by the contraction, not by this kernel
                const int64_t word = (rb * kw + sp * 4 + g) * 64 + lane;
                __builtin_nontemporal_store(v4u{h[0], h[1], h[2], h[3]}, reinterpret_cast<v4u*>(oh + word));
                if (yl) __builtin_nontemporal_store(v4u{l[0], l[1], l[2], l[3]}, reinterpret_cast<v4u*>(ol + word));
            }
        }
    }
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

// src [rows][cols] (leading dim lds) -> FP64 copy [rpad][cpad], zero padded.
__global__ void k_pad_f64(const double* __restrict__ src, int64_t lds, int rows, int64_t cols,
                          double* __restrict__ f64, int64_t cpad) {
    const int r = blockIdx.y;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cpad;
         c += (int64_t)gridDim.x * blockDim.x)
        f64[(int64_t)r * cpad + c] = (r < rows && c < cols) ? src[(int64_t)r * lds + c] : 0.0;
}

// Plane z = blockIdx.y of src (+ z * sstride; [rows][cols], leading dim lds)
// times scale[z] -> hi/lo panel planes (+ z * rpad * cpad) [rpad][cpad], zero
// padded, and for plane 0 optionally an unscaled FP32 row-major copy.  One
// lane per row and 8-element k-group (one 16-byte word per plane).  lo ==
// nullptr skips the lo planes.
template <int ET>
__global__ void k_split_panel(const double* __restrict__ src, int64_t sstride, int64_t lds, int rows,
                              int64_t cols, const double* __restrict__ scale, uint16_t* __restrict__ hi,
                              uint16_t* __restrict__ lo, float* __restrict__ f32, int rpad, int64_t cpad) {
    const int z = blockIdx.y;
    const int lane = threadIdx.x & 63;
    // a wave covers 16 rows x 4 k-groups of one 64-row block: 4 lanes per row,
    // so each row is read (and its FP32 copy written) in 256-byte runs
    const int64_t kw = cpad / 8, ks = cpad / 32, nw = (int64_t)(rpad / 64) * ks * 4;
    const double s = scale ? scale[z] : 1.0;
    const double* sp = src + z * sstride;
    uint4* oh = reinterpret_cast<uint4*>(hi + (int64_t)z * rpad * cpad);
    uint4* ol = lo ? reinterpret_cast<uint4*>(lo + (int64_t)z * rpad * cpad) : nullptr;
    const int64_t wstride = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; w < nw; w += wstride) {
        const int64_t rb = w / (ks * 4), rem = w % (ks * 4);
        const int row = (int)(rem & 3) * 16 + (lane >> 2);
        const int64_t g = (rem >> 2) * 4 + (lane & 3);
        const int64_t p = rb * 64 + row, k0 = g * 8;
        double v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            v[e] = (p < rows && k0 + e < cols) ? sp[p * lds + k0 + e] : 0.0;
        if (f32 && z == 0) {
            float4* d = reinterpret_cast<float4*>(f32 + p * cpad + k0);
            d[0] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
            d[1] = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
        }
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double a = v[2 * e] * s, b = v[2 * e + 1] * s;
            const uint16_t ha = Elem<ET>::bits((float)a), hb = Elem<ET>::bits((float)b);
            const uint16_t la = Elem<ET>::bits((float)(a - (double)Elem<ET>::val(ha)));
            const uint16_t lb = Elem<ET>::bits((float)(b - (double)Elem<ET>::val(hb)));
            h[e] = ha | ((uint32_t)hb << 16);
            l[e] = la | ((uint32_t)lb << 16);
        }
        const int64_t word = (rb * kw + g) * 64 + row;
        oh[word] = make_uint4(h[0], h[1], h[2], h[3]);
        if (lo) ol[word] = make_uint4(l[0], l[1], l[2], l[3]);
    }
}

// o_nm [S][N][n_mo] -> B^T rows c = s*n_mo + m: f64 [cpad][npad] (+ hi/lo panel
// planes of B * scale), LDS-tiled transpose, zero padded.  With rowsel, output row c takes
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
            if (bt64) bt64[(int64_t)c * npad + p] = v;
            if (bh) split_store<ET>(v * s, bh, bl, panel_off(c, p, npad));
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
// One 64 x 64 lower tile per workgroup: a wave reads or writes 512-byte row
// segments, and the tile goes through LDS for its mirror image.
__global__ __launch_bounds__(256) void k_finalize_lambda(double* __restrict__ E, int npad,
                                                         const int* __restrict__ idflag,
                                                         uint32_t* __restrict__ lmax) {
    __shared__ double tile[64][65];
    const int nt = npad / 64, T = nt * (nt + 1) / 2;
    const int f = blockIdx.x / T;
    int I, J;
    lower_tile32(blockIdx.x % T, I, J);
    double* Ef = E + (int64_t)f * npad * npad;
    const double id = idflag[f] ? 1.0 : 0.0;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double m = 0.0;
#pragma unroll 4
    for (int yy = ty; yy < 64; yy += 4) {
        const int P = I * 64 + yy, Q = J * 64 + tx;
        const double v = (I == J && Q > P) ? 0.0 : Ef[(int64_t)P * npad + Q];
        const double l = -v - (P == Q ? id : 0.0);
        tile[yy][tx] = l;
        m = fmax(m, fabs(l));
    }
    __syncthreads();
    if (I == J) {
        for (int yy = ty; yy < 64; yy += 4)
            if (tx > yy) tile[yy][tx] = tile[tx][yy];
        __syncthreads();
    }
#pragma unroll 4
    for (int yy = ty; yy < 64; yy += 4) {
        Ef[(int64_t)(I * 64 + yy) * npad + J * 64 + tx] = tile[yy][tx];
        if (I != J) Ef[(int64_t)(J * 64 + yy) * npad + I * 64 + tx] = tile[tx][yy];
    }
    if (lmax) {
        m = wave_max(m);
        if (tx == 0) atomic_absmax(lmax + f, m);
    }
}

// W_im[s][m][f] = sum_I partial[f][I][s*n_mo + m]
// W_im[c][node[f]] = sum_I partial[f][I][c] for the n_imp imaginary planes f
// (row stride n_freq, the full grid).
__global__ void k_reduce_w_im(const double* __restrict__ partial, int ni, int cpad, int n_imp,
                              const int* __restrict__ node, int n_freq, int ncols, double* __restrict__ w_im) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)ncols * n_imp) return;
    int c = (int)(t / n_imp), f = (int)(t % n_imp);
    double s = 0.0;
    for (int i = 0; i < ni; ++i) s += partial[((int64_t)f * ni + i) * cpad + c];
    w_im[(int64_t)c * n_freq + node[f]] = s;
}

// W at the nodes without a plane: W_im[c][rest[r]] = sum_j T[r][j] W_im[c][node[j]].
__global__ void k_interp_w_im(double* __restrict__ w_im, int n_freq, int ncols, int n_imp,
                              const int* __restrict__ node, int n_rest, const int* __restrict__ rest,
                              const double* __restrict__ T) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)ncols * n_rest) return;
    int c = (int)(t / n_rest), r = (int)(t % n_rest);
    double* row = w_im + (int64_t)c * n_freq;
    double s = 0.0;
    for (int j = 0; j < n_imp; ++j) s += T[(int64_t)r * n_imp + j] * row[node[j]];
    row[rest[r]] = s;
}

// Gershgorin bound of an imaginary-axis plane: rowsum[P] += sum_Q |E_PQ - delta_PQ|
// over the symmetric matrix stored in the lower triangle; one 64 x 64 tile
// per block, one row per wave at a time.
__global__ void k_rowabs(const double* __restrict__ E, int npad, double* __restrict__ rowsum) {
    __shared__ double cs[4][64];
    int t = blockIdx.x, I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const int q = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double csum = 0.0;
    for (int p = wv; p < 64; p += 4) {
        const int P = I * 64 + p, Q = J * 64 + q;
        const double v = (I == J && Q > P) ? 0.0 : fabs(E[(int64_t)P * npad + Q] - (P == Q ? 1.0 : 0.0));
        csum += v;
        double r = v;
        for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
        if (q == 0) atomicAdd(&rowsum[P], r);
    }
    cs[wv][q] = csum;
    __syncthreads();
    if (I != J && threadIdx.x < 64)
        atomicAdd(&rowsum[J * 64 + threadIdx.x], cs[0][threadIdx.x] + cs[1][threadIdx.x] + cs[2][threadIdx.x] +
                                                     cs[3][threadIdx.x]);
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

void launch_prescale(hipStream_t s, int et, const float* x32, int npad, int64_t kpad, const float* cw32,
                     const double* ys, const int* fmap, int nfb, uint16_t* yh, uint16_t* yl) {
    const int64_t waves = (int64_t)(npad / 64) * (kpad / 32);
    dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 8192)));
    if (et == 1)
        hipLaunchKernelGGL(k_prescale<1>, grid, dim3(256), 0, s, x32, npad, kpad, cw32, ys, fmap, nfb, yh, yl);
    else
        hipLaunchKernelGGL(k_prescale<0>, grid, dim3(256), 0, s, x32, npad, kpad, cw32, ys, fmap, nfb, yh, yl);
}

void launch_scales_w(hipStream_t s, const uint32_t* lmax, int n_f, double* sf, double* lam_scale, double* w_unscale) {
    hipLaunchKernelGGL(k_scales_w, dim3(1), dim3(256), 0, s, lmax, n_f, sf, lam_scale, w_unscale);
}

void launch_pad_f64(hipStream_t s, const double* src, int64_t lds, int rows, int64_t cols, double* f64, int rpad,
                    int64_t cpad) {
    dim3 grid(grid1(cpad, 2048), rpad);
    hipLaunchKernelGGL(k_pad_f64, grid, dim3(256), 0, s, src, lds, rows, cols, f64, cpad);
}

void launch_split_panel(hipStream_t s, int et, const double* src, int64_t sstride, int nz, int64_t lds, int rows,
                        int64_t cols, const double* scale, uint16_t* hi, uint16_t* lo, float* f32, int rpad,
                        int64_t cpad) {
    const int64_t waves = (int64_t)(rpad / 64) * (cpad / 32) * 4;
    dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 4096)), nz);
    if (et == 1)
        hipLaunchKernelGGL(k_split_panel<1>, grid, dim3(256), 0, s, src, sstride, lds, rows, cols, scale, hi, lo,
                           f32, rpad, cpad);
    else
        hipLaunchKernelGGL(k_split_panel<0>, grid, dim3(256), 0, s, src, sstride, lds, rows, cols, scale, hi, lo,
                           f32, rpad, cpad);
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
    int nt = npad / 64, T = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_finalize_lambda, dim3(T * n_f), dim3(256), 0, s, E, npad, idflag, lmax);
}

void launch_interp_w(hipStream_t s, double* w_im, int n_freq, int ncols, int n_imp, const int* node, int n_rest,
                     const int* rest, const double* T) {
    int64_t n = (int64_t)ncols * n_rest;
    if (n > 0)
        hipLaunchKernelGGL(k_interp_w_im, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w_im, n_freq, ncols,
                           n_imp, node, n_rest, rest, T);
}

void launch_rowabs(hipStream_t s, const double* E, int npad, double* rowsum) {
    const int nt = npad / 64;
    hipLaunchKernelGGL(k_rowabs, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, E, npad, rowsum);
}

void launch_extract_pi(hipStream_t s, const double* E, int npad, int n, int n_z, int q, double* out) {
    int64_t tot = (int64_t)n_z * n * n;
    hipLaunchKernelGGL(k_extract_pi, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, E, npad, n, n_z, q, out);
}

void launch_reduce_w(hipStream_t s, const double* partial_im, const double* partial_re, int ni, int cpad, int cfpad,
                     int n_imp, const int* node, int n_freq, int n_re, int ncols, int nfit, double* w_im,
                     double* w_re) {
    int64_t n1 = (int64_t)ncols * n_imp;
    if (n1 > 0)
        hipLaunchKernelGGL(k_reduce_w_im, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, partial_im, ni, cpad,
                           n_imp, node, n_freq, ncols, w_im);
    int64_t n2 = (int64_t)nfit * n_re;
    if (n2 > 0)
        hipLaunchKernelGGL(k_reduce_w_re, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, partial_re, ni, cfpad,
                           n_re, nfit, w_re);
}

}  // namespace cdwac
