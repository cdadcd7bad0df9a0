// Inversion of the dielectric matrix eps(z) = I - Pi(z) (Eq. bigLambda) by
// the blocked symmetric sweep (Gauss-Jordan without pivoting), FP64.
//
// Sweeping diagonal block k of a symmetric A with D = A_kk replaces
//   A_ij <- A_ij - A_ik D^-1 A_kj   (i, j != k)
//   A_ik <- A_ik D^-1,  A_kj <- D^-1 A_kj,  A_kk <- -D^-1
// and after every block has been swept A holds -A^-1.  For a symmetric A this
// costs N^3 flops, the same as Cholesky + triangular inverse + product, but
// every step is one rank-64 update of the whole (lower) matrix, which maps onto
// batched matrix-core tiles.  eps(i w) is symmetric positive definite
// (Pi(i w) <= 0), so no pivoting is needed there; at near-real z the matrix is
// complex symmetric and the same recursion is used without conjugation.
// Only the lower triangle of A is read and written.
#include "common.h"
#include "kernels.h"

namespace cdwac {

template <bool C>
struct Planes {
    double* re;
    double* im;
};

// Plane addresses of matrix `mat` in the E array: real matrices are planes
// 0..n_real-1; complex matrix j uses planes (cbase + 2j, cbase + 2j + 1).
__device__ inline double* plane(double* E, int64_t n2, int p) { return E + (int64_t)p * n2; }

template <bool C>
__device__ inline void mat_planes(double* E, int64_t n2, int mat, int cbase, double*& re, double*& im) {
    if (C) {
        re = plane(E, n2, cbase + 2 * mat);
        im = re + n2;
    } else {
        re = plane(E, n2, mat);
        im = nullptr;
    }
}

// ---------------------------------------------------------------------------
// 1. Invert the current diagonal block: Dinv = D^-1 (unblocked sweep in LDS).
// ---------------------------------------------------------------------------
template <bool C>
__global__ __launch_bounds__(256) void k_sweep_diag(double* __restrict__ E, int npad, int cbase,
                                                    int kb, double* __restrict__ dinv,
                                                    int* __restrict__ err) {
    __shared__ double dr[kNb][kNb + 1];
    __shared__ double di[C ? kNb : 1][C ? kNb + 1 : 1];
    const int mat = blockIdx.x;
    const int64_t n2 = (int64_t)npad * npad;
    double *Er, *Ei;
    mat_planes<C>(E, n2, mat, cbase, Er, Ei);
    const int k0 = kb * kNb;
    for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
        int i = e / kNb, j = e % kNb;
        int r = i >= j ? i : j, c = i >= j ? j : i;
        int64_t o = (int64_t)(k0 + r) * npad + k0 + c;
        dr[i][j] = Er[o];
        if (C) di[i][j] = Ei[o];
    }
    __syncthreads();
    for (int p = 0; p < kNb; ++p) {
        double nv_r[16], nv_i[16];
        cplx piv = cmk(dr[p][p], C ? di[p][p] : 0.0);
        cplx inv = cmk(1.0, 0.0) / piv;
        if (threadIdx.x == 0 && (!cfinite(inv) || (piv.re == 0.0 && piv.im == 0.0))) atomicOr(err, 1);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int e = threadIdx.x + 256 * q;
            int i = e / kNb, j = e % kNb;
            cplx aij = cmk(dr[i][j], C ? di[i][j] : 0.0);
            cplx aip = cmk(dr[i][p], C ? di[i][p] : 0.0);
            cplx apj = cmk(dr[p][j], C ? di[p][j] : 0.0);
            cplx v;
            if (i != p && j != p) v = aij - aip * (apj * inv);
            else if (i == p && j == p) v = cmk(-inv.re, -inv.im);
            else if (i == p) v = apj * inv;
            else v = aip * inv;
            nv_r[q] = v.re;
            nv_i[q] = v.im;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int e = threadIdx.x + 256 * q;
            dr[e / kNb][e % kNb] = nv_r[q];
            if (C) di[e / kNb][e % kNb] = nv_i[q];
        }
        __syncthreads();
    }
    // the block now holds -D^-1
    double* out = dinv + (int64_t)mat * (C ? 2 : 1) * kNb * kNb;
    for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
        out[e] = -dr[e / kNb][e % kNb];
        if (C) out[kNb * kNb + e] = -di[e / kNb][e % kNb];
    }
}

// ---------------------------------------------------------------------------
// 2. Panel: P_i = A_ik (old), Q_i = P_i D^-1 for every block row i != k.
//    Buffers [mat][plane][nblk][64][64], row-major [row][k].
// ---------------------------------------------------------------------------
template <bool C>
__global__ __launch_bounds__(256) void k_sweep_panel(double* __restrict__ E, int npad, int cbase,
                                                     int kb, const double* __restrict__ dinv,
                                                     double* __restrict__ pbuf,
                                                     double* __restrict__ qbuf) {
    __shared__ double pr[kNb][kNb + 1];
    __shared__ double pi[C ? kNb : 1][C ? kNb + 1 : 1];
    const int ib = blockIdx.x, mat = blockIdx.y;
    const int nblk = npad / kNb;
    if (ib == kb) return;
    const int64_t n2 = (int64_t)npad * npad;
    double *Er, *Ei;
    mat_planes<C>(E, n2, mat, cbase, Er, Ei);
    const int k0 = kb * kNb, i0 = ib * kNb;
    // load P_i = A_ik (stored directly below the diagonal block, or transposed)
    for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
        int a = e / kNb, b = e % kNb;
        if (ib > kb) {
            int64_t o = (int64_t)(i0 + a) * npad + k0 + b;     // row a, col b
            pr[a][b] = Er[o];
            if (C) pi[a][b] = Ei[o];
        } else {
            int64_t o = (int64_t)(k0 + a) * npad + i0 + b;     // A_ki[a][b] = P_i[b][a]
            pr[b][a] = Er[o];
            if (C) pi[b][a] = Ei[o];
        }
    }
    __syncthreads();
    const int planes = C ? 2 : 1;
    const int64_t blk = (int64_t)kNb * kNb;
    const double* Dr = dinv + (int64_t)mat * planes * blk;
    const double* Di = C ? Dr + blk : nullptr;
    double* Pb = pbuf + ((int64_t)mat * planes * nblk + ib) * blk;
    double* Qb = qbuf + ((int64_t)mat * planes * nblk + ib) * blk;
    const int64_t pstride = (int64_t)nblk * blk;   // plane stride inside a matrix
    // thread -> column c, rows r = t/64 + 4q
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    double accr[16], acci[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) { accr[q] = 0.0; acci[q] = 0.0; }
    for (int k = 0; k < kNb; ++k) {
        double dre = Dr[k * kNb + c];
        double dim = C ? Di[k * kNb + c] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int r = r0 + 4 * q;
            double a = pr[r][k];
            accr[q] += a * dre;
            if (C) {
                double b = pi[r][k];
                accr[q] -= b * dim;
                acci[q] += a * dim + b * dre;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        int r = r0 + 4 * q;
        Qb[r * kNb + c] = accr[q];
        Pb[r * kNb + c] = pr[r][c];
        if (C) {
            Qb[pstride + r * kNb + c] = acci[q];
            Pb[pstride + r * kNb + c] = pi[r][c];
        }
    }
}

// ---------------------------------------------------------------------------
// 3. Rank-64 update of every lower tile (I, J), I, J != k:
//    A_IJ -= Q_I P_J^T  (complex: re -= Qr Pr^T - Qi Pi^T, im -= Qr Pi^T + Qi Pr^T)
//    FP64 MFMA 16x16x4, 64 x 64 tile, 4 waves of 32 x 32.
//    With M3 the complex product takes three real products instead of four
//    (Gauss): T1 = Qr Pr^T, T2 = Qi Pi^T, T3 = (Qr + Qi)(Pr + Pi)^T, re = T1 - T2,
//    im = T3 - T1 - T2.  Its rounding error is bounded by (|Qr| + |Qi|)(|Pr| + |Pi|)
//    u per term, the size of the real part's, so it is used where the inputs
//    carry 16-bit contraction errors far above that.
// ---------------------------------------------------------------------------
constexpr int U_KC = 16, U_LD = kNb + 2;

// KW = panel width: 64 (one pivot block kb) or 128 (pivot blocks kb, kb + 1).
template <bool C, int KW = kNb, bool M3 = false>
__global__ __launch_bounds__(256) void k_sweep_update(double* __restrict__ E, int npad, int cbase,
                                                      int kb, const double* __restrict__ pbuf,
                                                      const double* __restrict__ qbuf) {
    __shared__ double sq[C ? 2 : 1][U_KC][U_LD];
    __shared__ double sp[C ? 2 : 1][U_KC][U_LD];
    const int nblk = npad / kNb, T = nblk * (nblk + 1) / 2;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int mat = bid / T;
    int I, J;
    sweep_tile_order(bid % T, nblk, I, J);
    constexpr int NK = KW / kNb;                 // pivot blocks of this step
    if ((I >= kb && I < kb + NK) || (J >= kb && J < kb + NK)) return;
    const int planes = C ? 2 : 1;
    const int64_t blk = (int64_t)kNb * KW, pstride = (int64_t)nblk * blk;
    const double* Q = qbuf + ((int64_t)mat * planes * nblk + I) * blk;
    const double* P = pbuf + ((int64_t)mat * planes * nblk + J) * blk;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const int row = threadIdx.x >> 2, kq = (threadIdx.x & 3) * 4;
    // the tile of A is read before the product so that its loads overlap it
    const int64_t n2 = (int64_t)npad * npad;
    double *Er, *Ei;
    mat_planes<C>(E, n2, mat, cbase, Er, Ei);
    double er[2][2][4], ei[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t o = (int64_t)(I * kNb + wr * 32 + bi * 16 + lk + 4 * r) * npad + J * kNb + wc * 32 +
                                  bj * 16 + lr;
                er[bi][bj][r] = Er[o];
                if (C) ei[bi][bj][r] = Ei[o];
            }
    v4d ar[2][2] = {}, ai[2][2] = {}, a2[M3 ? 2 : 1][M3 ? 2 : 1] = {};
    for (int k0 = 0; k0 < KW; k0 += U_KC) {
#pragma unroll
        for (int pl = 0; pl < planes; ++pl) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sq[pl][kq + e][row] = Q[pl * pstride + row * KW + k0 + kq + e];
                sp[pl][kq + e][row] = P[pl * pstride + row * KW + k0 + kq + e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < U_KC / 4; ++kk) {
            const int k = kk * 4 + lk;
            double qa[2], pa[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                qa[b] = sq[0][k][wr * 32 + b * 16 + lr];
                pa[b] = sp[0][k][wc * 32 + b * 16 + lr];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    ar[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[bi], pa[bj], ar[bi][bj], 0, 0, 0);
            if (C) {
                double qb[2], pb[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    qb[b] = sq[C ? 1 : 0][k][wr * 32 + b * 16 + lr];
                    pb[b] = sp[C ? 1 : 0][k][wc * 32 + b * 16 + lr];
                }
                if (M3) {
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj) {
                            a2[M3 ? bi : 0][M3 ? bj : 0] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                qb[bi], pb[bj], a2[M3 ? bi : 0][M3 ? bj : 0], 0, 0, 0);
                            ai[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[bi] + qb[bi], pa[bj] + pb[bj],
                                                                             ai[bi][bj], 0, 0, 0);
                        }
                } else {
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj) {
                            ar[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-qb[bi], pb[bj], ar[bi][bj], 0, 0, 0);
                            ai[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[bi], pb[bj], ai[bi][bj], 0, 0, 0);
                            ai[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(qb[bi], pa[bj], ai[bi][bj], 0, 0, 0);
                        }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int P_ = I * kNb + wr * 32 + bi * 16 + lk + 4 * r;
                int Q_ = J * kNb + wc * 32 + bj * 16 + lr;
                int64_t o = (int64_t)P_ * npad + Q_;
                if (C && M3) {
                    const double t1 = ar[bi][bj][r], t2 = a2[M3 ? bi : 0][M3 ? bj : 0][r];
                    Er[o] = er[bi][bj][r] - (t1 - t2);
                    Ei[o] = ei[bi][bj][r] - (ai[bi][bj][r] - t1 - t2);
                } else {
                    Er[o] = er[bi][bj][r] - ar[bi][bj][r];
                    if (C) Ei[o] = ei[bi][bj][r] - ai[bi][bj][r];
                }
            }
}

// ---------------------------------------------------------------------------
// 4. Write back: A_ik <- Q_i, A_ki <- Q_i^T, A_kk <- -D^-1.
// ---------------------------------------------------------------------------
template <bool C>
__global__ __launch_bounds__(256) void k_sweep_writeback(double* __restrict__ E, int npad, int cbase,
                                                         int kb, const double* __restrict__ dinv,
                                                         const double* __restrict__ qbuf) {
    const int ib = blockIdx.x, mat = blockIdx.y;
    const int nblk = npad / kNb;
    const int planes = C ? 2 : 1;
    const int64_t blk = (int64_t)kNb * kNb, pstride = (int64_t)nblk * blk;
    const int64_t n2 = (int64_t)npad * npad;
    double *Er, *Ei;
    mat_planes<C>(E, n2, mat, cbase, Er, Ei);
    const int k0 = kb * kNb, i0 = ib * kNb;
    if (ib == kb) {
        const double* D = dinv + (int64_t)mat * planes * blk;
        for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
            int a = e / kNb, b = e % kNb;
            int64_t o = (int64_t)(k0 + a) * npad + k0 + b;
            Er[o] = -D[e];
            if (C) Ei[o] = -D[blk + e];
        }
        return;
    }
    const double* Qb = qbuf + ((int64_t)mat * planes * nblk + ib) * blk;
    for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
        if (ib > kb) {
            int a = e / kNb, b = e % kNb;                 // Q[a][b] -> A[i0+a][k0+b]
            int64_t o = (int64_t)(i0 + a) * npad + k0 + b;
            Er[o] = Qb[a * kNb + b];
            if (C) Ei[o] = Qb[pstride + a * kNb + b];
        } else {
            int b = e / kNb, a = e % kNb;                 // Q[a][b] -> A[k0+b][i0+a]
            int64_t o = (int64_t)(k0 + b) * npad + i0 + a;
            Er[o] = Qb[a * kNb + b];
            if (C) Ei[o] = Qb[pstride + a * kNb + b];
        }
    }
}

// Sweeps every block of n_real real and n_cplx complex matrices in E.
void launch_sweep(hipStream_t s, double* E, int npad, int n_real, int n_cplx, int cbase, double* dinv_r,
                  double* pbuf_r, double* qbuf_r, double* dinv_c, double* pbuf_c, double* qbuf_c,
                  int* err, bool gauss3) {
    const int nblk = npad / kNb, T = nblk * (nblk + 1) / 2;
    for (int kb = 0; kb < nblk; ++kb) {
        if (n_real > 0) {
            hipLaunchKernelGGL(k_sweep_diag<false>, dim3(n_real), dim3(256), 0, s, E, npad, 0, kb, dinv_r, err);
            hipLaunchKernelGGL(k_sweep_panel<false>, dim3(nblk, n_real), dim3(256), 0, s, E, npad, 0, kb,
                               dinv_r, pbuf_r, qbuf_r);
            hipLaunchKernelGGL(k_sweep_update<false>, dim3(T * n_real), dim3(256), 0, s, E, npad, 0, kb,
                               pbuf_r, qbuf_r);
            hipLaunchKernelGGL(k_sweep_writeback<false>, dim3(nblk, n_real), dim3(256), 0, s, E, npad, 0,
                               kb, dinv_r, qbuf_r);
        }
        if (n_cplx > 0) {
            hipLaunchKernelGGL(k_sweep_diag<true>, dim3(n_cplx), dim3(256), 0, s, E, npad, cbase, kb, dinv_c,
                               err);
            hipLaunchKernelGGL(k_sweep_panel<true>, dim3(nblk, n_cplx), dim3(256), 0, s, E, npad, cbase, kb,
                               dinv_c, pbuf_c, qbuf_c);
            if (gauss3)
                hipLaunchKernelGGL((k_sweep_update<true, kNb, true>), dim3(T * n_cplx), dim3(256), 0, s, E, npad,
                                   cbase, kb, pbuf_c, qbuf_c);
            else
                hipLaunchKernelGGL(k_sweep_update<true>, dim3(T * n_cplx), dim3(256), 0, s, E, npad, cbase, kb,
                                   pbuf_c, qbuf_c);
            hipLaunchKernelGGL(k_sweep_writeback<true>, dim3(nblk, n_cplx), dim3(256), 0, s, E, npad, cbase,
                               kb, dinv_c, qbuf_c);
        }
    }
}

// ---------------------------------------------------------------------------
// Sweeps of 128-wide pivot blocks K = {kb, kb + 1}: the same recursion with
// D = A_KK (128 x 128), so each update is a rank-128 pass over the matrix and
// the matrix streams through HBM half as often as with 64-wide pivots.
// -D^-1 comes from sweeping a copy of A_KK with the 64-block kernels above.
// Panel buffers hold 64 x 128 blocks: [mat][plane][nblk][64][128].
// ---------------------------------------------------------------------------
constexpr int kNb2 = 2 * kNb;

// dscr[mat] (128 x 128, lower triangle) <- A_KK.
template <bool C>
__global__ __launch_bounds__(256) void k_sweep_gather(const double* __restrict__ E, int npad, int cbase, int kb,
                                                      double* __restrict__ dscr) {
    const int mat = blockIdx.x;
    const int64_t n2 = (int64_t)npad * npad, d2 = (int64_t)kNb2 * kNb2;
    double *Er, *Ei, *Dr, *Di;
    mat_planes<C>(const_cast<double*>(E), n2, mat, cbase, Er, Ei);
    mat_planes<C>(dscr, d2, mat, 0, Dr, Di);
    const int k0 = kb * kNb;
    for (int e = threadIdx.x; e < kNb2 * kNb2; e += 256) {
        const int r = e / kNb2, c = e % kNb2;
        if (c > r) continue;
        const int64_t o = (int64_t)(k0 + r) * npad + k0 + c;
        Dr[e] = Er[o];
        if (C) Di[e] = Ei[o];
    }
}

// P_i = A_iK (64 x 128, old values) and Q_i = P_i D^-1 for every block row
// i outside K; D^-1 = -(swept copy), read from its lower triangle.
template <bool C>
__global__ __launch_bounds__(256) void k_sweep_panel2(const double* __restrict__ E, int npad, int cbase, int kb,
                                                      const double* __restrict__ dscr, double* __restrict__ pbuf,
                                                      double* __restrict__ qbuf) {
    __shared__ double pr[kNb][kNb2 + 1];
    __shared__ double pi[C ? kNb : 1][C ? kNb2 + 1 : 1];
    const int ib = blockIdx.x, mat = blockIdx.y;
    const int nblk = npad / kNb;
    if (ib == kb || ib == kb + 1) return;
    const int64_t n2 = (int64_t)npad * npad, d2 = (int64_t)kNb2 * kNb2;
    double *Er, *Ei, *Dr, *Di;
    mat_planes<C>(const_cast<double*>(E), n2, mat, cbase, Er, Ei);
    mat_planes<C>(const_cast<double*>(dscr), d2, mat, 0, Dr, Di);
    const int i0 = ib * kNb;
    for (int e = threadIdx.x; e < kNb * kNb2; e += 256) {
        const int a = e / kNb2, b = e % kNb2;          // row a of block i, column b of K
        const int kc = kb * kNb + b;
        const int64_t o = ib > kb ? (int64_t)(i0 + a) * npad + kc      // A_iK stored in the lower triangle
                                  : (int64_t)kc * npad + i0 + a;       // or as A_Ki
        pr[a][b] = Er[o];
        if (C) pi[a][b] = Ei[o];
    }
    __syncthreads();
    const int planes = C ? 2 : 1;
    const int64_t blk = (int64_t)kNb * kNb2, pstride = (int64_t)nblk * blk;
    double* Pb = pbuf + ((int64_t)mat * planes * nblk + ib) * blk;
    double* Qb = qbuf + ((int64_t)mat * planes * nblk + ib) * blk;
    // thread -> column c, rows r = t/128 + 2q
    const int c = threadIdx.x & (kNb2 - 1), r0 = threadIdx.x >> 7;
    double accr[32], acci[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) { accr[q] = 0.0; acci[q] = 0.0; }
    for (int k = 0; k < kNb2; ++k) {
        const int64_t o = k >= c ? (int64_t)k * kNb2 + c : (int64_t)c * kNb2 + k;
        const double dre = -Dr[o];
        const double dim = C ? -Di[o] : 0.0;
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int r = r0 + 2 * q;
            const double a = pr[r][k];
            accr[q] += a * dre;
            if (C) {
                const double b = pi[r][k];
                accr[q] -= b * dim;
                acci[q] += a * dim + b * dre;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int r = r0 + 2 * q;
        Qb[r * kNb2 + c] = accr[q];
        Pb[r * kNb2 + c] = pr[r][c];
        if (C) {
            Qb[pstride + r * kNb2 + c] = acci[q];
            Pb[pstride + r * kNb2 + c] = pi[r][c];
        }
    }
}

// A_iK <- Q_i for every block row i outside K; A_KK <- -D^-1 (the swept copy).
template <bool C>
__global__ __launch_bounds__(256) void k_sweep_writeback2(double* __restrict__ E, int npad, int cbase, int kb,
                                                          const double* __restrict__ dscr,
                                                          const double* __restrict__ qbuf) {
    const int ib = blockIdx.x, mat = blockIdx.y;
    const int nblk = npad / kNb;
    const int planes = C ? 2 : 1;
    const int64_t blk = (int64_t)kNb * kNb2, pstride = (int64_t)nblk * blk;
    const int64_t n2 = (int64_t)npad * npad, d2 = (int64_t)kNb2 * kNb2;
    double *Er, *Ei, *Dr, *Di;
    mat_planes<C>(E, n2, mat, cbase, Er, Ei);
    mat_planes<C>(const_cast<double*>(dscr), d2, mat, 0, Dr, Di);
    const int k0 = kb * kNb, i0 = ib * kNb;
    if (ib == kb + 1) return;
    if (ib == kb) {
        for (int e = threadIdx.x; e < kNb2 * kNb2; e += 256) {
            const int r = e / kNb2, c = e % kNb2;
            if (c > r) continue;
            const int64_t o = (int64_t)(k0 + r) * npad + k0 + c;
            Er[o] = Dr[e];
            if (C) Ei[o] = Di[e];
        }
        return;
    }
    const double* Qb = qbuf + ((int64_t)mat * planes * nblk + ib) * blk;
    for (int e = threadIdx.x; e < kNb * kNb2; e += 256) {
        if (ib > kb) {
            const int a = e / kNb2, b = e % kNb2;          // Q[a][b] -> A[i0 + a][k0 + b]
            const int64_t o = (int64_t)(i0 + a) * npad + k0 + b;
            Er[o] = Qb[a * kNb2 + b];
            if (C) Ei[o] = Qb[pstride + a * kNb2 + b];
        } else {
            const int b = e / kNb, a = e % kNb;            // Q[a][b] -> A[k0 + b][i0 + a]
            const int64_t o = (int64_t)(k0 + b) * npad + i0 + a;
            Er[o] = Qb[a * kNb2 + b];
            if (C) Ei[o] = Qb[pstride + a * kNb2 + b];
        }
    }
}

// Sweeps every block of n_mat real (C = false) or complex (C = true,
// planes cbase + 2j) matrices in E with 128-wide pivots.  npad must be a
// multiple of 128.  dscr: [n_mat][planes][128][128]; dinv, pbuf, qbuf as for
// launch_sweep, with pbuf and qbuf twice as large.
template <bool C>
void launch_sweep2_t(hipStream_t s, double* E, int npad, int n_mat, int cbase, double* dscr, double* dinv,
                     double* pbuf, double* qbuf, int* err) {
    if (n_mat <= 0) return;
    const int nblk = npad / kNb, T = nblk * (nblk + 1) / 2;
    for (int kb = 0; kb < nblk; kb += 2) {
        hipLaunchKernelGGL(k_sweep_gather<C>, dim3(n_mat), dim3(256), 0, s, E, npad, cbase, kb, dscr);
        // -D^-1 of every pivot block: a 64-block sweep of the 128 x 128 copies
        if (C) launch_sweep(s, dscr, kNb2, 0, n_mat, 0, nullptr, nullptr, nullptr, dinv, pbuf, qbuf, err);
        else launch_sweep(s, dscr, kNb2, n_mat, 0, 0, dinv, pbuf, qbuf, nullptr, nullptr, nullptr, err);
        hipLaunchKernelGGL(k_sweep_panel2<C>, dim3(nblk, n_mat), dim3(256), 0, s, E, npad, cbase, kb, dscr, pbuf,
                           qbuf);
        hipLaunchKernelGGL((k_sweep_update<C, kNb2>), dim3(T * n_mat), dim3(256), 0, s, E, npad, cbase, kb, pbuf,
                           qbuf);
        hipLaunchKernelGGL(k_sweep_writeback2<C>, dim3(nblk, n_mat), dim3(256), 0, s, E, npad, cbase, kb, dscr,
                           qbuf);
    }
}

void launch_sweep2(hipStream_t s, double* E, int npad, int n_real, int n_cplx, int cbase, double* dscr_r,
                   double* dscr_c, double* dinv_r, double* pbuf_r, double* qbuf_r, double* dinv_c, double* pbuf_c,
                   double* qbuf_c, int* err) {
    launch_sweep2_t<false>(s, E, npad, n_real, 0, dscr_r, dinv_r, pbuf_r, qbuf_r, err);
    launch_sweep2_t<true>(s, E, npad, n_cplx, cbase, dscr_c, dinv_c, pbuf_c, qbuf_c, err);
}

// ---------------------------------------------------------------------------
// Residual check of the computed inverses.  Before the sweep, kFactCols
// columns eps_j of every plane are copied out of the lower-triangle storage;
// after Lambda = eps^-1 - I has been formed (Re plane: Re eps^-1 - I; Im
// plane: Im eps^-1), r = (Lambda + I) eps_j - e_j = eps^-1 eps_j - e_j is
// formed in FP64 together with the scale b = |eps^-1| |eps_j| (elementwise
// moduli).  A backward-stable inverse keeps max|r| / max b at a small multiple
// of the unit roundoff; element growth in the unpivoted sweep of an indefinite
// complex-symmetric eps(x + i eta) raises it by the growth factor.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fact_gather(const double* __restrict__ E, int npad,
                                                     const int* __restrict__ cols,
                                                     double* __restrict__ out) {
    const int f = blockIdx.x, c = blockIdx.y;
    const int j = cols[c];
    const double* Ef = E + (int64_t)f * npad * npad;
    double* o = out + ((int64_t)f * kFactCols + c) * npad;
    for (int i = threadIdx.x; i < npad; i += 256)
        o[i] = i >= j ? Ef[(int64_t)i * npad + j] : Ef[(int64_t)j * npad + i];
}

__device__ inline double wave_sum_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per row i of one matrix (4 rows per workgroup); res[mat][c] holds
// {max_i |r_i|, max_i b_i} as the bit patterns of non-negative doubles, which
// order like the values (atomicMax on 64-bit integers).
template <bool C>
__global__ __launch_bounds__(256) void k_fact_residual(const double* __restrict__ E, int npad, int cbase,
                                                       const int* __restrict__ cols,
                                                       const double* __restrict__ saved,
                                                       unsigned long long* __restrict__ res, int res_base) {
    const int mat = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= npad) return;
    const int64_t n2 = (int64_t)npad * npad;
    const int pr = C ? cbase + 2 * mat : cbase + mat;
    const double* Lr = E + (int64_t)pr * n2 + (int64_t)i * npad;
    const double* Li = Lr + n2;
    const double* sr = saved + (int64_t)pr * kFactCols * npad;
    const double* si = sr + (int64_t)kFactCols * npad;
    double ar[kFactCols], ai[kFactCols], b[kFactCols];
#pragma unroll
    for (int c = 0; c < kFactCols; ++c) ar[c] = ai[c] = b[c] = 0.0;
    for (int k = lane; k < npad; k += 64) {
        const double lr = Lr[k] + (k == i ? 1.0 : 0.0);
        const double li = C ? Li[k] : 0.0;
        const double lm = C ? sqrt(lr * lr + li * li) : fabs(lr);
#pragma unroll
        for (int c = 0; c < kFactCols; ++c) {
            const double er = sr[(int64_t)c * npad + k];
            const double ei = C ? si[(int64_t)c * npad + k] : 0.0;
            ar[c] += lr * er - li * ei;
            ai[c] += lr * ei + li * er;
            b[c] += lm * (C ? sqrt(er * er + ei * ei) : fabs(er));
        }
    }
#pragma unroll
    for (int c = 0; c < kFactCols; ++c) {
        const double rr = wave_sum_d(ar[c]) - (i == cols[c] ? 1.0 : 0.0);
        const double ri = wave_sum_d(ai[c]);
        const double bb = wave_sum_d(b[c]);
        if (lane == 0) {
            unsigned long long* o = res + 2 * ((int64_t)(res_base + mat) * kFactCols + c);
            atomicMax(o, (unsigned long long)__double_as_longlong(sqrt(rr * rr + ri * ri)));
            atomicMax(o + 1, (unsigned long long)__double_as_longlong(bb));
        }
    }
}

void launch_fact_gather(hipStream_t s, const double* E, int npad, int n_f, const int* cols, double* out) {
    if (n_f > 0) hipLaunchKernelGGL(k_fact_gather, dim3(n_f, kFactCols), dim3(256), 0, s, E, npad, cols, out);
}

void launch_fact_residual(hipStream_t s, const double* E, int npad, int n_real, int n_cplx, int cbase,
                          const int* cols, const double* saved, unsigned long long* res) {
    const unsigned gx = (unsigned)((npad + 3) / 4);
    if (n_real > 0)
        hipLaunchKernelGGL(k_fact_residual<false>, dim3(gx, n_real), dim3(256), 0, s, E, npad, 0, cols, saved, res,
                           0);
    if (n_cplx > 0)
        hipLaunchKernelGGL(k_fact_residual<true>, dim3(gx, n_cplx), dim3(256), 0, s, E, npad, cbase, cols, saved,
                           res, n_real);
}

}  // namespace cdwac
