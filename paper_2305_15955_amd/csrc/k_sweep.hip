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
// ---------------------------------------------------------------------------
constexpr int U_KC = 16, U_LD = kNb + 2;

template <bool C>
__global__ __launch_bounds__(256) void k_sweep_update(double* __restrict__ E, int npad, int cbase,
                                                      int kb, const double* __restrict__ pbuf,
                                                      const double* __restrict__ qbuf) {
    __shared__ double sq[C ? 2 : 1][U_KC][U_LD];
    __shared__ double sp[C ? 2 : 1][U_KC][U_LD];
    const int nblk = npad / kNb, T = nblk * (nblk + 1) / 2;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int mat = bid / T;
    const int t = bid % T;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    if (I == kb || J == kb) return;
    const int planes = C ? 2 : 1;
    const int64_t blk = (int64_t)kNb * kNb, pstride = (int64_t)nblk * blk;
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
    v4d ar[2][2] = {}, ai[2][2] = {};
    for (int k0 = 0; k0 < kNb; k0 += U_KC) {
#pragma unroll
        for (int pl = 0; pl < planes; ++pl) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sq[pl][kq + e][row] = Q[pl * pstride + row * kNb + k0 + kq + e];
                sp[pl][kq + e][row] = P[pl * pstride + row * kNb + k0 + kq + e];
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
                Er[o] = er[bi][bj][r] - ar[bi][bj][r];
                if (C) Ei[o] = ei[bi][bj][r] - ai[bi][bj][r];
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
                  int* err) {
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
            hipLaunchKernelGGL(k_sweep_update<true>, dim3(T * n_cplx), dim3(256), 0, s, E, npad, cbase, kb,
                               pbuf_c, qbuf_c);
            hipLaunchKernelGGL(k_sweep_writeback<true>, dim3(nblk, n_cplx), dim3(256), 0, s, E, npad, cbase,
                               kb, dinv_c, qbuf_c);
        }
    }
}

}  // namespace cdwac
