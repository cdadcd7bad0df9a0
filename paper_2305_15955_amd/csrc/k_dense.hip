// Dense contractions of the CD-WAC path on gfx950 matrix cores.
//
//  * Pi_f = X diag(c_f) X^T  (Eq. piriv in RI form): a symmetric rank-K
//    product per real weight vector c_f; only lower tiles are computed and
//    eps_f = delta_f I - Pi_f is stored (delta_f = 1 for the real part of a
//    frequency, 0 for an imaginary part).
//  * W^c_nm = sum_PQ O^nm_P Lambda_PQ O^nm_Q  (Eq. wriv): C = Lambda B^T with
//    B = O^T (one row per (n, m)), then a fused column dot with B.
//
// Arithmetic: FP64 MFMA (v_mfma_f64_16x16x4), or 16-bit MFMA
// (v_mfma_f32_32x32x16_{bf16,f16}) on operands split as hi + lo with the
// products hi*hi + hi*lo + lo*hi accumulated in FP32 and flushed into FP64
// every kFlush k-values, so the FP32 rounding of long sums stays bounded.
#include "common.h"
#include "kernels.h"

#include <algorithm>

namespace cdwac {

// ============================================================================
// FP64 MFMA tile machinery: 64 x 64 output tile, 4 waves of 32 x 32,
// K chunks of 16 staged in LDS as [k][row].
// ============================================================================

constexpr int F_BT = 64, F_KC = 16, F_LD = F_BT + 2;

struct F64Stage {
    double a[F_KC][F_LD];
    double b[F_KC][F_LD];
};

// acc[bi][bj] += A_tile * B_tile^T for one staged chunk.
__device__ inline void f64_chunk(const F64Stage& st, int wr, int wc, int lane, v4d (&acc)[2][2]) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < F_KC / 4; ++kk) {
        const int k = kk * 4 + lk;
        double a0 = st.a[k][wr * 32 + lr], a1 = st.a[k][wr * 32 + 16 + lr];
        double b0 = st.b[k][wc * 32 + lr], b1 = st.b[k][wc * 32 + 16 + lr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

// Thread t loads row t/4, k = (t%4)*4 .. +3 of a 64 x 16 chunk.
struct F64Frag {
    double a[4], b[4];
};

__device__ inline void f64_load(F64Frag& fr, const double* __restrict__ arow,
                                const double* __restrict__ brow, const double* __restrict__ cw,
                                int64_t k0) {
    const double2* pa = reinterpret_cast<const double2*>(arow + k0);
    const double2* pb = reinterpret_cast<const double2*>(brow + k0);
    double2 a01 = pa[0], a23 = pa[1], b01 = pb[0], b23 = pb[1];
    fr.a[0] = a01.x; fr.a[1] = a01.y; fr.a[2] = a23.x; fr.a[3] = a23.y;
    fr.b[0] = b01.x; fr.b[1] = b01.y; fr.b[2] = b23.x; fr.b[3] = b23.y;
    if (cw) {
        const double2* pc = reinterpret_cast<const double2*>(cw + k0);
        double2 c01 = pc[0], c23 = pc[1];
        fr.b[0] *= c01.x; fr.b[1] *= c01.y; fr.b[2] *= c23.x; fr.b[3] *= c23.y;
    }
}

__device__ inline void f64_store(F64Stage& st, const F64Frag& fr, int row, int kq) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        st.a[kq + e][row] = fr.a[e];
        st.b[kq + e][row] = fr.b[e];
    }
}

// Full K loop: acc = A[rows a0..a0+63] * (B[rows b0..b0+63] * diag(cw))^T.
__device__ inline void f64_tile_product(const double* __restrict__ A, int64_t lda,
                                        const double* __restrict__ B, int64_t ldb,
                                        const double* __restrict__ cw, int64_t K,
                                        F64Stage (&st)[2], v4d (&acc)[2][2]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row = t >> 2, kq = (t & 3) * 4;
    const double* arow = A + (int64_t)row * lda + kq;
    const double* brow = B + (int64_t)row * ldb + kq;
    const double* crow = cw ? cw + kq : nullptr;
    const int64_t nk = K / F_KC;
    F64Frag fr;
    f64_load(fr, arow, brow, crow, 0);
    f64_store(st[0], fr, row, kq);
    __syncthreads();
    for (int64_t i = 0; i < nk; ++i) {
        const int s = (int)(i & 1);
        if (i + 1 < nk) f64_load(fr, arow, brow, crow, (i + 1) * F_KC);
        f64_chunk(st[s], wr, wc, lane, acc);
        if (i + 1 < nk) f64_store(st[s ^ 1], fr, row, kq);
        __syncthreads();
    }
}

__device__ inline void lower_tile(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// eps_f = delta_f I - X diag(c_f) X^T on the lower 64 x 64 tiles, FP64.
__global__ __launch_bounds__(256) void k_pi_f64(const double* __restrict__ x, int64_t kpad,
                                                const double* __restrict__ cw,
                                                const int* __restrict__ idflag,
                                                double* __restrict__ E, int npad, int n_f) {
    __shared__ F64Stage st[2];
    const int nt = npad / F_BT, T = nt * (nt + 1) / 2;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int f = bid / T;
    int I, J;
    lower_tile(bid % T, I, J);
    v4d acc[2][2] = {};
    f64_tile_product(x + (int64_t)I * F_BT * kpad, kpad, x + (int64_t)J * F_BT * kpad, kpad,
                     cw + (int64_t)f * kpad, kpad, st, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const double id = idflag[f] ? 1.0 : 0.0;
    double* Ef = E + (int64_t)f * npad * npad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int P = I * F_BT + wr * 32 + bi * 16 + (lane >> 4) + 4 * r;
                int Q = J * F_BT + wc * 32 + bj * 16 + (lane & 15);
                Ef[(int64_t)P * npad + Q] = (P == Q ? id : 0.0) - acc[bi][bj][r];
            }
}

// partial[f][I][c] = sum_{P in tile I} B[c][P] (Lambda_f B^T)[P][c], FP64.
__global__ __launch_bounds__(256) void k_w_f64(const double* __restrict__ lam, int npad,
                                               const double* __restrict__ bt, int cpad,
                                               int f0, double* __restrict__ partial) {
    __shared__ F64Stage st[2];
    __shared__ double red[2][F_BT];
    const int ni = npad / F_BT, nc = cpad / F_BT;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int fl = bid / (ni * nc);
    const int rem = bid % (ni * nc);
    const int I = rem % ni, J = rem / ni;
    const double* L = lam + (int64_t)(f0 + fl) * npad * npad;
    v4d acc[2][2] = {};
    f64_tile_product(L + (int64_t)I * F_BT * npad, npad, bt + (int64_t)J * F_BT * npad, npad,
                     nullptr, npad, st, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int c = J * F_BT + wc * 32 + bj * 16 + (lane & 15);
        double s = 0.0;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int P = I * F_BT + wr * 32 + bi * 16 + (lane >> 4) + 4 * r;
                s += bt[(int64_t)c * npad + P] * acc[bi][bj][r];
            }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (lane < 16) red[wr][wc * 32 + bj * 16 + lane] = s;
    }
    __syncthreads();
    if (threadIdx.x < F_BT) {
        int c = J * F_BT + threadIdx.x;
        partial[((int64_t)fl * ni + I) * cpad + c] = red[0][threadIdx.x] + red[1][threadIdx.x];
    }
}


// ============================================================================
// Split 16-bit MFMA tile machinery: 128 x 128 output tile, 4 waves of 64 x 64
// (2 x 2 blocks of 32 x 32 x 16), K chunks of 32 staged in LDS as
// [k-group of 8][row] so that each lane's 16-byte fragment read is contiguous.
// ============================================================================

constexpr int B_BT = 128, B_KC = 32, kFlushChunks = 64;   // flush every 2048 k

struct SplitStage {
    uint4 ah[4][B_BT], al[4][B_BT], bh[4][B_BT], bl[4][B_BT];
};

struct SplitFrag {
    uint4 ah[2], al[2], bh[2], bl[2];
};

__device__ inline uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }

// Rescale the B operand by per-k weights and split again: y = (hi + lo) * c.
template <int ET>
__device__ inline void reweight(uint4& h, uint4& l, const float* c) {
    uint32_t hw[4] = {h.x, h.y, h.z, h.w}, lw[4] = {l.x, l.y, l.z, l.w};
    uint32_t oh[4], ol[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t rh = 0, rl = 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            uint16_t bh = (uint16_t)(hw[q] >> (16 * e)), bl = (uint16_t)(lw[q] >> (16 * e));
            float y = (Elem<ET>::val(bh) + Elem<ET>::val(bl)) * c[2 * q + e];
            uint16_t yh = Elem<ET>::bits(y);
            uint16_t yl = Elem<ET>::bits(y - Elem<ET>::val(yh));
            rh |= (uint32_t)yh << (16 * e);
            rl |= (uint32_t)yl << (16 * e);
        }
        oh[q] = rh;
        ol[q] = rl;
    }
    h = make_uint4(oh[0], oh[1], oh[2], oh[3]);
    l = make_uint4(ol[0], ol[1], ol[2], ol[3]);
}

__device__ inline void split_store_stage(SplitStage& st, const SplitFrag& fr, int row, int kg0) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        st.ah[kg0 + g][row] = fr.ah[g];
        st.al[kg0 + g][row] = fr.al[g];
        st.bh[kg0 + g][row] = fr.bh[g];
        st.bl[kg0 + g][row] = fr.bl[g];
    }
}

template <int ET, bool SPLIT>
__device__ inline void split_chunk(const SplitStage& st, int wr, int wc, int lane, v16f (&acc)[2][2]) {
    typedef typename Elem<ET>::vec V;
    const int r = lane & 31, hg = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int kg = ks * 2 + hg;
        V ahv[2], alv[2], bhv[2], blv[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            ahv[b] = __builtin_bit_cast(V, st.ah[kg][wr * 64 + b * 32 + r]);
            bhv[b] = __builtin_bit_cast(V, st.bh[kg][wc * 64 + b * 32 + r]);
            if (SPLIT) {
                alv[b] = __builtin_bit_cast(V, st.al[kg][wr * 64 + b * 32 + r]);
                blv[b] = __builtin_bit_cast(V, st.bl[kg][wc * 64 + b * 32 + r]);
            }
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                acc[bi][bj] = Elem<ET>::mfma(ahv[bi], bhv[bj], acc[bi][bj]);
                if (SPLIT) {
                    acc[bi][bj] = Elem<ET>::mfma(ahv[bi], blv[bj], acc[bi][bj]);
                    acc[bi][bj] = Elem<ET>::mfma(alv[bi], bhv[bj], acc[bi][bj]);
                }
            }
    }
}

// accd = A[rows] * (B[rows] diag(cw))^T over K (multiple of 32), FP32 products
// flushed into the FP64 accumulators every kFlushChunks chunks.
template <int ET, bool SPLIT, bool WEIGHTED>
__device__ inline void split_tile_product(const uint16_t* __restrict__ ah, const uint16_t* __restrict__ al,
                                          int64_t lda, const uint16_t* __restrict__ bh,
                                          const uint16_t* __restrict__ bl, int64_t ldb,
                                          const float* __restrict__ cw, int64_t K, SplitStage (&st)[2],
                                          double (&accd)[2][2][16]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row = t >> 1, kg0 = (t & 1) * 2;
    const uint16_t* pah = ah + (int64_t)row * lda + kg0 * 8;
    const uint16_t* pal = al + (int64_t)row * lda + kg0 * 8;
    const uint16_t* pbh = bh + (int64_t)row * ldb + kg0 * 8;
    const uint16_t* pbl = bl + (int64_t)row * ldb + kg0 * 8;
    const float* pc = WEIGHTED ? cw + kg0 * 8 : nullptr;
    const int64_t nk = K / B_KC;
    SplitFrag fr;
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            fr.ah[g] = ld16(pah + k0 + 8 * g);
            fr.bh[g] = ld16(pbh + k0 + 8 * g);
            if (SPLIT || WEIGHTED) {
                fr.al[g] = ld16(pal + k0 + 8 * g);
                fr.bl[g] = ld16(pbl + k0 + 8 * g);
            }
        }
        if (WEIGHTED) {
            float c[16];
            const float4* q4 = reinterpret_cast<const float4*>(pc + k0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float4 v = q4[q];
                c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
            }
            reweight<ET>(fr.bh[0], fr.bl[0], c);
            reweight<ET>(fr.bh[1], fr.bl[1], c + 8);
        }
    };
    v16f acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            acc[bi][bj] = v16f{};
#pragma unroll
            for (int v = 0; v < 16; ++v) accd[bi][bj][v] = 0.0;
        }
    auto flush = [&]() {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
                for (int v = 0; v < 16; ++v) accd[bi][bj][v] += (double)acc[bi][bj][v];
                acc[bi][bj] = v16f{};
            }
    };
    load(0);
    split_store_stage(st[0], fr, row, kg0);
    __syncthreads();
    for (int64_t i = 0; i < nk; ++i) {
        const int s = (int)(i & 1);
        if (i + 1 < nk) load((i + 1) * B_KC);
        split_chunk<ET, SPLIT>(st[s], wr, wc, lane, acc);
        if ((i + 1) % kFlushChunks == 0) flush();
        if (i + 1 < nk) split_store_stage(st[s ^ 1], fr, row, kg0);
        __syncthreads();
    }
    flush();
}

// eps_f = delta_f I - Pi_f on the lower 128 x 128 tiles; acc * pi_unscale[f] = Pi_f.
template <int ET, bool SPLIT>
__global__ __launch_bounds__(256) void k_pi_split(const uint16_t* __restrict__ xh,
                                                  const uint16_t* __restrict__ xl, int64_t kpad,
                                                  const float* __restrict__ cw,
                                                  const double* __restrict__ pi_unscale,
                                                  const int* __restrict__ idflag, double* __restrict__ E,
                                                  int npad) {
    __shared__ SplitStage st[2];
    const int nt = npad / B_BT, T = nt * (nt + 1) / 2;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int f = bid / T;
    int I, J;
    lower_tile(bid % T, I, J);
    double accd[2][2][16];
    const int64_t ai = (int64_t)I * B_BT * kpad, bj0 = (int64_t)J * B_BT * kpad;
    split_tile_product<ET, SPLIT, true>(xh + ai, xl + ai, kpad, xh + bj0, xl + bj0, kpad,
                                        cw + (int64_t)f * kpad, kpad, st, accd);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const double id = idflag[f] ? 1.0 : 0.0;
    const double us = pi_unscale[f];
    double* Ef = E + (int64_t)f * npad * npad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                int P = I * B_BT + wr * 64 + bi * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                int Q = J * B_BT + wc * 64 + bj * 32 + (lane & 31);
                Ef[(int64_t)P * npad + Q] = (P == Q ? id : 0.0) - accd[bi][bj][v] * us;
            }
}

// partial[f][I][c] = sum_{P in tile I} B[c][P] (Lambda_f B^T)[P][c]; acc * w_unscale[f] = Lambda B^T.
template <int ET, bool SPLIT>
__global__ __launch_bounds__(256) void k_w_split(const uint16_t* __restrict__ lh,
                                                 const uint16_t* __restrict__ ll, int npad,
                                                 const uint16_t* __restrict__ bh,
                                                 const uint16_t* __restrict__ bl,
                                                 const double* __restrict__ bt64, int cpad, int f0,
                                                 const double* __restrict__ w_unscale,
                                                 double* __restrict__ partial) {
    __shared__ SplitStage st[2];
    __shared__ double red[2][B_BT];
    const int ni = npad / B_BT, nc = cpad / B_BT;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int fl = bid / (ni * nc);
    const int rem = bid % (ni * nc);
    const int I = rem % ni, J = rem / ni;
    const int64_t lo = (int64_t)(f0 + fl) * npad * npad + (int64_t)I * B_BT * npad;
    const int64_t bo = (int64_t)J * B_BT * npad;
    double accd[2][2][16];
    split_tile_product<ET, SPLIT, false>(lh + lo, ll + lo, npad, bh + bo, bl + bo, npad, nullptr, npad, st, accd);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const double us = w_unscale[f0 + fl];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int c = J * B_BT + wc * 64 + bj * 32 + (lane & 31);
        const double* brow = bt64 + (int64_t)c * npad;
        double s = 0.0;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                int P = I * B_BT + wr * 64 + bi * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                s += brow[P] * accd[bi][bj][v];
            }
        s *= us;
        s += __shfl_xor(s, 32);
        if (lane < 32) red[wr][wc * 64 + bj * 32 + lane] = s;
    }
    __syncthreads();
    if (threadIdx.x < B_BT) {
        int c = J * B_BT + threadIdx.x;
        partial[((int64_t)fl * ni + I) * cpad + c] = red[0][threadIdx.x] + red[1][threadIdx.x];
    }
}

// ============================================================================
// Host launchers
// ============================================================================

void launch_pi(hipStream_t s, int prec, int npad, int64_t kpad, int n_f, const double* x64, const uint16_t* xh,
               const uint16_t* xl, const double* cw64, const float* cw32, const double* pi_unscale,
               const int* idflag, double* E) {
    if (prec == PREC_P64) {
        int nt = npad / F_BT, T = nt * (nt + 1) / 2;
        hipLaunchKernelGGL(k_pi_f64, dim3(T * n_f), dim3(256), 0, s, x64, kpad, cw64, idflag, E, npad, n_f);
        return;
    }
    int nt = npad / B_BT, T = nt * (nt + 1) / 2;
    dim3 g(T * n_f), b(256);
    if (prec == PREC_B16X3)
        hipLaunchKernelGGL((k_pi_split<0, true>), g, b, 0, s, xh, xl, kpad, cw32, pi_unscale, idflag, E, npad);
    else if (prec == PREC_B16)
        hipLaunchKernelGGL((k_pi_split<0, false>), g, b, 0, s, xh, xl, kpad, cw32, pi_unscale, idflag, E, npad);
    else
        hipLaunchKernelGGL((k_pi_split<1, true>), g, b, 0, s, xh, xl, kpad, cw32, pi_unscale, idflag, E, npad);
}

int w_partial_blocks(int prec, int npad) { return npad / (prec == PREC_P64 ? F_BT : B_BT); }

void launch_w(hipStream_t s, int prec, int npad, int f0, int nf, const double* lam64, const uint16_t* lh,
              const uint16_t* ll, const double* bt64, const uint16_t* bh, const uint16_t* bl, int cpad,
              const double* w_unscale, double* partial) {
    if (nf <= 0) return;
    if (prec == PREC_P64) {
        int ni = npad / F_BT, nc = cpad / F_BT;
        hipLaunchKernelGGL(k_w_f64, dim3(ni * nc * nf), dim3(256), 0, s, lam64, npad, bt64, cpad, f0, partial);
        return;
    }
    int ni = npad / B_BT, nc = cpad / B_BT;
    dim3 g(ni * nc * nf), b(256);
    if (prec == PREC_B16X3)
        hipLaunchKernelGGL((k_w_split<0, true>), g, b, 0, s, lh, ll, npad, bh, bl, bt64, cpad, f0, w_unscale, partial);
    else if (prec == PREC_B16)
        hipLaunchKernelGGL((k_w_split<0, false>), g, b, 0, s, lh, ll, npad, bh, bl, bt64, cpad, f0, w_unscale, partial);
    else
        hipLaunchKernelGGL((k_w_split<1, true>), g, b, 0, s, lh, ll, npad, bh, bl, bt64, cpad, f0, w_unscale, partial);
}

}  // namespace cdwac
