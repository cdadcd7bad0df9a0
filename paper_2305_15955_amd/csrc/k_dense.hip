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
// products hi*hi + hi*lo + lo*hi accumulated in FP32.
#include "common.h"
#include "kernels.h"

#include <algorithm>
#include <vector>

namespace cdwac {

// ============================================================================
// FP64 MFMA tile machinery: 128 x 128 output tile, 4 waves of 64 x 64 (4 x 4
// blocks of v_mfma_f64_16x16x4), K chunks of 16 staged in LDS as [k][row],
// double-buffered.  Per chunk a workgroup stages 32 KiB for 1024 matrix-core
// blocks (a 64 x 64 tile needs twice the bytes per flop, and ran 1.27x slower
// on the polarizability); two workgroups per CU.
// ============================================================================

constexpr int F_BT = 128, F_KC = 16, F_LD = F_BT + 2;

struct F64Stage {
    double a[F_KC][F_LD];
    double b[F_KC][F_LD];
};

__device__ inline void f64_chunk(const F64Stage& st, int wr, int wc, int lane, v4d (&acc)[4][4]) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < F_KC / 4; ++kk) {
        const int k = kk * 4 + lk;
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = st.a[k][wr * 64 + i * 16 + lr];
            b[i] = st.b[k][wc * 64 + i * 16 + lr];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// Thread t loads row t/2, k = (t%2)*8 .. +7 of a 128 x 16 chunk of A and of B
// (B scaled by cw when given).
struct F64Frag {
    double a[8], b[8];
};

__device__ inline void f64_load(F64Frag& fr, const double* __restrict__ arow, const double* __restrict__ brow,
                                 const double* __restrict__ cw, int64_t k0) {
    const double2* pa = reinterpret_cast<const double2*>(arow + k0);
    const double2* pb = reinterpret_cast<const double2*>(brow + k0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double2 x = pa[e], y = pb[e];
        fr.a[2 * e] = x.x;
        fr.a[2 * e + 1] = x.y;
        fr.b[2 * e] = y.x;
        fr.b[2 * e + 1] = y.y;
    }
    if (cw) {
        const double2* pc = reinterpret_cast<const double2*>(cw + k0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double2 c = pc[e];
            fr.b[2 * e] *= c.x;
            fr.b[2 * e + 1] *= c.y;
        }
    }
}

__device__ inline void f64_store(F64Stage& st, const F64Frag& fr, int row, int kq) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        st.a[kq + e][row] = fr.a[e];
        st.b[kq + e][row] = fr.b[e];
    }
}

// acc = A[128 rows] * (B[128 rows] * diag(cw))^T over the first K columns (a
// multiple of 16); the partial sum over the first 16 n_dbl columns is doubled
// before the rest is added (n_dbl < 0: never).
__device__ inline void f64_tile_product(const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                         int64_t ldb, const double* __restrict__ cw, int64_t K, int64_t n_dbl,
                                         F64Stage (&st)[2], v4d (&acc)[4][4]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row = t >> 1, kq = (t & 1) * 8;
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
        if (i == n_dbl)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] *= 2.0;
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

// eps_f = delta_f I - X diag(c_f) X^T on the lower 128 x 128 tiles, FP64
// (npad a multiple of 128, kpad of 16).
__global__ __launch_bounds__(256, 2) void k_pi_f64(const double* __restrict__ x, int64_t kpad,
                                                const double* __restrict__ cw,
                                                const int* __restrict__ idflag,
                                                double* __restrict__ E, int npad, int n_f) {
    __shared__ F64Stage st[2];
    const int nt = npad / F_BT, T = nt * (nt + 1) / 2;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int f = bid / T;
    int I, J;
    lower_tile(bid % T, I, J);
    v4d acc[4][4] = {};
    f64_tile_product(x + (int64_t)I * F_BT * kpad, kpad, x + (int64_t)J * F_BT * kpad, kpad,
                      cw + (int64_t)f * kpad, kpad, -1, st, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const double id = idflag[f] ? 1.0 : 0.0;
    double* Ef = E + (int64_t)f * npad * npad;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int P = I * F_BT + wr * 64 + bi * 16 + (lane >> 4) + 4 * r;
                int Q = J * F_BT + wc * 64 + bj * 16 + (lane & 15);
                Ef[(int64_t)P * npad + Q] = (P == Q ? id : 0.0) - acc[bi][bj][r];
            }
}

// partial[f][I][c] = sum_{P in tile I} B[c][P] (Lambda'_f B^T)[P][c], FP64,
// 128 x 128 tiles (npad and cpad multiples of 128), where Lambda' keeps the
// 128-row blocks of Lambda left of and on its diagonal only, the ones left of
// it doubled: Lambda is symmetric, so the partials of all row blocks still sum
// to the full quadratic form B[c] Lambda B[c]^T (Eq. wriv) at about half the
// products.  Row blocks go from the last (the longest contraction) down.
__global__ __launch_bounds__(256, 2) void k_w_f64(const double* __restrict__ lam, int npad,
                                                  const double* __restrict__ bt, int cpad,
                                                  int f0, double* __restrict__ partial) {
    __shared__ F64Stage st[2];
    __shared__ double red[2][F_BT];
    const int ni = npad / F_BT, nc = cpad / F_BT;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int fl = bid / (ni * nc);
    const int rem = bid % (ni * nc);
    const int I = ni - 1 - rem % ni, J = rem / ni;
    const double* L = lam + (int64_t)(f0 + fl) * npad * npad;
    v4d acc[4][4] = {};
    f64_tile_product(L + (int64_t)I * F_BT * npad, npad, bt + (int64_t)J * F_BT * npad, npad,
                      nullptr, (int64_t)(I + 1) * F_BT, (int64_t)I * (F_BT / F_KC), st, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
        const int c = J * F_BT + wc * 64 + bj * 16 + (lane & 15);
        double s = 0.0;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int P = I * F_BT + wr * 64 + bi * 16 + (lane >> 4) + 4 * r;
                s += bt[(int64_t)c * npad + P] * acc[bi][bj][r];
            }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (lane < 16) red[wr][wc * 64 + bj * 16 + lane] = s;
    }
    __syncthreads();
    if (threadIdx.x < F_BT) {
        int c = J * F_BT + threadIdx.x;
        partial[((int64_t)fl * ni + I) * cpad + c] = red[0][threadIdx.x] + red[1][threadIdx.x];
    }
}


// ============================================================================
// 16-bit split MFMA contraction (v_mfma_f32_32x32x16_{bf16,f16}).
//
// One workgroup of 8 waves computes a 256 x 256 tile of A B^T with both
// operands stored as hi/lo planes in the panel layout of panel_off (K is the
// leading dimension lda = ldb), so each wave-wide load of one 64-row block at
// one k-group reads 1 KiB of consecutive memory and lands in LDS through the
// direct global-to-LDS path.  The waves form a 4 x 2 grid; each owns a 64 x 128
// sub-tile (2 x 4 matrix-core blocks, 128 FP32 accumulators per lane).  K
// advances in chunks of 32 through an LDS ring of 128 KiB: 2 stages of 64 KiB
// with the hi/lo split (chunk i+1 in flight while chunk i is multiplied), 4
// stages of 32 KiB without it (three chunks in flight, since a chunk then
// carries a third of the matrix-core work per byte).  LDS layout per stage:
// [operand][plane][k-group of 8][row] x 16 bytes, so every fragment read is one
// contiguous 16-byte word per lane and a half-wave reads 512 consecutive
// bytes (no bank conflicts).  Products hi*hi + hi*lo + lo*hi accumulate in
// FP32 in the matrix cores over the whole contraction and are converted to
// FP64 at the end.  The polarizability's tiles come from a host-built work
// list (pi_worklist) in which the workgroups an XCD runs together share
// operand panels in its L2; the W contraction's from 4 x 8 blocks.
// ============================================================================

constexpr int GT = 256;
constexpr int kGemmThreads = 512;
// K chunk GKX (a multiple of 16), k-groups of 8 per chunk, uint4 slots of the
// LDS ring (SLOTSX: 8192 = 128 KiB), of one operand per stage, of a stage, and
// the ring depth
template <bool SPLIT, int GKX = 32, int SLOTSX = 8192>
struct Ring {
    static constexpr int GK = GKX;
    static constexpr int KG = GKX / 8;
    static constexpr int PL = SPLIT ? 2 : 1;
    static constexpr int SLOTS = SLOTSX;
    static constexpr int OP = PL * KG * GT;
    static constexpr int STAGE = 2 * OP;
    static constexpr int NST = SLOTS / STAGE;
    // 64-row-block loads per chunk and wave: 2 operands x PL planes x KG
    // k-groups x 4 row blocks over 8 waves
    static constexpr int LPW = 2 * PL * KG * 4 / 8;
};

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt immediates (gfx9 encoding): vmcnt(n) and lgkmcnt(0), expcnt open.
constexpr int wait_vm_lgkm0(int n) { return ((n >> 4) << 14) | (7 << 4) | (n & 15); }

// Workgroup barrier without the memory fence of __syncthreads(), whose
// release semantics would also wait for the global-to-LDS loads still in
// flight for the next chunk.  Callers wait for what must be complete first.
__device__ inline void stage_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Issues this wave's share of the row-block loads of chunk k0 into stage st.
template <bool SPLIT, class RG>
__device__ inline void gemm_issue(uint4* lds, int st, const uint16_t* __restrict__ ah, const uint16_t* __restrict__ al,
                                  const uint16_t* __restrict__ bh, const uint16_t* __restrict__ bl, int64_t K,
                                  int64_t k0, int w, int lane) {
    constexpr int per = RG::LPW, per_op = RG::PL * RG::KG * 4;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const int u = w * per + q;
        const int op = u / per_op;                    // operand A or B
        const int v = u % per_op;
        const int pl = v / (RG::KG * 4), kg = (v >> 2) % RG::KG, rb = v & 3;
        const uint16_t* base = op ? (pl ? bl : bh) : (pl ? al : ah);
        const uint16_t* g = base + (int64_t)rb * 64 * K + (k0 + kg * 8) * 64 + lane * 8;
        const int slot = op * RG::OP + (pl * RG::KG + kg) * GT + rb * 64;
        __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(lds + st * RG::STAGE + slot), 16, 0, 0);
    }
}

template <int ET, bool SPLIT, class RG>
__device__ inline void gemm_chunk(const uint4* lds, int st, int r0, int c0, int lane, v16f (&acc)[2][4]) {
    typedef typename Elem<ET>::vec V;
    const uint4* sa = lds + st * RG::STAGE;
    const uint4* sb = sa + RG::OP;
    const int r = lane & 31, hg = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < RG::GK / 16; ++ks) {
        const int kg = ks * 2 + hg;
        V ahv[2], alv[2], bhv[4], blv[4];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            ahv[b] = __builtin_bit_cast(V, sa[kg * GT + r0 + b * 32 + r]);
            if (SPLIT) alv[b] = __builtin_bit_cast(V, sa[(RG::KG + kg) * GT + r0 + b * 32 + r]);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            bhv[b] = __builtin_bit_cast(V, sb[kg * GT + c0 + b * 32 + r]);
            if (SPLIT) blv[b] = __builtin_bit_cast(V, sb[(RG::KG + kg) * GT + c0 + b * 32 + r]);
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                acc[bi][bj] = Elem<ET>::mfma(ahv[bi], bhv[bj], acc[bi][bj]);
                if (SPLIT) {
                    acc[bi][bj] = Elem<ET>::mfma(ahv[bi], blv[bj], acc[bi][bj]);
                    acc[bi][bj] = Elem<ET>::mfma(alv[bi], bhv[bj], acc[bi][bj]);
                }
            }
    }
}

// acc = A[rows 0..256) * B[rows 0..256)^T over the first nk chunks of RG::GK
// columns of K (the panels' K extent, a multiple of RG::GK); A and B point at
// the first row block of the tile.  The partial sum over the first n_dbl chunks
// is doubled before the rest is added (n_dbl < 0: never).  Wave w owns rows
// 64 (w / 2) .. +64 and columns 128 (w % 2) .. +128.
template <int ET, bool SPLIT, class RG>
__device__ inline void gemm_tile(uint4* lds, const uint16_t* __restrict__ ah, const uint16_t* __restrict__ al,
                                 const uint16_t* __restrict__ bh, const uint16_t* __restrict__ bl, int64_t K,
                                 int64_t nk, int64_t n_dbl, v16f (&acc)[2][4]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r0 = (w >> 1) * 64, c0 = (w & 1) * 128;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = v16f{};
    constexpr int NST = RG::NST;
    constexpr int ahead = (NST - 2) * RG::LPW;   // loads of later chunks left in flight
    static_assert(ahead < 64, "vmcnt holds at most 63 outstanding loads");
#pragma unroll
    for (int j = 0; j < NST - 1; ++j)
        if (j < nk) gemm_issue<SPLIT, RG>(lds, j, ah, al, bh, bl, K, j * RG::GK, w, lane);
    for (int64_t i = 0; i < nk; ++i) {
        // chunk i has landed (own loads) and every wave is done with chunk i-1
        if (i + NST - 2 < nk) __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(ahead));
        else __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
        stage_barrier();
        if (i + NST - 1 < nk)
            gemm_issue<SPLIT, RG>(lds, (int)((i + NST - 1) % NST), ah, al, bh, bl, K, (i + NST - 1) * RG::GK, w,
                                  lane);
        if (i == n_dbl)
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] *= 2.0f;
        gemm_chunk<ET, SPLIT, RG>(lds, (int)(i % NST), r0, c0, lane, acc);
    }
}

// Row and column inside the tile of the output element held by (lane, v) of
// block (bi, bj) of wave w.
__device__ inline int out_row(int w, int bi, int lane, int v) {
    return (w >> 1) * 64 + bi * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}
__device__ inline int out_col(int w, int bj, int lane) { return (w & 1) * 128 + bj * 32 + (lane & 31); }

// eps_f = delta_f I - Pi_f for the tiles of a work list (pi_worklist): entry
// {fb << 16 | I, J} is tile (I, J) of plane f = fmap[fb] (B = prescaled Y_f,
// batch slot fb); {-1, -1} is an empty slot.
// Ring of the polarizability contraction: 32-wide K chunks in 2 stages of
// 64 KiB with the split, 4 stages of 32 KiB without it.
template <bool SPLIT>
using PiRing = Ring<SPLIT, 32, 8192>;

template <int ET, bool SPLIT>
__global__ __launch_bounds__(kGemmThreads) void k_pi_gemm(const uint16_t* __restrict__ xh,
                                                          const uint16_t* __restrict__ xl,
                                                          const uint16_t* __restrict__ yh,
                                                          const uint16_t* __restrict__ yl, int64_t kpad,
                                                          const int2* __restrict__ work,
                                                          const int* __restrict__ fmap,
                                                          const double* __restrict__ pi_unscale,
                                                          const int* __restrict__ idflag, double* __restrict__ E,
                                                          int npad) {
    __shared__ uint4 lds[PiRing<SPLIT>::SLOTS];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int2 e = work[bid];
    if (e.x < 0) return;
    const int fb = e.x >> 16, I = e.x & 0xffff, J = e.y, f = fmap[fb];
    const int64_t ao = (int64_t)I * GT * kpad;
    const int64_t bo = (int64_t)fb * npad * kpad + (int64_t)J * GT * kpad;
    v16f acc[2][4];
    gemm_tile<ET, SPLIT, PiRing<SPLIT>>(lds, xh + ao, xl + ao, yh + bo, yl + bo, kpad, kpad / PiRing<SPLIT>::GK, -1,
                                        acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double id = idflag[f] ? 1.0 : 0.0;
    const double us = pi_unscale[f];
    double* Ef = E + (int64_t)f * npad * npad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int P = I * GT + out_row(w, bi, lane, v);
                const int Q = J * GT + out_col(w, bj, lane);
                Ef[(int64_t)P * npad + Q] = (P == Q ? id : 0.0) - (double)acc[bi][bj][v] * us;
            }
}

// Ring of the W contraction (same as the polarizability's).
template <bool SPLIT>
using WRing = Ring<SPLIT, 32, 8192>;

// partial[fl][I][c] = sum_{P in row block I} B[c][P] (Lambda'_f B^T)[P][c],
// where Lambda' keeps the 256-row blocks of Lambda left of and on its diagonal
// only, the ones left of it doubled (as in k_w_f64): the partials of all row
// blocks sum to B[c] Lambda_f B[c]^T (Eq. wriv) at about half the products.
template <int ET, bool SPLIT>
__global__ __launch_bounds__(kGemmThreads) void k_w_gemm(const uint16_t* __restrict__ lh,
                                                         const uint16_t* __restrict__ ll, int npad,
                                                         const uint16_t* __restrict__ bh,
                                                         const uint16_t* __restrict__ bl,
                                                         const double* __restrict__ bt64, int cpad,
                                                         const int2* __restrict__ tiles, int n_tiles, int f0,
                                                         const double* __restrict__ w_unscale,
                                                         double* __restrict__ partial) {
    __shared__ uint4 lds[WRing<SPLIT>::SLOTS];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int fl = bid / n_tiles;
    const int2 tile = tiles[bid % n_tiles];
    const int I = tile.x, J = tile.y;
    const int ni = npad / GT;
    const int64_t lo = (int64_t)(f0 + fl) * npad * npad + (int64_t)I * GT * npad;
    const int64_t bo = (int64_t)J * GT * npad;
    v16f acc[2][4];
    gemm_tile<ET, SPLIT, WRing<SPLIT>>(lds, lh + lo, ll + lo, bh + bo, bl + bo, npad,
                                       (int64_t)(I + 1) * (GT / WRing<SPLIT>::GK), (int64_t)I * (GT / WRing<SPLIT>::GK),
                                       acc);
    // the column sums reuse the ring once every wave is done reading it
    __syncthreads();
    double (*red)[GT] = reinterpret_cast<double (*)[GT]>(lds);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double us = w_unscale[f0 + fl];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
        const int c = J * GT + out_col(w, bj, lane);
        const double* brow = bt64 + (int64_t)c * npad + I * GT;
        double s = 0.0;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 16; ++v) s += brow[out_row(w, bi, lane, v)] * (double)acc[bi][bj][v];
        s *= us;
        s += __shfl_xor(s, 32);
        if (lane < 32) red[w >> 1][out_col(w, bj, lane)] = s;
    }
    __syncthreads();
    if (threadIdx.x < GT) {
        const int c = J * GT + threadIdx.x;
        partial[((int64_t)fl * ni + I) * cpad + c] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    }
}

// ============================================================================
// Host side: tile lists and launchers
// ============================================================================

// Number of 256 x 256 tiles (I, J), J <= I, covering the lower triangle of an
// npad x npad matrix.
int pi_tile_count(int npad) {
    const int n = npad / GT;
    return n * (n + 1) / 2;
}

// Planes per polarizability launch for n_planes planes, at most nb per batch
// (the Y buffers), n_tiles tiles per plane on n_cu CUs.  Batches are of
// near-equal size.  Every tile keeps one CU busy for the same time, so a launch
// takes ceil(tiles / CUs) waves of workgroups; the split with the fewest waves
// in total wins (a last wave that is mostly empty costs as much as a full
// one), then the one with the fewest launches.
int pi_batch_size(int n_planes, int nb, int n_tiles, int n_cu) {
    if (n_planes <= 0) return 1;
    nb = std::max(nb, 1);
    n_cu = std::max(n_cu, 1);
    const int min_batches = (n_planes + nb - 1) / nb;
    auto waves = [&](int per) {
        int64_t w = 0;
        for (int f0 = 0; f0 < n_planes; f0 += per)
            w += ((int64_t)std::min(per, n_planes - f0) * n_tiles + n_cu - 1) / n_cu;
        return w;
    };
    int best_per = (n_planes + min_batches - 1) / min_batches;
    int64_t best = waves(best_per);
    for (int nbat = min_batches + 1; nbat <= std::min(n_planes, min_batches + 4); ++nbat) {
        const int per = (n_planes + nbat - 1) / nbat;
        const int64_t w = waves(per);
        if (w < best) {
            best = w;
            best_per = per;
        }
    }
    return best_per;
}

// Work list of the polarizability contraction over nfb planes, for a device
// whose workgroups go round robin to kXcd XCDs of cu_per_xcd CUs each (one
// 256 x 256 tile per CU at a time, so an XCD runs its tiles in rounds of
// cu_per_xcd).  A round's tiles share operand panels in that XCD's L2:
// * the lower triangle is cut into 4-row bands, each into 4 x 4 pieces left
//   of its diagonal block and the diagonal triangle;
// * the list runs piece by piece, each piece over all planes, so that a round
//   holds the same piece of consecutive planes: one set of X row panels (the
//   same for every plane) and the Y_f panels of a few planes;
// * each XCD takes a contiguous run of whole rounds (entries are dealt so that
//   XCD x runs entries x q .. x q + q - 1 in order), padded with empty slots
//   {-1, -1} at the end of its run only, so that no round straddles a piece
//   boundary by a shift.
// Entries {fb << 16 | I, J}; length kXcd * q.
std::vector<int2> pi_worklist(int npad, int nfb, int cu_per_xcd) {
    constexpr int kXcd = 8;
    const int n = npad / GT;
    std::vector<int2> tiles;
    tiles.reserve((size_t)nfb * pi_tile_count(npad));
    for (int I0 = 0; I0 < n; I0 += 4) {
        const int I1 = std::min(n, I0 + 4);
        for (int c0 = 0; c0 <= I0; c0 += 4)            // c0 == I0: the diagonal triangle
            for (int fb = 0; fb < nfb; ++fb)
                for (int I = I0; I < I1; ++I) {
                    const int J1 = c0 == I0 ? I + 1 : c0 + 4;
                    for (int J = c0; J < J1; ++J) tiles.push_back(make_int2((fb << 16) | I, J));
                }
    }
    const int64_t total = (int64_t)tiles.size(), per_round = std::max(cu_per_xcd, 1);
    const int64_t q = per_round * ((total + kXcd * per_round - 1) / (kXcd * per_round));
    std::vector<int2> out((size_t)(kXcd * q), make_int2(-1, -1));
    for (int x = 0; x < kXcd; ++x)
        for (int64_t i = 0; i < q && x * q + i < total; ++i) out[(size_t)(x * q + i)] = tiles[(size_t)(x * q + i)];
    return out;
}

// Full ni x nc grid of W tiles in 4 x 8 blocks, from the last row block (the
// longest contraction, I + 1 chunks of 256) down, so that a launch ends on the
// short ones.
std::vector<int2> w_tiles(int npad, int cpad) {
    std::vector<int2> out;
    const int nI = npad / GT, nJ = cpad / GT;
    for (int I1 = nI; I1 > 0; I1 -= 4)
        for (int J0 = 0; J0 < nJ; J0 += 8)
            for (int I = I1 - 1; I >= std::max(0, I1 - 4); --I)
                for (int J = J0; J < std::min(nJ, J0 + 8); ++J) out.push_back(make_int2(I, J));
    return out;
}

void launch_pi_f64(hipStream_t s, int npad, int64_t kpad, int n_f, const double* x64, const double* cw64,
                   const int* idflag, double* E) {
    int nt = npad / F_BT, T = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_pi_f64, dim3(T * n_f), dim3(256), 0, s, x64, kpad, cw64, idflag, E, npad, n_f);
}

void launch_pi_gemm(hipStream_t s, int prec, int npad, int64_t kpad, const int* fmap, const uint16_t* xh,
                    const uint16_t* xl, const uint16_t* yh, const uint16_t* yl, const int2* work, int n_work,
                    const double* pi_unscale, const int* idflag, double* E) {
    dim3 g(n_work), b(kGemmThreads);
    if (prec == PREC_B16X3)
        hipLaunchKernelGGL((k_pi_gemm<0, true>), g, b, 0, s, xh, xl, yh, yl, kpad, work, fmap, pi_unscale,
                           idflag, E, npad);
    else if (prec == PREC_B16)
        hipLaunchKernelGGL((k_pi_gemm<0, false>), g, b, 0, s, xh, xl, yh, yl, kpad, work, fmap, pi_unscale,
                           idflag, E, npad);
    else if (prec == PREC_F16)
        hipLaunchKernelGGL((k_pi_gemm<1, false>), g, b, 0, s, xh, xl, yh, yl, kpad, work, fmap, pi_unscale,
                           idflag, E, npad);
    else
        hipLaunchKernelGGL((k_pi_gemm<1, true>), g, b, 0, s, xh, xl, yh, yl, kpad, work, fmap, pi_unscale,
                           idflag, E, npad);
}

int w_partial_blocks(int prec, int npad) { return npad / (prec == PREC_P64 ? F_BT : GT); }

void launch_w(hipStream_t s, int prec, int npad, int f0, int nf, const double* lam64, const uint16_t* lh,
              const uint16_t* ll, const double* bt64, const uint16_t* bh, const uint16_t* bl, int cpad,
              const int2* tiles, int n_tiles, const double* w_unscale, double* partial) {
    if (nf <= 0) return;
    if (prec == PREC_P64) {
        int ni = npad / F_BT, nc = cpad / F_BT;
        hipLaunchKernelGGL(k_w_f64, dim3(ni * nc * nf), dim3(256), 0, s, lam64, npad, bt64, cpad, f0, partial);
        return;
    }
    dim3 g(n_tiles * nf), b(kGemmThreads);
    if (prec == PREC_B16X3)
        hipLaunchKernelGGL((k_w_gemm<0, true>), g, b, 0, s, lh, ll, npad, bh, bl, bt64, cpad, tiles, n_tiles, f0,
                           w_unscale, partial);
    else if (prec == PREC_B16)
        hipLaunchKernelGGL((k_w_gemm<0, false>), g, b, 0, s, lh, ll, npad, bh, bl, bt64, cpad, tiles, n_tiles, f0,
                           w_unscale, partial);
    else
        hipLaunchKernelGGL((k_w_gemm<1, true>), g, b, 0, s, lh, ll, npad, bh, bl, bt64, cpad, tiles, n_tiles, f0,
                           w_unscale, partial);
}

}  // namespace cdwac
