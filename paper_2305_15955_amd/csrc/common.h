// Internal helpers shared by the gfx950 kernels of the CD-WAC library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdwac {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// Lane layouts of the two matrix-core forms used here (gfx950, wave64):
//  v_mfma_f64_16x16x4f64: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
//    D[i][j] in lane j + 16 (i % 4), element i / 4 (rows interleaved by 4).
//  v_mfma_f32_32x32x16_bf16: A[i][k] in lane i + 32 (k / 8), element k % 8;
//    B[k][j] in lane j + 32 (k / 8), element k % 8; D[i][j] in lane
//    j + 32 ((i / 4) % 2), element 4 (i / 8) + i % 4.
// Tile edge used for every padded dimension (auxiliary index, columns).
constexpr int kPad = 128;
// Block size of the blocked symmetric sweep (Gauss-Jordan) inversion.
constexpr int kNb = 64;
// Largest number of Pade reference points (a fit wave holds 4 per lane).
constexpr int kMaxPade = 256;

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---- panel layout of a 16-bit contraction operand ---------------------------
// Rows are padded to a multiple of 64 and K to a multiple of 32.  Each block
// of 64 rows is stored contiguously as [K / 8][64 rows][8], so the eight
// elements k .. k+7 (k % 8 == 0) of one row form one 16-byte word and the 64
// rows of a block at one k-group are 1 KiB of consecutive memory: one
// wave-wide 16-byte load fetches whole cache lines and lands in LDS as
// [k-group][row], the order the matrix-core fragments are read in.  Row block
// b starts at element b * 64 * K, as it would in row-major order.
__host__ __device__ inline int64_t panel_off(int64_t p, int64_t k, int64_t K) {
    return (((p >> 6) * (K >> 3) + (k >> 3)) * 64 + (p & 63)) * 8 + (k & 7);
}

// ---- bf16 split: x ~= hi + lo with hi = rn(x), lo = rn(x - hi) ------------
__device__ inline uint16_t bf16_bits(float x) {
    __bf16 h = (__bf16)x;                 // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Element types of the split operands: 0 = bf16 (8-bit significand),
// 1 = fp16 (11-bit significand; callers scale the values into its range).
template <int ET>
struct Elem;
template <>
struct Elem<0> {
    typedef v8bf vec;
    __device__ static uint16_t bits(float x) { return bf16_bits(x); }
    __device__ static float val(uint16_t b) { return bf16_float(b); }
    __device__ static v16f mfma(vec a, vec b, v16f c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Elem<1> {
    typedef v8h vec;
    __device__ static uint16_t bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
    __device__ static float val(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
    __device__ static v16f mfma(vec a, vec b, v16f c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// ---- complex double ---------------------------------------------------------
struct cplx {
    double re, im;
};
__host__ __device__ inline cplx cmk(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
// Division with Smith's scaling (avoids overflow in |b|^2).
__host__ __device__ inline cplx operator/(cplx a, cplx b) {
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        double r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
__host__ __device__ inline bool cfinite(cplx a) { return isfinite(a.re) && isfinite(a.im); }

// ---- XCD-aware tile order ---------------------------------------------------
// Workgroups are handed to the 8 XCDs round robin.  Remapping the linear
// block id so that XCD x receives a contiguous run of tiles keeps the tiles
// that share operand panels on the same L2.
__device__ inline int xcd_remap(int bid, int nblocks) {
    constexpr int kXcd = 8;
    int per = nblocks / kXcd;
    int full = per * kXcd;
    if (bid >= full) return bid;
    return (bid % kXcd) * per + bid / kXcd;
}

// Tile t of the lower triangle of an n x n grid of blocks (J <= I), in the
// order of the sweep's rank-k updates: bands of 4 block rows from the top,
// each cut into pieces of 8 block columns, a piece's tiles row by row.  Every
// 32 consecutive tiles (an XCD runs consecutive tiles together) then read 4
// row panels and 8 column panels instead of one row panel and 32 column
// panels, so that a band's column panels come from HBM about once per band
// instead of once per block row.
__host__ __device__ inline void sweep_tile_order(int t, int n, int& I, int& J) {
    // band b holds block rows 4b .. 4b + 3, starting at tile 4b (4b + 1) / 2
    int b = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.125);   // 2b (4b + 1) <= t, up to rounding
    while (b > 0 && 2 * b * (4 * b + 1) > t) --b;
    while (2 * (b + 1) * (4 * (b + 1) + 1) <= t && 4 * (b + 1) < n) ++b;
    int local = t - 2 * b * (4 * b + 1);
    const int r1 = n - 4 * b < 4 ? n - 4 * b : 4;   // rows in the band
    I = J = 0;   // not reached for 0 <= t < n (n + 1) / 2
    for (int c = 0; 8 * c < n; ++c)
        for (int r = 0; r < r1; ++r) {
            const int row = 4 * b + r, cnt = row + 1 - 8 * c;
            const int k = cnt < 0 ? 0 : (cnt > 8 ? 8 : cnt);
            if (local < k) {
                I = row;
                J = 8 * c + local;
                return;
            }
            local -= k;
        }
}

}  // namespace cdwac
