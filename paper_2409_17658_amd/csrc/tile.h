// tile.h -- the (min,+) tile routine shared by the single-product kernel and
// the persistent batched kernel.
//
// One workgroup computes a BM x BN block of C = A (x) B (Section 3:
// c_ij = min_k a_ik + b_kj).  K is walked in BK-deep slices that are copied
// from HBM into a double-buffered LDS stage with 16-byte loads; each lane
// then owns a TM x TN register tile of packed uint16 pairs and, for every k,
// issues one v_pk_add_u16 (clamp) and one v_pk_min_u16 per pair of outputs.
// The A operand needs no broadcast instruction: its two k values per VGPR
// are selected with the VOP3P op_sel / op_sel_hi modifiers, which the
// compiler folds from the .xx / .yy swizzles below.
//
// Infinity is 0xFFFF.  With finite inputs <= 0x7FFF the saturating add is
// exact for finite pairs and returns 0xFFFF whenever an operand is
// infinite, so no branch is needed anywhere in the inner loop; out-of-range
// rows, columns and k are loaded as infinity and drop out of the minimum.
#pragma once

#include "common.h"

namespace mpr {

template <int BM_, int BN_, int BK_, int TM_, int TN_>
struct TileCfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, TM = TM_, TN = TN_;
    static constexpr int TX = BN / TN;  // lanes along columns
    static constexpr int TY = BM / TM;  // lanes along rows
    static constexpr int NT = TX * TY;  // threads per workgroup
    static_assert(TN % 8 == 0 && BK % 8 == 0, "16-byte fragments");
    static_assert(NT % 64 == 0, "whole wavefronts");
    // Padded LDS row strides (elements).  A rows are BK + 8 long (a 16-byte
    // pad), so eight consecutive rows start in eight different 16-byte bank
    // groups; B rows get the same pad.
    static constexpr int LDA_S = BK + 8;
    static constexpr int LDB_S = BN + 8;
    static constexpr int A_STAGE = BM * LDA_S;
    static constexpr int B_STAGE = BK * LDB_S;
    static constexpr int LDS_ELEMS = 2 * (A_STAGE + B_STAGE);
    static constexpr int A_CH = BM * (BK / 8);  // 16-byte chunks per A slice
    static constexpr int B_CH = BK * (BN / 8);
    static constexpr int A_CPT = (A_CH + NT - 1) / NT;  // chunks per thread
    static constexpr int B_CPT = (B_CH + NT - 1) / NT;
    static constexpr int NACC = TN / 2;  // packed accumulators per row
};

// 8 consecutive uint16 starting at (row, col) of a row-major matrix, with
// infinity for everything outside rows x cols.  `vec` promises a 16-byte
// aligned base and a leading dimension that is a multiple of 8.
__device__ __forceinline__ uint4 load8(const u16 *__restrict__ base, int64_t ld, int64_t row, int64_t col,
                                       int64_t rows, int64_t cols, bool vec)
{
    const gu16 *g = glob(base);
    if (vec && row < rows && col + 8 <= cols) return gload16(g + row * ld + col);
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t c0 = col + 2 * q;
        const uint32_t lo = (row < rows && c0 < cols) ? g[row * ld + c0] : 0xFFFFu;
        const uint32_t hi = (row < rows && c0 + 1 < cols) ? g[row * ld + c0 + 1] : 0xFFFFu;
        w[q] = lo | (hi << 16);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <class T>
struct TileAcc {
    u16x2 v[T::TM][T::NACC];
};

// The k loop of one BM x BN block.  `aload(k0, row, kc)` returns the 8
// A-operand values of block row `row` at k = k0 + kc .. k0 + kc + 7 and
// `bload(k0, kr, jc)` the 8 B-operand values of k = k0 + kr at block columns
// jc .. jc + 7 (infinity outside the problem); nk is the number of BK-deep
// slices.  The plain product reads both operands directly; the compressed-K
// chain step gathers A's columns through an index list.
template <class T, class ALoad, class BLoad>
__device__ __forceinline__ void tile_mainloop_with(int64_t nk, ALoad aload, BLoad bload, u16 *lds, TileAcc<T> &acc)
{
    const int tid = threadIdx.x;
    const int tx = tid % T::TX, ty = tid / T::TX;
    // Stage s holds A at lds + s*STAGE and B at lds + s*STAGE + A_STAGE.
    constexpr int STAGE = T::A_STAGE + T::B_STAGE;

#pragma unroll
    for (int r = 0; r < T::TM; r++)
#pragma unroll
        for (int c = 0; c < T::NACC; c++) acc.v[r][c] = (u16x2){0xFFFF, 0xFFFF};

    if (nk == 0) return;

    uint4 ra[T::A_CPT], rb[T::B_CPT];
    auto gload = [&](int64_t kt) {
        const int64_t k0 = kt * T::BK;
#pragma unroll
        for (int q = 0; q < T::A_CPT; q++) {
            const int c = tid + q * T::NT;
            if (T::A_CH % T::NT == 0 || c < T::A_CH) ra[q] = aload(k0, c / (T::BK / 8), (c % (T::BK / 8)) * 8);
        }
#pragma unroll
        for (int q = 0; q < T::B_CPT; q++) {
            const int c = tid + q * T::NT;
            if (T::B_CH % T::NT == 0 || c < T::B_CH) rb[q] = bload(k0, c / (T::BN / 8), (c % (T::BN / 8)) * 8);
        }
    };
    auto sstore = [&](int stage) {
#pragma unroll
        for (int q = 0; q < T::A_CPT; q++) {
            const int c = tid + q * T::NT;
            if (T::A_CH % T::NT == 0 || c < T::A_CH) {
                const int row = c / (T::BK / 8), kc = (c % (T::BK / 8)) * 8;
                *(uint4 *)(lds + stage * STAGE + row * T::LDA_S + kc) = ra[q];
            }
        }
#pragma unroll
        for (int q = 0; q < T::B_CPT; q++) {
            const int c = tid + q * T::NT;
            if (T::B_CH % T::NT == 0 || c < T::B_CH) {
                const int kr = c / (T::BN / 8), jc = (c % (T::BN / 8)) * 8;
                *(uint4 *)(lds + stage * STAGE + T::A_STAGE + kr * T::LDB_S + jc) = rb[q];
            }
        }
    };
    gload(0);
    sstore(0);
    __syncthreads();

    for (int64_t kt = 0; kt < nk; kt++) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload(kt + 1);  // next slice in flight during the math
        const u16 *as = lds + cur * STAGE;
        const u16 *bs = as + T::A_STAGE;
#pragma unroll 1
        for (int kk = 0; kk < T::BK; kk += 8) {
            uint4 af[T::TM];
#pragma unroll
            for (int r = 0; r < T::TM; r++) af[r] = *(const uint4 *)(as + (ty + r * T::TY) * T::LDA_S + kk);
            // B fragments of row kk + kq; the next row's are read while this
            // one is consumed.
            uint4 bf[T::TN / 8], bn[T::TN / 8];
#pragma unroll
            for (int c8 = 0; c8 < T::TN / 8; c8++)
                bf[c8] = *(const uint4 *)(bs + kk * T::LDB_S + c8 * (T::TX * 8) + tx * 8);
#pragma unroll
            for (int kq = 0; kq < 8; kq++) {
                if (kq < 7) {
#pragma unroll
                    for (int c8 = 0; c8 < T::TN / 8; c8++)
                        bn[c8] = *(const uint4 *)(bs + (kk + kq + 1) * T::LDB_S + c8 * (T::TX * 8) + tx * 8);
                }
#pragma unroll
                for (int r = 0; r < T::TM; r++) {
                    const u16x2 ap = as_u16x2(comp(af[r], kq >> 1));
                    const u16x2 a2 = (kq & 1) ? ap.yy : ap.xx;
#pragma unroll
                    for (int c8 = 0; c8 < T::TN / 8; c8++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            u16x2 &d = acc.v[r][c8 * 4 + q];
                            d = min2(d, add_sat(a2, as_u16x2(comp(bf[c8], q))));
                        }
                }
#pragma unroll
                for (int c8 = 0; c8 < T::TN / 8; c8++) bf[c8] = bn[c8];
            }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
}


// The plain product's k loop: A is M x K (lda), B is K x N (ldb), block at (m0, n0).
template <class T>
__device__ __forceinline__ void tile_mainloop(const u16 *__restrict__ A, int64_t lda,
                                              const u16 *__restrict__ B, int64_t ldb,
                                              int64_t M, int64_t N, int64_t K, int64_t m0, int64_t n0,
                                              bool vec, u16 *lds, TileAcc<T> &acc)
{
    const int64_t nk = (K + T::BK - 1) / T::BK;
    tile_mainloop_with<T>(
        nk, [&](int64_t k0, int row, int kc) { return load8(A, lda, m0 + row, k0 + kc, M, K, vec); },
        [&](int64_t k0, int kr, int jc) { return load8(B, ldb, k0 + kr, n0 + jc, K, N, vec); }, lds, acc);
}

// Row of the block that accumulator row r of this lane holds.
template <class T>
__device__ __forceinline__ int tile_row(int r) { return (int)(threadIdx.x / T::TX) + r * T::TY; }
// First of the 8 block columns that accumulator group c8 of this lane holds.
template <class T>
__device__ __forceinline__ int tile_col(int c8) { return c8 * (T::TX * 8) + (int)(threadIdx.x % T::TX) * 8; }

template <class T>
__device__ __forceinline__ void tile_store(u16 *__restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t m0,
                                           int64_t n0, bool vec, const TileAcc<T> &acc)
{
#pragma unroll
    for (int r = 0; r < T::TM; r++) {
        const int64_t row = m0 + tile_row<T>(r);
        if (row >= M) continue;
#pragma unroll
        for (int c8 = 0; c8 < T::TN / 8; c8++) {
            const int64_t col = n0 + tile_col<T>(c8);
            uint4 v = make_uint4(as_u32(acc.v[r][c8 * 4 + 0]), as_u32(acc.v[r][c8 * 4 + 1]),
                                 as_u32(acc.v[r][c8 * 4 + 2]), as_u32(acc.v[r][c8 * 4 + 3]));
            gu16 *g = glob(C);
            if (vec && col + 8 <= N) {
                gstore16(g + row * ldc + col, v);
            } else {
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 8; e++)
                    if (col + e < N) g[row * ldc + col + e] = (u16)(w[e >> 1] >> ((e & 1) * 16));
            }
        }
    }
}

}  // namespace mpr
