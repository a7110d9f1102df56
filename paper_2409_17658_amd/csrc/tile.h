// tile.h -- the (min,+) tile routine shared by the single-product kernel and
// the batched kernel.
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
//
// The f16 form (H = true) runs the same loop on the f16 images of the
// operands (to_h16: small values are their own bit patterns, infinity is
// +inf), two k at a time: two v_pk_add_f16 and one v_pk_minimum3_f16 per
// pair of outputs, 3 instructions for 4 (add, min) pairs instead of 4.
// Round-to-nearest is monotone and exact below 2048, so a result below
// 0x800 is the exact minimum, +inf means every term had an infinite operand
// (exactly the uint16 infinity: finite sums never reach 0xFFFF), and any
// other result means the true minimum is >= 2048; a block that holds such a
// result recomputes its tile with the uint16 loop (tile_product).  The
// f16 form thus gives the uint16 product bit for bit on every input.
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

// 8 staged values as the k loop of form H reads them.
template <bool H>
__device__ __forceinline__ uint4 image(const uint4 &v)
{
    if constexpr (H) return make_uint4(to_h16(v.x), to_h16(v.y), to_h16(v.z), to_h16(v.w));
    return v;
}

// Operand staging.  The k loop asks an operand policy to `load(k0)` the
// BK-deep slice starting at k0 into registers (issued before the math on the
// current slice, so its latency is hidden) and later to `store(stage)` it
// into the LDS stage (`store<H>`, in the representation of form H): A as
// rows of BK (stride LDA_S), B as rows of BN (stride LDB_S).  ChunkA /
// ChunkB stage 16-byte chunks produced by a functor f(k0, row, kc) (8 A
// values: block row `row`, k = k0+kc..+7) or f(k0, kr, jc) (8 B values:
// k = k0+kr, block columns jc..+7).
template <class T, class F>
struct ChunkA {
    F f;
    uint4 r[T::A_CPT];
    __device__ __forceinline__ void load(int64_t k0)
    {
#pragma unroll
        for (int q = 0; q < T::A_CPT; q++) {
            const int c = threadIdx.x + q * T::NT;
            if (T::A_CH % T::NT == 0 || c < T::A_CH) r[q] = f(k0, c / (T::BK / 8), (c % (T::BK / 8)) * 8);
        }
    }
    template <bool H>
    __device__ __forceinline__ void store(u16 *as) const
    {
#pragma unroll
        for (int q = 0; q < T::A_CPT; q++) {
            const int c = threadIdx.x + q * T::NT;
            if (T::A_CH % T::NT == 0 || c < T::A_CH)
                *(uint4 *)(as + (c / (T::BK / 8)) * T::LDA_S + (c % (T::BK / 8)) * 8) = image<H>(r[q]);
        }
    }
};

template <class T, class F>
struct ChunkB {
    F f;
    uint4 r[T::B_CPT];
    __device__ __forceinline__ void load(int64_t k0)
    {
#pragma unroll
        for (int q = 0; q < T::B_CPT; q++) {
            const int c = threadIdx.x + q * T::NT;
            if (T::B_CH % T::NT == 0 || c < T::B_CH) r[q] = f(k0, c / (T::BN / 8), (c % (T::BN / 8)) * 8);
        }
    }
    template <bool H>
    __device__ __forceinline__ void store(u16 *bs) const
    {
#pragma unroll
        for (int q = 0; q < T::B_CPT; q++) {
            const int c = threadIdx.x + q * T::NT;
            if (T::B_CH % T::NT == 0 || c < T::B_CH)
                *(uint4 *)(bs + (c / (T::BN / 8)) * T::LDB_S + (c % (T::BN / 8)) * 8) = image<H>(r[q]);
        }
    }
};

template <class T, class F>
__device__ __forceinline__ ChunkA<T, F> chunk_a(F f)
{
    return ChunkA<T, F>{f, {}};
}
template <class T, class F>
__device__ __forceinline__ ChunkB<T, F> chunk_b(F f)
{
    return ChunkB<T, F>{f, {}};
}

// The k loop of one BM x BN block over nk BK-deep slices, in form H.
template <class T, bool H, class AOp, class BOp>
__device__ __forceinline__ void tile_kloop(int64_t nk, AOp &aop, BOp &bop, u16 *lds, TileAcc<T> &acc)
{
    const int tid = threadIdx.x;
    const int tx = tid % T::TX, ty = tid / T::TX;
    // Stage s holds A at lds + s*STAGE and B at lds + s*STAGE + A_STAGE.
    constexpr int STAGE = T::A_STAGE + T::B_STAGE;
    constexpr u16 INIT = H ? 0x7C00 : 0xFFFF;

#pragma unroll
    for (int r = 0; r < T::TM; r++)
#pragma unroll
        for (int c = 0; c < T::NACC; c++) acc.v[r][c] = (u16x2){INIT, INIT};

    if (nk == 0) return;

    aop.load(0);
    bop.load(0);
    aop.template store<H>(lds);
    bop.template store<H>(lds + T::A_STAGE);
    __syncthreads();

    for (int64_t kt = 0; kt < nk; kt++) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) {  // next slice in flight during the math
            aop.load((kt + 1) * T::BK);
            bop.load((kt + 1) * T::BK);
        }
        const u16 *as = lds + cur * STAGE;
        const u16 *bs = as + T::A_STAGE;
#pragma unroll 1
        for (int kk = 0; kk < T::BK; kk += 8) {
            uint4 af[T::TM];
#pragma unroll
            for (int r = 0; r < T::TM; r++) af[r] = *(const uint4 *)(as + (ty + r * T::TY) * T::LDA_S + kk);
            auto brow = [&](int k, int c8) {
                return *(const uint4 *)(bs + k * T::LDB_S + c8 * (T::TX * 8) + tx * 8);
            };
            if constexpr (!H) {
                // B fragments of row kk + kq; the next row's are read while
                // this one is consumed.  The four sums of a column group are
                // formed before its minima: a v_pk_min_u16 that reads the
                // high-half-broadcast add issued just before it costs a wait
                // state on gfx950.
                uint4 bf[T::TN / 8], bn[T::TN / 8];
#pragma unroll
                for (int c8 = 0; c8 < T::TN / 8; c8++) bf[c8] = brow(kk, c8);
#pragma unroll
                for (int kq = 0; kq < 8; kq++) {
                    if (kq < 7) {
#pragma unroll
                        for (int c8 = 0; c8 < T::TN / 8; c8++) bn[c8] = brow(kk + kq + 1, c8);
                    }
#pragma unroll
                    for (int r = 0; r < T::TM; r++) {
                        const u16x2 ap = as_u16x2(comp(af[r], kq >> 1));
                        const u16x2 a2 = (kq & 1) ? ap.yy : ap.xx;
#pragma unroll
                        for (int c8 = 0; c8 < T::TN / 8; c8++) {
                            u16x2 sum[4];
#pragma unroll
                            for (int q = 0; q < 4; q++) sum[q] = add_sat(a2, as_u16x2(comp(bf[c8], q)));
#pragma unroll
                            for (int q = 0; q < 4; q++) {
                                u16x2 &d = acc.v[r][c8 * 4 + q];
                                d = min2(d, sum[q]);
                            }
                        }
                    }
#pragma unroll
                    for (int c8 = 0; c8 < T::TN / 8; c8++) bf[c8] = bn[c8];
                }
            } else {
                // Rows kk + kq and kk + kq + 1 together; the A register holds
                // a_k in its low and a_(k+1) in its high half.
                uint4 b0[T::TN / 8], b1[T::TN / 8], n0[T::TN / 8], n1[T::TN / 8];
#pragma unroll
                for (int c8 = 0; c8 < T::TN / 8; c8++) {
                    b0[c8] = brow(kk, c8);
                    b1[c8] = brow(kk + 1, c8);
                }
#pragma unroll
                for (int kq = 0; kq < 8; kq += 2) {
                    if (kq < 6) {
#pragma unroll
                        for (int c8 = 0; c8 < T::TN / 8; c8++) {
                            n0[c8] = brow(kk + kq + 2, c8);
                            n1[c8] = brow(kk + kq + 3, c8);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < T::TM; r++) {
                        const h16x2 ap = as_h16x2(comp(af[r], kq >> 1));
                        const h16x2 alo = ap.xx, ahi = ap.yy;
#pragma unroll
                        for (int c8 = 0; c8 < T::TN / 8; c8++) {
                            // all eight sums first: a minimum3 that reads the
                            // add just before it costs a wait state
                            h16x2 s0[4], s1[4];
#pragma unroll
                            for (int q = 0; q < 4; q++) {
                                s0[q] = alo + as_h16x2(comp(b0[c8], q));
                                s1[q] = ahi + as_h16x2(comp(b1[c8], q));
                            }
#pragma unroll
                            for (int q = 0; q < 4; q++) {
                                u16x2 &d = acc.v[r][c8 * 4 + q];
                                const h16x2 m = __builtin_elementwise_minimum(
                                    __builtin_elementwise_minimum(as_h16x2(as_u32(d)), s0[q]), s1[q]);
                                d = as_u16x2(as_u32(m));
                            }
                        }
                    }
#pragma unroll
                    for (int c8 = 0; c8 < T::TN / 8; c8++) {
                        b0[c8] = n0[c8];
                        b1[c8] = n1[c8];
                    }
                }
            }
        }
        if (kt + 1 < nk) {
            aop.template store<H>(lds + (cur ^ 1) * STAGE);
            bop.template store<H>(lds + (cur ^ 1) * STAGE + T::A_STAGE);
        }
        __syncthreads();
    }
}

// Converts the accumulators of an f16 pass back to uint16 (+inf -> 0xFFFF)
// and returns true when one of them is not exact (finite, >= 0x800).  All
// packed: v + 0x8400 (wrapping) takes +inf to 0, the exact values below
// 0x800 to [0x8400, 0x8BFF] and the inexact ones to [0x8C00, 0xFFFF]; among
// the values kept only +inf has bit 14 set, which the shift pair spreads
// over the half.
template <class T>
__device__ __forceinline__ bool tile_from_h16(TileAcc<T> &acc)
{
    u16x2 worst = {0, 0};
#pragma unroll
    for (int r = 0; r < T::TM; r++)
#pragma unroll
        for (int c = 0; c < T::NACC; c++) {
            const u16x2 v = acc.v[r][c];
            worst = __builtin_elementwise_max(worst, v + (u16x2){0x8400, 0x8400});
            const i16x2 hi = __builtin_bit_cast(i16x2, v << (u16)1) >> (short)15;
            acc.v[r][c] = v | __builtin_bit_cast(u16x2, hi);
        }
    return worst.x >= 0x8C00 || worst.y >= 0x8C00;
}

// The (min,+) block product: form H, with the uint16 recomputation for the
// blocks whose f16 results are not all exact (block-uniform decision).
template <class T, bool H, class AOp, class BOp>
__device__ __forceinline__ void tile_product(int64_t nk, AOp &aop, BOp &bop, u16 *lds, TileAcc<T> &acc)
{
    if constexpr (H) {
        tile_kloop<T, true>(nk, aop, bop, lds, acc);
        if (!__syncthreads_or(tile_from_h16<T>(acc))) return;
    }
    tile_kloop<T, false>(nk, aop, bop, lds, acc);
}

// uint16 form only (kept for callers that stage operands themselves).
template <class T, class AOp, class BOp>
__device__ __forceinline__ void tile_mainloop_ops(int64_t nk, AOp &aop, BOp &bop, u16 *lds, TileAcc<T> &acc)
{
    tile_kloop<T, false>(nk, aop, bop, lds, acc);
}

// Functor form of the k loop (16-byte chunk producers for both operands).
template <class T, bool H = false, class ALoad, class BLoad>
__device__ __forceinline__ void tile_mainloop_with(int64_t nk, ALoad aload, BLoad bload, u16 *lds, TileAcc<T> &acc)
{
    auto aop = chunk_a<T>(aload);
    auto bop = chunk_b<T>(bload);
    tile_product<T, H>(nk, aop, bop, lds, acc);
}

// The plain product's k loop: A is M x K (lda), B is K x N (ldb), block at (m0, n0).
template <class T, bool H = false>
__device__ __forceinline__ void tile_mainloop(const u16 *__restrict__ A, int64_t lda,
                                              const u16 *__restrict__ B, int64_t ldb,
                                              int64_t M, int64_t N, int64_t K, int64_t m0, int64_t n0,
                                              bool vec, u16 *lds, TileAcc<T> &acc)
{
    const int64_t nk = (K + T::BK - 1) / T::BK;
    tile_mainloop_with<T, H>(
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
