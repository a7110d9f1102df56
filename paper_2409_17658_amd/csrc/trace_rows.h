// trace_rows.h -- the trace of a (min,+) product whose right operand is
// given through the canonical form of its transpose (Corollary 7 applied to
// P = (RX (+) X) (x) Y with Y[l][i] = CY[i] + YT[i][l]):
//     trace = min_i (RX[i] + CY[i] + min_l (X[i][l] + YT[i][l])).
// Row i of X and row i of YT are read side by side, so the pass is a plain
// stream of 2 n^2 uint16 values with 16-byte loads: one wave per row, sums
// in 32 bits (exact for every uint16 input), the offsets added once per row
// in int64.  No LDS, no barrier inside the row loop.
#pragma once

#include "trace_tile.h"

namespace mpr {

constexpr uint32_t TR_NONE = 0xFFFFFFFFu;  // no finite term

// 16-byte global load marked non-temporal: the passes read every operand
// byte once, so the caches need not keep it (measured: 0.96 GB read in 141
// instead of 155 us at the m = 9 size, 19.0 instead of 20.2 us at m = 8).
__device__ __forceinline__ uint4 gload16_nt(const gu16 *p)
{
    const u32x4 v = __builtin_nontemporal_load((const gu32x4 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
constexpr int TR_ROWS = 4;                 // rows per block of 256 threads: one per wave
constexpr int TR_TRIP = 8;                 // 16-byte chunks of each row per lane in flight per trip

__device__ __forceinline__ uint32_t tr_term(uint32_t x, uint32_t y, uint32_t best)
{
    const uint32_t s = (x == 0xFFFFu || y == 0xFFFFu) ? TR_NONE : x + y;
    return s < best ? s : best;
}

// The 8 positions of two 8-value chunks.
__device__ __forceinline__ uint32_t tr_min8(uint4 a, uint4 b, uint32_t best)
{
    const uint32_t xa[4] = {a.x, a.y, a.z, a.w}, yb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        best = tr_term(xa[q] & 0xFFFFu, yb[q] & 0xFFFFu, best);
        best = tr_term(xa[q] >> 16, yb[q] >> 16, best);
    }
    return best;
}

// Wave-wide min over l < n of x[l] + y[l] for one row (TR_NONE when every
// term has an infinite operand), returned to every lane.  `vec`: both rows
// 16-byte aligned.  Lane t reads the chunks at 8t, 8t + 512, ...; each trip
// issues up to TR_TRIP chunks of both rows before using any (chunks past
// the row's end are not loaded and count as infinite), so a row takes
// ceil(chunks per lane / TR_TRIP) memory round trips, the last one included.
__device__ __forceinline__ uint32_t tr_row_min(const u16 *x, const u16 *y, int64_t n, bool vec)
{
    const int lane = (int)(threadIdx.x & 63);
    const gu16 *gx = glob(x), *gy = glob(y);
    uint32_t best = TR_NONE;
    int64_t tail = 0;
    if (vec) {
        const int64_t n8 = n & ~(int64_t)7;
        const uint4 inf = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        for (int64_t c = (int64_t)lane * 8; c < n8; c += TR_TRIP * 512) {
            uint4 a[TR_TRIP], b[TR_TRIP];
#pragma unroll
            for (int q = 0; q < TR_TRIP; q++) {
                const bool in = c + q * 512 < n8;
                a[q] = in ? gload16_nt(gx + c + q * 512) : inf;
                b[q] = in ? gload16_nt(gy + c + q * 512) : inf;
            }
#pragma unroll
            for (int q = 0; q < TR_TRIP; q++) best = tr_min8(a[q], b[q], best);
        }
        tail = n8;
    }
    for (int64_t c = tail + lane; c < n; c += 64) best = tr_term(gx[c], gy[c], best);
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    return best;
}

// Blocks of one n x n trace.
__host__ __device__ __forceinline__ int64_t tr_blocks(int64_t n) { return (n + TR_ROWS - 1) / TR_ROWS; }

// Rows [r0, r0 + TR_ROWS) of one trace (256 threads, wave w takes row
// r0 + w); the block's minimum is folded into *out.
__device__ __forceinline__ void tr_rows(const u16 *__restrict__ X, const int64_t *__restrict__ RX,
                                        const u16 *__restrict__ YT, const int64_t *__restrict__ CY, int64_t n,
                                        int64_t ld, int64_t r0, bool vec, int64_t *out)
{
    __shared__ int64_t red[TR_ROWS];
    const int w = (int)(threadIdx.x >> 6);
    const int64_t i = r0 + w;
    int64_t best = ROW_NONE;
    if (i < n) {  // wave-uniform
        const int64_t rx = RX ? RX[i] : 0, cy = CY ? CY[i] : 0;  // in flight with the row
        const uint32_t m = tr_row_min(X + i * ld, YT + i * ld, n, vec);
        if (m != TR_NONE && rx != ROW_NONE && cy != ROW_NONE) best = rx + cy + (int64_t)m;
    }
    if ((threadIdx.x & 63) == 0) red[w] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t v = red[0];
        for (int q = 1; q < TR_ROWS; q++) v = red[q] < v ? red[q] : v;
        tp_fold_min(out, v);
    }
}

// ---- the same pass over byte copies of the operands
// Entries 0..TR8_FMAX are finite, 0xFF is infinity; no other value occurs
// (the producer checks it).  A finite sum is then at most 2 TR8_FMAX = 254
// and any sum with an infinite operand is at least 255, so a packed uint16
// add and min need no test per term: the even bytes (0, 2) and the odd
// bytes (1, 3) of a word are taken as two uint16 pairs (a byte sum is at
// most 510 and never carries into the next half), added, and folded into a
// running uint16-pair minimum.
constexpr uint32_t TR8_FMAX = 127;

__device__ __forceinline__ u16x2 tr8_even(uint32_t w) { return __builtin_bit_cast(u16x2, w & 0x00FF00FFu); }
__device__ __forceinline__ u16x2 tr8_odd(uint32_t w) { return __builtin_bit_cast(u16x2, (w >> 8) & 0x00FF00FFu); }

// 16 positions of two 16-byte chunks: the eight sums first, then their
// minima (a packed min reading the packed add issued just before it waits
// a cycle).
__device__ __forceinline__ u16x2 tr8_min16(uint4 a, uint4 b, u16x2 best)
{
    const uint32_t xa[4] = {a.x, a.y, a.z, a.w}, yb[4] = {b.x, b.y, b.z, b.w};
    u16x2 s[8];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        s[2 * q] = tr8_even(xa[q]) + tr8_even(yb[q]);
        s[2 * q + 1] = tr8_odd(xa[q]) + tr8_odd(yb[q]);
    }
#pragma unroll
    for (int q = 0; q < 8; q++) best = __builtin_elementwise_min(best, s[q]);
    return best;
}

// Launches the pass over all n rows (rowops.hip); *out is set first.
mpr_status trace_product_t_launch(const u16 *X, const int64_t *RX, const u16 *YT, const int64_t *CY, int64_t n,
                                  int64_t ld, int64_t *out, hipStream_t s);

}  // namespace mpr
