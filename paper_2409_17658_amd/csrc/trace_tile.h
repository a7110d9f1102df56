// trace_tile.h -- one tile of the trace of a (min,+) product without
// forming it (Corollary 7 applied to P = (RX (+) X) (x) (RY (+) Y)):
//     trace = min_i min_l RX[i] + X[i][l] + RY[l] + Y[l][i].
// The pass is bound by HBM: every entry of X and Y is read once.  A block
// takes rows i0.. of X and inner indices l0.. (a TPI x TPL tile of X and the
// matching TPL x TPI tile of Y), reads both with 16-byte loads, and keeps the
// Y tile in LDS so it can be read transposed.  Offsets are taken relative to
// the tile's least finite RX and RY, so the per-pair arithmetic is 32-bit;
// a tile whose finite offsets spread by 2^28 or more takes an int64 path
// instead (exact either way).
#pragma once

#include "common.h"

namespace mpr {

constexpr int TPI = 64;  // rows i of a tile
constexpr int TPL = 64;  // inner indices l of a tile
constexpr int TP_YS = TPI + 2;  // LDS row stride (u16) of the Y tile: odd dword stride

struct TPShared {
    u16 y[TPL * TP_YS];  // y[l * TP_YS + i] = Y[l0 + l][i0 + i]
    uint32_t rx[TPI], ry[TPL];
    int64_t rx64[TPI], ry64[TPL];
    int64_t base[2];
    int64_t red[4];
    uint32_t redu[4];
    int wide[2];  // offsets of the rows i / inner indices l spread by >= TP_SPREAD
};

constexpr uint32_t TP_BIG = 0x40000000u;  // an infinite term / an empty row
constexpr int64_t TP_SPREAD = 1ll << 28;   // offsets below this use 32-bit sums

// 8 consecutive entries of a row-major matrix, infinity outside n x n.
__device__ __forceinline__ uint4 tp_load8(const u16 *M, int64_t ld, int64_t n, int64_t r, int64_t c, bool vec)
{
    const gu16 *g = glob(M);
    if (vec && r < n && c + 8 <= n) return gload16(g + r * ld + c);
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t lo = (r < n && c + 2 * q < n) ? g[r * ld + c + 2 * q] : 0xFFFFu;
        const uint32_t hi = (r < n && c + 2 * q + 1 < n) ? g[r * ld + c + 2 * q + 1] : 0xFFFFu;
        w[q] = lo | (hi << 16);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Tile (ti, tl) of the t-th block of a tiles x tiles grid.  Blocks are taken
// in groups of TP_G tile-rows, walking down each group's columns, so the
// blocks in flight read both X (rows i, along l) and Y (rows l, along i) in
// runs of several KB per row instead of one 128-byte piece per row.
constexpr int TP_G = 32;
// Tiles per block.  Launches give every block `chunk` consecutive tiles
// (one grid of short-lived blocks, not a persistent grid-stride one: the
// CU's arbiter favours older waves, so of resident blocks that split the
// tiles statically the youngest finish last).  Large traces take 4 tiles a
// block, which keeps the blocks (and their folds) few; below 8192 tiles (2048
// blocks of 4, 8 per CU of 256) a trace is latency-bound and takes one tile
// a block, so that all its tiles run at once.
constexpr int TP_CHUNK = 4;
constexpr int64_t TP_CHUNK_FROM = 8192;
inline int tp_chunk(int64_t tiles) { return tiles * tiles >= TP_CHUNK_FROM ? TP_CHUNK : 1; }
inline int64_t tp_blocks(int64_t tiles)
{
    const int c = tp_chunk(tiles);
    return (tiles * tiles + c - 1) / c;
}
__device__ __forceinline__ void tp_tile_of(int64_t t, int64_t tiles, int64_t &ti, int64_t &tl)
{
    const int64_t width = TP_G * tiles;
    const int64_t first = (t / width) * TP_G;
    const int64_t gs = tiles - first < TP_G ? tiles - first : TP_G;
    const int64_t w = t % width;
    ti = first + w % gs;
    tl = w / gs;
}

// Folds a block's minimum into *out (thread 0).  The word only decreases,
// so a block whose minimum is not below what a relaxed load of it sees
// skips its atomic: with one atomic per block, tens of thousands of
// same-address atomics would serialise, while few blocks improve on the
// running minimum once the first ones have folded theirs.
__device__ __forceinline__ void tp_fold_min(int64_t *out, int64_t best)
{
    if (best == ROW_NONE) return;
    const int64_t seen = __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (best < seen) atomicMin((long long *)out, (long long)best);
}

// Block-wide (256 threads) minimum of the tile; the value is returned to
// every thread (ROW_NONE when the tile holds no finite term).
__device__ __forceinline__ int64_t tp_tile(const u16 *__restrict__ X, const int64_t *__restrict__ RX,
                                           const u16 *__restrict__ Y, const int64_t *__restrict__ RY, int64_t n,
                                           int64_t ld, int64_t i0, int64_t l0, bool vec, TPShared &sh)
{
    const int t = threadIdx.x;
    // Y tile into LDS, 2 chunks of 8 per thread
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int c = t + q * 256, l = c / (TPI / 8), i8 = (c % (TPI / 8)) * 8;
        const uint4 v = tp_load8(Y, ld, n, l0 + l, i0 + i8, vec);
        uint32_t *d = (uint32_t *)&sh.y[l * TP_YS + i8];  // 4-byte aligned (even offsets)
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
    }
    // offsets: wave 0 the rows i, wave 1 the inner indices l
    if (t < 128) {  // whole waves
        const bool is_x = t < 64;
        const int k = t & 63;
        const int64_t idx = (is_x ? i0 : l0) + k;
        const int64_t *R = is_x ? RX : RY;
        const int64_t r = idx >= n ? ROW_NONE : (R ? R[idx] : 0);
        const int64_t base = wave_min_i64(r);
        const int64_t rel = (r == ROW_NONE) ? -1 : r - base;
        const int wide = __any(rel >= TP_SPREAD) ? 1 : 0;
        (is_x ? sh.rx : sh.ry)[k] = rel < 0 ? TP_BIG : (uint32_t)(rel < TP_SPREAD ? rel : 0);
        (is_x ? sh.rx64 : sh.ry64)[k] = r;
        if (k == 0) {
            sh.base[is_x ? 0 : 1] = base;
            sh.wide[is_x ? 0 : 1] = wide;
        }
    }
    __syncthreads();
    const int64_t bx = sh.base[0], by = sh.base[1];
    if (bx == ROW_NONE || by == ROW_NONE) return ROW_NONE;  // block-uniform
    const int lc = (t % (TPL / 8)) * 8;                      // this lane's 8 inner indices
    if (!sh.wide[0] && !sh.wide[1]) {
        uint32_t best = 0xFFFFFFFFu;
#pragma unroll
        for (int pass = 0; pass < TPI / 32; pass++) {
            const int r = pass * 32 + t / (TPL / 8);
            const uint4 xv = tp_load8(X, ld, n, i0 + r, l0 + lc, vec);
            const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w};
            const uint32_t rxr = sh.rx[r];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t x = (xw[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
                const uint32_t y = sh.y[(lc + k) * TP_YS + r];
                const uint32_t s = (x == 0xFFFFu || y == 0xFFFFu) ? TP_BIG : x + y;
                const uint32_t v = s + rxr + sh.ry[lc + k];
                best = v < best ? v : best;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t o = __shfl_xor(best, off, 64);
            best = o < best ? o : best;
        }
        if ((t & 63) == 0) sh.redu[t >> 6] = best;
        __syncthreads();
        uint32_t m = sh.redu[0];
        for (int w = 1; w < 4; w++) m = sh.redu[w] < m ? sh.redu[w] : m;
        return m >= TP_BIG ? ROW_NONE : bx + by + (int64_t)m;
    }
    // wide offsets: the same minimum in int64
    int64_t best = ROW_NONE;
#pragma unroll
    for (int pass = 0; pass < TPI / 32; pass++) {
        const int r = pass * 32 + t / (TPL / 8);
        const uint4 xv = tp_load8(X, ld, n, i0 + r, l0 + lc, vec);
        const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w};
        const int64_t rxr = sh.rx64[r];
        if (rxr == ROW_NONE) continue;
        for (int k = 0; k < 8; k++) {
            const uint32_t x = (xw[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
            const uint32_t y = sh.y[(lc + k) * TP_YS + r];
            const int64_t ry = sh.ry64[lc + k];
            if (x == 0xFFFFu || y == 0xFFFFu || ry == ROW_NONE) continue;
            const int64_t v = rxr + ry + (int64_t)(x + y);
            best = v < best ? v : best;
        }
    }
    best = wave_min_i64(best);
    if ((t & 63) == 0) sh.red[t >> 6] = best;
    __syncthreads();
    int64_t m = sh.red[0];
    for (int w = 1; w < 4; w++) m = sh.red[w] < m ? sh.red[w] : m;
    return m;
}

}  // namespace mpr
