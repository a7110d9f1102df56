// sparse.hip -- the chain step N_k = N_(k-1) (x) A when A is sparse.
//
// A transfer matrix stays sparse (0.5 - 3 % finite for m = 6..9) while its
// powers are dense, so in the chain A^k = A^(k-1) (x) A only the rows l of A
// with a finite entry in an output column can contribute to that column.
// For a block J of BN output columns let L_J be those rows of A; then
//     C[:, J] = N[:, L_J] (x) A[L_J, J],
// a dense (min,+) product with inner dimension |L_J| instead of n.  A plan
// built once per matrix (on the device, no host round trip) stores, per
// block, the sorted list L_J (padded with row 0 to a multiple of BK) and the
// packed rows A[L_J, J] (padding rows infinite, so they never win).  The
// step runs the shared tile routine with the left operand gathered through
// L_J.  The result is the same product, entry for entry.
#include <algorithm>
#include <atomic>

#include "tile.h"

namespace mpr {

using SCfg = TileCfg<64, 64, 32, 4, 8>;  // 128 threads; 64-column blocks
constexpr int SBN = SCfg::BN;
constexpr int SBK = SCfg::BK;
// The entry-list form from this size on (m >= 8 transfer matrices); below
// it the tile form is faster (too few 512-row tiles to fill the device).
constexpr int64_t kEntryFormMinN = 7000;

// Does row l of A have a finite entry in columns [j0, j0 + SBN)?
__device__ __forceinline__ bool row_hits_block(const u16 *A, int64_t lda, int64_t l, int64_t j0, int64_t n, bool vec)
{
    const gu16 *row = glob(A) + l * lda;
    for (int64_t j = j0; j < j0 + SBN && j < n; j += 8) {
        if (vec && j + 8 <= n) {
            const uint4 v = gload16(row + j);
            if ((v.x & v.y & v.z & v.w) != 0xFFFFFFFFu) return true;
        } else {
            for (int64_t e = j; e < j + 8 && e < n; e++)
                if (row[e] != 0xFFFF) return true;
        }
    }
    return false;
}

// counts[J] = |L_J| rounded up to a multiple of SBK.
__global__ __launch_bounds__(256) void sp_count_kernel(const u16 *A, int64_t lda, int64_t n, int64_t *counts, int vec)
{
    __shared__ uint64_t sh[4];
    const int64_t j0 = (int64_t)blockIdx.x * SBN;
    uint64_t c = 0;
    for (int64_t l = threadIdx.x; l < n; l += 256) c += row_hits_block(A, lda, l, j0, n, vec != 0);
    c = wave_sum_u64(c);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t t = sh[0] + sh[1] + sh[2] + sh[3];
        counts[blockIdx.x] = (int64_t)((t + SBK - 1) / SBK * SBK);
    }
}

// off[J] = sum of counts before J; off[nblk] = total.  One block.
__global__ __launch_bounds__(1024) void sp_scan_kernel(const int64_t *counts, int64_t nblk, int64_t *off)
{
    __shared__ int64_t part[1024];
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t b0 = threadIdx.x * per;
    int64_t s = 0;
    for (int64_t b = b0; b < b0 + per && b < nblk; b++) s += counts[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < 1024; t++) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        off[nblk] = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t b = b0; b < b0 + per && b < nblk; b++) {
        off[b] = run;
        run += counts[b];
    }
}

// order[r] = the column block with the r-th largest |L_J| (ties by index):
// the step launches the costliest blocks first so the launch does not end
// on a few long blocks (|L_J| varies by 50x within one transfer matrix).
// One block.
__global__ __launch_bounds__(1024) void sp_order_kernel(const int64_t *counts, int64_t nblk, int32_t *order)
{
    for (int64_t J = threadIdx.x; J < nblk; J += 1024) {
        const int64_t c = counts[J];
        int64_t rank = 0;
        for (int64_t K = 0; K < nblk; K++) {
            const int64_t d = counts[K];
            rank += (d > c) || (d == c && K < J);
        }
        order[rank] = (int32_t)J;
    }
}

// Ordered compaction of block J: idx[off[J] + t] = t-th row of L_J and
// Bp[(off[J] + t) * SBN + c] = A[l][j0 + c]; padding rows are row 0 / infinite.
// A plan whose rows (off[nblk]) exceed the capacity `cap` of its workspace
// is not written: *st = MPR_ENOMEM, and the step kernel then does nothing.
__global__ __launch_bounds__(256) void sp_fill_kernel(const u16 *A, int64_t lda, int64_t n, const int64_t *off,
                                                      int64_t nblk, int64_t cap, int32_t *idx, u16 *Bp, int vec,
                                                      int32_t *st)
{
    __shared__ int wsum[4];
    __shared__ int64_t run;
    if (off[nblk] > cap) {  // uniform over the grid
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(st, MPR_ENOMEM);
        return;
    }
    const int64_t J = blockIdx.x, j0 = J * SBN;
    const int64_t base = off[J], end = off[J + 1];
    if (threadIdx.x == 0) run = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t l0 = 0; l0 < n; l0 += 256) {
        const int64_t l = l0 + threadIdx.x;
        const bool hit = l < n && row_hits_block(A, lda, l, j0, n, vec != 0);
        const uint64_t ball = __ballot(hit);
        const int before = __popcll(ball & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __popcll(ball);
        __syncthreads();
        int pre = 0;
        for (int q = 0; q < w; q++) pre += wsum[q];
        const int64_t t = base + run + pre + before;
        if (hit) {
            idx[t] = (int32_t)l;
            const gu16 *src = glob(A) + l * lda;
            gu16 *dst = glob(Bp) + t * SBN;
            for (int c = 0; c < SBN; c++) dst[c] = (j0 + c < n) ? src[j0 + c] : (u16)0xFFFF;
        }
        __syncthreads();
        if (threadIdx.x == 0) run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    // padding up to the multiple of SBK
    for (int64_t t = base + run + threadIdx.x; t < end; t += 256) {
        idx[t] = 0;
        gu16 *dst = glob(Bp) + t * SBN;
        for (int c = 0; c < SBN; c++) dst[c] = 0xFFFF;
    }
}

// One value's f16 image (to_h16 for a single uint16): signed, 0xFFFF is -1
// and survives min(., 0x800); unsigned, it then meets 0x7C00.
__device__ __forceinline__ u16 to_h16_1(u16 x)
{
    const short c = __builtin_elementwise_min((short)x, (short)0x800);
    return __builtin_elementwise_min((u16)c, (u16)0x7C00);
}

// Left operand of the compressed-K step: N[m0 + row][L_J[k]] for the BK-deep
// slice.  Thread t handles k = t % BK (fixed: NT is a multiple of BK), so it
// reads its index once per slice, and rows t / BK + e * (NT / BK); a wave thus
// reads 32 consecutive gathered columns (sorted, mostly adjacent) of two rows
// per instruction, and the values go to LDS one 16-bit store each.
template <class T>
struct GatherA {
    static_assert(T::NT % T::BK == 0, "fixed k per thread");
    static constexpr int PER = T::BM * T::BK / T::NT;  // values per thread
    static constexpr int RSTEP = T::NT / T::BK;        // rows between them
    const gu16 *N;
    int64_t ldn, n, m0;
    const __attribute__((address_space(1))) int32_t *idx;
    bool full;  // all BM rows of the block are < n (block-uniform)
    uint32_t v[PER];
    __device__ __forceinline__ void load(int64_t k0)
    {
        const int k = (int)(threadIdx.x % T::BK), r0 = (int)(threadIdx.x / T::BK);
        const int64_t col = idx[k0 + k];
        if (full) {
#pragma unroll
            for (int e = 0; e < PER; e++) v[e] = N[(m0 + r0 + e * RSTEP) * ldn + col];
            return;
        }
#pragma unroll
        for (int e = 0; e < PER; e++) {
            const int64_t r = m0 + r0 + e * RSTEP;
            v[e] = r < n ? (uint32_t)N[r * ldn + col] : 0xFFFFu;
        }
    }
    template <bool H>
    __device__ __forceinline__ void store(u16 *as) const
    {
        const int k = (int)(threadIdx.x % T::BK), r0 = (int)(threadIdx.x / T::BK);
#pragma unroll
        for (int e = 0; e < PER; e++)
            as[(r0 + e * RSTEP) * T::LDA_S + k] = H ? to_h16_1((u16)v[e]) : (u16)v[e];
    }
};

// One SCfg tile of C = N[:, L_J] (x) A[L_J, J], in form H (tile.h).
template <bool H>
__global__ __launch_bounds__(SCfg::NT) __attribute__((amdgpu_waves_per_eu(4))) void sp_step_kernel(const u16 *__restrict__ Np, int64_t ldn, int64_t n,
                                                           const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ order,
                                                           const int32_t *__restrict__ idx,
                                                           const u16 *__restrict__ Bp, u16 *__restrict__ C,
                                                           int64_t ldc, int tiles_m, int nblk, int64_t cap, int vec)
{
    __shared__ __attribute__((aligned(16))) u16 lds[SCfg::LDS_ELEMS];
    // Column blocks costliest first (order[]), all row tiles of one column
    // block consecutively; consecutive blocks go to different XCDs, so every
    // XCD gets the same mix of costs.
    const int t = (int)blockIdx.x;
    if (t >= tiles_m * nblk) return;
    const int tm = t % tiles_m, J = order[t / tiles_m];
    const int64_t m0 = (int64_t)tm * SCfg::BM, n0 = (int64_t)J * SBN;
    if (off[nblk] > cap) {
        // The plan did not fit its workspace (sp_fill_kernel reported it and
        // wrote nothing): the output is all infinite, so no later pass reads
        // stale values.
        TileAcc<SCfg> none;
#pragma unroll
        for (int r = 0; r < SCfg::TM; r++)
#pragma unroll
            for (int q = 0; q < SCfg::NACC; q++) none.v[r][q] = (u16x2){0xFFFF, 0xFFFF};
        tile_store<SCfg>(C, ldc, n, n, m0, n0, vec != 0, none);
        return;
    }
    const int64_t kbeg = off[J], K = off[J + 1] - kbeg;
    const gu16 *gN = glob(Np);
    const __attribute__((address_space(1))) int32_t *gi = glob(idx) + kbeg;
    const gu16 *gB = glob(Bp) + kbeg * SBN;
    TileAcc<SCfg> acc;
    GatherA<SCfg> aop{gN, ldn, n, m0, gi, m0 + SCfg::BM <= n, {}};
    auto bop = chunk_b<SCfg>([&](int64_t k0, int kr, int jc) { return gload16(gB + (k0 + kr) * SBN + jc); });
    tile_product<SCfg, H>(K / SBK, aop, bop, lds, acc);
    tile_store<SCfg>(C, ldc, n, n, m0, n0, vec != 0, acc);
}

// ------------------------------------------- entry-list form of the step
// The tile above multiplies whole 64-column rows of A[L_J, J]; for a
// transfer matrix about nine in ten of those entries are infinite (a
// column has 25 to 120 finite entries, its block's L_J ten times as many),
// so nine in ten of its pairs cannot win.  This form visits the finite
// entries only.  A block takes 512 rows and one column block; each of its
// eight waves owns 8 whole columns (all 512 rows, 8 per lane), so the
// entries of a column are the same for every lane of the wave.  Per slice
// of 32 rows of L_J, the gathered N[rows, L_J-slice] is stored in LDS
// transposed (l-major), and per column a wave holds the column's 32 values
// of A (one per lane, loaded a slice ahead straight into registers), turns
// the finite ones into a wave-uniform bit mask, and for each set bit l adds
// the scalar A[l][j] to the lane's eight values N[i][l] (one 16-byte LDS
// read) and keeps the minimum.  Two columns are walked together, two reads
// in flight; a column whose mask has run out adds infinity, which changes
// nothing, and a pair with many entries in the slice walks its rows in
// order (one read for both columns, infinity where one of them has no
// entry, rows where neither has one skipped).  The same
// plan, the same minimum over the same entries: the same bits as the tile
// form.
typedef const __attribute__((address_space(1))) unsigned char gbytes;
constexpr int EBM = 512;                 // rows per block
constexpr int ENT = 512;                 // threads: 8 waves
constexpr int ECOLS = SBN / (ENT / 64);  // columns per wave
constexpr int ERL = EBM / 64;            // rows per lane
constexpr int ELDN = EBM + 8;            // transposed slice row (u16), 16-byte aligned
constexpr int E_NT = SBK * ELDN;         // one transposed slice buffer
constexpr int ERP = ENT / SBK;           // row pairs staged per slice by one k
static_assert(ENT == EBM, "one output row per thread in the epilogue");
static_assert(EBM % (2 * ERP) == 0, "staging covers the tile's rows");
static_assert(ECOLS == 8 && ERL == 8, "a lane: 8 columns of A (one 16-byte load), 8 rows (one 16-byte read)");
static_assert(SBN * ELDN <= 2 * E_NT, "the output tile fits the two slice buffers");
constexpr int kEntryDense = 12;          // more entries than this in a column's slice: walk the rows in order
constexpr int ESV = EBM / ERP;           // values a thread stages per slice

// One 512-row tile of the entry-list step; FULL: every row of the tile is
// < n (so the gathers need no row test).
template <bool FULL>
__device__ __forceinline__ void entry_tile(const u16 *__restrict__ Np, int64_t ldn, int64_t n, int64_t m0,
                                           int64_t j0, const int32_t *__restrict__ idx, const u16 *__restrict__ Bp,
                                           int64_t kbeg, int64_t nk, u16 *__restrict__ C, int64_t ldc, int vec,
                                           u16 *nt)
{
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    u16x2 acc[ECOLS][ERL / 2];
#pragma unroll
    for (int c = 0; c < ECOLS; c++)
#pragma unroll
        for (int h = 0; h < ERL / 2; h++) acc[c][h] = (u16x2){0xFFFF, 0xFFFF};

    // staging: thread (k = t % 32, row pair p = t / 32) gathers
    // N[m0 + 2 ERP e + 2p + h][L_J[k]], h < 2.  The values stay as loaded
    // until they are stored (the wait for them falls after the slice's
    // compute), and the column index is read one slice ahead.
    const int sk = (int)(threadIdx.x % SBK), sp = (int)(threadIdx.x / SBK);  // sk == lane % 32
    const gu16 *gN = glob(Np);
    const gbytes *gNb = (const gbytes *)(gN + m0 * ldn);  // this tile's rows; offsets < 2^32 (host)
    const uint32_t rowb = (uint32_t)ldn * 2u;             // bytes per row
    const int nloc = (int)(n - m0 < EBM ? n - m0 : EBM);  // rows of the tile below n (>= 1)
    const __attribute__((address_space(1))) int32_t *gi = glob(idx) + kbeg;
    const gu16 *gB = glob(Bp) + kbeg * SBN;
    uint32_t sv[ESV];
    uint4 bn, bcur;  // A[L_J[32 sl + lane % 32]][j0 + 8 w .. + 7]: the next slice's, this one's
    auto row_of = [&](int e) { return (e >> 1) * (2 * ERP) + 2 * sp + (e & 1); };
    auto load = [&](int64_t sl, uint32_t col) {
        bn = gload16(gB + (sl * SBK + sk) * SBN + w * ECOLS);
        if (FULL) {
            const uint32_t o = (uint32_t)(2 * sp) * rowb + col * 2u;
#pragma unroll
            for (int e = 0; e < ESV; e++)
                sv[e] = *(const gu16 *)(gNb + (uint32_t)(o + (uint32_t)((e >> 1) * (2 * ERP) + (e & 1)) * rowb));
        } else {
            // rows past n read the last row (every load unconditional, so
            // none waits for another); store() puts infinity in their place
#pragma unroll
            for (int e = 0; e < ESV; e++) {
                const int r = row_of(e);
                const uint32_t rr = (uint32_t)(r < nloc ? r : nloc - 1);
                sv[e] = *(const gu16 *)(gNb + (uint32_t)(rr * rowb + col * 2u));
            }
        }
    };
    auto store = [&](int buf) {
        u16 *q = nt + buf * E_NT + sk * ELDN + 2 * sp;
#pragma unroll
        for (int e = 0; e < ESV / 2; e++) {
            uint32_t lo = sv[2 * e], hi = sv[2 * e + 1];
            if (!FULL) {
                lo = row_of(2 * e) < nloc ? lo : 0xFFFFu;
                hi = row_of(2 * e + 1) < nloc ? hi : 0xFFFFu;
            }
            *(uint32_t *)(q + 2 * ERP * e) = lo | (hi << 16);
        }
    };
    auto upd = [&](int c, const uint4 &v, uint32_t wgt) {
        const u16x2 a = (u16x2){(u16)wgt, (u16)wgt};
        const u16x2 s0 = add_sat(as_u16x2(v.x), a), s1 = add_sat(as_u16x2(v.y), a);
        const u16x2 s2 = add_sat(as_u16x2(v.z), a), s3 = add_sat(as_u16x2(v.w), a);
        acc[c][0] = min2(acc[c][0], s0);
        acc[c][1] = min2(acc[c][1], s1);
        acc[c][2] = min2(acc[c][2], s2);
        acc[c][3] = min2(acc[c][3], s3);
    };
    auto compute = [&](int buf) {
        const u16 *nl = nt + buf * E_NT + lane * ERL;
        // lanes 0-31: column c, lanes 32-63: column c + 1, k = lane % 32
        const int hsh = (lane >> 5) * 16;
#pragma unroll
        for (int c = 0; c < ECOLS; c += 2) {
            const uint32_t bv = (comp(bcur, c / 2) >> hsh) & 0xFFFFu;
            const uint64_t mask = __ballot(bv != 0xFFFFu);
            uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
            if (__builtin_popcount(lo) > kEntryDense || __builtin_popcount(hi) > kEntryDense) {
                const uint32_t any = lo | hi;  // rows where neither column has an entry are skipped
#pragma unroll
                for (int k = 0; k < SBK; k++) {
                    if (!((any >> k) & 1u)) continue;
                    const uint32_t wl = (uint32_t)__builtin_amdgcn_readlane((int)bv, k);
                    const uint32_t wh = (uint32_t)__builtin_amdgcn_readlane((int)bv, k + 32);
                    const uint4 v = *(const uint4 *)(nl + k * ELDN);
                    upd(c, v, wl);
                    upd(c + 1, v, wh);
                }
                continue;
            }
            while (lo | hi) {
                // an exhausted mask reads row 31 and adds infinity (no branch;
                // the test is on the scanned bit, so it stays scalar)
                const int kl = __builtin_ctz(lo | 0x80000000u), kh = __builtin_ctz(hi | 0x80000000u);
                const uint32_t rl = (uint32_t)__builtin_amdgcn_readlane((int)bv, kl);
                const uint32_t rh = (uint32_t)__builtin_amdgcn_readlane((int)bv, kh + 32);
                const uint32_t wl = (lo >> kl) & 1u ? rl : 0xFFFFu, wh = (hi >> kh) & 1u ? rh : 0xFFFFu;
                lo &= ~(1u << kl);
                hi &= ~(1u << kh);
                const uint4 vl = *(const uint4 *)(nl + kl * ELDN);
                const uint4 vh = *(const uint4 *)(nl + kh * ELDN);
                upd(c, vl, wl);
                upd(c + 1, vh, wh);
            }
        }
    };
    if (nk > 0) {
        uint32_t col = (uint32_t)gi[sk];
        load(0, col);
        col = nk > 1 ? (uint32_t)gi[SBK + sk] : 0u;
        store(0);
        bcur = bn;
        __syncthreads();
        for (int64_t sl = 0; sl < nk; sl++) {
            const int buf = (int)(sl & 1);
            if (sl + 1 < nk) {
                load(sl + 1, col);
                col = sl + 2 < nk ? (uint32_t)gi[(sl + 2) * SBK + sk] : 0u;
            }
            compute(buf);
            if (sl + 1 < nk) {
                store(buf ^ 1);
                bcur = bn;
            }
            __syncthreads();
        }
    }
    // epilogue: the tile through LDS as [column][row], then each thread
    // writes one row's 64 columns in 16-byte pieces
    u16 *ct = nt;
#pragma unroll
    for (int c = 0; c < ECOLS; c++)
        *(uint4 *)(ct + (w * ECOLS + c) * ELDN + lane * ERL) =
            make_uint4(as_u32(acc[c][0]), as_u32(acc[c][1]), as_u32(acc[c][2]), as_u32(acc[c][3]));
    __syncthreads();
    const int r = (int)threadIdx.x;
    const int64_t i = m0 + r;
    if (i >= n) return;
    gu16 *crow = glob(C) + i * ldc + j0;
#pragma unroll
    for (int c8 = 0; c8 < SBN; c8 += 8) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = ct[(c8 + q) * ELDN + r];
        if (vec && j0 + c8 + 8 <= n) {
            gstore16(crow + c8, make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                                           v[6] | (v[7] << 16)));
        } else {
            for (int q = 0; q < 8; q++)
                if (j0 + c8 + q < n) crow[c8 + q] = (u16)v[q];
        }
    }
}

__global__ __launch_bounds__(ENT) __attribute__((amdgpu_waves_per_eu(4))) void sp_entry_kernel(
    const u16 *__restrict__ Np, int64_t ldn, int64_t n, const int64_t *__restrict__ off,
    const int32_t *__restrict__ order, const int32_t *__restrict__ idx, const u16 *__restrict__ Bp,
    u16 *__restrict__ C, int64_t ldc, int tiles_m, int nblk, int64_t cap, int vec)
{
    __shared__ __attribute__((aligned(16))) u16 nt[2 * E_NT];
    const int t = (int)blockIdx.x;
    if (t >= tiles_m * nblk) return;
    // Column blocks costliest first, all row tiles of one column block
    // consecutively (one strip of rows at a time, blocks costliest first
    // within it, measured slower: the last strip's costly blocks start late).
    const int tm = t % tiles_m, J = order[t / tiles_m];
    const int64_t m0 = (int64_t)tm * EBM, j0 = (int64_t)J * SBN;
    // A plan that did not fit its workspace (sp_fill_kernel reported it and
    // wrote nothing) leaves the tile infinite, as the tile form does.
    const int64_t kbeg = off[J];
    const int64_t nk = off[nblk] > cap ? 0 : (off[J + 1] - kbeg) / SBK;
    if (m0 + EBM <= n)
        entry_tile<true>(Np, ldn, n, m0, j0, idx, Bp, kbeg, nk, C, ldc, vec, nt);
    else
        entry_tile<false>(Np, ldn, n, m0, j0, idx, Bp, kbeg, nk, C, ldc, vec, nt);
}

// ------------------------------------------------------------ host side
// Plan layout: counts[nblk + 1] | off[nblk + 1] | order[nblk] | idx[cap] |
// Bp[cap * SBN], every piece 256-byte aligned; cap (rows) follows from the
// bytes the caller gives the plan.  Its rows are sum_J |L_J| rounded up to
// SBK per block, at most nblk * round_up(n, SBK) (the worst case, a dense
// A); a transfer matrix needs a few per cent of that.
static int64_t plan_fixed_bytes(int64_t nblk)
{
    return round_up((nblk + 1) * 8, 256) * 2 + round_up(nblk * 4, 256);
}

size_t sparse_plan_bytes_rows(int64_t n, int64_t rows)
{
    const int64_t nblk = (n + SBN - 1) / SBN;
    return (size_t)(plan_fixed_bytes(nblk) + round_up(rows * 4, 256) + round_up(rows * SBN * 2, 256) + 256);
}

size_t sparse_plan_bytes(int64_t n)
{
    const int64_t nblk = (n + SBN - 1) / SBN;
    return sparse_plan_bytes_rows(n, nblk * round_up(n, SBK));
}

// Rows a plan workspace of `bytes` holds: the largest cap with
// sparse_plan_bytes_rows(n, cap) <= bytes (so a workspace sized for `rows`
// rows holds at least `rows`).  The first guess is at least that cap and
// the roundings to 256 bytes take it at most a few rows past it.
static int64_t plan_capacity(int64_t n, size_t bytes)
{
    const int64_t nblk = (n + SBN - 1) / SBN;
    const int64_t avail = (int64_t)bytes - plan_fixed_bytes(nblk) - 256;
    if (avail <= 0) return 0;
    int64_t cap = avail / (4 + SBN * 2);
    while (cap > 0 && sparse_plan_bytes_rows(n, cap) > bytes) cap--;
    return cap;
}

struct SparsePlan {
    int64_t nblk, cap;
    int64_t *counts, *off;
    int32_t *order, *idx;
    u16 *Bp;
};

static SparsePlan carve_plan(void *ws, int64_t n, size_t bytes)
{
    SparsePlan p;
    p.nblk = (n + SBN - 1) / SBN;
    p.cap = plan_capacity(n, bytes);
    char *c = (char *)ws;
    p.counts = (int64_t *)c;
    c += round_up((p.nblk + 1) * 8, 256);
    p.off = (int64_t *)c;
    c += round_up((p.nblk + 1) * 8, 256);
    p.order = (int32_t *)c;
    c += round_up(p.nblk * 4, 256);
    p.idx = (int32_t *)c;
    c += round_up(p.cap * 4, 256);
    p.Bp = (u16 *)c;
    return p;
}

// The counts and their prefix sums only (off[nblk] = the plan's rows).
static void plan_count(const u16 *A, int64_t n, int64_t lda, const SparsePlan &p, hipStream_t s)
{
    const int vec = aligned16(A) && lda % 8 == 0;
    hipLaunchKernelGGL(sp_count_kernel, dim3((unsigned)p.nblk), dim3(256), 0, s, A, lda, n, p.counts, vec);
    hipLaunchKernelGGL(sp_scan_kernel, dim3(1), dim3(1024), 0, s, (const int64_t *)p.counts, p.nblk, p.off);
}

mpr_status sparse_plan_rows(const u16 *A, int64_t n, int64_t lda, void *ws, hipStream_t s, int64_t *rows)
{
    SparsePlan p = carve_plan(ws, n, 0);
    plan_count(A, n, lda, p, s);
    if (check_launch() != MPR_OK) return MPR_EHIP;
    if (hipMemcpyAsync(rows, p.off + p.nblk, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MPR_EHIP;
    return MPR_OK;
}

mpr_status sparse_plan_launch(const u16 *A, int64_t n, int64_t lda, void *ws, size_t bytes, int32_t *st,
                              hipStream_t s)
{
    SparsePlan p = carve_plan(ws, n, bytes);
    const int vec = aligned16(A) && lda % 8 == 0;
    plan_count(A, n, lda, p, s);
    hipLaunchKernelGGL(sp_order_kernel, dim3(1), dim3(1024), 0, s, (const int64_t *)p.counts, p.nblk, p.order);
    hipLaunchKernelGGL(sp_fill_kernel, dim3((unsigned)p.nblk), dim3(256), 0, s, A, lda, n, (const int64_t *)p.off,
                       p.nblk, p.cap, p.idx, p.Bp, vec, st);
    return check_launch();
}

static std::atomic<int> g_sparse_arith{MPR_ARITH_U16};  // process-wide, set from any thread
static std::atomic<int> g_sparse_form{MPR_SPARSE_AUTO};

// The form a step of an n x n matrix takes: the entry-list form in uint16
// once it has enough blocks to fill the device, else the tile form.
static bool use_entry_form(int64_t n)
{
    if (g_sparse_arith == MPR_ARITH_F16) return false;
    const int form = g_sparse_form;
    if (form != MPR_SPARSE_AUTO) return form == MPR_SPARSE_ENTRIES;
    return n >= kEntryFormMinN;
}

mpr_status sparse_step_launch(const u16 *Np, int64_t ldn, int64_t n, void *ws, size_t bytes, u16 *C, int64_t ldc,
                              hipStream_t s)
{
    SparsePlan p = carve_plan(ws, n, bytes);
    const int vec = aligned16(C) && ldc % 8 == 0;
    if (use_entry_form(n) && (int64_t)EBM * ldn * 2 < ((int64_t)1 << 32)) {
        const int64_t tiles_m = (n + EBM - 1) / EBM;
        const int64_t tiles = tiles_m * p.nblk;
        if (tiles > (int64_t)INT32_MAX - 8) return MPR_EUNSUPPORTED;
        hipLaunchKernelGGL(sp_entry_kernel, dim3((unsigned)tiles), dim3(ENT), 0, s, Np, ldn, n,
                           (const int64_t *)p.off, (const int32_t *)p.order, (const int32_t *)p.idx,
                           (const u16 *)p.Bp, C, ldc, (int)tiles_m, (int)p.nblk, p.cap, vec);
        return check_launch();
    }
    const int64_t tiles_m = (n + SCfg::BM - 1) / SCfg::BM;
    const int64_t tiles = tiles_m * p.nblk;
    if (tiles > (int64_t)INT32_MAX - 8) return MPR_EUNSUPPORTED;
    auto kernel = g_sparse_arith == MPR_ARITH_F16 ? sp_step_kernel<true> : sp_step_kernel<false>;
    hipLaunchKernelGGL(kernel, dim3((unsigned)tiles), dim3(SCfg::NT), 0, s, Np, ldn, n, (const int64_t *)p.off,
                       (const int32_t *)p.order, (const int32_t *)p.idx, (const u16 *)p.Bp, C, ldc, (int)tiles_m,
                       (int)p.nblk, p.cap, vec);
    return check_launch();
}

}  // namespace mpr

extern "C" mpr_status mpr_set_sparse_form(int form)
{
    if (form != MPR_SPARSE_AUTO && form != MPR_SPARSE_TILES && form != MPR_SPARSE_ENTRIES) return MPR_EINVAL;
    mpr::g_sparse_form = form;
    return MPR_OK;
}

extern "C" mpr_status mpr_set_sparse_arith(int arith)
{
    if (arith != MPR_ARITH_U16 && arith != MPR_ARITH_F16) return MPR_EINVAL;
    mpr::g_sparse_arith = arith;
    return MPR_OK;
}
