// rowops.hip -- the memory-bound kernels around the product: row-min
// normalisation (canonical form), operand folding for products of powers,
// input validation, traces (Corollary 7), the class hash and exact compare of
// the period search, and small fills.  All of them stream rows with 16-byte
// loads and are bounded by HBM bandwidth.
#include <algorithm>

#include "common.h"
#include "trace_rows.h"
#include "trace_tile.h"

namespace mpr {

constexpr int RB = 256;  // threads per row block

__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t *sh)
{
    v = wave_min_u32(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    uint32_t r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); i++) r = sh[i] < r ? sh[i] : r;
    return r;
}
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *sh)
{
    v = wave_min_i64(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    int64_t r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); i++) r = sh[i] < r ? sh[i] : r;
    return r;
}
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *sh)
{
    v = wave_sum_u64(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    uint64_t r = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) r += sh[i];
    return r;
}

// Key of entry (i, j) with value v in the class hash; injective for
// i, j < 2^24.
__device__ __forceinline__ uint64_t entry_hash(int64_t i, int64_t j, uint32_t v)
{
    return mix64(((uint64_t)i << 40) ^ ((uint64_t)j << 16) ^ (uint64_t)v ^ 0x6A09E667F3BCC909ull);
}

// Subtract r from a packed pair, keeping infinity; flags results > FMAX.
__device__ __forceinline__ uint32_t sub_pair(uint32_t w, uint32_t r, bool &over)
{
    uint32_t lo = w & 0xFFFFu, hi = w >> 16;
    lo = lo == 0xFFFFu ? lo : lo - r;
    hi = hi == 0xFFFFu ? hi : hi - r;
    over |= (lo != 0xFFFFu && lo > FMAX16) || (hi != 0xFFFFu && hi > FMAX16);
    return lo | (hi << 16);
}

__device__ __forceinline__ uint32_t min_pair(uint32_t m, uint32_t w) { return min(m, min(w & 0xFFFFu, w >> 16)); }

constexpr int NCH = 12;  // 16-byte chunks a thread keeps in registers

// One block per row: r = least finite entry, row -= r, R_out = R_in + r (+ add).
// Rows of up to RB * 8 * NCH entries (24576) are read from HBM once and kept
// in registers between the minimum and the subtraction; longer rows are read
// twice.
__global__ __launch_bounds__(RB) void normalise_kernel(u16 *C, int64_t ldc, int64_t N, const int64_t *R_in,
                                                       const int64_t *add_scalar, int64_t *R_out, int32_t *st,
                                                       uint64_t *row_hash, int vec)
{
    __shared__ uint64_t sh[RB / 64];
    const int64_t i = blockIdx.x;
    u16 *row = C + i * ldc;
    uint32_t mn = 0xFFFFu;
    const bool resident = vec && N <= (int64_t)RB * 8 * NCH;
    uint4 keep[NCH];
    if (resident) {
#pragma unroll
        for (int q = 0; q < NCH; q++) {
            const int64_t c = ((int64_t)threadIdx.x + (int64_t)q * RB) * 8;
            keep[q] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
            if (c + 8 <= N) {
                keep[q] = *(const uint4 *)(row + c);
            } else if (c < N) {
                uint32_t w[4];
                for (int e = 0; e < 4; e++) {
                    const uint32_t lo = c + 2 * e < N ? row[c + 2 * e] : 0xFFFFu;
                    const uint32_t hi = c + 2 * e + 1 < N ? row[c + 2 * e + 1] : 0xFFFFu;
                    w[e] = lo | (hi << 16);
                }
                keep[q] = make_uint4(w[0], w[1], w[2], w[3]);
            }
            mn = min_pair(min_pair(mn, keep[q].x), keep[q].y);
            mn = min_pair(min_pair(mn, keep[q].z), keep[q].w);
        }
    } else if (vec) {
        for (int64_t c = (int64_t)threadIdx.x * 8; c < N; c += RB * 8) {
            if (c + 8 <= N) {
                const uint4 v = *(const uint4 *)(row + c);
                mn = min_pair(min_pair(mn, v.x), v.y);
                mn = min_pair(min_pair(mn, v.z), v.w);
            } else {
                for (int64_t j = c; j < N; j++) mn = min(mn, (uint32_t)row[j]);
            }
        }
    } else {
        for (int64_t j = threadIdx.x; j < N; j += RB) mn = min(mn, (uint32_t)row[j]);
    }
    const uint32_t r = block_min_u32(mn, (uint32_t *)sh);
    if (threadIdx.x == 0) {
        const int64_t rin = R_in ? R_in[i] : 0;
        const int64_t add = add_scalar ? *add_scalar : 0;
        const bool none = r == 0xFFFFu || rin == ROW_NONE || add == ROW_NONE;
        R_out[i] = none ? ROW_NONE : rin + (int64_t)r + add;
    }
    uint64_t h = 0;
    bool over = false;
    if (r != 0xFFFFu) {
        if (resident) {
#pragma unroll
            for (int q = 0; q < NCH; q++) {
                const int64_t c = ((int64_t)threadIdx.x + (int64_t)q * RB) * 8;
                if (c >= N) continue;
                uint32_t w[4] = {keep[q].x, keep[q].y, keep[q].z, keep[q].w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    w[e] = sub_pair(w[e], r, over);
                    if (row_hash) {
                        if (c + 2 * e < N) h += entry_hash(i, c + 2 * e, w[e] & 0xFFFFu);
                        if (c + 2 * e + 1 < N) h += entry_hash(i, c + 2 * e + 1, w[e] >> 16);
                    }
                }
                if (c + 8 <= N) {
                    *(uint4 *)(row + c) = make_uint4(w[0], w[1], w[2], w[3]);
                } else {
                    for (int e = 0; e < 8 && c + e < N; e++) row[c + e] = (u16)(w[e >> 1] >> ((e & 1) * 16));
                }
            }
        } else if (vec) {
            for (int64_t c = (int64_t)threadIdx.x * 8; c < N; c += RB * 8) {
                if (c + 8 <= N) {
                    uint4 v = *(const uint4 *)(row + c);
                    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        w[q] = sub_pair(w[q], r, over);
                        if (row_hash)
                            h += entry_hash(i, c + 2 * q, w[q] & 0xFFFFu) + entry_hash(i, c + 2 * q + 1, w[q] >> 16);
                    }
                    *(uint4 *)(row + c) = make_uint4(w[0], w[1], w[2], w[3]);
                } else {
                    for (int64_t j = c; j < N; j++) {
                        uint32_t x = row[j];
                        x = x == 0xFFFFu ? x : x - r;
                        over |= x != 0xFFFFu && x > FMAX16;
                        if (row_hash) h += entry_hash(i, j, x);
                        row[j] = (u16)x;
                    }
                }
            }
        } else {
            for (int64_t j = threadIdx.x; j < N; j += RB) {
                uint32_t x = row[j];
                x = x == 0xFFFFu ? x : x - r;
                over |= x != 0xFFFFu && x > FMAX16;
                if (row_hash) h += entry_hash(i, j, x);
                row[j] = (u16)x;
            }
        }
    } else if (row_hash) {
        for (int64_t j = threadIdx.x; j < N; j += RB) h += entry_hash(i, j, 0xFFFFu);
    }
    if (over) set_status(st, MPR_EOVERFLOW);
    if (row_hash) {
        const uint64_t t = block_sum_u64(h, sh);
        if (threadIdx.x == 0) row_hash[i] = t;
    }
}

mpr_status normalise_launch(int64_t M, int64_t N, u16 *C, int64_t ldc, const int64_t *R_in,
                            const int64_t *add_scalar, int64_t *R_out, int32_t *st, uint64_t *row_hash,
                            hipStream_t s)
{
    if (M == 0) return MPR_OK;
    if (M > INT32_MAX) return MPR_EUNSUPPORTED;
    const int vec = aligned16(C) && ldc % 8 == 0;
    hipLaunchKernelGGL(normalise_kernel, dim3((unsigned)M), dim3(RB), 0, s, C, ldc, N, R_in, add_scalar, R_out, st,
                       row_hash, vec);
    return check_launch();
}

// Flags a finite entry above MPR_FMAX.
__global__ void validate_kernel(const u16 *X, int64_t rows, int64_t cols, int64_t ld, int32_t *st)
{
    bool over = false;
    const int64_t total = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = X[(t / cols) * ld + t % cols];
        over |= v != 0xFFFFu && v > FMAX16;
    }
    if (over) set_status(st, MPR_EOVERFLOW);
}

mpr_status validate_launch(const u16 *X, int64_t rows, int64_t cols, int64_t ld, int32_t *st, hipStream_t s)
{
    if (!st || rows == 0 || cols == 0) return MPR_OK;
    const int64_t blocks = std::min<int64_t>((rows * cols + 255) / 256, 8192);
    hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, rows, cols, ld, st);
    return check_launch();
}

__global__ void copy_kernel(const u16 *src, int64_t lds, u16 *dst, int64_t ldd, int64_t rows, int64_t cols)
{
    const int64_t total = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / cols, j = t % cols;
        dst[i * ldd + j] = src[i * lds + j];
    }
}

mpr_status copy_launch(const u16 *src, int64_t lds, u16 *dst, int64_t ldd, int64_t rows, int64_t cols, hipStream_t s)
{
    if (rows == 0 || cols == 0) return MPR_OK;
    const int64_t blocks = std::min<int64_t>((rows * cols + 255) / 256, 16384);
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
    return check_launch();
}

// s = min over rows with an offset of Rb[l] (ROW_NONE if none).
__global__ __launch_bounds__(1024) void min_offset_kernel(const int64_t *R, int64_t n, int64_t *out)
{
    __shared__ int64_t sh[16];
    int64_t v = ROW_NONE;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v = R[i] < v ? R[i] : v;
    v = block_min_i64(v, sh);
    if (threadIdx.x == 0) *out = v;
}

// B'[l][j] = B[l][j] + (Rb[l] - s); infinity stays, an empty row stays empty.
__global__ void fold_kernel(const u16 *B, int64_t ldb, const int64_t *Rb, const int64_t *s_ptr, int64_t K, int64_t N,
                            u16 *Bp, int64_t ldp, int32_t *st)
{
    const int64_t s = *s_ptr;
    bool over = false;
    const int64_t total = K * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = t / N, j = t % N;
        const uint32_t b = B[l * ldb + j];
        const int64_t rb = Rb[l];
        uint32_t out = 0xFFFFu;
        if (b != 0xFFFFu && rb != ROW_NONE) {
            const int64_t v = (int64_t)b + (rb - s);
            over |= v > (int64_t)FMAX16;
            out = v > (int64_t)FMAX16 ? 0xFFFFu : (uint32_t)v;
        }
        Bp[l * ldp + j] = (u16)out;
    }
    if (over) set_status(st, MPR_EOVERFLOW);
}

mpr_status fold_launch(const u16 *B, int64_t ldb, const int64_t *Rb, int64_t K, int64_t N, u16 *Bp, int64_t ldp,
                       int64_t *s_out, int32_t *st, hipStream_t s)
{
    hipLaunchKernelGGL(min_offset_kernel, dim3(1), dim3(1024), 0, s, Rb, K, s_out);
    mpr_status e = check_launch();
    if (e != MPR_OK || K == 0 || N == 0) return e;
    const int64_t blocks = std::min<int64_t>((K * N + 255) / 256, 16384);
    hipLaunchKernelGGL(fold_kernel, dim3((unsigned)blocks), dim3(256), 0, s, B, ldb, Rb, (const int64_t *)s_out, K, N,
                       Bp, ldp, st);
    return check_launch();
}

// Corollary 7: min_i (R[i] + N[i][i]).
__global__ __launch_bounds__(1024) void trace_kernel(const u16 *N, int64_t n, int64_t ld, const int64_t *R,
                                                     int64_t *out)
{
    __shared__ int64_t sh[16];
    int64_t v = ROW_NONE;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t d = N[i * ld + i];
        const int64_t r = R ? R[i] : 0;
        if (d != 0xFFFFu && r != ROW_NONE) {
            const int64_t x = r + (int64_t)d;
            v = x < v ? x : v;
        }
    }
    v = block_min_i64(v, sh);
    if (threadIdx.x == 0) *out = v;
}

mpr_status trace_launch(const u16 *N, int64_t n, int64_t ld, const int64_t *R, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(1024), 0, s, N, n, ld, R, out);
    return check_launch();
}

__global__ void fill_i64_kernel(int64_t *p, int64_t count, int64_t v)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}
__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t v)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

mpr_status fill_i32_launch(int32_t *p, int64_t count, int32_t v, hipStream_t s)
{
    if (count == 0) return MPR_OK;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
    return check_launch();
}

// Trace of (RX (+) X) (x) (RY (+) Y): min over (i, l) of
// RX[i] + X[i][l] + RY[l] + Y[l][i], one tile per block (trace_tile.h).
__global__ __launch_bounds__(256) void trace_product_kernel(const u16 *X, const int64_t *RX, const u16 *Y,
                                                            const int64_t *RY, int64_t n, int64_t ld, int64_t *out,
                                                            int vec, int chunk)
{
    // `chunk` consecutive tiles per block, a running minimum, and one fold
    // into the result word per block.
    __shared__ TPShared sh;
    const int64_t tiles = (n + TPI - 1) / TPI, total = tiles * tiles;
    const int64_t t0 = (int64_t)blockIdx.x * chunk, t1 = t0 + chunk < total ? t0 + chunk : total;
    int64_t best = ROW_NONE;
    for (int64_t t = t0; t < t1; t++) {
        int64_t ti, tl;
        tp_tile_of(t, tiles, ti, tl);
        const int64_t v = tp_tile(X, RX, Y, RY, n, ld, ti * TPI, tl * TPL, vec != 0, sh);
        best = v < best ? v : best;
        __syncthreads();  // the next tile reuses sh
    }
    if (threadIdx.x == 0) tp_fold_min(out, best);
}

mpr_status trace_product_launch(const u16 *X, const int64_t *RX, const u16 *Y, const int64_t *RY, int64_t n,
                                int64_t ld, int64_t *out, hipStream_t s)
{
    static_assert(TPI == TPL, "square tiles");
    hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(64), 0, s, out, (int64_t)1, ROW_NONE);
    mpr_status e = check_launch();
    if (e != MPR_OK || n == 0) return e;
    const int64_t tiles = (n + TPI - 1) / TPI;
    const int vec = aligned16(X) && aligned16(Y) && ld % 8 == 0;
    const int64_t grid = tp_blocks(tiles);  // <= 2^18 for n <= 65536
    if (grid > INT32_MAX) return MPR_EUNSUPPORTED;
    hipLaunchKernelGGL(trace_product_kernel, dim3((unsigned)grid), dim3(256), 0, s, X, RX, Y, RY, n, ld, out, vec,
                       tp_chunk(tiles));
    return check_launch();
}

// Trace of (RX (+) X) (x) Y with Y given as the canonical form (YT, CY) of
// its transpose: TR_ROWS rows per block (trace_rows.h).
__global__ __launch_bounds__(256) void trace_product_t_kernel(const u16 *X, const int64_t *RX, const u16 *YT,
                                                              const int64_t *CY, int64_t n, int64_t ld,
                                                              int64_t *out, int vec)
{
    tr_rows(X, RX, YT, CY, n, ld, (int64_t)blockIdx.x * TR_ROWS, vec != 0, out);
}

mpr_status trace_product_t_launch(const u16 *X, const int64_t *RX, const u16 *YT, const int64_t *CY, int64_t n,
                                  int64_t ld, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(64), 0, s, out, (int64_t)1, ROW_NONE);
    mpr_status e = check_launch();
    if (e != MPR_OK || n == 0) return e;
    const int64_t grid = tr_blocks(n);
    if (grid > INT32_MAX) return MPR_EUNSUPPORTED;
    const int vec = aligned16(X) && aligned16(YT) && ld % 8 == 0;
    hipLaunchKernelGGL(trace_product_t_kernel, dim3((unsigned)grid), dim3(256), 0, s, X, RX, YT, CY, n, ld, out, vec);
    return check_launch();
}

// dst = src^T for an n x n matrix, 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_kernel(const u16 *src, int64_t lds, u16 *dst, int64_t ldd, int64_t n)
{
    __shared__ u16 t[64][66];
    const int64_t tiles = (n + 63) / 64;
    const int64_t i0 = ((int64_t)blockIdx.x / tiles) * 64, j0 = ((int64_t)blockIdx.x % tiles) * 64;
    const int c = (int)(threadIdx.x & 63), r = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int k = 0; k < 16; k++) {  // rows i0 + r + 4k of src, columns j0 + c
        const int64_t i = i0 + r + 4 * k, j = j0 + c;
        t[r + 4 * k][c] = (i < n && j < n) ? src[i * lds + j] : (u16)0xFFFF;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) {  // rows j0 + r + 4k of dst, columns i0 + c
        const int64_t j = j0 + r + 4 * k, i = i0 + c;
        if (i < n && j < n) dst[j * ldd + i] = t[c][r + 4 * k];
    }
}

mpr_status transpose_launch(const u16 *src, int64_t lds, u16 *dst, int64_t ldd, int64_t n, hipStream_t s)
{
    if (n == 0) return MPR_OK;
    const int64_t tiles = (n + 63) / 64;
    if (tiles * tiles > INT32_MAX) return MPR_EUNSUPPORTED;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(tiles * tiles)), dim3(256), 0, s, src, lds, dst, ldd, n);
    return check_launch();
}

// Class hash of a canonical form up to a scalar shift:
// sum of the row hashes of N plus a term per row for R[i] - min R.
__global__ __launch_bounds__(1024) void class_hash_kernel(const uint64_t *row_hash, const int64_t *R, int64_t n,
                                                          uint64_t *out)
{
    __shared__ int64_t shm[16];
    __shared__ uint64_t shs[16];
    int64_t v = ROW_NONE;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v = R[i] < v ? R[i] : v;
    const int64_t base = block_min_i64(v, shm);
    uint64_t h = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint64_t rel = R[i] == ROW_NONE ? 0xFFFFFFFFFFFFFFFFull : (uint64_t)(R[i] - base);
        h += row_hash[i] + mix64(mix64((uint64_t)i ^ 0xBB67AE8584CAA73Bull) + rel);
    }
    h = block_sum_u64(h, shs);
    if (threadIdx.x == 0) *out = h;
}

mpr_status class_hash_launch(const uint64_t *row_hash, const int64_t *R, int64_t n, uint64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(class_hash_kernel, dim3(1), dim3(1024), 0, s, row_hash, R, n, out);
    return check_launch();
}

// Exact compare of two canonical forms up to a scalar shift.
// out3[0] = number of differing entries of N plus rows whose emptiness
// differs, out3[1] / out3[2] = min / max of RY[i] - RX[i] over non-empty rows.
__global__ void compare_kernel(const u16 *X, const int64_t *RX, const u16 *Y, const int64_t *RY, int64_t n, int64_t ld,
                               int64_t *out3)
{
    int64_t diff = 0, lo = ROW_NONE, hi = -ROW_NONE;
    const int64_t total = n * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t % n;
        diff += X[i * ld + j] != Y[i * ld + j];
        if (j == 0) {
            const bool ex = RX[i] == ROW_NONE, ey = RY[i] == ROW_NONE;
            diff += ex != ey;
            if (!ex && !ey) {
                const int64_t d = RY[i] - RX[i];
                lo = d < lo ? d : lo;
                hi = d > hi ? d : hi;
            }
        }
    }
    if (diff) atomicAdd((unsigned long long *)&out3[0], (unsigned long long)diff);
    if (lo != ROW_NONE) atomicMin((long long *)&out3[1], (long long)lo);
    if (hi != -ROW_NONE) atomicMax((long long *)&out3[2], (long long)hi);
}

__global__ void compare_init_kernel(int64_t *out3)
{
    out3[0] = 0;
    out3[1] = ROW_NONE;
    out3[2] = -ROW_NONE;
}

mpr_status compare_launch(const u16 *X, const int64_t *RX, const u16 *Y, const int64_t *RY, int64_t n, int64_t ld,
                          int64_t *out3, hipStream_t s)
{
    hipLaunchKernelGGL(compare_init_kernel, dim3(1), dim3(1), 0, s, out3);
    mpr_status e = check_launch();
    if (e != MPR_OK || n == 0) return e;
    const int64_t blocks = std::min<int64_t>((n * n + 255) / 256, 16384);
    hipLaunchKernelGGL(compare_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, RX, Y, RY, n, ld, out3);
    return check_launch();
}

}  // namespace mpr
