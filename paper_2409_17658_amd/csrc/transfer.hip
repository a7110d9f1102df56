// transfer.hip -- the transfer matrix A(G) of Corollary 7 built on the GPU.
//
// States are the correct words of Definition 4 (no ad, da, ab, ba, bb as
// vertical neighbours) in increasing base-4 order, row 1 the most
// significant letter, a=0 b=1 c=2 d=3.  Instead of enumerating all 4^m
// words, each lane unranks its own words with a table of suffix counts:
// S[len][x] = number of correct words of length len that start with x.
// Entry (q, p) is 2 p(a) + p(b) when p can follow q (the rule lists of
// Section 4.1, with the intermediate-row "p_1 = d" read as p_i = d), else
// infinity.
#include <string.h>

#include "common.h"

namespace mpr {

constexpr int MAXM = 12;

struct WordTable {
    int m;
    int64_t S[MAXM + 1][4];  // S[len][first letter]
};

// May letter y sit directly below letter x in a column?
__host__ __device__ __forceinline__ bool adjacent_ok(int x, int y)
{
    // forbidden vertical pairs: ad, da, ab, ba, bb  (bit 4*x + y)
    constexpr uint32_t bad = (1u << (0 * 4 + 3)) | (1u << (3 * 4 + 0)) | (1u << (0 * 4 + 1)) | (1u << (1 * 4 + 0)) |
                             (1u << (1 * 4 + 1));
    return !((bad >> (4 * x + y)) & 1u);
}

static void make_table(int m, WordTable &t)
{
    memset(&t, 0, sizeof(t));
    t.m = m;
    for (int x = 0; x < 4; x++) t.S[1][x] = 1;
    for (int len = 2; len <= m; len++)
        for (int x = 0; x < 4; x++)
            for (int y = 0; y < 4; y++)
                if (adjacent_ok(x, y)) t.S[len][x] += t.S[len - 1][y];
}

static int64_t word_count(const WordTable &t)
{
    int64_t c = 0;
    for (int x = 0; x < 4; x++) c += t.S[t.m][x];
    return c;
}

// Letters of the word of rank r, packed two bits per row, row 0 in bits 0-1.
__host__ __device__ __forceinline__ uint32_t unrank(const WordTable &t, int64_t r)
{
    uint32_t w = 0;
    int prev = -1;
    for (int i = 0; i < t.m; i++) {
        const int len = t.m - i;
        for (int x = 0; x < 4; x++) {
            if (prev >= 0 && !adjacent_ok(prev, x)) continue;
            if (r < t.S[len][x]) {
                w |= (uint32_t)x << (2 * i);
                prev = x;
                break;
            }
            r -= t.S[len][x];
        }
    }
    return w;
}

// Letters allowed for p_i after q_i: always (first mask) or only when a
// vertical neighbour of p_i in the new column is an a (second mask).
//   q_i = a: p_i in {a, c}
//   q_i = b: p_i = d, or p_i = c next to an a
//   q_i = c: p_i in {a, b, d}, or p_i = c next to an a
//   q_i = d: p_i = a
__device__ __constant__ uint8_t kAlways[4] = {(1 << 0) | (1 << 2), (1 << 3), (1 << 0) | (1 << 1) | (1 << 3), (1 << 0)};
__device__ __constant__ uint8_t kWithA[4] = {0, (1 << 2), (1 << 2), 0};

__global__ __launch_bounds__(256) void transfer_kernel(WordTable t, int64_t n, u16 *A, int64_t lda)
{
    const int64_t q = blockIdx.x;
    const uint32_t wq = unrank(t, q);
    const int m = t.m;
    for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
        const uint32_t wp = unrank(t, p);
        bool ok = true;
        uint32_t weight = 0;
        for (int i = 0; i < m; i++) {
            const int qi = (wq >> (2 * i)) & 3, pi = (wp >> (2 * i)) & 3;
            const bool a_up = i > 0 && ((wp >> (2 * (i - 1))) & 3) == 0;
            const bool a_down = i + 1 < m && ((wp >> (2 * (i + 1))) & 3) == 0;
            const uint32_t allowed = kAlways[qi] | ((a_up || a_down) ? kWithA[qi] : 0);
            ok = ok && ((allowed >> pi) & 1u);
            weight += pi == 0 ? 2u : (pi == 1 ? 1u : 0u);
        }
        A[q * lda + p] = ok ? (u16)weight : (u16)0xFFFF;
    }
}

// Border ("loss") matrix of the appendix for a strip of m rows.  Rows
// 1..m-1 follow the rule lists above; the m-th row need not be dominated,
// so after q_m = d everything allowed after q_m = c is allowed.  The arc
// label is 10 p(a) + 5 p(b) - 2 nd(q, p), nd(q, p) = newly dominated
// vertices by Algorithm 3 (per row: (a,a) 1, (b,c) 1, (c,a) 2, (c|d, b|c) 1,
// (d,a) 3; plus 1 when p_m = a, for the vertex below the strip).  Labels
// can be negative down to -2 (3m + 1); entries are stored shifted by
// shift = 2 (3m + 1) so that they fit uint16, and every closed walk of n
// arcs then weighs n * shift more.
__global__ __launch_bounds__(256) void border_transfer_kernel(WordTable t, int64_t n, u16 *A, int64_t lda, int shift)
{
    const int64_t q = blockIdx.x;
    const uint32_t wq = unrank(t, q);
    const int m = t.m;
    for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
        const uint32_t wp = unrank(t, p);
        bool ok = true;
        int label = 0, nd = 0;
        for (int i = 0; i < m; i++) {
            const int qi = (wq >> (2 * i)) & 3, pi = (wp >> (2 * i)) & 3;
            const bool a_up = i > 0 && ((wp >> (2 * (i - 1))) & 3) == 0;
            const bool a_down = i + 1 < m && ((wp >> (2 * (i + 1))) & 3) == 0;
            const int qr = (i == m - 1 && qi == 3) ? 2 : qi;  // last row: d behaves like c
            const uint32_t allowed = kAlways[qr] | ((a_up || a_down) ? kWithA[qr] : 0);
            ok = ok && ((allowed >> pi) & 1u);
            label += pi == 0 ? 10 : (pi == 1 ? 5 : 0);
            if (qi == 0 && pi == 0) nd += 1;
            else if (qi == 1 && pi == 2) nd += 1;
            else if (qi == 2 && pi == 0) nd += 2;
            else if (qi >= 2 && (pi == 1 || pi == 2)) nd += 1;
            else if (qi == 3 && pi == 0) nd += 3;
        }
        if (((wp >> (2 * (m - 1))) & 3) == 0) nd += 1;
        A[q * lda + p] = ok ? (u16)(label - 2 * nd + shift) : (u16)0xFFFF;
    }
}

int border_shift(int m) { return 2 * (3 * m + 1); }

mpr_status border_transfer_launch(int m, u16 *A, int64_t lda, hipStream_t s)
{
    WordTable t;
    make_table(m, t);
    const int64_t n = word_count(t);
    if (lda < n) return MPR_EINVAL;
    hipLaunchKernelGGL(border_transfer_kernel, dim3((unsigned)n), dim3(256), 0, s, t, n, A, lda, border_shift(m));
    return check_launch();
}

mpr_status transfer_launch(int m, u16 *A, int64_t lda, hipStream_t s)
{
    WordTable t;
    make_table(m, t);
    const int64_t n = word_count(t);
    if (lda < n) return MPR_EINVAL;
    hipLaunchKernelGGL(transfer_kernel, dim3((unsigned)n), dim3(256), 0, s, t, n, A, lda);
    return check_launch();
}

int64_t transfer_size(int m)
{
    WordTable t;
    make_table(m, t);
    return word_count(t);
}

void transfer_words(int m, uint8_t *out, int64_t count)
{
    WordTable t;
    make_table(m, t);
    for (int64_t r = 0; r < count; r++) {
        const uint32_t w = unrank(t, r);
        for (int i = 0; i < m; i++) out[r * m + i] = (uint8_t)((w >> (2 * i)) & 3);
    }
}

}  // namespace mpr
