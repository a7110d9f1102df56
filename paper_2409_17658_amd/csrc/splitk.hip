// splitk.hip -- the (min,+) product of small matrices with its inner
// dimension split.
//
// C[i][j] = min_k A[i][k] + B[k][j] is a minimum over k, so it can be taken
// in parts: over S ranges of k, then the minimum of the S partial results,
// exactly (Section 3's product; the minimum is associative and commutative).
// A product whose tiles are too few to fill the device (N = 848: 196 tiles
// of 64 x 64 for 256 CUs) runs S blocks per tile instead, each over one
// range of k, writing a partial tile; a light elementwise pass then takes
// the minimum of the partial products into C.  Used by the chain step for
// small matrices when its workspace holds the partial products.
#include <algorithm>

#include "tile.h"

namespace mpr {

using SplitCfg = TileCfg<64, 64, 32, 4, 8>;  // 128 threads, 64 x 64 tiles

// Block b: tile b % tiles of split b / tiles, over k in [s * kchunk, ...);
// split 0 writes C, split s > 0 partial product s - 1 (row stride ldp).
template <bool H>
__global__ __launch_bounds__(SplitCfg::NT) __attribute__((amdgpu_waves_per_eu(4))) void splitk_kernel(
    const u16 *__restrict__ A, int64_t lda, const u16 *__restrict__ B, int64_t ldb, u16 *__restrict__ C, int64_t ldc,
    u16 *__restrict__ P, int64_t ldp, int64_t M, int64_t N, int64_t K, int tiles_m, int tiles_n, int64_t kchunk,
    int vec)
{
    using T = SplitCfg;
    __shared__ __attribute__((aligned(16))) u16 lds[T::LDS_ELEMS];
    const int tiles = tiles_m * tiles_n;
    const int tile = (int)(blockIdx.x % (unsigned)tiles), s = (int)(blockIdx.x / (unsigned)tiles);
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
    const int64_t k0 = (int64_t)s * kchunk, kk = K - k0 < kchunk ? K - k0 : kchunk;  // kk >= 1 (host)
    TileAcc<T> acc;
    tile_mainloop<T, H>(A + k0, lda, B + k0 * ldb, ldb, M, N, kk, m0, n0, vec != 0, lds, acc);
    u16 *out = s == 0 ? C : P + (int64_t)(s - 1) * M * ldp;
    tile_store<T>(out, s == 0 ? ldc : ldp, M, N, m0, n0, vec != 0, acc);
}

// C = min(C, P_0, ..., P_(parts-1)) elementwise, 8 entries at a time where
// the rows allow 16-byte accesses.
__global__ __launch_bounds__(256) void min_parts_kernel(u16 *C, int64_t ldc, const u16 *P, int64_t ldp, int64_t M,
                                                        int64_t N, int parts, int vec)
{
    const int64_t cpr = (N + 7) / 8, total = M * cpr;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / cpr, j0 = (t % cpr) * 8;
        gu16 *c = glob(C) + i * ldc + j0;
        if (vec && j0 + 8 <= N) {
            uint4 v = gload16(c);
            u16x2 w[4] = {as_u16x2(v.x), as_u16x2(v.y), as_u16x2(v.z), as_u16x2(v.w)};
            for (int p = 0; p < parts; p++) {
                const uint4 q = gload16(glob(P) + (int64_t)p * M * ldp + i * ldp + j0);
                w[0] = min2(w[0], as_u16x2(q.x));
                w[1] = min2(w[1], as_u16x2(q.y));
                w[2] = min2(w[2], as_u16x2(q.z));
                w[3] = min2(w[3], as_u16x2(q.w));
            }
            gstore16(c, make_uint4(as_u32(w[0]), as_u32(w[1]), as_u32(w[2]), as_u32(w[3])));
        } else {
            for (int64_t j = j0; j < j0 + 8 && j < N; j++) {
                u16 m = c[j - j0];
                for (int p = 0; p < parts; p++) {
                    const u16 q = glob(P)[(int64_t)p * M * ldp + i * ldp + j];
                    m = q < m ? q : m;
                }
                c[j - j0] = m;
            }
        }
    }
}

// Splits of the product of an M x K and a K x N matrix: enough blocks for
// every CU to hold a few, each range of k at least 4 slices deep; 1 when
// the tiles alone fill the device.
int splitk_parts(int64_t M, int64_t N, int64_t K)
{
    const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
    const int64_t want = 4 * (int64_t)device_cu_count();
    if (tiles >= want / 2 || K < 8 * SplitCfg::BK) return 1;
    int64_t s = (want + tiles - 1) / tiles;
    s = s < K / (4 * SplitCfg::BK) ? s : K / (4 * SplitCfg::BK);
    return (int)(s < 8 ? (s > 1 ? s : 1) : 8);
}

// Bytes of the partial products for `parts` splits (row stride round_up(N, 8)).
size_t splitk_bytes(int64_t M, int64_t N, int parts)
{
    return parts > 1 ? (size_t)(parts - 1) * (size_t)M * (size_t)round_up(N, 8) * sizeof(u16) : 0;
}

// C = A (x) B in `parts` splits of k, the partial products in P (at least
// splitk_bytes bytes); parts <= 1 takes the plain launch.
mpr_status splitk_launch(int parts, int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda, const u16 *B,
                         int64_t ldb, u16 *C, int64_t ldc, u16 *P, hipStream_t s)
{
    if (parts <= 1 || M == 0 || N == 0 || K == 0 || !P) return gemm_launch(-1, M, N, K, A, lda, B, ldb, C, ldc, s);
    const int64_t slices = (K + SplitCfg::BK - 1) / SplitCfg::BK;
    const int64_t kchunk = ((slices + parts - 1) / parts) * SplitCfg::BK;
    const int real = (int)((K + kchunk - 1) / kchunk);  // every split non-empty
    const int tiles_m = (int)((M + 63) / 64), tiles_n = (int)((N + 63) / 64);
    const int64_t ldp = round_up(N, 8);
    const bool vec = aligned16(A) && aligned16(B) && aligned16(C) && aligned16(P) && lda % 8 == 0 && ldb % 8 == 0 &&
                     ldc % 8 == 0;
    const unsigned grid = (unsigned)((int64_t)tiles_m * tiles_n * real);
    if (current_arith() == MPR_ARITH_F16)
        hipLaunchKernelGGL(splitk_kernel<true>, dim3(grid), dim3(SplitCfg::NT), 0, s, A, lda, B, ldb, C, ldc, P, ldp, M,
                           N, K, tiles_m, tiles_n, kchunk, vec ? 1 : 0);
    else
        hipLaunchKernelGGL(splitk_kernel<false>, dim3(grid), dim3(SplitCfg::NT), 0, s, A, lda, B, ldb, C, ldc, P, ldp,
                           M, N, K, tiles_m, tiles_n, kchunk, vec ? 1 : 0);
    mpr_status e = check_launch();
    if (e != MPR_OK || real <= 1) return e;
    const int64_t chunks = M * ((N + 7) / 8);
    const int blocks = (int)std::min<int64_t>((chunks + 255) / 256, 4096);
    hipLaunchKernelGGL(min_parts_kernel, dim3(blocks), dim3(256), 0, s, C, ldc, P, ldp, M, N, real - 1, vec ? 1 : 0);
    return check_launch();
}

}  // namespace mpr
