// gemm.hip -- single (min,+) product C = A (x) B over a grid of tiles, the
// compiled tile configurations, the size -> configuration table and the
// autotuner that fills it.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "tile.h"

namespace mpr {

// Compiled configurations: (BM, BN, BK, TM, TN).
using Cfg0 = TileCfg<128, 128, 32, 8, 8>;    // 256 threads, 8x8 per lane
using Cfg1 = TileCfg<128, 256, 32, 8, 16>;   // 256 threads, 8x16 per lane
using Cfg2 = TileCfg<256, 128, 32, 16, 8>;   // 256 threads, 16x8 per lane
using Cfg3 = TileCfg<64, 64, 32, 4, 8>;      // 128 threads, small problems
using Cfg4 = TileCfg<64, 256, 32, 8, 16>;    // 128 threads, 8x16 per lane
using Cfg5 = TileCfg<128, 128, 16, 8, 8>;    // shallow k slices
using Cfg6 = TileCfg<256, 128, 32, 8, 8>;    // 512 threads, 8x8 per lane

// Blocks are handed to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Renumber so that each XCD receives a contiguous run of tiles, and walk the
// tiles in groups of G tile-rows so that the blocks resident on one XCD share
// A row panels and B column panels in that XCD's L2.
__device__ __forceinline__ bool tile_of_block(int tiles_m, int tiles_n, int &tm, int &tn)
{
    const int nb = (int)gridDim.x;  // a multiple of 8
    const int b = (int)blockIdx.x;
    const int t = (b & 7) * (nb >> 3) + (b >> 3);
    if (t >= tiles_m * tiles_n) return false;
    constexpr int G = 8;
    const int width = G * tiles_n;
    const int first = (t / width) * G;
    const int gs = min(tiles_m - first, G);
    const int w = t % width;
    tm = first + w % gs;
    tn = w / gs;
    return true;
}

// Waves per SIMD the register allocation must allow: 4 (<= 128 VGPRs) for
// tiles of up to 64 outputs per lane, 2 for the larger ones.
template <class T>
struct GemmWaves {
    static constexpr int value = T::TM * T::TN <= 64 ? 4 : 2;
};

template <class T, bool H>
__global__ __launch_bounds__(T::NT) __attribute__((amdgpu_waves_per_eu(GemmWaves<T>::value))) void gemm_kernel(const u16 *__restrict__ A, int64_t lda,
                                                     const u16 *__restrict__ B, int64_t ldb,
                                                     u16 *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                                     int64_t K, int tiles_m, int tiles_n, int vec)
{
    __shared__ __attribute__((aligned(16))) u16 lds[T::LDS_ELEMS];
    int tm, tn;
    if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
    const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
    TileAcc<T> acc;
    tile_mainloop<T, H>(A, lda, B, ldb, M, N, K, m0, n0, vec != 0, lds, acc);
    tile_store<T>(C, ldc, M, N, m0, n0, vec != 0, acc);
}

// An empty inner dimension: every entry of C is infinite.
__global__ void fill_inf_kernel(u16 *C, int64_t ldc, int64_t M, int64_t N)
{
    const int64_t total = M * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        C[(t / N) * ldc + t % N] = 0xFFFF;
}

template <class T, bool H>
static mpr_status launch_cfg(int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda, const u16 *B,
                             int64_t ldb, u16 *C, int64_t ldc, hipStream_t s, size_t pad_lds = 0)
{
    const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
    const int64_t tiles = tiles_m * tiles_n;
    if (tiles > (int64_t)INT32_MAX - 8) return MPR_EUNSUPPORTED;
    const int64_t blocks = round_up(tiles, 8);
    const bool vec = aligned16(A) && aligned16(B) && aligned16(C) && lda % 8 == 0 && ldb % 8 == 0 && ldc % 8 == 0;
    hipLaunchKernelGGL((gemm_kernel<T, H>), dim3((unsigned)blocks), dim3(T::NT), pad_lds, s, A, lda, B, ldb, C, ldc, M,
                       N, K, (int)tiles_m, (int)tiles_n, vec ? 1 : 0);
    return check_launch();
}

// Workgroups of a configuration resident per CU, and its static LDS bytes.
template <class T, bool H>
static void residency(int *blocks, size_t *lds)
{
    int b = 0;
    hipFuncAttributes fa{};
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)gemm_kernel<T, H>, T::NT, 0) != hipSuccess ||
        hipFuncGetAttributes(&fa, (const void *)gemm_kernel<T, H>) != hipSuccess) {
        (void)hipGetLastError();
        b = 0;
    }
    *blocks = b;
    *lds = fa.sharedSizeBytes;
}

struct CfgInfo {
    int bm, bn, bk, tm, tn, nt, arith;
    mpr_status (*launch)(int64_t, int64_t, int64_t, const u16 *, int64_t, const u16 *, int64_t, u16 *, int64_t,
                         hipStream_t, size_t);
    void (*residency)(int *, size_t *);
};

// Configurations 0..5 compute in uint16 (MPR_ARITH_U16); 6..11 are the
// same tiles in the f16 form with the uint16 recomputation of inexact blocks
// (MPR_ARITH_F16), which gives the same product bit for bit.  12 is a
// 512-thread tile in uint16, 13 the same in the f16 form.
#define MPR_CFG(T, H)                                                                                 \
    {T::BM, T::BN, T::BK, T::TM, T::TN, T::NT, H ? MPR_ARITH_F16 : MPR_ARITH_U16, launch_cfg<T, H>,       \
     residency<T, H>}
static const CfgInfo kCfgs[] = {MPR_CFG(Cfg0, false), MPR_CFG(Cfg1, false), MPR_CFG(Cfg2, false),
                                MPR_CFG(Cfg3, false), MPR_CFG(Cfg4, false), MPR_CFG(Cfg5, false),
                                MPR_CFG(Cfg0, true),  MPR_CFG(Cfg1, true),  MPR_CFG(Cfg2, true),
                                MPR_CFG(Cfg3, true),  MPR_CFG(Cfg4, true),  MPR_CFG(Cfg5, true),
                                MPR_CFG(Cfg6, false), MPR_CFG(Cfg6, true)};
#undef MPR_CFG
static constexpr int kNumCfgs = (int)(sizeof(kCfgs) / sizeof(kCfgs[0]));

// Arithmetic of the products whose configuration the library picks (the
// tile table, chain and period steps, batched plans, server builds):
// MPR_ARITH_U16 by default, MPR_ARITH_F16 on request.  Process-wide.
static std::atomic<int> g_arith{MPR_ARITH_U16};
int current_arith() { return g_arith.load(); }

// Size -> configuration tables (largest dimension, ascending), one per
// arithmetic.  The defaults are replaced by mpr_set_tile_table with the
// autotuner's measurements.
static std::mutex g_table_mu;
static std::vector<std::pair<int64_t, int>> g_table[2] = {{{96, 3}, {1024, 0}, {INT64_MAX, 0}},
                                                          {{96, 9}, {1024, 6}, {INT64_MAX, 6}}};

int pick_config_arith(int arith, int64_t M, int64_t N, int64_t K)
{
    const int64_t d = std::max(M, std::max(N, K));
    std::lock_guard<std::mutex> lk(g_table_mu);
    const auto &t = g_table[arith == MPR_ARITH_F16 ? 1 : 0];
    for (auto &e : t)
        if (d <= e.first) return e.second;
    return t.back().second;
}

int pick_config(int64_t M, int64_t N, int64_t K) { return pick_config_arith(current_arith(), M, N, K); }

mpr_status gemm_launch(int cfg, int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda, const u16 *B,
                       int64_t ldb, u16 *C, int64_t ldc, hipStream_t s)
{
    if (M == 0 || N == 0) return MPR_OK;
    if (K == 0) {
        const int64_t total = M * N;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(fill_inf_kernel, dim3(blocks), dim3(256), 0, s, C, ldc, M, N);
        return check_launch();
    }
    if (cfg < 0) cfg = pick_config(M, N, K);
    if (cfg >= kNumCfgs) return MPR_EINVAL;
    return kCfgs[cfg].launch(M, N, K, A, lda, B, ldb, C, ldc, s, 0);
}

// LDS of one CU on gfx950.
constexpr size_t kLdsPerCU = 160 * 1024;

mpr_status gemm_launch_spare(int cfg, int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda, const u16 *B,
                             int64_t ldb, u16 *C, int64_t ldc, hipStream_t s)
{
    if (M == 0 || N == 0 || K == 0) return gemm_launch(cfg, M, N, K, A, lda, B, ldb, C, ldc, s);
    if (cfg < 0) cfg = pick_config(M, N, K);
    if (cfg >= kNumCfgs) return MPR_EINVAL;
    // The plain launch, with extra dynamic LDS per workgroup so that one
    // workgroup fewer fits on a CU than registers and static LDS allow: the
    // blocks still retire and refill as usual, and the slot left over (its
    // registers, and a few KB of LDS) takes the waves of other launches.  A
    // configuration of fewer than 3 workgroups per CU gives way to the
    // 128 x 128 tile of the same arithmetic (4 per CU).
    static std::atomic<int> res_blocks[kNumCfgs];   // 0: not yet asked
    static std::atomic<size_t> res_lds[kNumCfgs];
    auto info = [&](int c, int &blocks, size_t &lds) {
        blocks = res_blocks[c].load();
        if (blocks == 0) {
            size_t l = 0;
            kCfgs[c].residency(&blocks, &l);
            res_lds[c] = l;
            res_blocks[c] = blocks > 0 ? blocks : -1;
        }
        lds = res_lds[c].load();
    };
    int blocks = 0;
    size_t lds = 0;
    info(cfg, blocks, lds);
    if (blocks < 3) {
        cfg = kCfgs[cfg].arith == MPR_ARITH_F16 ? 6 : 0;  // Cfg0 in either arithmetic
        info(cfg, blocks, lds);
    }
    if (blocks < 3) return kCfgs[cfg].launch(M, N, K, A, lda, B, ldb, C, ldc, s, 0);
    // (blocks - 1) workgroups of `per` bytes fit with 4 KB to spare, blocks do not
    const size_t per = ((kLdsPerCU - 4096) / (size_t)(blocks - 1)) & ~(size_t)1023;
    const size_t pad = per > lds ? per - lds : 0;
    return kCfgs[cfg].launch(M, N, K, A, lda, B, ldb, C, ldc, s, pad);
}

}  // namespace mpr

using namespace mpr;

extern "C" int mpr_gemm_config_count(void) { return kNumCfgs; }

extern "C" mpr_status mpr_gemm_config_info(int cfg, int *bm, int *bn, int *bk, int *tm, int *tn, int *threads,
                                           int *arith)
{
    if (cfg < 0 || cfg >= kNumCfgs) return MPR_EINVAL;
    const CfgInfo &c = kCfgs[cfg];
    if (bm) *bm = c.bm;
    if (bn) *bn = c.bn;
    if (bk) *bk = c.bk;
    if (tm) *tm = c.tm;
    if (tn) *tn = c.tn;
    if (threads) *threads = c.nt;
    if (arith) *arith = c.arith;
    return MPR_OK;
}

extern "C" int mpr_gemm_pick_config(int64_t M, int64_t N, int64_t K) { return pick_config(M, N, K); }

extern "C" mpr_status mpr_set_tile_table(const int64_t *max_dim_host, const int *cfg_host, int entries)
{
    if (entries <= 0 || !max_dim_host || !cfg_host) return MPR_EINVAL;
    std::vector<std::pair<int64_t, int>> t;
    int arith = -1;
    for (int i = 0; i < entries; i++) {
        if (cfg_host[i] < 0 || cfg_host[i] >= kNumCfgs) return MPR_EINVAL;
        if (i > 0 && max_dim_host[i] <= max_dim_host[i - 1]) return MPR_EINVAL;
        if (arith >= 0 && kCfgs[cfg_host[i]].arith != arith) return MPR_EINVAL;  // one arithmetic per table
        arith = kCfgs[cfg_host[i]].arith;
        t.push_back({max_dim_host[i], cfg_host[i]});
    }
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_table[arith == MPR_ARITH_F16 ? 1 : 0] = t;
    return MPR_OK;
}

extern "C" mpr_status mpr_set_arith(int arith)
{
    if (arith != MPR_ARITH_U16 && arith != MPR_ARITH_F16) return MPR_EINVAL;
    g_arith = arith;
    return mpr_set_sparse_arith(arith);
}

extern "C" int mpr_get_arith(void) { return current_arith(); }

__global__ void tune_fill_kernel(u16 *X, int64_t count, uint64_t seed)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t z = mix64(seed + (uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull);
        X[t] = (z >> 32) < 1288490189ull ? (u16)0xFFFF : (u16)(z & 15);  // 30 % infinite, else 0..15
    }
}

extern "C" mpr_status mpr_autotune_gemm(int64_t n, int reps, float *ms_host, int *best_host, mpr_stream stream)
{
    if (n <= 0 || reps <= 0 || !ms_host) return MPR_EINVAL;
    mpr_status st = ensure_init();
    if (st != MPR_OK) return st;
    hipStream_t s = as_stream(stream);
    const int64_t ld = round_up(n, 8);
    u16 *buf = nullptr;
    if (hipMalloc(&buf, (size_t)(3 * n * ld) * sizeof(u16)) != hipSuccess) return MPR_ENOMEM;
    u16 *A = buf, *B = buf + n * ld, *C = buf + 2 * n * ld;
    hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, s, buf, 2 * n * ld, (uint64_t)n);
    st = check_launch();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == MPR_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = MPR_EHIP;
    float best = 1e30f;
    int besti = -1;
    for (int c = 0; c < kNumCfgs && st == MPR_OK; c++) {
        st = kCfgs[c].launch(n, n, n, A, ld, B, ld, C, ld, s, 0);  // warm-up
        if (st == MPR_OK && hipEventRecord(e0, s) != hipSuccess) st = MPR_EHIP;
        for (int r = 0; r < reps && st == MPR_OK; r++) st = kCfgs[c].launch(n, n, n, A, ld, B, ld, C, ld, s, 0);
        float ms = 0.f;
        if (st == MPR_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = MPR_EHIP;
        if (st != MPR_OK) break;
        ms_host[c] = ms / reps;
        if (ms_host[c] < best) {
            best = ms_host[c];
            besti = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);  // nothing of the timing still reads buf
    (void)hipFree(buf);
    if (best_host) *best_host = besti;
    return st;
}
