// batch.hip -- many independent power chains in one launch.
//
// Row i of A^k = A^(k-1) (x) A depends only on row i of A^(k-1) and on A, and
// the row-min normalisation is per row, so a block of rows (a "panel") of one
// chain can run all of its e-1 steps without ever waiting for another
// panel.  The batch is cut into panels of BM rows; a work list of
// (instance, first row) items, longest first, is consumed by a grid of one
// workgroup per item, each taking the next item with one atomic add when it
// starts, so the k-th workgroup to start runs the k-th longest item.  By
// default the grid is not persistent (a persistent form, a grid of resident
// workgroups looping over the list, is kept for comparison and is slower):
// the CU's wave arbiter favours older waves, so of the workgroups sharing a
// CU the youngest ones progress slowest (on MI355X, four resident workgroups of the 64-row f16
// configuration ran at 123, 45, 22 and 16 G pairs/s).  A persistent
// workgroup never gets older than its neighbours, so the ones that started
// last kept their long first items to the very end of the launch; with one
// workgroup per item the oldest waves hold the longest items and the
// youngest the shortest.  Per step, a panel computes its BM x n slice of
// the raw product column tile by column tile (the shared tile routine),
// keeps the running row minima in LDS, then rewrites the slice normalised.
// Only workgroup barriers separate the phases: no data crosses workgroups.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "tile.h"

namespace mpr {

struct DevChain {
    const u16 *A;
    int64_t n, lda, e;
    u16 *N_out;
    int64_t ldo;
    int64_t *R_out;
    u16 *P;  // second panel buffer (workspace), n x ldp
    int64_t ldp;
};

struct BatchItem {
    int32_t inst;
    int32_t row0;
};

using BCfg0 = TileCfg<64, 128, 32, 4, 8>;   // 256 threads, 64-row panels
using BCfg1 = TileCfg<32, 128, 32, 4, 8>;   // 128 threads, 32-row panels
using BCfg2 = TileCfg<128, 128, 32, 8, 8>;  // 256 threads, 128-row panels
using BCfg3 = TileCfg<64, 128, 32, 8, 8>;   // 128 threads, 64-row panels, 8x8 per lane
using BCfg4 = TileCfg<64, 256, 32, 8, 16>;  // 128 threads, 64-row panels, 8x16 per lane
using BCfg5 = TileCfg<64, 64, 32, 4, 8>;    // 128 threads, 64-row panels, 64-column tiles

// A panel's global writes are read back only by the workgroup that wrote
// them (all its waves run on one CU and share its L1 and its XCD's L2), so a
// workgroup barrier -- a workgroup-scope release/acquire -- orders them.  An
// agent-scope fence would write back and invalidate the whole L2 of the XCD
// on every step.

// Rewrites rows [r0, r0+rows) of src (raw values) into dst, subtracting the
// row minima in rmin[] (infinity stays) and adding them to R (or setting R
// when first).  Flags normalised values above MPR_FMAX.  Rows are walked in
// 8-element chunks (16-byte accesses when `vec`).
__device__ __forceinline__ uint32_t sub_keep_inf(uint32_t v, uint32_t r)
{
    return (r == 0xFFFFu || v == 0xFFFFu) ? v : v - r;
}

template <int NT>
__device__ void panel_normalise(const u16 *src, int64_t lds_, u16 *dst, int64_t ldd, int64_t r0, int rows, int64_t n,
                                const uint32_t *rmin, int64_t *R, bool first, bool vec, int32_t *st)
{
    bool over = false;
    const int64_t cpr = (n + 7) / 8;  // chunks per row
    const int64_t total = (int64_t)rows * cpr;
    for (int64_t t = threadIdx.x; t < total; t += NT) {
        const int rr = (int)(t / cpr);
        const int64_t j0 = (t % cpr) * 8;
        const uint32_t r = rmin[rr];
        const gu16 *sp = glob(src) + (r0 + rr) * lds_ + j0;
        gu16 *dp = glob(dst) + (r0 + rr) * ldd + j0;
        if (vec && j0 + 8 <= n) {
            const uint4 v = gload16(sp);
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t lo = sub_keep_inf(w[q] & 0xFFFFu, r), hi = sub_keep_inf(w[q] >> 16, r);
                over |= (lo != 0xFFFFu && lo > FMAX16) || (hi != 0xFFFFu && hi > FMAX16);
                w[q] = lo | (hi << 16);
            }
            gstore16(dp, make_uint4(w[0], w[1], w[2], w[3]));
        } else {
            for (int64_t j = j0; j < j0 + 8 && j < n; j++) {
                const uint32_t x = sub_keep_inf(sp[j - j0], r);
                over |= x != 0xFFFFu && x > FMAX16;
                dp[j - j0] = (u16)x;
            }
        }
    }
    for (int rr = threadIdx.x; rr < rows; rr += NT) {
        const uint32_t r = rmin[rr];
        __attribute__((address_space(1))) int64_t &Rv = glob(R)[r0 + rr];
        if (first)
            Rv = r == 0xFFFFu ? ROW_NONE : (int64_t)r;
        else
            Rv = (r == 0xFFFFu || Rv == ROW_NONE) ? ROW_NONE : Rv + (int64_t)r;
    }
    if (over) set_status(st, MPR_EOVERFLOW);
}

// Row minima of rows [r0, r0+rows) of A into rmin[] (already 0xFFFF).
template <int NT>
__device__ void panel_rowmin(const u16 *A, int64_t lda, int64_t r0, int rows, int64_t n, uint32_t *rmin, bool vec)
{
    const int64_t cpr = (n + 7) / 8;
    const int64_t total = (int64_t)rows * cpr;
    for (int64_t t = threadIdx.x; t < total; t += NT) {
        const int rr = (int)(t / cpr);
        const int64_t j0 = (t % cpr) * 8;
        const gu16 *sp = glob(A) + (r0 + rr) * lda + j0;
        uint32_t m = 0xFFFFu;
        if (vec && j0 + 8 <= n) {
            const uint4 v = gload16(sp);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; q++) m = min(m, min(w[q] & 0xFFFFu, w[q] >> 16));
        } else {
            for (int64_t j = j0; j < j0 + 8 && j < n; j++) m = min(m, (uint32_t)sp[j - j0]);
        }
        atomicMin(&rmin[rr], m);
    }
}

// Register budget: the 4x8-per-lane configurations are held to 128 VGPRs
// (4 waves per SIMD), the larger tiles to 256.
template <class T>
struct BatchWaves {
    static constexpr int value = (T::TM * T::TN <= 32) ? 4 : 2;
};

// Largest value a panel may carry into the next product without being
// normalised first.  Row i of (s (+) N) (x) A is s_i (+) the row of N (x) A
// (the scalar rule of Section 3), so a panel can skip the per-step
// normalisation and keep its row offsets inside its values for as long as
// they stay small: in uint16 every finite input <= MPR_FMAX is exact; in the
// f16 form inputs up to 1023 keep the sums with A's small entries inside
// the exact range (larger ones would only send tiles to the uint16 redo).
// The row minima are still taken every step, and the canonical form is
// written at the last step, so the results are the same bits.
template <bool H>
struct LazyMax {
    static constexpr uint32_t value = H ? 0x3FFu : FMAX16;
};

// One panel: all e - 1 chain steps of rows [row0, row0 + BM) of one chain.
// A step computes the raw product of the panel with A column tile by column
// tile, keeping each row's least value and largest finite value in LDS; the
// panel is normalised in place (offsets into R) only when a row's largest
// value passes LazyMax, and at the last step.
template <class T, bool H>
__device__ __forceinline__ void batch_item(const DevChain *__restrict__ chains, const BatchItem item, u16 *lds,
                                           uint32_t *rmin, uint32_t *rmax, int32_t *st)
{
    const DevChain c = chains[item.inst];
    const int64_t n = c.n, r0 = item.row0;
    const int rows = (int)min<int64_t>(T::BM, n - r0);
    // Step k writes buffer (e - k) % 2 so that step e lands in N_out.
    u16 *buf[2] = {c.N_out, c.P};
    const int64_t ld[2] = {c.ldo, c.ldp};
    int b = (int)((c.e - 1) & 1);

    const bool vec = ((uintptr_t)c.A % 16 == 0) && c.lda % 8 == 0 && ((uintptr_t)c.N_out % 16 == 0) &&
                     c.ldo % 8 == 0 && ((uintptr_t)c.P % 16 == 0) && c.ldp % 8 == 0;
    // Step 1: the panel of A itself, normalised.
    for (int rr = threadIdx.x; rr < T::BM; rr += T::NT) rmin[rr] = 0xFFFFu;
    __syncthreads();
    panel_rowmin<T::NT>(c.A, c.lda, r0, rows, n, rmin, vec);
    __syncthreads();
    panel_normalise<T::NT>(c.A, c.lda, buf[b], ld[b], r0, rows, n, rmin, c.R_out, true, vec, st);

    for (int64_t k = 2; k <= c.e; k++) {
        __syncthreads();
        const int nb = b ^ 1;
        for (int rr = threadIdx.x; rr < T::BM; rr += T::NT) {
            rmin[rr] = 0xFFFFu;
            rmax[rr] = 0u;
        }
        // (visibility of rmin is covered by the barriers inside the tile loop)
        // 32-bit offsets: n <= 32768 and leading dimensions <= 65528.
        const gu16 *Lp = glob(buf[b]) + r0 * ld[b];
        gu16 *Op = glob(buf[nb]) + r0 * ld[nb];
        const gu16 *Ap = glob(c.A);
        const int ldl = (int)ld[b], ldo = (int)ld[nb], lda = (int)c.lda, nn = (int)n;
        for (int n0 = 0; n0 < nn; n0 += T::BN) {
            TileAcc<T> acc;
            // Left operand: rows r0.. of the previous power (rows beyond
            // `rows` read as infinity); right operand: A.
            tile_mainloop_with<T, H>(
                (nn + T::BK - 1) / T::BK,
                [&](int64_t k0, int row, int kc) {
                    const int k = (int)k0 + kc;
                    if (vec && row < rows && k + 8 <= nn) return gload16(Lp + (row * ldl + k));
                    uint32_t w[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const uint32_t lo = (row < rows && k + 2 * q < nn) ? Lp[row * ldl + k + 2 * q] : 0xFFFFu;
                        const uint32_t hi =
                            (row < rows && k + 2 * q + 1 < nn) ? Lp[row * ldl + k + 2 * q + 1] : 0xFFFFu;
                        w[q] = lo | (hi << 16);
                    }
                    return make_uint4(w[0], w[1], w[2], w[3]);
                },
                [&](int64_t k0, int kr, int jc) {
                    const int k = (int)k0 + kr, j = n0 + jc;
                    if (vec && k < nn && j + 8 <= nn) return gload16(Ap + (k * lda + j));
                    uint32_t w[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const uint32_t lo = (k < nn && j + 2 * q < nn) ? Ap[k * lda + j + 2 * q] : 0xFFFFu;
                        const uint32_t hi = (k < nn && j + 2 * q + 1 < nn) ? Ap[k * lda + j + 2 * q + 1] : 0xFFFFu;
                        w[q] = lo | (hi << 16);
                    }
                    return make_uint4(w[0], w[1], w[2], w[3]);
                },
                lds, acc);
#pragma unroll
            for (int r = 0; r < T::TM; r++) {
                const int row = tile_row<T>(r);
                if (row >= rows) continue;
#pragma unroll
                for (int c8 = 0; c8 < T::TN / 8; c8++) {
                    const int col = n0 + tile_col<T>(c8);
                    const uint4 v = make_uint4(as_u32(acc.v[r][c8 * 4 + 0]), as_u32(acc.v[r][c8 * 4 + 1]),
                                               as_u32(acc.v[r][c8 * 4 + 2]), as_u32(acc.v[r][c8 * 4 + 3]));
                    if (vec && col + 8 <= nn) {
                        gstore16(Op + (row * ldo + col), v);
                    } else {
                        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int e = 0; e < 8; e++)
                            if (col + e < nn) Op[row * ldo + col + e] = (u16)(w[e >> 1] >> ((e & 1) * 16));
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < T::TM; r++) {
                // Least value, and largest finite value + 1 (infinity wraps to
                // 0), two columns per packed instruction; columns past the end
                // of the chain are infinite (A was read as infinity there).
                u16x2 mn = {0xFFFF, 0xFFFF}, mx = {0, 0};
#pragma unroll
                for (int q = 0; q < T::NACC; q++) {
                    mn = min2(mn, acc.v[r][q]);
                    mx = __builtin_elementwise_max(mx, acc.v[r][q] + (u16x2){1, 1});
                }
                uint32_t m = min((uint32_t)mn.x, (uint32_t)mn.y), x = max((uint32_t)mx.x, (uint32_t)mx.y);
                // lanes tx = 0..TX-1 of one row group are consecutive
#pragma unroll
                for (int off = 1; off < T::TX; off <<= 1) {
                    m = min(m, (uint32_t)__shfl_xor(m, off, 64));
                    x = max(x, (uint32_t)__shfl_xor(x, off, 64));
                }
                if (threadIdx.x % T::TX == 0) {
                    atomicMin(&rmin[tile_row<T>(r)], m);
                    atomicMax(&rmax[tile_row<T>(r)], x);
                }
            }
        }
        __syncthreads();
        // Rows past the chain's end hold only infinity (x = 0), so they never
        // ask for a normalisation.
        bool wide = false;
        for (int rr = threadIdx.x; rr < rows; rr += T::NT) wide |= rmax[rr] > LazyMax<H>::value + 1u;
        if (__syncthreads_or(wide) || k == c.e)
            panel_normalise<T::NT>(buf[nb], ld[nb], buf[nb], ld[nb], r0, rows, n, rmin, c.R_out, false, vec, st);
        b = nb;
    }
}

template <class T, bool H>
__global__ __launch_bounds__(T::NT) __attribute__((amdgpu_waves_per_eu(BatchWaves<T>::value)))
void batch_kernel(const DevChain *__restrict__ chains, const BatchItem *__restrict__ items, int n_items,
                  int *counter, int persistent, int32_t *st)
{
    __shared__ __attribute__((aligned(16))) u16 lds[T::LDS_ELEMS];
    __shared__ uint32_t rmin[T::BM], rmax[T::BM];
    __shared__ int next;
    // Each workgroup takes the next item with one atomic add, so the k-th item
    // taken is the k-th longest.  One workgroup per item by default; in the
    // persistent form a grid of resident workgroups loops until the list is
    // empty.
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();  // every thread has read `next` before it changes
        if (it >= n_items) return;  // block-uniform
        batch_item<T, H>(chains, items[it], lds, rmin, rmax, st);
        if (!persistent) return;
        __syncthreads();  // the next item reuses lds, rmin and rmax
    }
}

__global__ void reset_counter_kernel(int *counter) { *counter = 0; }

// ------------------------------------------------------------ host side
struct BatchCfgInfo {
    int bm, nt, arith;
    const void *kernel;
};
// 0..5 compute in uint16, 6..11 are the same tiles in the f16 form (same
// results bit for bit; see tile.h).
#define MPR_BCFG(T, H) {T::BM, T::NT, H ? MPR_ARITH_F16 : MPR_ARITH_U16, (const void *)batch_kernel<T, H>}
static const BatchCfgInfo kBatchCfgs[] = {
    MPR_BCFG(BCfg0, false), MPR_BCFG(BCfg1, false), MPR_BCFG(BCfg2, false),
    MPR_BCFG(BCfg3, false), MPR_BCFG(BCfg4, false), MPR_BCFG(BCfg5, false),
    MPR_BCFG(BCfg0, true),  MPR_BCFG(BCfg1, true),  MPR_BCFG(BCfg2, true),
    MPR_BCFG(BCfg3, true),  MPR_BCFG(BCfg4, true),  MPR_BCFG(BCfg5, true),
};
#undef MPR_BCFG
static constexpr int kNumBatchCfgs = (int)(sizeof(kBatchCfgs) / sizeof(kBatchCfgs[0]));

struct BatchPlan {
    int cfg;
    int n_items;
    int grid;
    int persistent;
    DevChain *chains;
    BatchItem *items;
    int *counter;
};

static std::mutex g_plan_mu;
static std::map<void *, BatchPlan> g_plans;

struct BatchLayout {
    size_t chains_off, items_off, counter_off, bufs_off, bytes;
    std::vector<size_t> buf_off;
    std::vector<int64_t> ldp;
};

static BatchLayout batch_layout(const mpr_chain_desc *d, int count, int bm)
{
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (size_t)round_up((int64_t)off, 256);
        const size_t at = off;
        off += bytes;
        return at;
    };
    int64_t n_items = 0;
    for (int i = 0; i < count; i++) n_items += (d[i].n + bm - 1) / bm;
    L.chains_off = take(sizeof(DevChain) * (size_t)count);
    L.items_off = take(sizeof(BatchItem) * (size_t)std::max<int64_t>(n_items, 1));
    L.counter_off = take(256);
    for (int i = 0; i < count; i++) {
        const int64_t ldp = round_up(std::max<int64_t>(d[i].n, 1), 8);
        L.ldp.push_back(ldp);
        L.buf_off.push_back(take((size_t)(d[i].n * ldp) * sizeof(u16)));
    }
    L.bytes = off + 256;
    return L;
}

static int occupancy(int cfg)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kBatchCfgs[cfg].kernel, kBatchCfgs[cfg].nt, 0) !=
            hipSuccess ||
        blocks < 1)
        blocks = 1;
    return blocks;
}

// Longest-first greedy schedule of the items on `slots` equal workers;
// returns the modelled makespan in units of pair-operations per worker.
static double lpt_makespan(const std::vector<double> &work_sorted, int slots)
{
    std::vector<double> heap(slots, 0.0);  // min-heap of finish times
    std::make_heap(heap.begin(), heap.end(), std::greater<double>());
    for (double w : work_sorted) {
        std::pop_heap(heap.begin(), heap.end(), std::greater<double>());
        heap.back() += w;
        std::push_heap(heap.begin(), heap.end(), std::greater<double>());
    }
    return *std::max_element(heap.begin(), heap.end());
}

// Modelled cost of one panel: the tile routine computes all BM rows of a
// panel (rows past the end of the matrix read as infinity), so a ragged last
// panel costs as much as a full one and is ordered with them.
static double panel_cost(const mpr_chain_desc &d, int bm)
{
    return (double)d.e * (double)bm * (double)d.n * (double)d.n;
}

// Relative throughput of each configuration on a full chip (uniform
// batches of 128 chains of N = 1024, e = 17, measured on MI355X; the f16
// 64x128 4x8 configuration = 1).  The schedule model below scores load
// balance; these weigh in how fast each tile shape runs.  They are the
// compiled-in prior: the batch autotuner measures its own and installs them
// with mpr_set_batch_weights.
static const double kBatchRel[] = {0.79, 0.63, 0.75, 0.69, 0.49, 0.70,   // uint16 0..5
                                   1.00, 0.77, 0.93, 0.86, 0.63, 0.88};  // f16 6..11
static_assert(sizeof(kBatchRel) / sizeof(kBatchRel[0]) == kNumBatchCfgs, "one prior per configuration");
static std::mutex g_weights_mu;
static std::vector<double> g_batch_rel(kBatchRel, kBatchRel + kNumBatchCfgs);

// Configuration of a batch in arithmetic `arith`: the one whose modelled
// makespan (longest-first schedule of its panels, weighed by the
// configuration's relative throughput) is least.
static int choose_batch_cfg(const mpr_chain_desc *d, int count, int arith)
{
    std::vector<double> rel;
    {
        std::lock_guard<std::mutex> lk(g_weights_mu);
        rel = g_batch_rel;
    }
    const int cus = device_cu_count();
    int best = -1;
    double best_t = 1e300;
    for (int c = 0; c < kNumBatchCfgs; c++) {
        if (kBatchCfgs[c].arith != arith || !(rel[c] > 0.0)) continue;
        const int bm = kBatchCfgs[c].bm;
        std::vector<double> w;
        for (int i = 0; i < count; i++)
            for (int64_t r0 = 0; r0 < d[i].n; r0 += bm) w.push_back(panel_cost(d[i], bm));
        std::sort(w.begin(), w.end(), std::greater<double>());
        // A worker's speed is the CU's rate (rel) shared among its resident
        // workers.
        const int per_cu = std::max(1, occupancy(c));
        const double t = lpt_makespan(w, cus * per_cu) * per_cu / rel[c];
        if (t < best_t) {
            best_t = t;
            best = c;
        }
    }
    return best;
}

// Process-wide settings, read when a plan is made (atomic: set and read from
// any thread).
static std::atomic<int> g_forced_batch_cfg{-1};
static std::atomic<int> g_batch_persistent{0};

}  // namespace mpr

using namespace mpr;

extern "C" int mpr_batch_config_count(void) { return kNumBatchCfgs; }

extern "C" mpr_status mpr_batch_config_info(int cfg, int *panel_rows, int *threads, int *arith)
{
    if (cfg < 0 || cfg >= kNumBatchCfgs) return MPR_EINVAL;
    if (panel_rows) *panel_rows = kBatchCfgs[cfg].bm;
    if (threads) *threads = kBatchCfgs[cfg].nt;
    if (arith) *arith = kBatchCfgs[cfg].arith;
    return MPR_OK;
}

extern "C" mpr_status mpr_set_batch_persistent(int on)
{
    if (on != 0 && on != 1) return MPR_EINVAL;
    g_batch_persistent = on;
    return MPR_OK;
}

extern "C" mpr_status mpr_set_batch_weights(const double *rel_host, int count)
{
    if (count != kNumBatchCfgs) return MPR_EINVAL;
    std::vector<double> w(kBatchRel, kBatchRel + kNumBatchCfgs);
    if (rel_host) {
        bool any[2] = {false, false};
        for (int c = 0; c < count; c++) {
            if (!(rel_host[c] >= 0.0) || rel_host[c] > 1e6) return MPR_EINVAL;
            any[kBatchCfgs[c].arith == MPR_ARITH_F16] |= rel_host[c] > 0.0;
            w[c] = rel_host[c];
        }
        if (!any[0] || !any[1]) return MPR_EINVAL;  // every arithmetic keeps a configuration
    }
    std::lock_guard<std::mutex> lk(g_weights_mu);
    g_batch_rel = w;
    return MPR_OK;
}

extern "C" mpr_status mpr_get_batch_weights(double *rel_host, int count)
{
    if (!rel_host || count < kNumBatchCfgs) return MPR_EINVAL;
    std::lock_guard<std::mutex> lk(g_weights_mu);
    for (int c = 0; c < kNumBatchCfgs; c++) rel_host[c] = g_batch_rel[c];
    return MPR_OK;
}

extern "C" mpr_status mpr_set_batch_config(int cfg)
{
    if (cfg < -1 || cfg >= kNumBatchCfgs) return MPR_EINVAL;
    g_forced_batch_cfg = cfg;
    return MPR_OK;
}

static mpr_status check_descs(const mpr_chain_desc *d, int count)
{
    if (count < 0 || (count && !d)) return MPR_EINVAL;
    for (int i = 0; i < count; i++) {
        if (d[i].n < 1 || d[i].n > 32768 || d[i].e < 1) return MPR_EINVAL;
        if (!d[i].A || !d[i].N_out || !d[i].R_out) return MPR_EINVAL;
        if (d[i].lda < d[i].n || d[i].ldo < d[i].n || d[i].lda > 65528 || d[i].ldo > 65528) return MPR_EINVAL;
    }
    return MPR_OK;
}

extern "C" mpr_status mpr_batch_workspace_size(const mpr_chain_desc *descs_host, int count, size_t *bytes_host)
{
    mpr_status e = check_descs(descs_host, count);
    if (e != MPR_OK || !bytes_host) return e != MPR_OK ? e : MPR_EINVAL;
    size_t mx = 0;
    for (int c = 0; c < kNumBatchCfgs; c++) mx = std::max(mx, batch_layout(descs_host, count, kBatchCfgs[c].bm).bytes);
    *bytes_host = mx;
    return MPR_OK;
}

extern "C" mpr_status mpr_batch_plan(const mpr_chain_desc *descs_host, int count, void *ws, size_t ws_bytes,
                                     mpr_stream stream)
{
    mpr_status e = check_descs(descs_host, count);
    if (e != MPR_OK) return e;
    if (!ws) return MPR_EINVAL;
    if ((e = ensure_init()) != MPR_OK) return e;
    const int forced = g_forced_batch_cfg.load();
    const int cfg = forced >= 0 ? forced : choose_batch_cfg(descs_host, count, current_arith());
    const int bm = kBatchCfgs[cfg].bm;
    BatchLayout L = batch_layout(descs_host, count, bm);
    if (ws_bytes < L.bytes) return MPR_ENOMEM;
    char *base = (char *)ws;
    std::vector<DevChain> chains(count);
    std::vector<std::pair<double, BatchItem>> items;
    for (int i = 0; i < count; i++) {
        const mpr_chain_desc &d = descs_host[i];
        chains[i] = DevChain{d.A, d.n, d.lda, d.e, d.N_out, d.ldo, d.R_out, (u16 *)(base + L.buf_off[i]), L.ldp[i]};
        for (int64_t r0 = 0; r0 < d.n; r0 += bm) items.push_back({panel_cost(d, bm), BatchItem{i, (int32_t)r0}});
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<double, BatchItem> &a, const std::pair<double, BatchItem> &b) {
                         return a.first > b.first;
                     });
    if (items.size() > (size_t)INT32_MAX) return MPR_EUNSUPPORTED;  // one workgroup per panel
    std::vector<BatchItem> flat;
    for (auto &p : items) flat.push_back(p.second);
    hipStream_t s = as_stream(stream);
    if (count && hipMemcpyAsync(base + L.chains_off, chains.data(), sizeof(DevChain) * count, hipMemcpyHostToDevice,
                                s) != hipSuccess)
        return MPR_EHIP;
    if (!flat.empty() && hipMemcpyAsync(base + L.items_off, flat.data(), sizeof(BatchItem) * flat.size(),
                                        hipMemcpyHostToDevice, s) != hipSuccess)
        return MPR_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MPR_EHIP;
    BatchPlan plan;
    plan.cfg = cfg;
    plan.n_items = (int)flat.size();
    plan.persistent = g_batch_persistent;
    plan.grid = plan.persistent ? std::max(1, std::min(plan.n_items, device_cu_count() * occupancy(cfg)))
                                : std::max(1, plan.n_items);
    plan.chains = (DevChain *)(base + L.chains_off);
    plan.items = (BatchItem *)(base + L.items_off);
    plan.counter = (int *)(base + L.counter_off);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[ws] = plan;
    return MPR_OK;
}

extern "C" mpr_status mpr_batch_launch(void *ws, int32_t *d_status, mpr_stream stream)
{
    BatchPlan p;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(ws);
        if (it == g_plans.end()) return MPR_EINVAL;
        p = it->second;
    }
    if (p.n_items == 0) return MPR_OK;
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, p.counter);
    mpr_status e = check_launch();
    if (e != MPR_OK) return e;
    const void *args_k = kBatchCfgs[p.cfg].kernel;
    void *args[] = {&p.chains, &p.items, &p.n_items, &p.counter, &p.persistent, &d_status};
    if (hipLaunchKernel(args_k, dim3(p.grid), dim3(kBatchCfgs[p.cfg].nt), args, 0, s) != hipSuccess) return MPR_EHIP;
    return check_launch();
}

extern "C" mpr_status mpr_batch_plan_info(void *ws, int *cfg, int *grid, int *panels)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(ws);
    if (it == g_plans.end()) return MPR_EINVAL;
    if (cfg) *cfg = it->second.cfg;
    if (grid) *grid = it->second.grid;
    if (panels) *panels = it->second.n_items;
    return MPR_OK;
}

extern "C" mpr_status mpr_batch_power(const mpr_chain_desc *descs_host, int count, void *ws, size_t ws_bytes,
                                      int32_t *d_status, mpr_stream stream)
{
    mpr_status e = mpr_batch_plan(descs_host, count, ws, ws_bytes, stream);
    return e != MPR_OK ? e : mpr_batch_launch(ws, d_status, stream);
}

extern "C" mpr_status mpr_batch_graph_create(void *ws, int32_t *d_status, mpr_stream stream, void **graph_host)
{
    if (!graph_host) return MPR_EINVAL;
    hipStream_t s = as_stream(stream);
    if (!s) return MPR_EINVAL;  // the null stream can not be captured
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPR_EHIP;
    mpr_status e = mpr_batch_launch(ws, d_status, stream);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess || e != MPR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e != MPR_OK ? e : MPR_EHIP;
    }
    hipGraphExec_t x = nullptr;
    const bool ok = hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
    (void)hipGraphDestroy(g);
    if (!ok) return MPR_EHIP;
    *graph_host = (void *)x;
    return MPR_OK;
}

extern "C" mpr_status mpr_graph_launch(void *graph, mpr_stream stream)
{
    if (!graph) return MPR_EINVAL;
    return hipGraphLaunch((hipGraphExec_t)graph, as_stream(stream)) == hipSuccess ? MPR_OK : MPR_EHIP;
}

extern "C" mpr_status mpr_graph_destroy(void *graph)
{
    if (!graph) return MPR_EINVAL;
    return hipGraphExecDestroy((hipGraphExec_t)graph) == hipSuccess ? MPR_OK : MPR_EHIP;
}
