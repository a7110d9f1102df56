// serve.hip -- a continuous-batching query engine for gamma_R(P_m x C_n).
//
// For each m the engine keeps a "ladder" of canonical powers resident in
// HBM: baby steps (A^T)^1 .. (A^T)^B, the transposes of A^1 .. A^B (a chain
// over the compressed rows of the sparse transfer matrix, transposed), and
// giant steps A^B, A^2B, ... (A^B by the same chain on A, the rest by dense
// products), plus byte copies of both when their entries fit; it answers
// n = B*i + j (1 <= j <= B) as the trace of A^(B i) (x) A^j, i.e. one
// HBM-bound pass per query reading both operands along rows (Corollary 7;
// the product is never formed).  n <= B is read off the baby traces
// computed once at build time.
//
// A worker thread owns every HIP call.  Each tick it gathers the requests
// whose ladder is ready into ONE grouped launch on the query stream (up to
// `slots` launches in flight), while ladder builds run on a separate build
// stream, so queries for warm m keep flowing while a cold m is built.  A
// ladder is admitted only if its bytes fit the HBM budget; idle ladders are
// evicted least-recently-used to make room, and requests that do not fit
// wait in an admission queue.
//
// The labelled fast mode (period_mode) answers from Proposition 8 instead:
// the build of m searches the period of A (compressed-K chain, ring of
// powers, class hashes) up to max_n on a host thread and stream of its own,
// keeps the traces of A^1 .. A^max_n on the host (those past the confirmed
// period filled from it) and releases its device memory; a query is then a
// table read, with no GPU work.
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"
#include "trace_rows.h"

namespace mpr {

mpr_status transfer_launch(int m, u16 *A, int64_t lda, hipStream_t s);
mpr_status transpose_launch(const u16 *src, int64_t lds, u16 *dst, int64_t ldd, int64_t n, hipStream_t s);
int64_t transfer_size(int m);

// ------------------------------------------------------------ grouped trace-of-product
// A query n = B i + j is the trace of A^(B i) (x) A^j (Corollary 7).  The
// giant powers A^(B i) are kept in canonical form (rows), the baby powers as
// the canonical forms of (A^T)^j = (A^j)^T, so one query is a row-streaming
// pass over two matrices (trace_rows.h).
struct TRDesc {
    const u16 *X;     // A^(B i), canonical rows
    const int64_t *RX;
    const u16 *YT;    // (A^T)^j, canonical rows
    const int64_t *CY;
    const uint8_t *X8, *YT8;  // their byte copies, used when `narrow`
    int64_t n, ld, ld8, first_block;
    int vec, narrow;
    int gpos, gsize;  // position in its group, and (at position 0) the group's size
};

// Blocks of one query of n x n operands.
static inline int64_t trace_blocks(int64_t n) { return tr_blocks(n); }

// Queries that share a giant power (same m and i) in one pass.
constexpr int TR_GROUP = 8;

// Result words of a launch.  Folding thousands of block minima into one
// 64-bit word serialises them on its cache line at the memory side (a
// relaxed agent-scope load, and an atomic when it lowers the word): at
// m = 8 that cost about a sixth of the pass.  Block b folds into slot
// b % TR_SLOTS instead, and query q's slot s is the word s * nqpad + q with
// nqpad a multiple of 16, so the slots of one query lie on distinct 128-byte
// lines; the host takes the minimum over the slots.
constexpr int TR_SLOTS = 32;
static inline int64_t slot_pitch(int64_t nq) { return (nq + 15) / 16 * 16; }

// Rows [r0, r0 + TR_ROWS) of the nq <= TR_GROUP queries of a group, which
// share X = A^(B i) and differ in YT (byte copies): wave w streams row r0 + w
// of X once, and the same row of every YT_q beside it, so a group of q
// queries reads X once instead of q times.  Query q's minimum is folded
// into out[q].
__device__ __forceinline__ void tr8_group_rows(const TRDesc *__restrict__ g, int nq, int64_t r0, int64_t *out)
{
    __shared__ int64_t red[TR_GROUP][TR_ROWS];
    typedef const __attribute__((address_space(1))) uint8_t gbyte;
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t n = g[0].n, ld8 = g[0].ld8, i = r0 + w;
    if (i < n) {  // wave-uniform
        gbyte *gx = (gbyte *)g[0].X8 + i * ld8;
        u16x2 best[TR_GROUP];
#pragma unroll
        for (int q = 0; q < TR_GROUP; q++) best[q] = (u16x2){0xFFFF, 0xFFFF};
        const int64_t n16 = n & ~(int64_t)15;
        const uint4 inf = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        for (int64_t c = (int64_t)lane * 16; c < n16; c += TR_TRIP * 1024) {
            uint4 a[TR_TRIP];
#pragma unroll
            for (int k = 0; k < TR_TRIP; k++)
                a[k] = c + k * 1024 < n16 ? gload16_nt((const gu16 *)(gx + c + k * 1024)) : inf;
#pragma unroll
            for (int q = 0; q < TR_GROUP; q++) {
                if (q >= nq) break;  // uniform
                gbyte *gy = (gbyte *)g[q].YT8 + i * ld8;
                uint4 b[TR_TRIP];
#pragma unroll
                for (int k = 0; k < TR_TRIP; k++)
                    b[k] = c + k * 1024 < n16 ? gload16_nt((const gu16 *)(gy + c + k * 1024)) : inf;
#pragma unroll
                for (int k = 0; k < TR_TRIP; k++) best[q] = tr8_min16(a[k], b[k], best[q]);
            }
        }
        const int64_t rx = g[0].RX ? g[0].RX[i] : 0;
#pragma unroll
        for (int q = 0; q < TR_GROUP; q++) {
            if (q >= nq) break;
            gbyte *gy = (gbyte *)g[q].YT8 + i * ld8;
            uint32_t m = best[q].x < best[q].y ? best[q].x : best[q].y;
            for (int64_t c = n16 + lane; c < n; c += 64) {
                const uint32_t s = (uint32_t)gx[c] + (uint32_t)gy[c];
                m = s < m ? s : m;
            }
            for (int off = 32; off > 0; off >>= 1) {
                const uint32_t o = __shfl_xor(m, off, 64);
                m = o < m ? o : m;
            }
            const int64_t cy = g[q].CY ? g[q].CY[i] : 0;
            int64_t v = ROW_NONE;
            if (m < 255u && rx != ROW_NONE && cy != ROW_NONE) v = rx + cy + (int64_t)m;
            if (lane == 0) red[q][w] = v;
        }
    } else if ((threadIdx.x & 63) == 0) {
        for (int q = 0; q < nq; q++) red[q][w] = ROW_NONE;
    }
    __syncthreads();
    if ((int)threadIdx.x < nq) {
        int64_t v = red[threadIdx.x][0];
        for (int k = 1; k < TR_ROWS; k++) v = red[threadIdx.x][k] < v ? red[threadIdx.x][k] : v;
        tp_fold_min(&out[threadIdx.x], v);
    }
}

// One launch for all queries of a batch.  Queries come in groups (the
// queries of a group are consecutive and share the giant power; a group of
// one otherwise); every query of a group carries the group's first block,
// and the group owns the blocks [first_block, first_block +
// trace_blocks(n)); each block takes TR_ROWS rows of its group and folds
// their minima into the queries' words of its result slot.
__global__ __launch_bounds__(256) void grouped_trace_rows_kernel(const TRDesc *__restrict__ d, int nq,
                                                                   int64_t nqpad, int64_t *out)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nq - 1;  // last q with first_block <= b (every thread, same answer)
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (d[mid].first_block <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    TRDesc q = d[lo];
    int lead = lo;
    if (q.gpos != 0) {  // a member of a group: its leader carries the group
        lead = lo - q.gpos;
        q = d[lead];
    }
    const int64_t r0 = (b - q.first_block) * TR_ROWS;
    int64_t *o = out + (b % TR_SLOTS) * nqpad + lead;
    if (q.narrow)  // block-uniform
        tr8_group_rows(&d[lead], q.gsize, r0, o);
    else
        tr_rows(q.X, q.RX, q.YT, q.CY, q.n, q.ld, r0, q.vec != 0, o);
}

// Byte copy of an n x n canonical power (0xFFFF -> 0xFF), one row per
// block; *wide is set when a finite entry exceeds TR8_FMAX (the copy is then
// not used).  Entries of canonical Roman powers stay below 2m + 1.
__global__ __launch_bounds__(256) void pack8_kernel(const u16 *src, int64_t ld, uint8_t *dst, int64_t ld8, int64_t n,
                                                    int vec, int32_t *wide)
{
    const int64_t i = blockIdx.x;
    const gu16 *s = glob(src) + i * ld;
    uint8_t *d = dst + i * ld8;
    bool w = false;
    for (int64_t j = (int64_t)threadIdx.x * 8; j < n; j += 256 * 8) {
        const bool full = vec && j + 8 <= n;
        uint32_t v[8];
        if (full) {
            const uint4 q = gload16(s + j);
            const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = (qw[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu;
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = j + e < n ? (uint32_t)s[j + e] : 0xFFFFu;
        }
        uint32_t b[2] = {0, 0};
#pragma unroll
        for (int e = 0; e < 8; e++) {
            w |= v[e] != 0xFFFFu && v[e] > TR8_FMAX;
            b[e >> 2] |= (v[e] == 0xFFFFu ? 0xFFu : (v[e] & 0xFFu)) << ((e & 3) * 8);
        }
        if (full) {
            *(uint2 *)(d + j) = make_uint2(b[0], b[1]);  // 8-byte aligned: ld8 % 16 == 0
        } else {
#pragma unroll
            for (int e = 0; e < 8; e++)
                if (j + e < n) d[j + e] = (uint8_t)(b[e >> 2] >> ((e & 3) * 8));
        }
    }
    if (w) atomicOr(wide, 1);
}

__global__ void fill_none_kernel(int64_t *p, int count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = ROW_NONE;
}

// ------------------------------------------------------------ engine
using Clock = std::chrono::steady_clock;

// A period-mode build in flight: its thread writes the fields, then `done`.
struct PeriodBuild {
    std::thread th;
    std::atomic<bool> done{false};
    mpr_status status = MPR_OK;
    std::vector<int64_t> traces;  // [k] = trace of A^k, k = 1..max_n
};

struct Ladder {
    int m = 0;
    int64_t n = 0, ld = 0;
    enum State { NONE, BUILDING, READY, FAILED } state = NONE;
    int fail_status = MPR_OK;  // why a FAILED ladder failed
    void *mem = nullptr;
    size_t bytes = 0;
    std::vector<u16 *> Nb, Ng;        // baby[1..B] = (A^T)^j, giant[1..G] = A^(B i), canonical forms
    std::vector<int64_t *> Rb, Rg;
    std::vector<uint8_t *> Nb8, Ng8;  // byte copies (row stride ld8), when the server keeps them
    int64_t ld8 = 0;
    int32_t *wide_dev = nullptr;      // set by the pack pass when an entry does not fit a byte
    // Pinned host copy of the build's words (baby traces, status word,
    // byte-copy flag), refreshed by the build stream before each of its
    // events, so the worker reads them without a HIP call of its own (a
    // blocking copy could wait behind the build on a shared hardware queue).
    volatile int64_t *info = nullptr;
    bool narrow = false;              // queries read the byte copies
    std::vector<int64_t> baby_trace;  // host, index j = 1..B
    hipEvent_t ready = nullptr;
    // Progressive readiness while the ladder builds: step_ev[i] (i = 1..G)
    // completes once the babies, their traces and the giants A^B .. A^(B i)
    // (with their byte copies) are written; `avail` is the largest such i
    // seen complete with a clean status word, so queries n <= B (avail + 1)
    // are answered before the build ends.
    std::vector<hipEvent_t> step_ev;
    int avail = 0;
    bool failing = false;  // the build failed; no new queries while earlier ones drain
    // Giant products are handed to the build stream a few at a time (the
    // worker tops them up as they finish), so whatever shares the stream's
    // hardware queue, and the builds of other m, wait for at most those.
    int next_giant = 0;      // next giant to enqueue
    bool submitted = false;  // every step enqueued and `ready` recorded
    u16 *Bp = nullptr;       // the folded A^B, right operand of every giant product
    int64_t *scal = nullptr; // the build's scalar words on the device
    int64_t *trace_dev = nullptr;
    int32_t *status_dev = nullptr;
    int inflight = 0;
    double last_use = 0;
    double build_s0 = 0, build_s = 0;
    bool period = false;                  // period mode: answers from `table`
    std::shared_ptr<PeriodBuild> pb;      // the build, while it runs
    std::vector<int64_t> table;           // period mode: [n] = gamma_R(P_m x C_n)
};

struct Request {
    int64_t tag;
    int m;
    int64_t n;
    double t_submit;
    bool cold = false;
};

struct Slot {
    hipStream_t stream = nullptr;  // the query stream, or the early stream (the last slot)
    bool busy = false;
    hipEvent_t done = nullptr;
    TRDesc *desc_host = nullptr;  // pinned
    TRDesc *desc_dev = nullptr;
    int64_t *out_dev = nullptr;
    int64_t *out_host = nullptr;  // pinned
    std::vector<Request> reqs;
    double t_launch = 0;
};

struct Server {
    mpr_server_options opt;
    int device = 0;
    // queries of ready ladders / builds / queries of ladders still building
    hipStream_t qstream = nullptr, bstream = nullptr, estream = nullptr;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_in, cv_out;
    std::deque<Request> inbox;
    std::vector<int64_t> cancels;  // tags to cancel (mpr_server_cancel)
    std::deque<mpr_query_result> outbox;
    bool stop = false;
    std::thread worker;
    // worker-owned
    std::map<int, Ladder> ladders;
    std::map<int, std::deque<Request>> waiting;  // per m, ladder not ready
    std::deque<int> admission;                   // m values waiting for memory
    std::vector<Slot> slots;
    size_t resident = 0;
    int64_t *info_host = nullptr;  // pinned, info_words(baby) words per m = 0..11
    mpr_server_stats stats;
    std::string fatal;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

// The worker's writes to the counters that mpr_server_stats_get reads.
template <class F>
static void stats_update(Server &S, F f)
{
    std::lock_guard<std::mutex> lk(S.mu);
    f(S.stats);
}

static size_t ladder_bytes(int m, int B, int G, bool bytes8, int64_t *n_out, int64_t *ld_out)
{
    const int64_t n = transfer_size(m), ld = round_up(n, 8);
    const size_t mat = (size_t)round_up(n * ld * 2, 256), vec = (size_t)round_up(n * 8, 256);
    // A, B babies, G giants, one folded operand; the scalars; the
    // compressed-K plan (of A for the first giant, then of A^T for the
    // babies); the byte copies of the babies and giants
    const size_t count = 1 + (size_t)B + (size_t)G + 1;
    const size_t mat8 = bytes8 ? (size_t)round_up(n * round_up(n, 16), 256) : 0;
    if (n_out) *n_out = n;
    if (ld_out) *ld_out = ld;
    return count * (mat + vec) + (size_t)round_up((int64_t)(B + 8) * 8, 256) + sparse_plan_bytes(n) +
           (size_t)(B + G) * mat8;
}

static int giant_count(const mpr_server_options &o) { return (int)((o.max_n - 1) / o.baby); }

// A ladder's pinned word copy: words 1 .. B + 3 of its scalar block, i.e.
// the B baby traces, one unused word, the status word and the byte-copy
// flag (each int32 in the low half of its word).
static inline int info_words(int B) { return B + 3; }
static inline int32_t info_status(volatile const int64_t *info, int B)
{
    return ((volatile const int32_t *)(info + B + 1))[0];
}
static inline int32_t info_wide(volatile const int64_t *info, int B)
{
    return ((volatile const int32_t *)(info + B + 2))[0];
}

// Ring powers of a period-mode search: confirms periods up to 7.
constexpr int kPeriodSlots = 8;
constexpr int kPeriodFlags = MPR_PERIOD_SPARSE | MPR_PERIOD_EXTEND | MPR_PERIOD_PIPELINE;

// Device bytes of a period-mode build of m: A, then the search's workspace
// (sized with a compressed-K plan for a dense A, since the bytes are
// admitted before A exists; the search sizes the plan for A itself and
// gives the rest to its ring).  Released when the build ends.
static size_t period_build_bytes(int m, int64_t *n_out, int64_t *ld_out)
{
    const int64_t n = transfer_size(m), ld = round_up(n, 8);
    size_t ws = 0;
    if (mpr_period_workspace_size_ex(n, kPeriodSlots, kPeriodFlags, &ws) != MPR_OK) return SIZE_MAX;
    if (n_out) *n_out = n;
    if (ld_out) *ld_out = ld;
    return (size_t)round_up(n * ld * 2, 256) + ws;
}

// Device bytes a build of m takes in this server's mode.
static size_t build_bytes(const Server &S, int m)
{
    if (S.opt.period_mode) return period_build_bytes(m, nullptr, nullptr);
    return ladder_bytes(m, S.opt.baby, giant_count(S.opt), !S.opt.wide_only, nullptr, nullptr);
}

// Starts a period-mode build of L.m on its own thread and stream.
static mpr_status start_period_build(Server &S, Ladder &L)
{
    L.bytes = period_build_bytes(L.m, &L.n, &L.ld);
    if (L.bytes == SIZE_MAX) return MPR_EINVAL;
    if (hipMalloc(&L.mem, L.bytes) != hipSuccess) return MPR_ENOMEM;
    auto pb = std::make_shared<PeriodBuild>();
    pb->traces.assign((size_t)S.opt.max_n + 1, ROW_NONE);
    const int dev = S.device, m = L.m;
    const int64_t n = L.n, ld = L.ld, kmax = S.opt.max_n;
    char *mem = (char *)L.mem;
    const size_t bytes = L.bytes, mat = (size_t)round_up(n * ld * 2, 256);
    PeriodBuild *b = pb.get();  // owned by the ladder until the worker joins the thread
    try {
        pb->th = std::thread([b, dev, m, n, ld, kmax, mem, bytes, mat]() {
            mpr_status e = hipSetDevice(dev) == hipSuccess ? MPR_OK : MPR_EHIP;
            hipStream_t s = nullptr;
            if (e == MPR_OK && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) e = MPR_EHIP;
            if (e == MPR_OK) e = transfer_launch(m, (u16 *)mem, ld, s);
            int64_t mu = 0, lam = 0, c = 0;
            if (e == MPR_OK)
                e = mpr_find_period_ex((const uint16_t *)mem, n, ld, kmax, kPeriodFlags, &mu, &lam, &c,
                                       b->traces.data(), mem + mat, bytes - mat, (mpr_stream)s);
            if (e == MPR_ENOTFOUND) e = MPR_OK;  // no repeat up to max_n: every trace was computed directly
            if (s) {
                if (hipStreamSynchronize(s) != hipSuccess && e == MPR_OK) e = MPR_EHIP;
                (void)hipStreamDestroy(s);
            }
            b->status = e;
            b->done.store(true, std::memory_order_release);
        });
    } catch (...) {
        return MPR_EHIP;
    }
    L.pb = pb;
    L.period = true;
    L.state = Ladder::BUILDING;
    L.build_s0 = S.now();
    S.resident += L.bytes;
    stats_update(S, [](mpr_server_stats &t) { t.builds++; });
    return MPR_OK;
}

// Giant products are scheduled across the ladders being built, shortest
// first: a small ladder (N < kBigLadder, products of microseconds) keeps up
// to kSmallAhead of its products enqueued; of the large ones (milliseconds
// to a third of a second each) at most one product is enqueued at a time,
// taken from the ladder with the least N.  So a launch behind the build on
// a shared hardware queue waits for at most one large product, and a
// smaller ladder is never stuck behind a larger one's products (the
// worker's tick between two large products costs well under 1 %).
constexpr int64_t kBigLadder = 4096;
constexpr int kSmallAhead = 8;

// Giant products of L enqueued and not yet finished.
static inline int giants_in_flight(const Ladder &L) { return (L.next_giant - 1) - std::max(L.avail, 1); }

// The build's words into the pinned copy (L.info), ahead of an event.
static mpr_status publish_build(Server &S, Ladder &L)
{
    return hipMemcpyAsync((void *)L.info, L.scal + 1, 8 * (size_t)info_words(S.opt.baby), hipMemcpyDeviceToHost,
                          S.bstream) == hipSuccess
               ? MPR_OK
               : MPR_EHIP;
}

// Byte copy of one finished ladder matrix for the query pass (half the
// bytes per query); ladder buffers are 256-byte aligned.
static mpr_status pack_build(Server &S, Ladder &L, const u16 *src, uint8_t *dst)
{
    if (S.opt.wide_only || L.n == 0) return MPR_OK;
    hipLaunchKernelGGL(pack8_kernel, dim3((unsigned)L.n), dim3(256), 0, S.bstream, src, L.ld, dst, L.ld8, L.n,
                       L.ld % 8 == 0 ? 1 : 0, L.wide_dev);
    return check_launch();
}

// The build's last words and its `ready` event, after everything enqueued.
static mpr_status finish_build(Server &S, Ladder &L)
{
    mpr_status e = publish_build(S, L);
    if (hipEventRecord(L.ready, S.bstream) != hipSuccess) {
        // Unrecorded, the event reads as complete: wait here for the work
        // already enqueued instead.
        (void)hipStreamSynchronize(S.bstream);
        e = MPR_EHIP;
    }
    L.submitted = true;
    return e;
}

// Enqueues giants L.next_giant .. upto (each with its byte copy, the words
// and its event), then finishes the build once the last one is enqueued.
// A failure marks the build failing and finishes it.
static mpr_status enqueue_giants(Server &S, Ladder &L, int upto)
{
    const int G = (int)L.step_ev.size() - 1;
    const int64_t n = L.n, ld = L.ld;
    hipStream_t s = S.bstream;
    mpr_status e = MPR_OK;
    for (; !L.failing && L.next_giant <= std::min(upto, G) && e == MPR_OK; L.next_giant++) {
        const int i = L.next_giant;
        // large products leave one workgroup slot per CU to the queries
        // that run beside the build
        e = n >= kBigLadder ? gemm_launch_spare(-1, n, n, n, L.Ng[i - 1], ld, L.Bp, ld, L.Ng[i], ld, s)
                            : gemm_launch(-1, n, n, n, L.Ng[i - 1], ld, L.Bp, ld, L.Ng[i], ld, s);
        if (e == MPR_OK)
            e = normalise_launch(n, n, L.Ng[i], ld, L.Rg[i - 1], L.scal, L.Rg[i], L.status_dev, nullptr, s);
        if (e == MPR_OK) e = pack_build(S, L, L.Ng[i], L.Ng8[i]);
        if (e == MPR_OK) e = publish_build(S, L);
        if (e == MPR_OK && hipEventRecord(L.step_ev[i], s) != hipSuccess) e = MPR_EHIP;
    }
    if (e != MPR_OK) L.failing = true;
    if (!L.submitted && (L.failing || L.next_giant > G)) {
        const mpr_status f = finish_build(S, L);
        if (e == MPR_OK) e = f;
        if (f != MPR_OK) L.failing = true;
    }
    return e;
}

// Enqueues a ladder build on the build stream: A, the chain to A^B, the
// babies and their traces at once, then the first giant products (the
// worker enqueues the rest as earlier ones finish).
static mpr_status start_build(Server &S, Ladder &L)
{
    const int B = S.opt.baby, G = giant_count(S.opt);
    const bool bytes8 = !S.opt.wide_only;
    L.bytes = ladder_bytes(L.m, B, G, bytes8, &L.n, &L.ld);
    if (hipMalloc(&L.mem, L.bytes) != hipSuccess) return MPR_ENOMEM;
    const int64_t n = L.n, ld = L.ld;
    const size_t mat = (size_t)round_up(n * ld * 2, 256), vec = (size_t)round_up(n * 8, 256);
    char *p = (char *)L.mem;
    auto take_mat = [&]() { u16 *r = (u16 *)p; p += mat; return r; };
    auto take_vec = [&]() { int64_t *r = (int64_t *)p; p += vec; return r; };
    u16 *A = take_mat();
    (void)take_vec();
    L.Nb.assign(B + 1, nullptr);
    L.Rb.assign(B + 1, nullptr);
    for (int j = 1; j <= B; j++) {
        L.Nb[j] = take_mat();
        L.Rb[j] = take_vec();
    }
    L.Ng.assign(G + 1, nullptr);
    L.Rg.assign(G + 1, nullptr);
    for (int i = 1; i <= G; i++) {
        L.Ng[i] = take_mat();
        L.Rg[i] = take_vec();
    }
    u16 *Bp = take_mat();
    int64_t *Rp = take_vec();
    int64_t *scal = (int64_t *)p;  // [0] s of the fold, [1..B] traces, the status word, the byte-copy flag
    p += round_up((int64_t)(B + 8) * 8, 256);
    void *plan = p;
    const size_t plan_bytes = sparse_plan_bytes(n);
    p += plan_bytes;
    L.trace_dev = scal + 1;
    L.status_dev = (int32_t *)(scal + 2 + B);
    L.wide_dev = (int32_t *)(scal + 3 + B);
    L.info = S.info_host + (size_t)L.m * info_words(B);  // words 1 .. B + 3 of scal
    L.ld8 = round_up(n, 16);
    const size_t mat8 = (size_t)round_up(n * L.ld8, 256);
    L.Nb8.assign(B + 1, nullptr);
    L.Ng8.assign(G + 1, nullptr);
    if (bytes8) {
        for (int j = 1; j <= B; j++, p += mat8) L.Nb8[j] = (uint8_t *)p;
        for (int i = 1; i <= G; i++, p += mat8) L.Ng8[i] = (uint8_t *)p;
    }
    hipStream_t s = S.bstream;
    L.scal = scal;
    auto pack = [&](const u16 *src, uint8_t *dst) { return pack_build(S, L, src, dst); };
    L.step_ev.assign(G + 1, nullptr);
    for (int i = 1; i <= G; i++)
        if (hipEventCreateWithFlags(&L.step_ev[i], hipEventDisableTiming) != hipSuccess) return MPR_EHIP;
    if (hipEventCreateWithFlags(&L.ready, hipEventDisableTiming) != hipSuccess) return MPR_EHIP;
    mpr_status e = fill_i32_launch(L.status_dev, 1, 0, s);
    if (e == MPR_OK) e = fill_i32_launch(L.wide_dev, 1, 0, s);
    if (e == MPR_OK) e = transfer_launch(L.m, A, ld, s);
    // The first giant A^B by the compressed-K chain on A (A stays sparse;
    // identical results), alternating between Ng[1] and Bp so that step B
    // lands in Ng[1].
    if (G >= 1) {
        u16 *buf[2] = {L.Ng[1], Bp};
        int64_t *R[2] = {L.Rg[1], Rp};
        int b = (B - 1) & 1;
        if (e == MPR_OK) e = copy_launch(A, ld, buf[b], ld, n, n, s);
        if (e == MPR_OK) e = normalise_launch(n, n, buf[b], ld, nullptr, nullptr, R[b], L.status_dev, nullptr, s);
        if (e == MPR_OK && B >= 2) e = sparse_plan_launch(A, n, ld, plan, plan_bytes, L.status_dev, s);
        for (int k = 2; k <= B && e == MPR_OK; k++) {
            e = sparse_step_launch(buf[b], ld, n, plan, plan_bytes, buf[b ^ 1], ld, s);
            if (e == MPR_OK)
                e = normalise_launch(n, n, buf[b ^ 1], ld, R[b], nullptr, R[b ^ 1], L.status_dev, nullptr, s);
            b ^= 1;
        }
    }
    // Baby steps: the canonical forms of (A^T)^j = (A^j)^T by the same chain
    // on A^T (plan built from the raw A^T before it is normalised in place).
    if (e == MPR_OK) e = transpose_launch(A, ld, L.Nb[1], ld, n, s);
    if (e == MPR_OK && B >= 2) e = sparse_plan_launch(L.Nb[1], n, ld, plan, plan_bytes, L.status_dev, s);
    if (e == MPR_OK) e = normalise_launch(n, n, L.Nb[1], ld, nullptr, nullptr, L.Rb[1], L.status_dev, nullptr, s);
    for (int j = 2; j <= B && e == MPR_OK; j++) {
        e = sparse_step_launch(L.Nb[j - 1], ld, n, plan, plan_bytes, L.Nb[j], ld, s);
        if (e == MPR_OK)
            e = normalise_launch(n, n, L.Nb[j], ld, L.Rb[j - 1], nullptr, L.Rb[j], L.status_dev, nullptr, s);
    }
    for (int j = 1; j <= B && e == MPR_OK; j++) e = trace_launch(L.Nb[j], n, ld, L.Rb[j], L.trace_dev + (j - 1), s);
    for (int j = 1; j <= B && e == MPR_OK; j++) e = pack(L.Nb[j], L.Nb8[j]);
    // Then the giants in order, each announced by its event once written
    // (with its byte copy): the queries that need no later giant go ahead.
    if (G >= 1 && e == MPR_OK) e = pack(L.Ng[1], L.Ng8[1]);
    if (G >= 1 && e == MPR_OK) e = publish_build(S, L);
    if (G >= 1 && e == MPR_OK && hipEventRecord(L.step_ev[1], s) != hipSuccess) e = MPR_EHIP;
    if (G >= 2 && e == MPR_OK) e = fold_launch(L.Ng[1], ld, L.Rg[1], n, n, Bp, ld, scal, L.status_dev, s);
    if (e != MPR_OK) return e;
    L.Bp = Bp;
    L.next_giant = 2;
    (void)enqueue_giants(S, L, 1);  // no giant yet (the worker schedules them); finishes when G <= 1
    L.state = Ladder::BUILDING;
    L.build_s0 = S.now();
    S.resident += L.bytes;
    stats_update(S, [](mpr_server_stats &t) { t.builds++; });
    return MPR_OK;
}

static void free_ladder(Server &S, Ladder &L)
{
    if (L.pb && L.pb->th.joinable()) L.pb->th.join();  // a period-mode build still running
    if (L.ready) (void)hipEventDestroy(L.ready);
    for (hipEvent_t ev : L.step_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (L.mem) (void)hipFree(L.mem);
    S.resident -= L.bytes;
    L = Ladder();
}

static void complete(Server &S, const Request &r, int64_t gamma, int status, double t_start)
{
    mpr_query_result q;
    q.tag = r.tag;
    q.m = r.m;
    q.n = r.n;
    q.gamma = gamma;
    q.status = status;
    q.t_submit_s = r.t_submit;
    q.t_start_s = t_start;
    q.t_done_s = S.now();
    q.cold = r.cold ? 1 : 0;
    std::lock_guard<std::mutex> lk(S.mu);
    S.outbox.push_back(q);
    S.stats.completed++;
    S.cv_out.notify_all();
}

// Device memory free right now (0 if it can not be read).
static size_t free_device_bytes()
{
    size_t fr = 0, total = 0;
    if (hipMemGetInfo(&fr, &total) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return fr;
}

// Headroom kept free on the device beyond a ladder's own bytes.
constexpr size_t kFreeMargin = (size_t)256 << 20;

// Try to admit ladder m; evicts idle ladders LRU until the ladder fits both
// the byte budget and the device's free memory.  True when building (or
// failed, the failure recorded for the waiting requests); false when it
// must wait for memory that a running build or query will release.
static bool admit(Server &S, int m)
{
    const size_t need = build_bytes(S, m);
    if (need > S.opt.hbm_budget_bytes) return false;
    for (;;) {
        const bool budget_ok = S.resident + need <= S.opt.hbm_budget_bytes;
        const bool free_ok = need + kFreeMargin <= free_device_bytes();
        if (budget_ok && free_ok) break;
        Ladder *victim = nullptr;
        bool busy = false;  // some ladder of this server will release memory later
        for (auto &kv : S.ladders) {
            Ladder &L = kv.second;
            busy |= L.state == Ladder::BUILDING || (L.state == Ladder::READY && L.inflight > 0);
            if (L.state != Ladder::READY || L.inflight > 0 || !S.waiting[kv.first].empty() || L.bytes == 0)
                continue;  // (a period-mode table holds no device memory)
            if (!victim || L.last_use < victim->last_use) victim = &L;
        }
        if (victim) {
            free_ladder(S, *victim);
            stats_update(S, [](mpr_server_stats &t) { t.evictions++; });
            continue;
        }
        if (!budget_ok || busy) return false;  // wait: our own memory comes back later
        // Within the budget, but the device does not have the memory and
        // nothing of this server can release it: fail the build (the waiting
        // requests get MPR_ENOMEM; a later request tries again).
        Ladder &L = S.ladders[m];
        L.m = m;
        L.state = Ladder::FAILED;
        L.fail_status = MPR_ENOMEM;
        return true;
    }
    Ladder &L = S.ladders[m];
    L.m = m;
    const mpr_status e = S.opt.period_mode ? start_period_build(S, L) : start_build(S, L);
    if (e != MPR_OK) {
        if (L.mem) {
            (void)hipStreamSynchronize(S.bstream);  // part of the build may be enqueued
            (void)hipFree(L.mem);
            L.mem = nullptr;
        }
        if (L.ready) {
            (void)hipEventDestroy(L.ready);
            L.ready = nullptr;
        }
        for (hipEvent_t &ev : L.step_ev)
            if (ev) {
                (void)hipEventDestroy(ev);
                ev = nullptr;
            }
        L.state = Ladder::FAILED;
        L.fail_status = e;
    }
    return true;  // building, or failed (reported to the waiting requests)
}

// One grouped launch of `batch` on a free slot's stream.
static void launch_batch(Server &S, Slot *slot, std::vector<Request> &batch)
{
    if (!slot || batch.empty()) return;
    const int64_t B = S.opt.baby;
    // Queries on byte copies that share a giant power (same m and i)
    // go in groups of up to TR_GROUP, which read it once; the order
    // of the batch follows the groups.
    std::stable_sort(batch.begin(), batch.end(), [B](const Request &x, const Request &y) {
        const int64_t ix = (x.n - 1) / B, iy = (y.n - 1) / B;
        return x.m != y.m ? x.m < y.m : ix < iy;
    });
    int64_t blocks = 0, shared = 0;
    int lead = 0;
    for (size_t q = 0; q < batch.size(); q++) {
        const Request &r = batch[q];
        Ladder &L = S.ladders[r.m];
        const int64_t i = (r.n - 1) / B, j = r.n - B * i;
        const int vec = aligned16(L.Ng[i]) && aligned16(L.Nb[j]) && L.ld % 8 == 0;
        const TRDesc &head = slot->desc_host[lead];  // of the group the query may join
        const bool join = q > 0 && L.narrow && head.narrow && head.X8 == L.Ng8[i] && head.gsize < TR_GROUP;
        if (!join) lead = (int)q;
        const int64_t first = join ? head.first_block : blocks;
        slot->desc_host[q] = TRDesc{L.Ng[i], L.Rg[i], L.Nb[j], L.Rb[j], L.Ng8[i], L.Nb8[j],
                                    L.n,     L.ld,     L.ld8,    first,    vec,      L.narrow ? 1 : 0,
                                    (int)q - lead, 1};
        if (join) {
            slot->desc_host[lead].gsize++;
            shared++;
        } else
            blocks += trace_blocks(L.n);
        L.inflight++;
        L.last_use = S.now();
    }
    const int nq = (int)batch.size();
    hipStream_t s = slot->stream;
    bool ok = hipMemcpyAsync(slot->desc_dev, slot->desc_host, sizeof(TRDesc) * nq, hipMemcpyHostToDevice,
                             s) == hipSuccess;
    const int64_t pitch = slot_pitch(nq);
    const int words = (int)(TR_SLOTS * pitch);
    hipLaunchKernelGGL(fill_none_kernel, dim3((words + 255) / 256), dim3(256), 0, s, slot->out_dev, words);
    hipLaunchKernelGGL(grouped_trace_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, slot->desc_dev,
                       nq, pitch, slot->out_dev);
    ok = ok && hipGetLastError() == hipSuccess;
    ok = ok && hipMemcpyAsync(slot->out_host, slot->out_dev, 8 * (size_t)words, hipMemcpyDeviceToHost, s) ==
                   hipSuccess;
    ok = ok && hipEventRecord(slot->done, s) == hipSuccess;
    if (!ok) {
        S.fatal = "launch failed";
        for (auto &r : batch) {
            S.ladders[r.m].inflight--;
            complete(S, r, ROW_NONE, MPR_EHIP, S.now());
        }
        return;
    }
    slot->reqs = batch;
    slot->busy = true;
    slot->t_launch = S.now();
    stats_update(S, [nq, shared](mpr_server_stats &t) {
        t.batches++;
        t.shared_reads += shared;
        t.max_batch_seen = std::max<int64_t>(t.max_batch_seen, nq);
    });
}

static void worker_main(Server *Sp)
{
    Server &S = *Sp;
    (void)hipSetDevice(S.device);
    // The short waits below bound the completion latency only if the kernel
    // keeps them short: the default timer slack of a thread (50 us) would
    // stretch every 5 us wait to about 55 us.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    const int B = S.opt.baby;
    for (;;) {
        std::vector<Request> fresh;
        std::vector<int64_t> cancels;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            // A finished query launch is seen on the next pass, so the wait is
            // short while launches are in flight (it bounds the completion
            // latency); builds and admission are polled more slowly.
            bool queries = false, other = !S.admission.empty();
            for (auto &sl : S.slots) queries |= sl.busy;
            for (auto &kv : S.ladders) other |= kv.second.state == Ladder::BUILDING;
            const int wait_us = queries ? 5 : other ? 50 : 2000;
            if (S.inbox.empty() && S.cancels.empty() && !S.stop) {
                if (S.opt.busy_poll) {
                    lk.unlock();
                    std::this_thread::yield();
                    lk.lock();
                } else {
                    S.cv_in.wait_for(lk, std::chrono::microseconds(wait_us));
                }
            }
            if (S.stop) break;
            while (!S.inbox.empty()) {
                fresh.push_back(S.inbox.front());
                S.inbox.pop_front();
            }
            cancels.swap(S.cancels);
        }
        // 0. cancellations and deadlines of requests not yet launched
        if (!cancels.empty() || S.opt.request_timeout_s > 0) {
            const double now = S.now(), limit = S.opt.request_timeout_s;
            auto drop = [&](const Request &r) {
                if (std::find(cancels.begin(), cancels.end(), r.tag) != cancels.end()) {
                    complete(S, r, ROW_NONE, MPR_ECANCELED, now);
                    return true;
                }
                if (limit > 0 && now - r.t_submit > limit) {
                    complete(S, r, ROW_NONE, MPR_ETIMEDOUT, now);
                    return true;
                }
                return false;
            };
            fresh.erase(std::remove_if(fresh.begin(), fresh.end(), drop), fresh.end());
            for (auto &kv : S.waiting) kv.second.erase(std::remove_if(kv.second.begin(), kv.second.end(), drop),
                                                       kv.second.end());
            cancels.clear();
        }
        // 1. retire finished batches
        for (auto &sl : S.slots) {
            if (!sl.busy || hipEventQuery(sl.done) != hipSuccess) continue;
            const int64_t pitch = slot_pitch((int64_t)sl.reqs.size());
            for (size_t q = 0; q < sl.reqs.size(); q++) {
                const Request &r = sl.reqs[q];
                Ladder &L = S.ladders[r.m];
                L.inflight--;
                int64_t g = ROW_NONE;
                for (int k = 0; k < TR_SLOTS; k++) g = std::min(g, sl.out_host[k * pitch + (int64_t)q]);
                complete(S, r, g, MPR_OK, sl.t_launch);
            }
            sl.reqs.clear();
            sl.busy = false;
        }
        // 2. builds that finished
        for (auto &kv : S.ladders) {
            Ladder &L = kv.second;
            if (L.state != Ladder::BUILDING || !L.period) continue;
            if (!L.pb->done.load(std::memory_order_acquire)) continue;
            L.pb->th.join();
            const mpr_status st = L.pb->status;
            L.build_s = S.now() - L.build_s0;
            L.last_use = S.now();
            if (st == MPR_OK) {
                L.table = std::move(L.pb->traces);
                L.pb.reset();
                (void)hipFree(L.mem);  // the table is all a period-mode query reads
                L.mem = nullptr;
                S.resident -= L.bytes;
                L.bytes = 0;
                L.state = Ladder::READY;
            } else {
                free_ladder(S, L);
                L.m = kv.first;
                L.state = Ladder::FAILED;
                L.fail_status = st;
            }
        }
        // The status word, the byte-copy flag and (first time) the baby
        // traces, from the pinned copy the build wrote before the event
        // just seen complete.
        auto read_build = [&](Ladder &L, bool traces) {
            const int32_t st = info_status(L.info, B), wide = info_wide(L.info, B);
            if (traces) {
                L.baby_trace.assign(B + 1, ROW_NONE);
                for (int j = 1; j <= B; j++) L.baby_trace[j] = L.info[j - 1];
            }
            // The flag only rises: a launch that read byte copies did so
            // while every copy it read was known to fit.
            L.narrow = !S.opt.wide_only && wide == 0;
            return st;
        };
        for (auto &kv : S.ladders) {
            Ladder &L = kv.second;
            if (L.state != Ladder::BUILDING || L.period) continue;
            // Events complete in order: find the last one passed (among the
            // recorded ones: an event never recorded reads as complete), then
            // read the words once for all of them.
            const int G = (int)L.step_ev.size() - 1;
            const int recorded = std::min(G, L.next_giant - 1);
            int k = L.avail;
            while (!L.failing && k < recorded && hipEventQuery(L.step_ev[k + 1]) == hipSuccess) k++;
            if (k > L.avail) {
                if (read_build(L, L.avail == 0) == 0)
                    L.avail = k;
                else
                    L.failing = true;  // reported once the build's last event has passed
            }
        }
        {  // schedule the next giant products (shortest ladder first)
            std::vector<Ladder *> order;
            int big = 0;
            for (auto &kv : S.ladders) {
                Ladder &L = kv.second;
                if (L.state != Ladder::BUILDING || L.period || L.submitted) continue;
                order.push_back(&L);
                if (L.n >= kBigLadder) big += giants_in_flight(L);
            }
            std::sort(order.begin(), order.end(), [](const Ladder *x, const Ladder *y) { return x->n < y->n; });
            for (Ladder *L : order) {
                const int from = std::max(L->avail, 1);
                if (L->failing)
                    (void)enqueue_giants(S, *L, 0);  // finishes the build
                else if (L->n < kBigLadder)
                    (void)enqueue_giants(S, *L, from + kSmallAhead);
                else if (big == 0) {
                    (void)enqueue_giants(S, *L, from + 1);
                    big += giants_in_flight(*L);
                }
            }
        }
        for (auto &kv : S.ladders) {
            Ladder &L = kv.second;
            if (L.state != Ladder::BUILDING || L.period) continue;
            const int G = (int)L.step_ev.size() - 1;
            if (!L.submitted || hipEventQuery(L.ready) != hipSuccess) continue;
            const int32_t st = L.failing ? MPR_EHIP : read_build(L, L.avail == 0);
            if (st == 0) {
                if (L.narrow) stats_update(S, [](mpr_server_stats &t) { t.narrow_builds++; });
                L.build_s = S.now() - L.build_s0;
                L.last_use = S.now();
                L.avail = G;
                L.state = Ladder::READY;
                continue;
            }
            // The build is done with its memory: once no launch reads it any
            // more, release it and keep the verdict.
            L.failing = true;
            if (L.inflight > 0) continue;
            int32_t why = info_status(L.info, B);
            if (why == 0) why = MPR_EHIP;
            free_ladder(S, L);
            L.m = kv.first;
            L.state = Ladder::FAILED;
            L.fail_status = why;
        }
        // 3. route new requests
        for (auto &r : fresh) {
            if (r.m < 1 || r.m > 11 || r.n < 3 || r.n > S.opt.max_n) {
                complete(S, r, ROW_NONE, MPR_EINVAL, S.now());
                continue;
            }
            if (build_bytes(S, r.m) > S.opt.hbm_budget_bytes) {
                complete(S, r, ROW_NONE, MPR_ENOMEM, S.now());  // could never be admitted
                continue;
            }
            auto it = S.ladders.find(r.m);
            if (it == S.ladders.end() || it->second.state == Ladder::NONE) {
                r.cold = true;
                bool queued = std::find(S.admission.begin(), S.admission.end(), r.m) != S.admission.end();
                if (!queued && !admit(S, r.m)) {
                    S.admission.push_back(r.m);
                    stats_update(S, [](mpr_server_stats &t) { t.admission_waits++; });
                }
            } else if (it->second.state == Ladder::BUILDING) {
                r.cold = true;
            }
            S.waiting[r.m].push_back(r);
        }
        // 4. admission queue (memory may have been released)
        for (size_t k = 0; k < S.admission.size();) {
            const int m = S.admission[k];
            if (admit(S, m))
                S.admission.erase(S.admission.begin() + k);
            else
                k++;
        }
        // 5. one grouped launch for everything that is ready, and one on the
        // early stream for queries of ladders still building: their passes
        // share the device with the build's products, and behind them on
        // one stream the warm queries would wait for those products too.
        Slot *slot = nullptr, *eslot = nullptr;
        for (auto &sl : S.slots)
            if (!sl.busy) {
                Slot *&to = sl.stream == S.estream ? eslot : slot;
                if (!to) to = &sl;
            }
        std::vector<Request> batch, ebatch;
        int64_t batch_blocks = 0, ebatch_blocks = 0;  // grids of the grouped launches
        for (auto &kv : S.waiting) {
            Ladder &L = S.ladders[kv.first];
            if (L.state == Ladder::FAILED) {
                // Report the failure to the requests that waited for this
                // build, then forget it: a later request builds again (a
                // failure may be transient, e.g. memory another process held).
                for (auto &r : kv.second) complete(S, r, ROW_NONE, L.fail_status, S.now());
                kv.second.clear();
                L = Ladder();
                continue;
            }
            // A ready ladder answers every query; one still building, those
            // whose giant is already written.
            const bool early = L.state == Ladder::BUILDING && !L.period && !L.failing && L.avail >= 1;
            if (L.state != Ladder::READY && !early) continue;
            auto &dq = kv.second;
            if (L.period) {  // the labelled fast mode: a table read per query
                const int64_t cnt = (int64_t)dq.size();
                for (; !dq.empty(); dq.pop_front()) complete(S, dq.front(), L.table[dq.front().n], MPR_OK, S.now());
                L.last_use = S.now();
                if (cnt) stats_update(S, [cnt](mpr_server_stats &t) { t.period_answers += cnt; });
                continue;
            }
            int64_t answered_early = 0;
            for (auto it = dq.begin(); it != dq.end();) {
                const Request r = *it;
                const int64_t i = (r.n - 1) / B, j = r.n - B * i;
                if (i > L.avail) {  // its giant is not written yet (only while building)
                    ++it;
                    continue;
                }
                if (i == 0) {  // read off the build's trace of A^j
                    it = dq.erase(it);
                    L.last_use = S.now();
                    answered_early += early;
                    complete(S, r, L.baby_trace[j], MPR_OK, S.now());
                    continue;
                }
                const int64_t qb = trace_blocks(L.n);
                Slot *to = early ? eslot : slot;
                std::vector<Request> &tb = early ? ebatch : batch;
                int64_t &tbb = early ? ebatch_blocks : batch_blocks;
                if (!to || (int)tb.size() >= S.opt.max_batch || tbb + qb > INT32_MAX) break;
                it = dq.erase(it);
                answered_early += early;
                tb.push_back(r);
                tbb += qb;
            }
            if (answered_early)
                stats_update(S, [answered_early](mpr_server_stats &t) { t.early_answers += answered_early; });
        }
        launch_batch(S, slot, batch);
        launch_batch(S, eslot, ebatch);
        stats_update(S, [&S](mpr_server_stats &t) { t.resident_bytes = (int64_t)S.resident; });
    }
}

}  // namespace mpr

using namespace mpr;

extern "C" mpr_status mpr_server_create(const mpr_server_options *opt, void **server_host)
{
    if (!opt || !server_host) return MPR_EINVAL;
    if (opt->baby < 1 || opt->max_n < 3 || opt->max_batch < 1 || opt->slots < 1 || opt->slots > 64)
        return MPR_EINVAL;
    if (hipSetDevice(opt->device) != hipSuccess) return MPR_EUNSUPPORTED;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    Server *S = new Server();
    S->opt = *opt;
    S->device = opt->device;
    memset(&S->stats, 0, sizeof(S->stats));
    S->t0 = Clock::now();
    bool ok = hipStreamCreateWithFlags(&S->qstream, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&S->bstream, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&S->estream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&S->info_host, 8 * (size_t)12 * (size_t)info_words(opt->baby)) == hipSuccess;
    S->slots.resize(opt->slots + 1);  // the last one launches on the early stream
    for (size_t k = 0; k < S->slots.size(); k++) {
        Slot &sl = S->slots[k];
        sl.stream = k + 1 < S->slots.size() ? S->qstream : S->estream;
        ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&sl.desc_host, sizeof(TRDesc) * opt->max_batch) == hipSuccess;
        const size_t words = (size_t)TR_SLOTS * (size_t)slot_pitch(opt->max_batch);
        ok = ok && hipHostMalloc((void **)&sl.out_host, 8 * words) == hipSuccess;
        ok = ok && hipMalloc((void **)&sl.desc_dev, sizeof(TRDesc) * opt->max_batch) == hipSuccess;
        ok = ok && hipMalloc((void **)&sl.out_dev, 8 * words) == hipSuccess;
    }
    if (!ok) {
        mpr_server_destroy(S);
        return MPR_EHIP;
    }
    S->worker = std::thread(worker_main, S);
    *server_host = S;
    return MPR_OK;
}

extern "C" mpr_status mpr_server_submit(void *server, int m, int64_t n, int64_t tag)
{
    Server *S = (Server *)server;
    if (!S) return MPR_EINVAL;
    Request r;
    r.tag = tag;
    r.m = m;
    r.n = n;
    r.t_submit = S->now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->inbox.push_back(r);
        S->stats.submitted++;
    }
    S->cv_in.notify_one();
    return MPR_OK;
}

extern "C" mpr_status mpr_server_cancel(void *server, int64_t tag)
{
    Server *S = (Server *)server;
    if (!S) return MPR_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cancels.push_back(tag);
    }
    S->cv_in.notify_one();
    return MPR_OK;
}

extern "C" mpr_status mpr_server_poll(void *server, mpr_query_result *out_host, int capacity, int *count_host,
                                      int wait_ms)
{
    Server *S = (Server *)server;
    if (!S || !out_host || !count_host || capacity < 1) return MPR_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->outbox.empty() && wait_ms > 0) S->cv_out.wait_for(lk, std::chrono::milliseconds(wait_ms));
    int c = 0;
    while (c < capacity && !S->outbox.empty()) {
        out_host[c++] = S->outbox.front();
        S->outbox.pop_front();
    }
    *count_host = c;
    return MPR_OK;
}

extern "C" mpr_status mpr_server_stats_get(void *server, mpr_server_stats *out_host)
{
    Server *S = (Server *)server;
    if (!S || !out_host) return MPR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out_host = S->stats;
    return MPR_OK;
}

extern "C" double mpr_server_now(void *server)
{
    Server *S = (Server *)server;
    return S ? S->now() : 0.0;
}

extern "C" int64_t mpr_server_ladder_bytes(int m, int baby, int64_t max_n, int wide_only)
{
    if (m < 1 || m > 11 || baby < 1 || max_n < 3) return -1;
    return (int64_t)ladder_bytes(m, baby, (int)((max_n - 1) / baby), wide_only == 0, nullptr, nullptr);
}

extern "C" int64_t mpr_server_period_bytes(int m)
{
    if (m < 1 || m > 11) return -1;
    const size_t b = period_build_bytes(m, nullptr, nullptr);
    return b == SIZE_MAX ? -1 : (int64_t)b;
}

extern "C" mpr_status mpr_server_destroy(void *server)
{
    Server *S = (Server *)server;
    if (!S) return MPR_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_in.notify_all();
    if (S->worker.joinable()) S->worker.join();
    if (S->qstream) (void)hipStreamSynchronize(S->qstream);
    if (S->bstream) (void)hipStreamSynchronize(S->bstream);
    if (S->estream) (void)hipStreamSynchronize(S->estream);
    for (auto &kv : S->ladders)
        if (kv.second.mem) free_ladder(*S, kv.second);
    for (auto &sl : S->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.desc_host) (void)hipHostFree(sl.desc_host);
        if (sl.out_host) (void)hipHostFree(sl.out_host);
        if (sl.desc_dev) (void)hipFree(sl.desc_dev);
        if (sl.out_dev) (void)hipFree(sl.out_dev);
    }
    if (S->qstream) (void)hipStreamDestroy(S->qstream);
    if (S->bstream) (void)hipStreamDestroy(S->bstream);
    if (S->estream) (void)hipStreamDestroy(S->estream);
    if (S->info_host) (void)hipHostFree(S->info_host);
    delete S;
    return MPR_OK;
}
