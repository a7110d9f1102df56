// abi.hip -- the extern "C" entry points of libmpr: argument checks, device
// set-up, workspace layouts, and the host-side schedules built from the
// kernels (chain and binary powering, products of canonical forms, the
// period search of Algorithm 2).
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "trace_rows.h"

namespace mpr {

mpr_status transfer_launch(int m, u16 *A, int64_t lda, hipStream_t s);
mpr_status border_transfer_launch(int m, u16 *A, int64_t lda, hipStream_t s);
int border_shift(int m);
int64_t transfer_size(int m);
void transfer_words(int m, uint8_t *out, int64_t count);

hipStream_t as_stream(mpr_stream s) { return reinterpret_cast<hipStream_t>(s); }

mpr_status check_launch()
{
    return hipGetLastError() == hipSuccess ? MPR_OK : MPR_EHIP;
}

// Device memory of the allocation-free power entry point
// (mpr_minplus_power_noalloc): a fixed array that every GPU the library runs
// on holds from module load until the process ends.  Host code never uses
// its name as an address; it uses the per-device address that init records.
__device__ __align__(256) unsigned char scratch[MPR_NOALLOC_SCRATCH_BYTES];

static std::mutex g_init_mu;
static std::vector<int> g_cus;  // per device: CU count, 0 = not gfx950, -1 = unknown
static std::vector<void *> g_scratch;   // per device: device address of `scratch`, nullptr if unknown

static mpr_status init_device(int dev)
{
    std::lock_guard<std::mutex> lk(g_init_mu);
    if ((int)g_cus.size() <= dev) g_cus.resize(dev + 1, -1);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (g_cus[dev] > 0) return MPR_OK;
    if (g_cus[dev] == 0) return MPR_EUNSUPPORTED;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MPR_EHIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_cus[dev] = 0;
        return MPR_EUNSUPPORTED;
    }
    // The scratch array's address on this device, taken with the device
    // current (each GPU holds its own copy at its own address).
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MPR_EHIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return MPR_EHIP;
    void *p = nullptr;
    const hipError_t se = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev && hipSetDevice(cur) != hipSuccess) return MPR_EHIP;
    if (se != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the next launch check
        p = nullptr;
    }
    g_scratch[dev] = p;
    g_cus[dev] = prop.multiProcessorCount;
    return MPR_OK;
}

// Address of the current device's scratch copy (nullptr when unavailable).
static void *device_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_init_mu);
    return dev < (int)g_scratch.size() ? g_scratch[dev] : nullptr;
}

mpr_status ensure_init()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MPR_EUNSUPPORTED;
    return init_device(dev);
}

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(g_init_mu);
    return (dev < (int)g_cus.size() && g_cus[dev] > 0) ? g_cus[dev] : 256;
}

// ------------------------------------------------------------ workspace carving
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class X>
    X *take(size_t count)
    {
        used = (size_t)round_up((int64_t)used, 256);
        X *p = base ? (X *)(base + used) : nullptr;
        used += count * sizeof(X);
        return p;
    }
};

static bool ld_ok(int64_t ld, int64_t cols) { return ld >= (cols > 0 ? cols : 1); }

// Canonical product (Rc, C) = canon((Ra (+) A) (x) (Rb (+) B)) on carved scratch.
static mpr_status gemm_norm_impl(int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda, const int64_t *Ra,
                                 const u16 *B, int64_t ldb, const int64_t *Rb, u16 *C, int64_t ldc, int64_t *Rc,
                                 int64_t *s_scalar, u16 *Bp, int64_t ldp, int32_t *st, hipStream_t s)
{
    mpr_status e;
    if (Rb) {
        e = fold_launch(B, ldb, Rb, K, N, Bp, ldp, s_scalar, st, s);
        if (e != MPR_OK) return e;
        B = Bp;
        ldb = ldp;
    }
    e = gemm_launch(-1, M, N, K, A, lda, B, ldb, C, ldc, s);
    if (e != MPR_OK) return e;
    return normalise_launch(M, N, C, ldc, Ra, Rb ? s_scalar : nullptr, Rc, st, nullptr, s);
}

static size_t gemm_norm_ws(int64_t K, int64_t N, int64_t *ldp_out)
{
    const int64_t ldp = round_up(N > 0 ? N : 1, 8);
    Carver c(nullptr);
    c.take<int64_t>(1);
    c.take<u16>((size_t)(K * ldp));
    if (ldp_out) *ldp_out = ldp;
    return c.used + 256;
}

// ------------------------------------------------------------ powers
// splitk.hip: small products with the inner dimension split.
int splitk_parts(int64_t M, int64_t N, int64_t K);
size_t splitk_bytes(int64_t M, int64_t N, int parts);
mpr_status splitk_launch(int parts, int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda, const u16 *B,
                         int64_t ldb, u16 *C, int64_t ldc, u16 *P, hipStream_t s);

struct PowerWs {
    u16 *P, *acc, *Bp, *C;
    int64_t *RP, *Racc, *RC, *s;
    void *plan;         // compressed-K plan of A (MPR_CHAIN_SPARSE)
    size_t plan_bytes;  // its share of the workspace
    bool plan_full;     // sized for the worst case (any A fits)
    u16 *split;         // MPR_CHAIN: partial products of a split-k step, the rest of the workspace
    size_t split_bytes;
    int64_t ld;
    size_t bytes;       // needed (without the optional partial products)
};

// Workspace layout of mpr_minplus_power.  The compressed-K plan takes the
// rest of a workspace of ws_bytes, up to its worst case; ws_bytes = 0 (or
// more than needed) sizes it for the worst case.
static PowerWs carve_power(void *ws, int64_t n, int schedule, size_t ws_bytes = 0)
{
    PowerWs w{};
    w.ld = round_up(n > 0 ? n : 1, 8);
    Carver c(ws);
    w.P = c.take<u16>((size_t)(n * w.ld));
    if (schedule == MPR_SQUARE) {
        w.acc = c.take<u16>((size_t)(n * w.ld));
        w.Bp = c.take<u16>((size_t)(n * w.ld));
        w.C = c.take<u16>((size_t)(n * w.ld));
        w.RP = c.take<int64_t>((size_t)n);
        w.Racc = c.take<int64_t>((size_t)n);
        w.RC = c.take<int64_t>((size_t)n);
        w.s = c.take<int64_t>(1);
    }
    if (schedule == MPR_CHAIN_SPARSE) {
        const size_t at = (size_t)round_up((int64_t)c.used, 256), worst = sparse_plan_bytes(n);
        w.plan_bytes = (ws_bytes > at + 256 && ws_bytes - at - 256 < worst) ? ws_bytes - at - 256 : worst;
        w.plan_full = w.plan_bytes == worst;
        w.plan = c.take<char>(w.plan_bytes);
    }
    w.bytes = c.used + 256;
    if (schedule == MPR_CHAIN && ws_bytes > w.bytes + 256) {  // room for the partial products of small steps
        const size_t at = (size_t)round_up((int64_t)c.used, 256);
        w.split = ws ? (u16 *)((char *)ws + at) : nullptr;
        w.split_bytes = ws_bytes - at - 256;
    }
    return w;
}

// Workspace that mpr_power_workspace_size reports: the layout plus, for the
// chain of a small matrix, the partial products of its split-k steps.
static size_t power_ws_recommended(int64_t n, int schedule)
{
    const PowerWs w = carve_power(nullptr, n, schedule);
    size_t extra = 0;
    if (schedule == MPR_CHAIN && n > 0) extra = splitk_bytes(n, n, splitk_parts(n, n, n));
    return w.bytes + (extra ? extra + 256 : 0);
}

// e - 1 chain steps from a first power: A itself (normalised), or, when N0
// is given, the canonical form (N0, R0) of a power saved earlier, so a chain
// resumes where it stopped (row i of the next power needs row i of this one
// and A only).
static mpr_status power_chain(const u16 *A, int64_t n, int64_t lda, int64_t e, u16 *N_out, int64_t ldo,
                              int64_t *R_out, const PowerWs &w, int32_t *st, hipStream_t s, bool sparse,
                              const u16 *N0 = nullptr, const int64_t *R0 = nullptr, int64_t ld0 = 0)
{
    // Step k writes buffer (e - k) % 2, so step e lands in N_out.
    u16 *buf[2] = {N_out, w.P};
    const int64_t ld[2] = {ldo, w.ld};
    int b = (int)((e - 1) & 1);
    mpr_status r;
    if (N0) {
        r = N0 == buf[b] ? MPR_OK : copy_launch(N0, ld0, buf[b], ld[b], n, n, s);
        if (r == MPR_OK && R0 != R_out &&
            hipMemcpyAsync(R_out, R0, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
            r = MPR_EHIP;
    } else {
        r = copy_launch(A, lda, buf[b], ld[b], n, n, s);
        if (r == MPR_OK) r = normalise_launch(n, n, buf[b], ld[b], nullptr, nullptr, R_out, st, nullptr, s);
    }
    if (r == MPR_OK && sparse && e >= 2) r = sparse_plan_launch(A, n, lda, w.plan, w.plan_bytes, st, s);
    // a small matrix's steps split k when the workspace holds the partial products
    int parts = sparse ? 1 : splitk_parts(n, n, n);
    while (parts > 1 && splitk_bytes(n, n, parts) > w.split_bytes) parts--;
    for (int64_t k = 2; k <= e && r == MPR_OK; k++) {
        const int nb = b ^ 1;
        r = sparse ? sparse_step_launch(buf[b], ld[b], n, w.plan, w.plan_bytes, buf[nb], ld[nb], s)
                   : splitk_launch(parts, n, n, n, buf[b], ld[b], A, lda, buf[nb], ld[nb], w.split, s);
        if (r == MPR_OK) r = normalise_launch(n, n, buf[nb], ld[nb], R_out, nullptr, R_out, st, nullptr, s);
        b = nb;
    }
    return r;
}

static mpr_status power_square(const u16 *A, int64_t n, int64_t lda, int64_t e, u16 *N_out, int64_t ldo,
                               int64_t *R_out, const PowerWs &w, int32_t *st, hipStream_t s)
{
    u16 *P = w.P, *acc = w.acc, *C = w.C;
    int64_t *RP = w.RP, *Racc = w.Racc, *RC = w.RC;
    const int64_t ld = w.ld;
    mpr_status r = copy_launch(A, lda, P, ld, n, n, s);
    if (r == MPR_OK) r = normalise_launch(n, n, P, ld, nullptr, nullptr, RP, st, nullptr, s);
    bool have = false;
    while (r == MPR_OK) {
        if (e & 1) {
            if (!have) {
                r = copy_launch(P, ld, acc, ld, n, n, s);
                if (r == MPR_OK && hipMemcpyAsync(Racc, RP, (size_t)n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
                    r = MPR_EHIP;
                have = true;
            } else {
                r = gemm_norm_impl(n, n, n, acc, ld, Racc, P, ld, RP, C, ld, RC, w.s, w.Bp, ld, st, s);
                std::swap(acc, C);
                std::swap(Racc, RC);
            }
        }
        e >>= 1;
        if (!e || r != MPR_OK) break;
        r = gemm_norm_impl(n, n, n, P, ld, RP, P, ld, RP, C, ld, RC, w.s, w.Bp, ld, st, s);
        std::swap(P, C);
        std::swap(RP, RC);
    }
    if (r == MPR_OK) r = copy_launch(acc, ld, N_out, ldo, n, n, s);
    if (r == MPR_OK && hipMemcpyAsync(R_out, Racc, (size_t)n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        r = MPR_EHIP;
    return r;
}

// ------------------------------------------------------------ period search
// Process-wide observer of long period searches: called on the calling
// thread after every power (its index and trace).
static std::mutex g_progress_mu;
static void (*g_progress_fn)(int64_t, int64_t, void *) = nullptr;
static void *g_progress_user = nullptr;

static void report_progress(int64_t k, int64_t trace)
{
    void (*fn)(int64_t, int64_t, void *);
    void *user;
    {
        std::lock_guard<std::mutex> lk(g_progress_mu);
        fn = g_progress_fn;
        user = g_progress_user;
    }
    if (fn) fn(k, trace, user);
}

constexpr int kPeriodFlagsAll = MPR_PERIOD_SPARSE | MPR_PERIOD_EXTEND | MPR_PERIOD_REUSE_A | MPR_PERIOD_PIPELINE;

struct PeriodWs {
    uint64_t *row_hash;
    int64_t *hold_R;  // offsets of the power kept in A's buffer (MPR_PERIOD_REUSE_A)
    void *plan;
    size_t plan_bytes;
    int64_t *scal;  // [0] hash, [1] trace, [2] status (int32 in low half), [3..5] compare
    int64_t slots;
    int64_t ld;
    size_t slot_elems;  // u16 per slot (matrix) + R follows after padding
    char *slot_base;
    size_t slot_bytes;
    size_t fixed;
};

// Workspace layout of the period search: the per-row hashes and scalars,
// then (MPR_PERIOD_SPARSE) the compressed-K plan of plan_bytes (the worst
// case when 0), then the ring of power slots.
static PeriodWs carve_period(void *ws, int64_t n, size_t ws_bytes, int64_t slots_req, int flags,
                             size_t plan_bytes = 0)
{
    PeriodWs w{};
    w.ld = round_up(n > 0 ? n : 1, 8);
    Carver c(ws);
    w.row_hash = c.take<uint64_t>((size_t)n);
    w.scal = c.take<int64_t>(8);
    w.hold_R = (flags & MPR_PERIOD_REUSE_A) ? c.take<int64_t>((size_t)n) : nullptr;
    if (flags & MPR_PERIOD_SPARSE) {
        w.plan_bytes = plan_bytes ? plan_bytes : sparse_plan_bytes(n);
        w.plan = (void *)c.take<char>(w.plan_bytes);
    }
    w.fixed = (size_t)round_up((int64_t)c.used, 256);
    w.slot_elems = (size_t)(n * w.ld);
    w.slot_bytes = (size_t)round_up((int64_t)(w.slot_elems * 2), 256) + (size_t)round_up(n * 8, 256);
    w.slot_base = ws ? (char *)ws + w.fixed : nullptr;
    if (slots_req > 0)
        w.slots = slots_req;
    else
        w.slots = ws_bytes > w.fixed ? (int64_t)((ws_bytes - w.fixed) / w.slot_bytes) : 0;
    return w;
}

static inline u16 *slot_N(const PeriodWs &w, int64_t k) { return (u16 *)(w.slot_base + (size_t)k * w.slot_bytes); }
static inline int64_t *slot_R(const PeriodWs &w, int64_t k)
{
    return (int64_t *)(w.slot_base + (size_t)k * w.slot_bytes + (size_t)round_up((int64_t)(w.slot_elems * 2), 256));
}

}  // namespace mpr

using namespace mpr;

// ================================================================== C ABI
extern "C" int mpr_version(void) { return 100; }

extern "C" const char *mpr_status_string(int status)
{
    switch (status) {
    case MPR_OK: return "ok";
    case MPR_EINVAL: return "invalid argument";
    case MPR_ENOMEM: return "workspace too small";
    case MPR_EOVERFLOW: return "finite value above 0x7FFF would enter a product";
    case MPR_ENOTFOUND: return "no periodic regime found";
    case MPR_EHIP: return "HIP runtime error";
    case MPR_EUNSUPPORTED: return "unsupported device or size";
    case MPR_ETIMEDOUT: return "request waited past its deadline";
    case MPR_ECANCELED: return "request cancelled";
    default: return "unknown status";
    }
}

extern "C" mpr_status mpr_init(int device)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MPR_EUNSUPPORTED;
    return init_device(device);
}

extern "C" mpr_status mpr_transfer_size(int m, int64_t *n_states_host)
{
    if (m < 1 || m > 12 || !n_states_host) return MPR_EINVAL;
    *n_states_host = transfer_size(m);
    return MPR_OK;
}

extern "C" mpr_status mpr_transfer_words(int m, uint8_t *words_host, int64_t capacity_words)
{
    if (m < 1 || m > 12 || !words_host) return MPR_EINVAL;
    const int64_t n = transfer_size(m);
    if (capacity_words < n) return MPR_ENOMEM;
    transfer_words(m, words_host, n);
    return MPR_OK;
}

extern "C" mpr_status mpr_build_transfer(int m, uint16_t *A, int64_t lda, mpr_stream stream)
{
    if (m < 1 || m > 11 || !A) return MPR_EINVAL;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    if (lda < transfer_size(m)) return MPR_EINVAL;
    return transfer_launch(m, A, lda, as_stream(stream));
}

extern "C" mpr_status mpr_build_border_transfer(int m, uint16_t *A, int64_t lda, int64_t *shift_host,
                                                mpr_stream stream)
{
    if (m < 1 || m > 11 || !A || !shift_host) return MPR_EINVAL;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    if (lda < transfer_size(m)) return MPR_EINVAL;
    *shift_host = border_shift(m);
    return border_transfer_launch(m, A, lda, as_stream(stream));
}

static mpr_status gemm_args(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B, int64_t ldb,
                            const void *C, int64_t ldc)
{
    if (M < 0 || N < 0 || K < 0) return MPR_EINVAL;
    if ((M && K && !A) || (K && N && !B) || (M && N && !C)) return MPR_EINVAL;
    if (!ld_ok(lda, K) || !ld_ok(ldb, N) || !ld_ok(ldc, N)) return MPR_EINVAL;
    if (M > (1ll << 31) || N > (1ll << 31) || K > (1ll << 31)) return MPR_EUNSUPPORTED;
    return MPR_OK;
}

extern "C" mpr_status mpr_minplus_gemm_cfg(int cfg, int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t lda,
                                           const uint16_t *B, int64_t ldb, uint16_t *C, int64_t ldc,
                                           int32_t *d_status, mpr_stream stream)
{
    mpr_status e = gemm_args(M, N, K, A, lda, B, ldb, C, ldc);
    if (e != MPR_OK) return e;
    if (cfg < -1 || cfg >= mpr_gemm_config_count()) return MPR_EINVAL;
    if ((e = ensure_init()) != MPR_OK) return e;
    hipStream_t s = as_stream(stream);
    if (d_status) {
        if ((e = validate_launch(A, M, K, lda, d_status, s)) != MPR_OK) return e;
        if ((e = validate_launch(B, K, N, ldb, d_status, s)) != MPR_OK) return e;
    }
    return gemm_launch(cfg, M, N, K, A, lda, B, ldb, C, ldc, s);
}

extern "C" mpr_status mpr_minplus_gemm_spare(int cfg, int64_t M, int64_t N, int64_t K, const uint16_t *A,
                                             int64_t lda, const uint16_t *B, int64_t ldb, uint16_t *C, int64_t ldc,
                                             int32_t *d_status, mpr_stream stream)
{
    mpr_status e = gemm_args(M, N, K, A, lda, B, ldb, C, ldc);
    if (e != MPR_OK) return e;
    if (cfg < -1 || cfg >= mpr_gemm_config_count()) return MPR_EINVAL;
    if ((e = ensure_init()) != MPR_OK) return e;
    hipStream_t s = as_stream(stream);
    if (d_status) {
        if ((e = validate_launch(A, M, K, lda, d_status, s)) != MPR_OK) return e;
        if ((e = validate_launch(B, K, N, ldb, d_status, s)) != MPR_OK) return e;
    }
    return gemm_launch_spare(cfg, M, N, K, A, lda, B, ldb, C, ldc, s);
}

extern "C" mpr_status mpr_minplus_gemm(int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t lda,
                                       const uint16_t *B, int64_t ldb, uint16_t *C, int64_t ldc, int32_t *d_status,
                                       mpr_stream stream)
{
    return mpr_minplus_gemm_cfg(-1, M, N, K, A, lda, B, ldb, C, ldc, d_status, stream);
}

extern "C" mpr_status mpr_normalise(int64_t M, int64_t N, uint16_t *C, int64_t ldc, const int64_t *R_in,
                                    int64_t *R_out, int32_t *d_status, mpr_stream stream)
{
    if (M < 0 || N < 0 || (M && (!C || !R_out)) || !ld_ok(ldc, N)) return MPR_EINVAL;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    return normalise_launch(M, N, C, ldc, R_in, nullptr, R_out, d_status, nullptr, as_stream(stream));
}

extern "C" mpr_status mpr_gemm_norm_workspace_size(int64_t K, int64_t N, size_t *bytes_host)
{
    if (K < 0 || N < 0 || !bytes_host) return MPR_EINVAL;
    *bytes_host = gemm_norm_ws(K, N, nullptr);
    return MPR_OK;
}

extern "C" mpr_status mpr_minplus_gemm_norm(int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t lda,
                                            const int64_t *Ra, const uint16_t *B, int64_t ldb, const int64_t *Rb,
                                            uint16_t *C, int64_t ldc, int64_t *Rc, void *ws, size_t ws_bytes,
                                            int32_t *d_status, mpr_stream stream)
{
    mpr_status e = gemm_args(M, N, K, A, lda, B, ldb, C, ldc);
    if (e != MPR_OK) return e;
    if (M && !Rc) return MPR_EINVAL;
    int64_t ldp = 0;
    const size_t need = gemm_norm_ws(K, N, &ldp);
    if (Rb && (!ws || ws_bytes < need)) return MPR_ENOMEM;
    if ((e = ensure_init()) != MPR_OK) return e;
    hipStream_t s = as_stream(stream);
    if (d_status) {
        if ((e = validate_launch(A, M, K, lda, d_status, s)) != MPR_OK) return e;
        if ((e = validate_launch(B, K, N, ldb, d_status, s)) != MPR_OK) return e;
    }
    Carver c(ws);
    int64_t *sc = c.take<int64_t>(1);
    u16 *Bp = c.take<u16>((size_t)(K * ldp));
    return gemm_norm_impl(M, N, K, A, lda, Ra, B, ldb, Rb, C, ldc, Rc, sc, Bp, ldp, d_status, s);
}

extern "C" mpr_status mpr_power_workspace_size(int64_t n, int64_t e, int schedule, size_t *bytes_host)
{
    if (n < 0 || e < 1 || !bytes_host || schedule < MPR_CHAIN || schedule > MPR_CHAIN_SPARSE) return MPR_EINVAL;
    *bytes_host = power_ws_recommended(n, schedule);
    return MPR_OK;
}

extern "C" mpr_status mpr_minplus_power(const uint16_t *A, int64_t n, int64_t lda, int64_t e, int schedule,
                                        uint16_t *N_out, int64_t ldo, int64_t *R_out, void *ws, size_t ws_bytes,
                                        int32_t *d_status, mpr_stream stream)
{
    if (n < 0 || e < 1 || schedule < MPR_CHAIN || schedule > MPR_CHAIN_SPARSE) return MPR_EINVAL;
    if (n && (!A || !N_out || !R_out)) return MPR_EINVAL;
    if (!ld_ok(lda, n) || !ld_ok(ldo, n)) return MPR_EINVAL;
    if (n == 0) return MPR_OK;
    PowerWs w = carve_power(ws, n, schedule, ws_bytes);
    if (!ws || ws_bytes < w.bytes) return MPR_ENOMEM;
    if (schedule == MPR_CHAIN_SPARSE && !w.plan_full) {
        // A plan smaller than the worst case: too small even for the counts,
        // or no status word to report a plan that does not fit.
        if (w.plan_bytes < sparse_plan_bytes_rows(n, 0)) return MPR_ENOMEM;
        if (!d_status) return MPR_EINVAL;
    }
    mpr_status r = ensure_init();
    if (r != MPR_OK) return r;
    hipStream_t s = as_stream(stream);
    if ((r = validate_launch(A, n, n, lda, d_status, s)) != MPR_OK) return r;
    if (schedule == MPR_SQUARE) return power_square(A, n, lda, e, N_out, ldo, R_out, w, d_status, s);
    return power_chain(A, n, lda, e, N_out, ldo, R_out, w, d_status, s, schedule == MPR_CHAIN_SPARSE);
}

extern "C" mpr_status mpr_chain_resume(const uint16_t *A, int64_t n, int64_t lda, const uint16_t *N_k, int64_t ldk,
                                       const int64_t *R_k, int64_t steps, int schedule, uint16_t *N_out, int64_t ldo,
                                       int64_t *R_out, void *ws, size_t ws_bytes, int32_t *d_status, mpr_stream stream)
{
    if (n < 0 || steps < 0 || (schedule != MPR_CHAIN && schedule != MPR_CHAIN_SPARSE)) return MPR_EINVAL;
    if (n && (!A || !N_k || !R_k || !N_out || !R_out)) return MPR_EINVAL;
    if (!ld_ok(lda, n) || !ld_ok(ldk, n) || !ld_ok(ldo, n)) return MPR_EINVAL;
    if (N_k == N_out && ldk != ldo) return MPR_EINVAL;
    if (n == 0) return MPR_OK;
    PowerWs w = carve_power(ws, n, schedule, ws_bytes);
    if (!ws || ws_bytes < w.bytes) return MPR_ENOMEM;
    if (schedule == MPR_CHAIN_SPARSE && !w.plan_full) {
        if (w.plan_bytes < sparse_plan_bytes_rows(n, 0)) return MPR_ENOMEM;
        if (!d_status) return MPR_EINVAL;
    }
    mpr_status r = ensure_init();
    if (r != MPR_OK) return r;
    hipStream_t s = as_stream(stream);
    if ((r = validate_launch(A, n, n, lda, d_status, s)) != MPR_OK) return r;
    if ((r = validate_launch(N_k, n, n, ldk, d_status, s)) != MPR_OK) return r;
    return power_chain(A, n, lda, steps + 1, N_out, ldo, R_out, w, d_status, s, schedule == MPR_CHAIN_SPARSE, N_k, R_k,
                       ldk);
}

extern "C" mpr_status mpr_minplus_power_noalloc(const uint16_t *A, int64_t n, int64_t lda, int64_t e, int schedule,
                                                uint16_t *N_out, int64_t ldo, int64_t *R_out, int32_t *d_status,
                                                mpr_stream stream)
{
    if (n < 0 || e < 1 || schedule < MPR_CHAIN || schedule > MPR_CHAIN_SPARSE) return MPR_EINVAL;
    if (n && (!A || !N_out || !R_out)) return MPR_EINVAL;
    if (!ld_ok(lda, n) || !ld_ok(ldo, n)) return MPR_EINVAL;
    if (n == 0) return MPR_OK;
    if (carve_power(nullptr, n, schedule).bytes > (size_t)MPR_NOALLOC_SCRATCH_BYTES) return MPR_ENOMEM;
    mpr_status r = ensure_init();
    if (r != MPR_OK) return r;
    void *ws = device_scratch();
    if (!ws) return MPR_EHIP;
    return mpr_minplus_power(A, n, lda, e, schedule, N_out, ldo, R_out, ws, (size_t)MPR_NOALLOC_SCRATCH_BYTES,
                             d_status, stream);
}

extern "C" mpr_status mpr_sparse_plan_bytes(const uint16_t *A, int64_t n, int64_t lda, size_t *bytes_host,
                                            mpr_stream stream)
{
    if (n < 1 || !A || !bytes_host || !ld_ok(lda, n)) return MPR_EINVAL;
    mpr_status r = ensure_init();
    if (r != MPR_OK) return r;
    hipStream_t s = as_stream(stream);
    const size_t tmp_bytes = sparse_plan_bytes_rows(n, 0);
    void *tmp = nullptr;
    if (hipMallocAsync(&tmp, tmp_bytes, s) != hipSuccess) return MPR_ENOMEM;
    int64_t rows = 0;
    r = sparse_plan_rows(A, n, lda, tmp, s, &rows);
    if (hipFreeAsync(tmp, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) r = r != MPR_OK ? r : MPR_EHIP;
    if (r == MPR_OK) *bytes_host = sparse_plan_bytes_rows(n, rows);
    return r;
}

extern "C" mpr_status mpr_trace_min(const uint16_t *N, int64_t n, int64_t ld, const int64_t *R, int64_t *d_gamma,
                                    mpr_stream stream)
{
    if (n < 0 || !d_gamma || (n && !N) || !ld_ok(ld, n)) return MPR_EINVAL;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    return trace_launch(N, n, ld, R, d_gamma, as_stream(stream));
}

extern "C" mpr_status mpr_trace_of_product(const uint16_t *X, const int64_t *RX, const uint16_t *Y,
                                           const int64_t *RY, int64_t n, int64_t ld, int64_t *d_gamma,
                                           mpr_stream stream)
{
    if (n < 0 || !d_gamma || (n && (!X || !Y)) || !ld_ok(ld, n)) return MPR_EINVAL;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    return trace_product_launch(X, RX, Y, RY, n, ld, d_gamma, as_stream(stream));
}

extern "C" mpr_status mpr_trace_of_product_t(const uint16_t *X, const int64_t *RX, const uint16_t *YT,
                                             const int64_t *CY, int64_t n, int64_t ld, int64_t *d_gamma,
                                             mpr_stream stream)
{
    if (n < 0 || !d_gamma || (n && (!X || !YT)) || !ld_ok(ld, n)) return MPR_EINVAL;
    mpr_status e = ensure_init();
    if (e != MPR_OK) return e;
    return trace_product_t_launch(X, RX, YT, CY, n, ld, d_gamma, as_stream(stream));
}

extern "C" mpr_status mpr_period_workspace_size_ex(int64_t n, int64_t slots, int flags, size_t *bytes_host)
{
    if (n < 0 || slots < 2 || !bytes_host || (flags & ~kPeriodFlagsAll)) return MPR_EINVAL;
    if ((flags & MPR_PERIOD_PIPELINE) && (flags & MPR_PERIOD_REUSE_A)) return MPR_EINVAL;
    PeriodWs w = carve_period(nullptr, n, 0, slots, flags);
    // MPR_PERIOD_PIPELINE: one more buffer, for the power computed ahead
    const int64_t bufs = slots + ((flags & MPR_PERIOD_PIPELINE) ? 1 : 0);
    *bytes_host = w.fixed + (size_t)bufs * w.slot_bytes;
    return MPR_OK;
}

extern "C" mpr_status mpr_period_workspace_size(int64_t n, int64_t slots, size_t *bytes_host)
{
    return mpr_period_workspace_size_ex(n, slots, 0, bytes_host);
}

extern "C" mpr_status mpr_find_period_ex(const uint16_t *A, int64_t n, int64_t lda, int64_t kmax, int flags,
                                         int64_t *mu_host, int64_t *lam_host, int64_t *c_host, int64_t *traces_host,
                                         void *ws, size_t ws_bytes, mpr_stream stream)
{
    if (n < 1 || kmax < 1 || !A || !mu_host || !lam_host || !c_host || !ld_ok(lda, n)) return MPR_EINVAL;
    if (flags & ~kPeriodFlagsAll) return MPR_EINVAL;
    const bool sparse = (flags & MPR_PERIOD_SPARSE) != 0;
    const bool reuse_a = (flags & MPR_PERIOD_REUSE_A) != 0;
    const bool pipeline = (flags & MPR_PERIOD_PIPELINE) != 0;
    if (pipeline && reuse_a) return MPR_EINVAL;
    // A's buffer can hold a power only once nothing reads A any more (the
    // compressed-K plan replaces it after the first power) and only in the
    // ring's layout (the compare reads both powers with one row stride).
    if (reuse_a && (!sparse || lda != round_up(n, 8))) return MPR_EINVAL;
    if (!ws) return MPR_ENOMEM;
    mpr_status r = ensure_init();
    if (r != MPR_OK) return r;
    hipStream_t s = as_stream(stream);
    // The compressed-K plan is sized for this A (its rows are counted first,
    // one host round trip), so the ring gets every byte the plan does not use.
    size_t plan_bytes = 0;
    if (sparse) {
        PeriodWs probe = carve_period(ws, n, ws_bytes, 0, flags & ~MPR_PERIOD_SPARSE);  // the part before the plan
        if (ws_bytes < probe.fixed + sparse_plan_bytes_rows(n, 0)) return MPR_ENOMEM;
        int64_t rows = 0;
        if ((r = sparse_plan_rows(A, n, lda, (char *)ws + probe.fixed, s, &rows)) != MPR_OK) return r;
        plan_bytes = sparse_plan_bytes_rows(n, rows);
    }
    PeriodWs w = carve_period(ws, n, ws_bytes, 0, flags, plan_bytes);
    if (w.slots < (pipeline ? 3 : 2)) return MPR_ENOMEM;
    int32_t *st = (int32_t *)&w.scal[2];
    if ((r = fill_i32_launch(st, 2, 0, s)) != MPR_OK) return r;
    if ((r = validate_launch(A, n, n, lda, st, s)) != MPR_OK) return r;
    if (sparse && (r = sparse_plan_launch(A, n, lda, w.plan, w.plan_bytes, st, s)) != MPR_OK) return r;
    if (traces_host) traces_host[0] = MPR_ROW_NONE;

    // Power k lives in slot (k - 1) % slots (a ring), so a repeat of the class
    // of power j can be confirmed exactly while k - j < slots.  With
    // MPR_PERIOD_REUSE_A a repeat the ring can no longer confirm (power j
    // gone) is confirmed one period later instead: power k is kept in A's
    // buffer and compared with power k + (k - j) when the chain gets there.
    std::unordered_multimap<uint64_t, int64_t> seen;  // class hash -> k
    bool found = false;
    int64_t mu = 0, lam = 0, cval = 0;
    int64_t prev_slot = -1;
    bool held = false;           // a power waits in A's buffer
    int64_t held_k = 0, held_lam = 0;
    u16 *hold_N = reuse_a ? const_cast<u16 *>(A) : nullptr;

    // Exact comparison of (X, RX) with (Y, RY) (same N and emptiness, one
    // offset shift c over the non-empty rows; c = 0 when no row has one).
    auto same_class = [&](const u16 *X, const int64_t *RX, const u16 *Y, const int64_t *RY, bool &eq,
                          int64_t &c) -> mpr_status {
        int64_t *out3 = &w.scal[3];
        mpr_status e = compare_launch(X, RX, Y, RY, n, w.ld, out3, s);
        if (e != MPR_OK) return e;
        int64_t cmp[3];
        if (hipMemcpyAsync(cmp, out3, sizeof(cmp), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MPR_EHIP;
        const bool no_rows = cmp[1] == MPR_ROW_NONE && cmp[2] == -MPR_ROW_NONE;
        eq = cmp[0] == 0 && (cmp[1] == cmp[2] || no_rows);
        c = no_rows ? 0 : cmp[1];
        return MPR_OK;
    };
    if (pipeline) {
        // Power k + 1 is enqueued before the host waits for the class hash
        // and trace of power k (copied to pinned memory, each with its
        // event), so the round trip overlaps a power's work instead of
        // following it.  Power k + 1 overwrites power k + 1 - M of the ring
        // of M buffers, so a repeat of power j is confirmed while
        // k - j < M - 1: the workspace of `slots` holds M = slots + 1.
        const int64_t M = w.slots;
        int64_t *pin = nullptr;  // two records of the 8 scalar words
        hipEvent_t ev[2] = {nullptr, nullptr};
        auto finish = [&](mpr_status e) {
            if (hipStreamSynchronize(s) != hipSuccess && e == MPR_OK) e = MPR_EHIP;  // the power computed ahead
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            if (pin) (void)hipHostFree(pin);
            return e;
        };
        if (hipHostMalloc((void **)&pin, 2 * 8 * sizeof(int64_t)) != hipSuccess) return MPR_ENOMEM;
        if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess)
            return finish(MPR_EHIP);
        auto enqueue = [&](int64_t k) -> mpr_status {
            const int64_t slot = (k - 1) % M;
            u16 *Nk = slot_N(w, slot);
            int64_t *Rk = slot_R(w, slot);
            mpr_status e;
            if (k == 1) {
                e = copy_launch(A, lda, Nk, w.ld, n, n, s);
                if (e == MPR_OK) e = normalise_launch(n, n, Nk, w.ld, nullptr, nullptr, Rk, st, w.row_hash, s);
            } else {
                const int64_t ps = (k - 2) % M;
                e = sparse ? sparse_step_launch(slot_N(w, ps), w.ld, n, w.plan, w.plan_bytes, Nk, w.ld, s)
                           : gemm_launch(-1, n, n, n, slot_N(w, ps), w.ld, A, lda, Nk, w.ld, s);
                if (e == MPR_OK)
                    e = normalise_launch(n, n, Nk, w.ld, slot_R(w, ps), nullptr, Rk, st, w.row_hash, s);
            }
            if (e == MPR_OK) e = class_hash_launch(w.row_hash, Rk, n, (uint64_t *)&w.scal[0], s);
            if (e == MPR_OK) e = trace_launch(Nk, n, w.ld, Rk, &w.scal[1], s);
            if (e == MPR_OK && (hipMemcpyAsync(pin + 8 * (k & 1), w.scal, 8 * sizeof(int64_t), hipMemcpyDeviceToHost,
                                               s) != hipSuccess ||
                                hipEventRecord(ev[k & 1], s) != hipSuccess))
                e = MPR_EHIP;
            return e;
        };
        if ((r = enqueue(1)) != MPR_OK) return finish(r);
        for (int64_t k = 1; k <= kmax; k++) {
            if (k + 1 <= kmax && (r = enqueue(k + 1)) != MPR_OK) return finish(r);
            if (hipEventSynchronize(ev[k & 1]) != hipSuccess) return finish(MPR_EHIP);
            const volatile int64_t *rec = pin + 8 * (k & 1);
            const int64_t hash = rec[0], trace = rec[1];
            const int32_t stv = (int32_t)(rec[2] & 0xFFFFFFFF);
            if (stv != 0) return finish((mpr_status)stv);
            if (traces_host) traces_host[k] = trace;
            report_progress(k, trace);
            if (!found) {
                const uint64_t h = (uint64_t)hash;
                auto range = seen.equal_range(h);
                for (auto it = range.first; it != range.second && !found; ++it) {
                    const int64_t j = it->second;
                    if (k - j >= M - 1) continue;  // power j overwritten (by power k + 1 at the latest)
                    const int64_t sj = (j - 1) % M, sk = (k - 1) % M;
                    bool eq = false;
                    int64_t c = 0;
                    if ((r = same_class(slot_N(w, sj), slot_R(w, sj), slot_N(w, sk), slot_R(w, sk), eq, c)) != MPR_OK)
                        return finish(r);
                    if (eq) {
                        found = true;
                        mu = j;
                        lam = k - j;
                        cval = c;
                    }
                }
                if (!found) seen.emplace(h, k);
            }
            if (found && !traces_host) break;
            if (found && (flags & MPR_PERIOD_EXTEND)) {
                for (int64_t j = k + 1; j <= kmax; j++)
                    traces_host[j] =
                        traces_host[j - lam] == MPR_ROW_NONE ? MPR_ROW_NONE : traces_host[j - lam] + cval;
                break;
            }
        }
        if ((r = finish(MPR_OK)) != MPR_OK) return r;
        if (!found) return MPR_ENOTFOUND;
        *mu_host = mu;
        *lam_host = lam;
        *c_host = cval;
        return MPR_OK;
    }
    for (int64_t k = 1; k <= kmax; k++) {
        const int64_t slot = (k - 1) % w.slots;
        u16 *Nk = slot_N(w, slot);
        int64_t *Rk = slot_R(w, slot);
        if (k == 1) {
            r = copy_launch(A, lda, Nk, w.ld, n, n, s);
            if (r == MPR_OK) r = normalise_launch(n, n, Nk, w.ld, nullptr, nullptr, Rk, st, w.row_hash, s);
        } else {
            r = sparse ? sparse_step_launch(slot_N(w, prev_slot), w.ld, n, w.plan, w.plan_bytes, Nk, w.ld, s)
                       : gemm_launch(-1, n, n, n, slot_N(w, prev_slot), w.ld, A, lda, Nk, w.ld, s);
            if (r == MPR_OK)
                r = normalise_launch(n, n, Nk, w.ld, slot_R(w, prev_slot), nullptr, Rk, st, w.row_hash, s);
        }
        if (r == MPR_OK) r = class_hash_launch(w.row_hash, Rk, n, (uint64_t *)&w.scal[0], s);
        if (r == MPR_OK) r = trace_launch(Nk, n, w.ld, Rk, &w.scal[1], s);
        if (r != MPR_OK) return r;
        int64_t host[3];
        if (hipMemcpyAsync(host, w.scal, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MPR_EHIP;
        if ((int32_t)(host[2] & 0xFFFFFFFF) != 0) return (mpr_status)(int32_t)(host[2] & 0xFFFFFFFF);
        if (traces_host) traces_host[k] = host[1];
        report_progress(k, host[1]);
        prev_slot = slot;
        if (!found && held && k == held_k + held_lam) {
            // the power kept one period ago: the relation A^(k) = c (x)
            // A^(k - lam) confirmed exactly at n0 = k - lam
            bool eq = false;
            int64_t c = 0;
            if ((r = same_class(hold_N, w.hold_R, Nk, Rk, eq, c)) != MPR_OK) return r;
            held = false;
            if (eq) {
                found = true;
                mu = held_k;
                lam = held_lam;
                cval = c;
            }
        }
        if (!found) {
            const uint64_t h = (uint64_t)host[0];
            auto range = seen.equal_range(h);
            for (auto it = range.first; it != range.second && !found; ++it) {
                const int64_t j = it->second;
                if (k - j >= w.slots) {  // power j is no longer resident
                    if (reuse_a && !held) {
                        if ((r = copy_launch(Nk, w.ld, hold_N, lda, n, n, s)) != MPR_OK) return r;
                        if (hipMemcpyAsync(w.hold_R, Rk, (size_t)n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
                            return MPR_EHIP;
                        held = true;
                        held_k = k;
                        held_lam = k - j;
                    }
                    continue;
                }
                const int64_t sj = (j - 1) % w.slots;
                bool eq = false;
                int64_t c = 0;
                if ((r = same_class(slot_N(w, sj), slot_R(w, sj), Nk, Rk, eq, c)) != MPR_OK) return r;
                if (eq) {
                    found = true;
                    mu = j;
                    lam = k - j;
                    cval = c;
                }
            }
            if (!found) seen.emplace(h, k);
        }
        if (found && !traces_host) break;
        if (found && (flags & MPR_PERIOD_EXTEND)) {
            for (int64_t j = k + 1; j <= kmax; j++)
                traces_host[j] = traces_host[j - lam] == MPR_ROW_NONE ? MPR_ROW_NONE : traces_host[j - lam] + cval;
            break;
        }
    }
    if (!found) return MPR_ENOTFOUND;
    *mu_host = mu;
    *lam_host = lam;
    *c_host = cval;
    return MPR_OK;
}

extern "C" mpr_status mpr_set_period_progress(void (*fn)(int64_t k, int64_t trace, void *user), void *user)
{
    std::lock_guard<std::mutex> lk(g_progress_mu);
    g_progress_fn = fn;
    g_progress_user = user;
    return MPR_OK;
}

// ------------------------------------------------------------ Proposition 8
extern "C" mpr_status mpr_gamma_from_period(int64_t mu, int64_t lam, int64_t c, const int64_t *traces_host,
                                            int64_t kmax, int64_t n, int64_t *gamma_host)
{
    if (mu < 1 || lam < 1 || !traces_host || !gamma_host || n < 1 || mu + lam - 1 > kmax) return MPR_EINVAL;
    if (n < mu) {
        if (n > kmax) return MPR_EINVAL;
        *gamma_host = traces_host[n];
        return MPR_OK;
    }
    const int64_t q = (n - mu) / lam, r = (n - mu) % lam;
    // A residue class whose traces have no finite term stays empty
    // (trace(k + lam) = c + trace(k) keeps +infinity).
    const int64_t t = traces_host[mu + r];
    *gamma_host = t == MPR_ROW_NONE ? MPR_ROW_NONE : t + c * q;
    return MPR_OK;
}

extern "C" mpr_status mpr_period_formula(int64_t mu, int64_t lam, int64_t c, const int64_t *traces_host,
                                         int64_t kmax, int64_t *numer_host)
{
    if (mu < 1 || lam < 1 || !traces_host || !numer_host || mu + lam - 1 > kmax) return MPR_EINVAL;
    for (int64_t r = 0; r < lam; r++) {
        const int64_t k = mu + r;  // residue class of k modulo lam
        // an empty residue class (no finite trace) is reported as MPR_ROW_NONE
        numer_host[k % lam] = traces_host[k] == MPR_ROW_NONE ? MPR_ROW_NONE : lam * traces_host[k] - c * k;
    }
    return MPR_OK;
}

extern "C" mpr_status mpr_find_period(const uint16_t *A, int64_t n, int64_t lda, int64_t kmax, int64_t *mu_host,
                                      int64_t *lam_host, int64_t *c_host, int64_t *traces_host, void *ws,
                                      size_t ws_bytes, mpr_stream stream)
{
    return mpr_find_period_ex(A, n, lda, kmax, 0, mu_host, lam_host, c_host, traces_host, ws, ws_bytes, stream);
}
