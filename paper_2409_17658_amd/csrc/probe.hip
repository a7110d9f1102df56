// probe.hip -- measures the VALU rate of the (min,+) instruction mixes on
// the device itself, to confirm the peak the kernels are priced against:
// a register-only kernel issuing the inner-loop instructions of each form
// (uint16: v_pk_add_u16 clamp + v_pk_min_u16, 2 pairs per 2 instructions;
// f16 form: 2 v_pk_add_f16 + 1 v_pk_minimum3_f16, 4 pairs per 3), with
// enough independent accumulators per lane that dependences never stall
// the issue, on every CU.  One wave also reads the shader clock counter and
// the constant-rate wall clock at both ends, which gives the clock the
// chip ran at during the probe.
#include "common.h"

namespace mpr {

constexpr int PROBE_CHAINS = 16;  // independent accumulator pairs per lane

template <bool H>
__global__ __launch_bounds__(256) void valu_probe_kernel(uint32_t seed, int iters, uint32_t *sink,
                                                         unsigned long long *clk)
{
    const uint32_t t = seed ^ (blockIdx.x * 256u + threadIdx.x);
    uint32_t x[PROBE_CHAINS], y[PROBE_CHAINS];
#pragma unroll
    for (int q = 0; q < PROBE_CHAINS; q++) {
        x[q] = (t * 0x9E3779B9u + (uint32_t)q) & 0x03FF03FFu;
        y[q] = (t * 0x85EBCA6Bu + (uint32_t)q * 7u) & 0x03FF03FFu;
    }
    // per-lane constants (held in VGPRs, as the operands of the tile loop are)
    const uint32_t c1 = ((t & 7u) | 1u) * 0x00010001u, c2 = c1 + 0x00020002u;
    unsigned long long t0 = 0, w0 = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        t0 = clock64();
        w0 = wall_clock64();
    }
    for (int i = 0; i < iters; i++) {
        if constexpr (H) {
            // x = minimum3(x, y + c1, y + c2): 4 (add, min) pairs in 3
            // instructions.  Every sum of a round is formed before its
            // minima, as in the tile loop (a minimum3 that reads the add
            // issued just before it waits a cycle).
            h16x2 a[PROBE_CHAINS], b[PROBE_CHAINS];
#pragma unroll
            for (int q = 0; q < PROBE_CHAINS; q++) {
                a[q] = as_h16x2(y[q]) + as_h16x2(c1);
                b[q] = as_h16x2(y[q]) + as_h16x2(c2);
            }
#pragma unroll
            for (int q = 0; q < PROBE_CHAINS; q++)
                x[q] = as_u32(__builtin_elementwise_minimum(__builtin_elementwise_minimum(as_h16x2(x[q]), a[q]), b[q]));
#pragma unroll
            for (int q = 0; q < PROBE_CHAINS; q++) {
                a[q] = as_h16x2(x[q]) + as_h16x2(c1);
                b[q] = as_h16x2(x[q]) + as_h16x2(c2);
            }
#pragma unroll
            for (int q = 0; q < PROBE_CHAINS; q++)
                y[q] = as_u32(__builtin_elementwise_minimum(__builtin_elementwise_minimum(as_h16x2(y[q]), a[q]), b[q]));
        } else {
            // x = min(x, y.xx + c1) saturating: 2 pairs in 2 instructions,
            // one operand broadcast by op_sel as in the tile loop
#pragma unroll
            for (int q = 0; q < PROBE_CHAINS; q++) {
                const u16x2 yv = as_u16x2(y[q]);
                x[q] = as_u32(min2(as_u16x2(x[q]), add_sat(__builtin_shufflevector(yv, yv, 0, 0), as_u16x2(c1))));
            }
#pragma unroll
            for (int q = 0; q < PROBE_CHAINS; q++) {
                const u16x2 xv = as_u16x2(x[q]);
                y[q] = as_u32(min2(as_u16x2(y[q]), add_sat(__builtin_shufflevector(xv, xv, 1, 1), as_u16x2(c2))));
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = clock64() - t0;
        clk[1] = wall_clock64() - w0;
    }
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < PROBE_CHAINS; q++) v ^= x[q] ^ y[q];
    if (v == 0x12345678u) sink[0] = v;  // keeps the work observable; almost never stored
}

}  // namespace mpr

using namespace mpr;

extern "C" mpr_status mpr_valu_probe(int arith, int iters, double *pairs_per_s_host, double *clock_ghz_host,
                                     mpr_stream stream)
{
    if ((arith != MPR_ARITH_U16 && arith != MPR_ARITH_F16) || iters < 1 || iters > (1 << 24) ||
        !pairs_per_s_host || !clock_ghz_host)
        return MPR_EINVAL;
    mpr_status st = ensure_init();
    if (st != MPR_OK) return st;
    hipStream_t s = as_stream(stream);
    int dev = 0, wall_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
        return MPR_EHIP;
    void *buf = nullptr;
    if (hipMalloc(&buf, 256) != hipSuccess) return MPR_ENOMEM;
    uint32_t *sink = (uint32_t *)buf;
    unsigned long long *clk = (unsigned long long *)((char *)buf + 128);
    // 8 workgroups of 4 waves per CU: 8 waves per SIMD, every SIMD busy.
    const int blocks = device_cu_count() * 8;
    auto kernel = arith == MPR_ARITH_F16 ? valu_probe_kernel<true> : valu_probe_kernel<false>;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    unsigned long long host_clk[2] = {0, 0};
    st = MPR_EHIP;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, s, 1u, iters / 8 + 1, sink, clk);  // warm-up
        const bool rec0 = hipEventRecord(e0, s) == hipSuccess;
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, s, 2u, iters, sink, clk);
        const bool rec1 = hipEventRecord(e1, s) == hipSuccess;
        if (rec0 && rec1 && check_launch() == MPR_OK && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            hipMemcpy(host_clk, clk, sizeof(host_clk), hipMemcpyDeviceToHost) == hipSuccess && ms > 0.f &&
            host_clk[1] > 0)
            st = MPR_OK;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (st != MPR_OK) return st;
    // pairs per lane per iteration: 2 statements x 2 halves per chain (uint16),
    // 2 statements x 4 pairs per chain (f16 form)
    const double per_iter = arith == MPR_ARITH_F16 ? 8.0 * PROBE_CHAINS : 4.0 * PROBE_CHAINS;
    *pairs_per_s_host = (double)blocks * 256.0 * (double)iters * per_iter / (ms * 1e-3);
    *clock_ghz_host = (double)host_clk[0] / (double)host_clk[1] * (double)wall_khz * 1e-6;
    return MPR_OK;
}
