// common.h -- shared definitions of the libmpr HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpr.h"

namespace mpr {

typedef uint16_t u16;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr u16 INF16 = 0xFFFF;
constexpr u16 FMAX16 = 0x7FFF;
constexpr int64_t ROW_NONE = INT64_MAX;

// Device memory the kernels read and write is global memory; pointers that
// reach a kernel through a descriptor are generic, so accesses cast them to
// the global address space explicitly (global, not flat, instructions).
typedef __attribute__((address_space(1))) u16 gu16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;
template <class X>
__device__ __forceinline__ __attribute__((address_space(1))) X *glob(X *p)
{
    return (__attribute__((address_space(1))) X *)p;
}
template <class X>
__device__ __forceinline__ const __attribute__((address_space(1))) X *glob(const X *p)
{
    return (const __attribute__((address_space(1))) X *)p;
}

// 16-byte global load / store through the global address space.
__device__ __forceinline__ uint4 gload16(const gu16 *p)
{
    const u32x4 v = *(const gu32x4 *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore16(gu16 *p, const uint4 &v)
{
    u32x4 w = {v.x, v.y, v.z, v.w};
    *(gu32x4 *)p = w;
}

__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// Saturating packed add (v_pk_add_u16 ... clamp): any sum with an operand
// 0xFFFF stays 0xFFFF, so infinity absorbs.
__device__ __forceinline__ u16x2 add_sat(u16x2 a, u16x2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ u16x2 min2(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }

// The f16 image of a (min,+) value, used by the f16 form of the tile
// routine.  A finite uint16 x < 0x800 is, read as an f16 bit pattern, the
// number x * 2^-24 (subnormals and the first binade share the spacing
// 2^-24), so sums of such values below 2048 are exact and their bit
// patterns are the integer sums.  Infinity 0xFFFF becomes +inf (0x7C00);
// finite values >= 0x800 are clamped to 0x800, which keeps every sum they
// enter at or above 0x800 (flagged by tile_from_h16) and far from overflow.
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h16x2 as_h16x2(uint32_t v) { return __builtin_bit_cast(h16x2, v); }
__device__ __forceinline__ uint32_t as_u32(h16x2 v) { return __builtin_bit_cast(uint32_t, v); }
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t to_h16(uint32_t x)
{
    // Signed, 0xFFFF is -1 and survives min(., 0x800); unsigned, it then
    // meets 0x7C00 while the clamped finite values pass: two v_pk_min.
    const i16x2 c = __builtin_elementwise_min(__builtin_bit_cast(i16x2, x), (i16x2){0x800, 0x800});
    return as_u32(min2(__builtin_bit_cast(u16x2, c), (u16x2){0x7C00, 0x7C00}));
}

__device__ __forceinline__ uint32_t comp(const uint4 &v, int q)
{
    return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014), used only to hash the
// class of a power for the period search.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Wave-level reductions (64 lanes).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
    for (int off = 32; off > 0; off >>= 1) {
        int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void set_status(int32_t *st, int32_t code)
{
    if (st) __hip_atomic_store(st, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ---------------------------------------------------------------- host-side
// Internal entry points shared between translation units.
hipStream_t as_stream(mpr_stream s);
mpr_status check_launch();
mpr_status ensure_init();
int device_cu_count();

// gemm.hip
mpr_status gemm_launch(int cfg, int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda,
                       const u16 *B, int64_t ldb, u16 *C, int64_t ldc, hipStream_t s);
// The same product holding one workgroup per CU fewer than it could (extra
// LDS per workgroup), so that work on other streams finds free slots while
// it runs.
mpr_status gemm_launch_spare(int cfg, int64_t M, int64_t N, int64_t K, const u16 *A, int64_t lda,
                             const u16 *B, int64_t ldb, u16 *C, int64_t ldc, hipStream_t s);
int pick_config(int64_t M, int64_t N, int64_t K);
int pick_config_arith(int arith, int64_t M, int64_t N, int64_t K);
int current_arith();

// sparse.hip
size_t sparse_plan_bytes(int64_t n);                      // worst case (dense A)
size_t sparse_plan_bytes_rows(int64_t n, int64_t rows);   // a plan of `rows` rows
mpr_status sparse_plan_rows(const u16 *A, int64_t n, int64_t lda, void *ws, hipStream_t s, int64_t *rows);
mpr_status sparse_plan_launch(const u16 *A, int64_t n, int64_t lda, void *ws, size_t bytes, int32_t *st,
                              hipStream_t s);
mpr_status sparse_step_launch(const u16 *Np, int64_t ldn, int64_t n, void *ws, size_t bytes, u16 *C, int64_t ldc,
                              hipStream_t s);

// rowops.hip
mpr_status validate_launch(const u16 *X, int64_t rows, int64_t cols, int64_t ld, int32_t *st, hipStream_t s);
mpr_status normalise_launch(int64_t M, int64_t N, u16 *C, int64_t ldc, const int64_t *R_in,
                            const int64_t *add_scalar, int64_t *R_out, int32_t *st,
                            uint64_t *row_hash, hipStream_t s);
mpr_status copy_launch(const u16 *src, int64_t lds, u16 *dst, int64_t ldd, int64_t rows, int64_t cols,
                       hipStream_t s);
mpr_status fold_launch(const u16 *B, int64_t ldb, const int64_t *Rb, int64_t K, int64_t N, u16 *Bp,
                       int64_t ldp, int64_t *s_out, int32_t *st, hipStream_t s);
mpr_status trace_launch(const u16 *N, int64_t n, int64_t ld, const int64_t *R, int64_t *out, hipStream_t s);
mpr_status class_hash_launch(const uint64_t *row_hash, const int64_t *R, int64_t n, uint64_t *out,
                             hipStream_t s);
mpr_status compare_launch(const u16 *X, const int64_t *RX, const u16 *Y, const int64_t *RY, int64_t n,
                          int64_t ld, int64_t *out3, hipStream_t s);
mpr_status fill_i32_launch(int32_t *p, int64_t count, int32_t v, hipStream_t s);
mpr_status trace_product_launch(const u16 *X, const int64_t *RX, const u16 *Y, const int64_t *RY, int64_t n,
                                int64_t ld, int64_t *out, hipStream_t s);

}  // namespace mpr
