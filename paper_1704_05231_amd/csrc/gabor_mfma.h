// Device building blocks shared by the matrix-core kernels of the bank
// (gabor_fused.hip, gabor_ws.hip): the operand formats and matrix-core step
// of each arithmetic form, boundary folding of indices, the XCD-aware
// workgroup order, LDS-only barriers and raw buffer resources.
#pragma once

#include "gabor_internal.h"

namespace gabor {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));


// Operand storage and matrix-core step for each arithmetic form.  A pack
// is what one lane feeds one instruction: a float (FP32) or eight 16-bit
// values in 16 bytes.  A fragment of Q consecutive values is Q / PER packs;
// split forms hold a hi and a lo fragment.
template <int OP> struct Form;

// Wait until the last FP32 matrix-core result is written before any vector
// instruction reads it.  The compiler schedules reads of a
// v_mfma_f32_16x16x4_f32 result 10 wait states after the instruction, and on
// gfx950 such reads of the last accumulator register returned stale values;
// 16 wait states remove the race.  The accumulators are asm operands kept in
// AGPRs, so no copy of them can be placed before the wait.
__device__ __forceinline__ void f32_mfma_drain(f4_t& x, f4_t& y)
{
    asm volatile("s_nop 7\n\ts_nop 7" : "+a"(x), "+a"(y));
}
__device__ __forceinline__ void f32_mfma_drain(f4_t& x, f4_t& y, f4_t& z, f4_t& u)
{
    asm volatile("s_nop 7\n\ts_nop 7" : "+a"(x), "+a"(y), "+a"(z), "+a"(u));
}

template <> struct Form<FUSED_F32> {
    using T = float;                      // LDS element
    using Pack = float;
    static constexpr int PER = 1;         // values per pack
    static constexpr bool split = false;
    static constexpr bool drain = true;
    static constexpr bool scaled = false; // range scaling (float16 only)
    static constexpr bool centred = true;    // local offset removed before accumulating
    static constexpr int centre_from_q = 33; // only for quarters above 32 (R > 56)
    // n consecutive floats -> packs (hi only)
    template <int N>
    static __device__ __forceinline__ void pack(const float (&x)[N], Pack* hi, Pack* lo)
    {
        (void)lo;
#pragma unroll
        for (int e = 0; e < N; ++e) hi[e] = x[e];
    }
    static __device__ __forceinline__ void mma1(f4_t& acc, Pack ah, Pack al, Pack bh, Pack bl)
    {
        (void)al; (void)bl;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ah, bh, acc, 0, 0, 0);
    }
    // the products of mma1 one at a time (term t of TERMS), so that several
    // accumulators can be advanced in turn
    static constexpr int TERMS = 1;
    static __device__ __forceinline__ void mmat(int t, f4_t& acc, Pack ah, Pack al, Pack bh, Pack bl)
    {
        (void)t;
        mma1(acc, ah, al, bh, bl);
    }
    // two floats -> LDS words (used for image slabs and J rows)
    typedef float W2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ void cvt2(float x0, float x1, W2& hi, W2& lo)
    {
        hi[0] = x0; hi[1] = x1; lo = hi;
    }
};

template <typename E> struct Vec;
template <> struct Vec<__bf16> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    typedef __bf16 v2 __attribute__((ext_vector_type(2)));
};
template <> struct Vec<_Float16> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    typedef _Float16 v2 __attribute__((ext_vector_type(2)));
};

__device__ __forceinline__ f4_t mfma16(f4_t acc, Vec<__bf16>::v8 a, Vec<__bf16>::v8 b)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(f4_t acc, Vec<_Float16>::v8 a, Vec<_Float16>::v8 b)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
}

template <typename E, bool SPLIT> struct Form16 {
    using T = E;
    using Pack = typename Vec<E>::v8;
    static constexpr int PER = 8;
    static constexpr bool split = SPLIT;
    static constexpr bool drain = false;
    static constexpr bool scaled = __is_same(E, _Float16);
    static constexpr bool centred = !SPLIT;  // local offset removed before rounding
    static constexpr int centre_from_q = 0;
    template <int N>
    static __device__ __forceinline__ void pack(const float (&x)[N], Pack* hi, Pack* lo)
    {
#pragma unroll
        for (int p = 0; p < N / 8; ++p)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const E h = (E)x[8 * p + e];
                hi[p][e] = h;
                if (SPLIT) lo[p][e] = (E)(x[8 * p + e] - (float)h);
            }
    }
    static __device__ __forceinline__ void mma1(f4_t& acc, const Pack& ah, const Pack& al,
                                                const Pack& bh, const Pack& bl)
    {
        if (SPLIT) {
            acc = mfma16(acc, al, bh);
            acc = mfma16(acc, ah, bl);
        }
        acc = mfma16(acc, ah, bh);
    }
    // term t of mma1 (lo*hi, hi*lo, hi*hi in that order for the split
    // forms): a loop over t outside a loop over accumulators keeps the
    // dependent products of one accumulator apart, with the same sum order
    static constexpr int TERMS = SPLIT ? 3 : 1;
    static __device__ __forceinline__ void mmat(int t, f4_t& acc, const Pack& ah, const Pack& al,
                                                const Pack& bh, const Pack& bl)
    {
        if (SPLIT && t == 0) acc = mfma16(acc, al, bh);
        else if (SPLIT && t == 1) acc = mfma16(acc, ah, bl);
        else acc = mfma16(acc, ah, bh);
    }
    typedef typename Vec<E>::v2 W2;
    // x -> hi = round(x) and lo = round(x - hi), two values at a time (one
    // packed conversion each; a bfloat16's float value is its bits in the
    // upper half of a word)
    static __device__ __forceinline__ void cvt2(float x0, float x1, W2& hi, W2& lo)
    {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 x = {x0, x1};
        hi = __builtin_convertvector(x, W2);
        if (SPLIT) {
            f2 h;
            if constexpr (__is_same(E, __bf16)) {
                const uint32_t b = __builtin_bit_cast(uint32_t, hi);
                h[0] = __builtin_bit_cast(float, b << 16);
                h[1] = __builtin_bit_cast(float, b & 0xFFFF0000u);
            } else {
                h = __builtin_convertvector(hi, f2);
            }
            lo = __builtin_convertvector(x - h, W2);
        } else {
            lo = hi;
        }
    }
};

template <> struct Form<FUSED_BF16> : Form16<__bf16, false> {};
template <> struct Form<FUSED_BF16X3> : Form16<__bf16, true> {};
template <> struct Form<FUSED_F16> : Form16<_Float16, false> {};
template <> struct Form<FUSED_F16X3> : Form16<_Float16, true> {};

__device__ __forceinline__ int fold_index(int i, int n, int boundary)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (boundary == 0) return -1;
    if (n == 1) return 0;
    const int p = 2 * (n - 1);
    int r = i % p;
    if (r < 0) r += p;
    return r < n ? r : p - r;
}

// Same mapping for indices at most n - 1 outside [0, n): one reflection,
// straight-line code.
__device__ __forceinline__ int fold_once(int i, int n, int boundary)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (boundary == 0) return -1;
    return i < 0 ? -i : 2 * (n - 1) - i;
}

// Workgroup id remap: the hardware deals consecutive ids round-robin to the
// eight XCDs; give each XCD a contiguous range of logical work items so that
// strips sharing image rows meet in the same L2.
__device__ __forceinline__ int xcd_local_id(int b, int nb)
{
    const int q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + min(x, r) + b / 8;
}

// Workgroup barrier that orders LDS only: global loads and stores stay in
// flight across it (a full __syncthreads would wait for the output stores).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Buffer resources: raw buffer loads past num_records return 0 and stores
// past it are dropped, so edge handling needs no branch around a memory
// instruction and the outstanding-access counts stay static.
typedef int i2_t __attribute__((ext_vector_type(2)));
constexpr uint32_t kOutside = 0xFFFFFFF0u;   // an offset past every resource

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

}  // namespace
}  // namespace gabor
