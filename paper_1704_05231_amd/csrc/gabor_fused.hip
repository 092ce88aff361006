// Fused streaming kernel of the Gabor bank (Sec. II, Algorithm 1) on the
// matrix cores.  One workgroup owns one frequency, one horizontal result
// (an orientation theta and, when present, its pi - theta partner, Eq. (13))
// and one 64-column strip of an image row segment.  It walks down the strip
// 16 rows at a time:
//   - the horizontal pass (Eq. (3), (5)-(6)) turns a 16-row image slab into
//     16 new rows of J, kept in an LDS ring of the last L + 16 rows;
//   - the vertical pass (Eq. (4), (7)-(10); Eq. (15)-(16) for the partner)
//     reads the L-row window of J under the next 16 output rows and writes
//     them to memory.
// J never leaves the chip, and each J row is computed once per strip
// segment (plus an L-row lead-in at the segment top).
//
// Both 1-D passes are banded-Toeplitz contractions.  For 16 outputs at
// o = 0..15 along the contracted axis the inputs are k = 0..L-1 starting R
// before the first output; the band entry is krev[k - o] with
// krev[T] = k(R - T) the reversed complex tap k(t) = S(t) exp(i w t), split
// into its cosine (c) and sine (d) parts, and zero outside 0 <= T <= 2R.
// The band is the same for every block, so each wave builds its band
// fragments once and keeps them in registers.
//
//   horizontal:  J[y][x] = sum_k f[y][x0-R+k] * B[k][x]       (A = image)
//   vertical:    F[y][x] = sum_k B[y][k] * J[y0-R+k][x]       (B = J)
//
// The vertical pass forms, with J = a + ib and taps c + id, the products
// P1 = c.a, P2 = d.b, P3 = d.a, P4 = c.b and
//   F_theta = (P1 - P2) + i (P3 + P4),  F_(pi-theta) = (P1 + P2) + i (P3 - P4).
//
// Matrix-core operand layout (16 x 16 output block, lane l = o + 16 g): the
// contracted range of L = 4Q values is split into four contiguous quarters;
// lane group g supplies k = Q g .. Q g + Q - 1 of its row (A) or column (B).
// A 16-bit instruction v_mfma_f32_16x16x32_{bf16,f16} consumes 8 of them per
// lane, the FP32 instruction v_mfma_f32_16x16x4f32 one; every instruction
// pairs the same k on the A and B sides, so the sum runs over all L values.
// Split forms store x = hi + lo in 16-bit and accumulate lo*hi + hi*lo +
// hi*hi in FP32.  Operands are stored in LDS already converted.
#include "gabor_internal.h"

namespace gabor {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kSX = 64;           // strip width: four 16-column blocks, one per wave
constexpr int kThreads = 256;

// Operand storage and matrix-core step for each arithmetic form.
template <int OP> struct Form;

template <> struct Form<FUSED_F32> {
    using T = float;
    static constexpr bool split = false;
    static constexpr int per_mma = 1;     // k values per lane per instruction
    static __device__ __forceinline__ void cvt(float x, T& hi, T& lo) { hi = x; lo = 0.0f; }
    template <int Q>
    static __device__ __forceinline__ void mma(f4_t& acc, const T* ah, const T* al, const T* bh, const T* bl)
    {
        (void)al; (void)bl;
#pragma unroll
        for (int m = 0; m < Q; ++m) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[m], bh[m], acc, 0, 0, 0);
    }
};

template <typename E> struct Vec8;
template <> struct Vec8<__bf16> { typedef __bf16 type __attribute__((ext_vector_type(8))); };
template <> struct Vec8<_Float16> { typedef _Float16 type __attribute__((ext_vector_type(8))); };

__device__ __forceinline__ f4_t mfma16(f4_t acc, Vec8<__bf16>::type a, Vec8<__bf16>::type b)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(f4_t acc, Vec8<_Float16>::type a, Vec8<_Float16>::type b)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
}

template <typename E, bool SPLIT> struct Form16 {
    using T = E;
    static constexpr bool split = SPLIT;
    static constexpr int per_mma = 8;
    static __device__ __forceinline__ void cvt(float x, T& hi, T& lo)
    {
        hi = (T)x;
        lo = SPLIT ? (T)(x - (float)hi) : (T)0.0f;
    }
    using V = typename Vec8<E>::type;
    static __device__ __forceinline__ f4_t one(f4_t acc, const T* a, const T* b)
    {
        V va, vb;
#pragma unroll
        for (int e = 0; e < 8; ++e) { va[e] = a[e]; vb[e] = b[e]; }
        return mfma16(acc, va, vb);
    }
    template <int Q>
    static __device__ __forceinline__ void mma(f4_t& acc, const T* ah, const T* al, const T* bh, const T* bl)
    {
#pragma unroll
        for (int m = 0; m < Q; m += 8) {
            if (SPLIT) {
                acc = one(acc, al + m, bh + m);
                acc = one(acc, ah + m, bl + m);
            }
            acc = one(acc, ah + m, bh + m);
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

// Workgroup id remap: the hardware deals consecutive ids round-robin to the
// eight XCDs; give each XCD a contiguous range of logical work items so that
// strips sharing image rows meet in the same L2.
__device__ __forceinline__ int xcd_local_id(int b, int nb)
{
    const int q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + min(x, r) + b / 8;
}

// 16-byte LDS copies of Q consecutive operand values.
template <typename T, int Q>
__device__ __forceinline__ void lds_get(T* dst, const T* src)
{
    constexpr int per = 16 / sizeof(T);
    static_assert(Q % per == 0, "quarter must be whole 16-byte pieces");
#pragma unroll
    for (int p = 0; p < Q; p += per) *reinterpret_cast<float4*>(dst + p) = *reinterpret_cast<const float4*>(src + p);
}

template <int OP, int Q>
__global__ __launch_bounds__(kThreads) void k_stream(StreamArgs a)
{
    using F = Form<OP>;
    using T = typename F::T;
    constexpr bool SPLIT = F::split;
    constexpr int L = 4 * Q;                 // contracted length per 16-block
    constexpr int RING = L + 16;             // J rows held
    constexpr int PAD = 16 / sizeof(T);
    constexpr int RP = RING + PAD;           // J row pitch (per column)
    constexpr int WF = 48 + L;               // image slab columns
    constexpr int WP = WF + PAD;
    constexpr int NPL = SPLIT ? 2 : 1;       // hi (+ lo) copies
    constexpr int JPLANE = kSX * RP;         // one J component of one copy
    constexpr int FBUF = 16 * WP;            // one slab of one copy

    extern __shared__ float4 stream_lds4[];
    T* Jst = reinterpret_cast<T*>(stream_lds4);             // [NPL][2 comps][kSX][RP]
    T* Fst = Jst + NPL * 2 * JPLANE;                         // [NPL][2 bufs][16][WP]

    const int lid = xcd_local_id(blockIdx.x, gridDim.x);
    const int job = lid % a.n_jobs;
    const int rest = lid / a.n_jobs;
    const int xs = rest % a.n_xs, ys = rest / a.n_xs;
    const FusedJob jb = a.jobs[job];
    const int x0 = xs * kSX, yseg = ys * a.seg_rows;
    const int nsteps = (min(a.seg_rows, a.H - yseg) + 15) / 16;
    const int R = a.R;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int o = lane & 15, g = lane >> 4;
    const bool jr = jb.j_real != 0, cr = jb.c_real != 0;
    const float* tab = a.taps + jb.tap_off;                  // [4][L + 16]: row c, row d, col c, col d
    constexpr int KT = L + 16;

    // Band fragments: lane (o, g) holds krev[Q g + e - o], e = 0..Q-1
    // (entry m of a table holds krev[m - 16]).
    T rch[Q], rcl[Q], rdh[Q], rdl[Q], cch[Q], ccl[Q], cdh[Q], cdl[Q];
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        const int m = 16 + Q * g + e - o;
        F::cvt(tab[m] * a.tap_scale[0], rch[e], rcl[e]);
        F::cvt(tab[KT + m] * a.tap_scale[0], rdh[e], rdl[e]);
        F::cvt(tab[2 * KT + m] * a.tap_scale[1], cch[e], ccl[e]);
        F::cvt(tab[3 * KT + m] * a.tap_scale[1], cdh[e], cdl[e]);
    }

    // ---- image slab staging: rows yseg - R + 16 b + i, columns x0 - R + c
    constexpr int SLAB = 16 * WF;
    constexpr int PER_T = (SLAB + kThreads - 1) / kThreads;
    float pre[PER_T];
    auto slab_load = [&](int b) {
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int idx = tid + k * kThreads;
            float v = 0.0f;
            if (idx < SLAB) {
                const int r = idx / WF, c = idx - r * WF;
                const int yy = fold_index(yseg - R + 16 * b + r, a.H, a.boundary);
                const int xx = fold_index(x0 - R + c, a.W, a.boundary);
                if (yy >= 0 && xx >= 0) v = a.img[(int64_t)yy * a.stride + xx];
            }
            pre[k] = v * a.in_scale;
        }
    };
    auto slab_store = [&](int b) {
        T* hi = Fst + (b & 1) * FBUF;
        T* lo = hi + 2 * FBUF;
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int idx = tid + k * kThreads;
            if (idx < SLAB) {
                const int r = idx / WF, c = idx - r * WF;
                T h, l;
                F::cvt(pre[k], h, l);
                hi[r * WP + c] = h;
                if (SPLIT) lo[r * WP + c] = l;
            }
        }
    };

    // ---- horizontal pass of J block b (16 rows) for column block w
    auto row_pass = [&](int b) {
        const T* fh = Fst + (b & 1) * FBUF + o * WP + 16 * w + Q * g;
        const T* fl = fh + 2 * FBUF;
        T ah[Q], al[Q];
        lds_get<T, Q>(ah, fh);
        if (SPLIT) lds_get<T, Q>(al, fl);
        f4_t re = {0.f, 0.f, 0.f, 0.f}, im = re;
        F::template mma<Q>(re, ah, al, rch, rcl);
        if (!jr) F::template mma<Q>(im, ah, al, rdh, rdl);
        // lane holds J rows 16 b + 4 g + r of column 16 w + o
        const int slot = (16 * b) % RING + 4 * g;
        T* ja = Jst + (16 * w + o) * RP + slot;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T h, l;
            F::cvt(re[r] * a.mid_scale, h, l);
            ja[r] = h;                                  // hi, real part
            if (SPLIT) ja[2 * JPLANE + r] = l;          // lo, real part
            F::cvt(im[r] * a.mid_scale, h, l);
            ja[JPLANE + r] = h;                         // hi, imaginary part
            if (SPLIT) ja[3 * JPLANE + r] = l;          // lo, imaginary part
        }
    };

    // ---- vertical pass of output rows 16 s .. 16 s + 15, column block w
    const int64_t plane = (int64_t)a.H * a.W;
    float2* oa = a.out + (int64_t)jb.out_a * plane;
    float2* ob = jb.out_b >= 0 ? a.out + (int64_t)jb.out_b * plane : nullptr;
    auto col_pass = [&](int s) {
        T bah[Q], bal[Q], bbh[Q], bbl[Q];
        const T* base = Jst + (16 * w + o) * RP;
        constexpr int per = 16 / sizeof(T);
        int slot = (16 * s + Q * g) % RING;
#pragma unroll
        for (int p = 0; p < Q; p += per) {
            const T* src = base + slot;
            *reinterpret_cast<float4*>(bah + p) = *reinterpret_cast<const float4*>(src);
            if (SPLIT) *reinterpret_cast<float4*>(bal + p) = *reinterpret_cast<const float4*>(src + 2 * JPLANE);
            if (!jr) {
                *reinterpret_cast<float4*>(bbh + p) = *reinterpret_cast<const float4*>(src + JPLANE);
                if (SPLIT) *reinterpret_cast<float4*>(bbl + p) = *reinterpret_cast<const float4*>(src + 3 * JPLANE);
            }
            slot += per;
            if (slot >= RING) slot -= RING;
        }
        f4_t P1 = {0.f, 0.f, 0.f, 0.f}, P2 = P1, P3 = P1, P4 = P1;
        F::template mma<Q>(P1, cch, ccl, bah, bal);
        if (!cr) F::template mma<Q>(P3, cdh, cdl, bah, bal);
        if (!jr) {
            F::template mma<Q>(P4, cch, ccl, bbh, bbl);
            if (!cr) F::template mma<Q>(P2, cdh, cdl, bbh, bbl);
        }
        const int x = x0 + 16 * w + o;
        if (x < a.W) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = yseg + 16 * s + 4 * g + r;
                if (y < a.H && 16 * s + 4 * g + r < a.seg_rows) {
                    const float p1 = P1[r] * a.out_scale, p2 = P2[r] * a.out_scale;
                    const float p3 = P3[r] * a.out_scale, p4 = P4[r] * a.out_scale;
                    oa[(int64_t)y * a.W + x] = make_float2(p1 - p2, p3 + p4);
                    if (ob) ob[(int64_t)y * a.W + x] = make_float2(p1 + p2, p3 - p4);
                }
            }
        }
    };

    // ---- lead-in: J blocks 0 .. L/16 - 1, then the slab of block L/16
    constexpr int LEAD = L / 16;
    for (int b = 0; b < LEAD; ++b) {
        slab_load(b);
        slab_store(b);
        __syncthreads();
        row_pass(b);
    }
    if (nsteps > 1) {
        slab_load(LEAD);
        slab_store(LEAD);
    }
    __syncthreads();

    // ---- stream: iteration s computes J block s + LEAD (needed by step
    // s + 1) and output step s; the slab for the next block is fetched from
    // memory during the iteration and staged before the barrier.
    for (int s = 0; s < nsteps; ++s) {
        const bool more = s + 1 < nsteps;         // block s + LEAD is needed
        const bool fetch = s + 2 < nsteps;        // block s + LEAD + 1 is needed
        if (fetch) slab_load(s + LEAD + 1);
        if (more) row_pass(s + LEAD);
        col_pass(s);
        if (fetch) slab_store(s + LEAD + 1);
        __syncthreads();
    }
}

template <int OP, int Q>
hipError_t launch_q(const StreamArgs& a, int n_blocks, hipStream_t stream)
{
    const size_t lds = stream_lds_bytes(OP, Q);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_stream<OP, Q>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_stream<OP, Q>), dim3(n_blocks), dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}

template <int OP>
hipError_t launch_16(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream)
{
    switch (Q) {
        case 8: return launch_q<OP, 8>(a, n_blocks, stream);
        case 16: return launch_q<OP, 16>(a, n_blocks, stream);
        case 24: return launch_q<OP, 24>(a, n_blocks, stream);
        case 32: return launch_q<OP, 32>(a, n_blocks, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_f32(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream)
{
    switch (Q) {
        case 4: return launch_q<FUSED_F32, 4>(a, n_blocks, stream);
        case 8: return launch_q<FUSED_F32, 8>(a, n_blocks, stream);
        case 12: return launch_q<FUSED_F32, 12>(a, n_blocks, stream);
        case 16: return launch_q<FUSED_F32, 16>(a, n_blocks, stream);
        case 20: return launch_q<FUSED_F32, 20>(a, n_blocks, stream);
        case 24: return launch_q<FUSED_F32, 24>(a, n_blocks, stream);
        case 28: return launch_q<FUSED_F32, 28>(a, n_blocks, stream);
        case 32: return launch_q<FUSED_F32, 32>(a, n_blocks, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int stream_quarter(int op, int R)
{
    const int need = 16 + 2 * R;                         // inputs per 16-block
    if (op == FUSED_F32) return ((need + 15) / 16) * 4;  // L multiple of 16
    return ((need + 31) / 32) * 8;                       // L multiple of 32
}

size_t stream_lds_bytes(int op, int Q)
{
    const int L = 4 * Q, RING = L + 16, WF = 48 + L;
    const size_t es = op == FUSED_F32 ? 4 : 2;
    const int pad = (int)(16 / es);
    const size_t npl = (op == FUSED_BF16X3 || op == FUSED_F16X3) ? 2 : 1;
    return npl * es * (2 * (size_t)kSX * (RING + pad) + 2 * 16 * (size_t)(WF + pad));
}

int stream_strip_width() { return kSX; }

hipError_t launch_stream(int op, const StreamArgs& a, int Q, hipStream_t stream)
{
    if (a.n_jobs <= 0) return hipSuccess;
    if (a.seg_rows <= 0 || a.seg_rows % 16 != 0 || 16 + 2 * a.R > 4 * Q || Q > kStreamMaxQuarter)
        return hipErrorInvalidValue;
    const long long nb = (long long)a.n_xs * a.n_ys * a.n_jobs;
    if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return launch_f32(a, Q, (int)nb, stream);
        case FUSED_BF16: return launch_16<FUSED_BF16>(a, Q, (int)nb, stream);
        case FUSED_BF16X3: return launch_16<FUSED_BF16X3>(a, Q, (int)nb, stream);
        case FUSED_F16: return launch_16<FUSED_F16>(a, Q, (int)nb, stream);
        case FUSED_F16X3: return launch_16<FUSED_F16X3>(a, Q, (int)nb, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace gabor
