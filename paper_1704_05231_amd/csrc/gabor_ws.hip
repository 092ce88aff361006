// Wave-specialised streaming kernel of the Gabor bank (Sec. II,
// Algorithm 1) on the matrix cores.  A workgroup owns one frequency, one
// horizontal result (an orientation theta and, when present, its pi - theta
// partner, Eq. (13)) and a segment of one 64-column strip, as the streaming
// kernel of gabor_fused.hip does, but its eight waves split the two passes:
//   - four row waves (one per 16-column block) stage the image slabs and
//     run the horizontal pass (Eq. (3), (5)-(6)): 16 new rows of J per step
//     into an LDS ring;
//   - four column waves (one per 16-column block) run the vertical pass
//     (Eq. (4), (7)-(10); Eq. (15)-(16) for the partner) over the last L
//     rows of J and write the outputs.
// Step t: the row waves compute J block t from slab t, stage slab t + 1 and
// fetch slab t + 2; the column waves compute output block t - L/16 from J
// blocks t - L/16 .. t - 1.  One LDS barrier per step orders everything: the
// ring holds L/16 + 1 blocks (the block being written is never one being
// read) and the slab is double-buffered.  Each wave holds only the band
// fragments of its own pass, so both passes of a column block run
// concurrently on one SIMD, and a matrix-core chain of one wave hides the
// memory and LDS latency of the other.
//
// Operand layout and arithmetic forms are those of gabor_fused.hip: a
// banded-Toeplitz contraction per 16-output block over L = 4Q inputs, lane
// group g supplying the contiguous quarter k = Q g .. Q g + Q - 1; FP32 on
// v_mfma_f32_16x16x4f32, 16-bit forms on v_mfma_f32_16x16x32_{bf16,f16},
// split forms accumulating lo*hi + hi*lo + hi*hi.
#include "gabor_mfma.h"

namespace gabor {
namespace {

constexpr int kWSX = 64;           // strip width: four 16-column blocks
// Cache policy of the output stores: non-temporal (the outputs are written
// once and not read again by the kernel)
constexpr int kStoreNT = 2;
constexpr int kWThreads = 512;     // four row waves, then four column waves
constexpr int kRowThreads = 256;

template <int OP, int Q>
struct WsShape {
    using T = typename Form<OP>::T;
    static constexpr bool SPLIT = Form<OP>::split;
    static constexpr int L = 4 * Q;              // contracted length per 16-block
    static constexpr int LEAD = L / 16;          // J blocks under one output block
    static constexpr int RB = LEAD + 1;          // ring blocks
    static constexpr int RING = 16 * RB;         // ring rows
    static constexpr int PAD = 16 / sizeof(T);
    static constexpr int RP = RING + PAD;        // ring pitch per column
    static constexpr int WF = 48 + L;            // slab columns
    static constexpr int WP = WF + PAD;
    static constexpr int NPL = SPLIT ? 2 : 1;    // hi (+ lo) copies
    static constexpr int JPLANE = kWSX * RP;     // one J component of one copy
    static constexpr int SLAB2 = 16 * WF / 2;    // column pairs per slab
    static constexpr int PER_T = (SLAB2 + kRowThreads - 1) / kRowThreads;
    static constexpr int FROWS = (2 * PER_T * kRowThreads + WF - 1) / WF;
    static constexpr int FBUF = FROWS * WP;      // one slab of one copy (+ padding rows)
    static constexpr size_t lds_bytes = sizeof(T) * ((size_t)NPL * 2 * JPLANE + (size_t)2 * NPL * FBUF);
};

// JR: J is real (horizontal taps have no sine part); CR: vertical taps have
// no sine part (compile-time, so no branch separates a matrix-core chain
// from the reads of its result).  LS: a localized SDFT job (Sec. III): the
// taps are formed from the window weights and twiddles in lt for bins
// (u, v), and the job also stores conj(F_a) and conj(F_b) to the planes
// out_c, out_d (Eq. (20)).
template <int OP, int Q, bool JR, bool CR, bool LS = false>
__device__ __forceinline__ void ws_body(const StreamArgs& a, const FusedJob& jb, int job_rest,
                                        const LsdftTaps* lt = nullptr, int u = 0, int v = 0)
{
    using F = Form<OP>;
    using S = WsShape<OP, Q>;
    using T = typename F::T;
    using Pack = typename F::Pack;
    using W2 = typename F::W2;
    constexpr bool SPLIT = F::split;
    constexpr int NP = Q / F::PER;
    constexpr int L = S::L, LEAD = S::LEAD, RB = S::RB, RING = S::RING, PAD = S::PAD, RP = S::RP;
    constexpr int WF = S::WF, WP = S::WP, NPL = S::NPL, JPLANE = S::JPLANE, SLAB2 = S::SLAB2;
    constexpr int PER_T = S::PER_T, FBUF = S::FBUF;
    constexpr int KT = L + 16;
    constexpr int NCH = Q / PAD;                 // 16-byte operand chunks per fragment
    constexpr int PPC = PAD / F::PER;            // packs per chunk
    constexpr bool CENTRE = F::centred && Q >= F::centre_from_q;   // local offset (see gabor_fused.hip)
    static_assert(16 % sizeof(T) == 0 && Q % (16 / sizeof(T)) == 0, "16-byte pieces");

    extern __shared__ float4 ws_lds4[];
    T* Jst = reinterpret_cast<T*>(ws_lds4);              // [NPL][2 comps][kWSX][RP]
    T* Fst = Jst + NPL * 2 * JPLANE;                       // [2 buffers][NPL][FROWS][WP]
    float* red = reinterpret_cast<float*>(ws_lds4);       // prologue only: 4 partial sums

    const int xs = job_rest % a.n_xs, ys = job_rest / a.n_xs;
    const int x0 = xs * kWSX, yseg = ys * a.seg_rows;
    const int nsteps = (min(a.seg_rows, a.H - yseg) + 15) / 16;   // output blocks
    const int nt = nsteps + LEAD;                                    // steps
    const int R = a.R;
    const int tid = threadIdx.x;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int w = wid & 3, lane = tid & 63, o = lane & 15, g = lane >> 4;
    // [4][L + 16]: row c, row d, col c, col d.  A localized SDFT job forms
    // them first: krev[T] = w[j] exp(-i 2 pi b j / M) at window offset
    // j = T - (R - M/2) (Eq. (17)-(18)), b = u along x and v along y, the FP64
    // product of the window weight and the exact twiddle of index b j mod M
    // rounded once; the table sits in the J ring, which no pass uses before
    // every wave has read its bands.
    const float* tab = a.taps + jb.tap_off;
    const float* tab_raw = tab;                    // unscaled, for the tap sums
    // float16 forms: a copy of the table scaled for range (taps x 2^k, exact)
    // staged in LDS, so that forming the band fragments takes no multiply
    // (with it the Q = 40 split kernel spilled 67 registers to scratch, and
    // every float16 kernel held 8-32 registers more)
    constexpr bool PRESCALED = F::scaled && !LS;
    if constexpr (PRESCALED) {
        float* tl = reinterpret_cast<float*>(ws_lds4) + 16;      // past the prologue sums
        for (int i = tid; i < 4 * KT; i += kWThreads)
            tl[i] = tab[i] * (i < 2 * KT ? a.tap_scale[0] : a.tap_scale[1]);
        lds_barrier();                                             // B0 (this form only)
        tab = tl;
    }
    if constexpr (LS) {
        float* tl = reinterpret_cast<float*>(ws_lds4) + 16;      // past the prologue sums
        for (int i = tid; i < 4 * KT; i += kWThreads) {
            const int set = i / KT, axis = set >> 1;
            const int M = lt->m[axis], j = i - set * KT - 16 - (R - M / 2);
            float val = 0.0f;
            if (j >= 0 && j < M) {
                const int idx = ((axis ? v : u) * j) % M;
                const double wgt = lt->win[axis][j];
                val = (set & 1) ? (float)(-wgt * lt->tw[axis][1][idx]) : (float)(wgt * lt->tw[axis][0][idx]);
            }
            tl[i] = val;
        }
        lds_barrier();                                             // B0 (this job kind only)
        tab = tl;
        tab_raw = tl;
    }
    const float in_s = F::scaled ? a.in_scale : 1.0f, mid_s = F::scaled ? a.mid_scale : 1.0f;
    const float out_s = F::scaled ? a.out_scale : 1.0f;
    auto sc = [](float x, float k) { return F::scaled ? x * k : x; };
    auto uni = [](float x) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
    };

    // Band fragments of one pass: lane (o, g) holds krev[Q g + e - o],
    // e = 0..Q-1, of tap sets c (first) and d (second); entry m of a table
    // row holds krev[m - 16].
    auto band = [&](int row, float scale, Pack (&ch)[NP], Pack (&cl)[NP], Pack (&dh)[NP], Pack (&dl)[NP]) {
        float xc[Q], xd[Q];
#pragma unroll
        for (int e = 0; e < Q; ++e) {
            const int m = 16 + Q * g + e - o;
            xc[e] = PRESCALED ? tab[row * KT + m] : sc(tab[row * KT + m], scale);
            xd[e] = PRESCALED ? tab[(row + 1) * KT + m] : sc(tab[(row + 1) * KT + m], scale);
        }
        F::template pack<Q>(xc, ch, cl);
        F::template pack<Q>(xd, dh, dl);
    };
    // Sum of one tap set (unscaled): lanes o = 0 hold krev[0 .. L-1] between
    // the four lane groups.
    auto tap_sum = [&](int row) {
        float v = 0.f;
        if (o == 0)
#pragma unroll
            for (int e = 0; e < Q; ++e) v += tab_raw[row * KT + 16 + Q * g + e];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        return __shfl(v, 0);
    };

    if (wid < 4) {
        // ================= row waves: slabs and the horizontal pass =================
        Pack bch[NP], bcl[NP], bdh[NP], bdl[NP];
        band(0, F::scaled ? a.tap_scale[0] : 1.0f, bch, bcl, bdh, bdl);
        const int htid = tid;                                  // 0..255
        const __amdgpu_buffer_rsrc_t img_rsrc =
            make_rsrc(a.img, (uint32_t)(((int64_t)(a.H - 1) * a.stride + a.W) * 4));
        // per thread and column pair k: folded columns (fixed for the strip),
        // byte offsets relative to the slab's first row when nothing folds,
        // and LDS positions; lanes past the slab read the first element and
        // write the padding rows
        int col_of[2 * PER_T], lds_at[PER_T], row_of[PER_T];
        uint32_t rel4[2 * PER_T];
        const int xs0 = x0 - R;
        const bool cols_inside = xs0 >= 0 && xs0 + WF <= a.W;
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int idx = htid + k * kRowThreads;
            const int e = 2 * idx;
            const int r = e / WF, c = e - r * WF;
            const bool live = idx < SLAB2;
            row_of[k] = r;
            lds_at[k] = r * WP + c;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                col_of[2 * k + h] = live ? fold_index(xs0 + c + h, a.W, a.boundary) : -1;
                rel4[2 * k + h] = live ? (uint32_t)(r * a.stride + (xs0 + c + h)) * 4u : 0u;
            }
        }
        const bool one_fold = 2 * R + 64 <= a.H;
        // Interior slabs address each element as the thread's fixed offset
        // rel4 (a vector register that lives across the loop) plus the
        // wave-uniform row offset in a scalar register, so that a load's
        // destination never reuses the address register of a load still in
        // flight (which would make the next slab's loads wait for this one's).
        auto slab_rows = [&](int row0, float (&pre)[2 * PER_T]) {
            if (cols_inside && row0 >= 0 && row0 + 16 <= a.H) {
                const int base4 = __builtin_amdgcn_readfirstlane((int)((uint32_t)row0 * (uint32_t)a.stride * 4u));
#pragma unroll
                for (int k = 0; k < 2 * PER_T; ++k)
                    pre[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img_rsrc, (int)rel4[k], base4, 0));
            } else {
                uint32_t off[2 * PER_T];
#pragma unroll
                for (int k = 0; k < PER_T; ++k) {
                    const int yy = one_fold ? fold_once(row0 + row_of[k], a.H, a.boundary)
                                            : fold_index(row0 + row_of[k], a.H, a.boundary);
                    const uint32_t rowoff = (uint32_t)yy * (uint32_t)a.stride;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int cx = col_of[2 * k + h];
                        off[2 * k + h] = (yy >= 0 && cx >= 0) ? (rowoff + (uint32_t)cx) * 4u : kOutside;
                    }
                }
#pragma unroll
                for (int k = 0; k < 2 * PER_T; ++k)
                    pre[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img_rsrc, (int)off[k], 0, 0));
            }
        };
        auto slab_load = [&](int b, float (&pre)[2 * PER_T]) { slab_rows(yseg - R + 16 * b, pre); };
        float cs = 0.f;
        auto slab_store = [&](const float (&pre)[2 * PER_T], int buf) {
            T* hi = Fst + buf * NPL * FBUF;
            T* lo = hi + FBUF;
#pragma unroll
            for (int k = 0; k < PER_T; ++k) {
                W2 h, l;
                if constexpr (CENTRE)
                    F::cvt2(sc(pre[2 * k] - cs, in_s), sc(pre[2 * k + 1] - cs, in_s), h, l);
                else
                    F::cvt2(sc(pre[2 * k], in_s), sc(pre[2 * k + 1], in_s), h, l);
                *reinterpret_cast<W2*>(hi + lds_at[k]) = h;
                if (SPLIT) *reinterpret_cast<W2*>(lo + lds_at[k]) = l;
            }
        };
        // horizontal pass of J block b (16 rows) for column block w, from slab
        // buffer buf; each 16-byte operand chunk is read one chunk ahead of
        // the products that use it
        auto row_pass = [&](int b, int buf) {
            const T* fh = Fst + buf * NPL * FBUF + o * WP + 16 * w + Q * g;
            Pack ch[2][2][PPC];                                  // [buffer][hi, lo][pack]
            auto rd = [&](int c, int k) {
                *reinterpret_cast<float4*>(&ch[k][0][0]) = *reinterpret_cast<const float4*>(fh + c * PAD);
                if (SPLIT) *reinterpret_cast<float4*>(&ch[k][1][0]) = *reinterpret_cast<const float4*>(fh + FBUF + c * PAD);
            };
            f4_t re = {0.f, 0.f, 0.f, 0.f}, im = re;
            rd(0, 0);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (c + 1 < NCH) rd(c + 1, (c + 1) & 1);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < PPC; ++q) {
                    const int p = c * PPC + q;
#pragma unroll
                    for (int t = 0; t < F::TERMS; ++t) {
                        if constexpr (JR) {
                            // real J: even and odd packs on two accumulators
                            // (independent chains), added at the end
                            F::mmat(t, (p & 1) ? im : re, ch[c & 1][0][q], ch[c & 1][1][q], bch[p], bcl[p]);
                        } else {
                            F::mmat(t, re, ch[c & 1][0][q], ch[c & 1][1][q], bch[p], bcl[p]);
                            F::mmat(t, im, ch[c & 1][0][q], ch[c & 1][1][q], bdh[p], bdl[p]);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (F::drain) f32_mfma_drain(re, im);
            if constexpr (JR) re += im;
            // lane holds J rows 16 b + 4 g + r of column 16 w + o
            const int slot = 16 * (b % RB) + 4 * g;
            T* ja = Jst + (16 * w + o) * RP + slot;
            W2 h0, l0, h1, l1;
            F::cvt2(sc(re[0], mid_s), sc(re[1], mid_s), h0, l0);
            F::cvt2(sc(re[2], mid_s), sc(re[3], mid_s), h1, l1);
            reinterpret_cast<W2*>(ja)[0] = h0;
            reinterpret_cast<W2*>(ja)[1] = h1;
            if (SPLIT) {
                reinterpret_cast<W2*>(ja + 2 * JPLANE)[0] = l0;
                reinterpret_cast<W2*>(ja + 2 * JPLANE)[1] = l1;
            }
            if constexpr (!JR) {
                F::cvt2(sc(im[0], mid_s), sc(im[1], mid_s), h0, l0);
                F::cvt2(sc(im[2], mid_s), sc(im[3], mid_s), h1, l1);
                reinterpret_cast<W2*>(ja + JPLANE)[0] = h0;
                reinterpret_cast<W2*>(ja + JPLANE)[1] = h1;
                if (SPLIT) {
                    reinterpret_cast<W2*>(ja + 3 * JPLANE)[0] = l0;
                    reinterpret_cast<W2*>(ja + 3 * JPLANE)[1] = l1;
                }
            }
        };

        float pre_a[2 * PER_T], pre_b[2 * PER_T];
        slab_load(0, pre_a);
        slab_load(1, pre_b);
        if constexpr (CENTRE) {
            // mean of the strip's middle slab over the live lanes, summed in a
            // fixed order, rounded to 8 significant bits
            float mid[2 * PER_T];
            slab_rows(a.H > 16 ? a.H / 2 - 8 : 0, mid);
            float v = 0.f;
#pragma unroll
            for (int k = 0; k < PER_T; ++k)
                if (htid + k * kRowThreads < SLAB2) v += mid[2 * k] + mid[2 * k + 1];
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
            if (lane == 0) red[w] = v;
        }
        lds_barrier();                                             // B1: partial sums visible
        if constexpr (CENTRE) {
            const float mean = ((red[0] + red[1]) + (red[2] + red[3])) * (1.0f / (16 * WF));
            cs = uni(__builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, mean) + 0x8000u) & 0xFFFF0000u));
        }
        slab_store(pre_a, 0);
        lds_barrier();                                             // B2: slab 0 visible, sums read
        // step t: fetch slab t + 2, J block t from slab t (LDS buffer t & 1),
        // stage slab t + 1 (into buffer (t + 1) & 1)
        auto hstep = [&](int t, float (&fet)[2 * PER_T], const float (&stg)[2 * PER_T], int buf) {
            if (t < nt - 1) {
                slab_load(t + 2, fet);
                row_pass(t, buf);
                slab_store(stg, buf ^ 1);
            }
            lds_barrier();
        };
        for (int t = 0; t < nt; t += 2) {
            hstep(t, pre_a, pre_b, 0);
            hstep(t + 1, pre_b, pre_a, 1);
        }
    } else {
        // ================= column waves: the vertical pass and the stores =================
        Pack cch[NP], ccl[NP], cdh[NP], cdl[NP];
        band(2, F::scaled ? a.tap_scale[1] : 1.0f, cch, ccl, cdh, cdl);
        float2 dc_a = make_float2(0.f, 0.f), dc_b = dc_a;
        float tsum[4] = {0.f, 0.f, 0.f, 0.f};
        if constexpr (CENTRE)
#pragma unroll
            for (int k = 0; k < 4; ++k) tsum[k] = tap_sum(k);
        const int64_t plane = (int64_t)a.H * a.W;
        const uint32_t plane_bytes = (uint32_t)(plane * 8);
        const __amdgpu_buffer_rsrc_t out_a = make_rsrc(a.out + (int64_t)jb.out_a * plane, plane_bytes);
        const __amdgpu_buffer_rsrc_t out_b = jb.out_b >= 0
            ? make_rsrc(a.out + (int64_t)jb.out_b * plane, plane_bytes)
            : make_rsrc(a.out, 0u);                              // no partner: every store dropped
        const __amdgpu_buffer_rsrc_t out_c = LS && jb.out_c >= 0
            ? make_rsrc(a.out + (int64_t)jb.out_c * plane, plane_bytes) : make_rsrc(a.out, 0u);
        const __amdgpu_buffer_rsrc_t out_d = LS && jb.out_d >= 0
            ? make_rsrc(a.out + (int64_t)jb.out_d * plane, plane_bytes) : make_rsrc(a.out, 0u);
        // Output offsets: a per-lane base plus a wave-uniform row term.  The
        // last block of a segment that reaches the image bottom may pass it
        // (at most 15 rows: no 32-bit wrap for planes of at most 2^30 bytes);
        // the range check drops those rows.  Lanes of columns past the image
        // store at kOutside.
        const uint32_t W8 = (uint32_t)a.W * 8u;
        const int xcol = x0 + 16 * w + o;
        const bool col_live = xcol < a.W;
        const uint32_t lane_off = ((uint32_t)(yseg + 4 * g) * (uint32_t)a.W + (uint32_t)xcol) * 8u;
        // vertical pass of output block s; each 16-byte operand chunk is read
        // one chunk ahead of the products that use it
        auto col_pass = [&](int s) {
            const T* base = Jst + (16 * w + o) * RP;
            // ring row of each chunk (the window wraps at most once)
            int slot[NCH];
            {
                int sl = (16 * s + Q * g) % RING;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    slot[c] = sl;
                    sl += PAD;
                    if (sl >= RING) sl -= RING;
                }
            }
            Pack ch[2][4][PPC];                                  // [buffer][a hi, a lo, b hi, b lo][pack]
            auto rd = [&](int c, int k) {
                const T* src = base + slot[c];
                *reinterpret_cast<float4*>(&ch[k][0][0]) = *reinterpret_cast<const float4*>(src);
                if (SPLIT) *reinterpret_cast<float4*>(&ch[k][1][0]) = *reinterpret_cast<const float4*>(src + 2 * JPLANE);
                if constexpr (!JR) {
                    *reinterpret_cast<float4*>(&ch[k][2][0]) = *reinterpret_cast<const float4*>(src + JPLANE);
                    if (SPLIT) *reinterpret_cast<float4*>(&ch[k][3][0]) = *reinterpret_cast<const float4*>(src + 3 * JPLANE);
                }
            };
            f4_t P1 = {0.f, 0.f, 0.f, 0.f}, P2 = P1, P3 = P1, P4 = P1;
            rd(0, 0);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (c + 1 < NCH) rd(c + 1, (c + 1) & 1);
                __builtin_amdgcn_sched_barrier(0);
                const int k = c & 1;
#pragma unroll
                for (int q = 0; q < PPC; ++q) {
                    const int p = c * PPC + q;
#pragma unroll
                    for (int t = 0; t < F::TERMS; ++t) {
                        F::mmat(t, P1, cch[p], ccl[p], ch[k][0][q], ch[k][1][q]);
                        if constexpr (!CR) F::mmat(t, P3, cdh[p], cdl[p], ch[k][0][q], ch[k][1][q]);
                        if constexpr (!JR) {
                            F::mmat(t, P4, cch[p], ccl[p], ch[k][2][q], ch[k][3][q]);
                            if constexpr (!CR) F::mmat(t, P2, cdh[p], cdl[p], ch[k][2][q], ch[k][3][q]);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (F::drain) f32_mfma_drain(P1, P2, P3, P4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t off = col_live ? lane_off + (uint32_t)(16 * s + r) * W8 : kOutside;
                const float p1 = sc(P1[r], out_s), p2 = sc(P2[r], out_s);
                const float p3 = sc(P3[r], out_s), p4 = sc(P4[r], out_s);
                i2_t va, vb;
                if constexpr (CENTRE) {
                    va[0] = __builtin_bit_cast(int, (p1 - p2) + dc_a.x);
                    va[1] = __builtin_bit_cast(int, (p3 + p4) + dc_a.y);
                    vb[0] = __builtin_bit_cast(int, (p1 + p2) + dc_b.x);
                    vb[1] = __builtin_bit_cast(int, (p3 - p4) + dc_b.y);
                } else {
                    va[0] = __builtin_bit_cast(int, p1 - p2);
                    va[1] = __builtin_bit_cast(int, p3 + p4);
                    vb[0] = __builtin_bit_cast(int, p1 + p2);
                    vb[1] = __builtin_bit_cast(int, p3 - p4);
                }
                __builtin_amdgcn_raw_buffer_store_b64(va, out_a, (int)off, 0, kStoreNT);
                if constexpr (!JR) __builtin_amdgcn_raw_buffer_store_b64(vb, out_b, (int)off, 0, kStoreNT);
                if constexpr (LS) {
                    // the conjugate bins; absent planes have empty resources
                    va[1] ^= (int)0x80000000;
                    vb[1] ^= (int)0x80000000;
                    __builtin_amdgcn_raw_buffer_store_b64(va, out_c, (int)off, 0, kStoreNT);
                    if constexpr (!JR) __builtin_amdgcn_raw_buffer_store_b64(vb, out_d, (int)off, 0, kStoreNT);
                }
            }
        };
        lds_barrier();                                             // B1
        if constexpr (CENTRE) {
            const float mean = ((red[0] + red[1]) + (red[2] + red[3])) * (1.0f / (16 * WF));
            const float cs = uni(__builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, mean) + 0x8000u) & 0xFFFF0000u));
            // c times the constant responses (hc + i hd)(vc + i vd), (hc - i hd)(vc + i vd)
            const float hc = tsum[0], hd = tsum[1], vc = tsum[2], vd = tsum[3];
            dc_a = make_float2(uni(cs * (vc * hc - vd * hd)), uni(cs * (vc * hd + vd * hc)));
            dc_b = make_float2(uni(cs * (vc * hc + vd * hd)), uni(cs * (vd * hc - vc * hd)));
        }
        lds_barrier();                                             // B2
        // the same number of barriers as the row waves: steps in pairs
        for (int t = 0; t < nt; t += 2) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (t + k >= LEAD && t + k < nt) col_pass(t + k - LEAD);
                lds_barrier();
            }
        }
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kWThreads) void k_ws(StreamArgs a)
{
    int lid = xcd_local_id(blockIdx.x, gridDim.x);
    if (a.n_images > 1) {
        // strided batch: image-major workgroup ids, each image's own grid after
        const int per = a.n_xs * a.n_ys * a.n_jobs;
        const int b = lid / per;
        lid -= b * per;
        a.img += b * a.img_bstride;
        a.out += b * a.out_bstride;
    }
    const FusedJob jb = a.jobs[lid % a.n_jobs];
    const int rest = lid / a.n_jobs;
    if (jb.j_real) ws_body<OP, Q, true, false>(a, jb, rest);
    else if (jb.c_real) ws_body<OP, Q, false, true>(a, jb, rest);
    else ws_body<OP, Q, false, false>(a, jb, rest);
}

// Batched tiles: workgroup b takes tile b of a table sorted by decreasing
// cost, so the dispatcher hands out the longest tiles first and the rest as
// workgroups free up (a dynamic queue without atomics).
template <int OP, int Q>
__device__ __forceinline__ void ws_tile(const WsTilesArgs& t, const BatchTile& tl, const BatchImage& im,
                                        const BatchFreq& fq)
{
    StreamArgs a{};
    a.img = im.img;
    a.stride = im.stride;
    a.H = im.H;
    a.W = im.W;
    a.boundary = t.boundary;
    a.R = fq.R;
    a.seg_rows = fq.seg_rows;
    a.n_xs = im.n_xs;
    a.jobs = t.jobs;
    a.taps = t.taps;
    a.out = im.out;
    a.in_scale = fq.in_scale;
    a.mid_scale = fq.mid_scale;
    a.out_scale = fq.out_scale;
    a.tap_scale[0] = fq.tap_scale[0];
    a.tap_scale[1] = fq.tap_scale[1];
    const FusedJob jb = t.jobs[tl.job];
    if (jb.j_real) ws_body<OP, Q, true, false>(a, jb, tl.rest);
    else if (jb.c_real) ws_body<OP, Q, false, true>(a, jb, tl.rest);
    else ws_body<OP, Q, false, false>(a, jb, tl.rest);
}

template <int OP, int Q>
__global__ __launch_bounds__(kWThreads) void k_ws_tiles(WsTilesArgs t)
{
    const BatchTile tl = t.tiles[blockIdx.x];
    ws_tile<OP, Q>(t, tl, t.images[tl.image], t.freqs[tl.freq]);
}

// Tiles of several small quarters in one launch (sorted by decreasing cost
// across them): each workgroup runs the body of its tile's quarter.  The
// launch holds the largest member's registers and LDS, which for these
// quarters leaves as many workgroups per compute unit as that member alone.
template <int OP, int... Qs>
__device__ __forceinline__ void ws_tile_any(const WsTilesArgs& t, const BatchTile& tl, const BatchImage& im,
                                            const BatchFreq& fq)
{
    bool done = false;
    ((!done && fq.q == Qs ? (ws_tile<OP, Qs>(t, tl, im, fq), done = true) : false), ...);
}

template <int OP>
__global__ __launch_bounds__(kWThreads) void k_ws_tiles_small(WsTilesArgs t)
{
    const BatchTile tl = t.tiles[blockIdx.x];
    const BatchImage im = t.images[tl.image];
    const BatchFreq fq = t.freqs[tl.freq];
    if constexpr (OP == FUSED_F32) ws_tile_any<OP, 4, 8, 12, 16>(t, tl, im, fq);
    else ws_tile_any<OP, 8, 16>(t, tl, im, fq);
}
static_assert(kWsSmallQuarter == 16, "the small launch's quarter lists end at 16");

// Localized SDFT (Sec. III) on the wave-specialised structure: job (u, v),
// u <= Mx/2, v <= My/2, computes J_u once (Eq. (18)), F_{u,v} and
// F_{Mx-u,v} from J_u and its conjugate (Eq. (19)), and stores the
// conjugates to F_{Mx-u,My-v} and F_{u,My-v} (Eq. (20)); planes are indexed
// v Mx + u.  Bins u in {0, Mx/2} have a real J_u and no partner; v in
// {0, My/2} real vertical taps, whose conjugate outputs coincide with the
// direct ones.
template <int OP, int Q>
__global__ __launch_bounds__(kWThreads) void k_ws_lsdft(StreamArgs a, LsdftTaps t)
{
    const int lid = xcd_local_id(blockIdx.x, gridDim.x);
    const int job = lid % a.n_jobs, rest = lid / a.n_jobs;
    const int mx = t.m[0], my = t.m[1], nu = mx / 2 + 1;
    const int u = job % nu, v = job / nu;
    const int mu = u == 0 ? 0 : mx - u, mv = v == 0 ? 0 : my - v;
    FusedJob jb{};
    jb.j_real = u == mu;
    jb.c_real = v == mv;
    jb.out_a = v * mx + u;
    jb.out_b = jb.j_real ? -1 : v * mx + mu;
    jb.out_c = jb.c_real ? -1 : mv * mx + mu;
    jb.out_d = (jb.c_real || jb.j_real) ? -1 : mv * mx + u;
    if (jb.j_real) ws_body<OP, Q, true, false, true>(a, jb, rest, &t, u, v);
    else if (jb.c_real) ws_body<OP, Q, false, true, true>(a, jb, rest, &t, u, v);
    else ws_body<OP, Q, false, false, true>(a, jb, rest, &t, u, v);
}

// Dynamic-LDS limits of the two kernels of one form and quarter (raised at
// plan creation, so that no launch captured in a graph needs to).
template <int OP, int Q>
LdsLimit ws_tiles_limit;
template <int OP, int Q>
LdsLimit ws_limit;

template <int OP, int Q>
hipError_t launch_ws_tiles_q(const WsTilesArgs& t, hipStream_t stream)
{
    const size_t lds = WsShape<OP, Q>::lds_bytes;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    {
        const hipError_t e = ws_tiles_limit<OP, Q>.ensure((const void*)k_ws_tiles<OP, Q>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_ws_tiles<OP, Q>), dim3(t.n_tiles), dim3(kWThreads), lds, stream, t);
    return hipGetLastError();
}

template <int OP, int... Qs>
hipError_t launch_ws_tiles_list(const WsTilesArgs& t, int Q, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_ws_tiles_q<OP, Qs>(t, stream)) : (void)0), ...);
    return e;
}

template <int OP, int Q>
hipError_t launch_ws_q(const StreamArgs& a, int n_blocks, hipStream_t stream)
{
    const size_t lds = WsShape<OP, Q>::lds_bytes;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    {
        const hipError_t e = ws_limit<OP, Q>.ensure((const void*)k_ws<OP, Q>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_ws<OP, Q>), dim3(n_blocks), dim3(kWThreads), lds, stream, a);
    return hipGetLastError();
}

template <int OP, int Q>
LdsLimit ws_lsdft_limit;

template <int OP, int Q>
hipError_t launch_ws_lsdft_q(const StreamArgs& a, const LsdftTaps& t, int n_blocks, hipStream_t stream)
{
    const size_t lds = WsShape<OP, Q>::lds_bytes;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    {
        const hipError_t e = ws_lsdft_limit<OP, Q>.ensure((const void*)k_ws_lsdft<OP, Q>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_ws_lsdft<OP, Q>), dim3(n_blocks), dim3(kWThreads), lds, stream, a, t);
    return hipGetLastError();
}

template <int OP, int... Qs>
hipError_t launch_ws_lsdft_list(const StreamArgs& a, const LsdftTaps& t, int Q, int n_blocks, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_ws_lsdft_q<OP, Qs>(a, t, n_blocks, stream)) : (void)0), ...);
    return e;
}

template <int OP, int Q>
hipError_t prepare_ws_q()
{
    const size_t lds = WsShape<OP, Q>::lds_bytes;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = ws_limit<OP, Q>.ensure((const void*)k_ws<OP, Q>, lds);
    if (e == hipSuccess) e = ws_tiles_limit<OP, Q>.ensure((const void*)k_ws_tiles<OP, Q>, lds);
    return e;
}

template <int OP, int... Qs>
hipError_t prepare_ws_list(int Q)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = prepare_ws_q<OP, Qs>()) : (void)0), ...);
    return e;
}

template <int OP, int... Qs>
hipError_t launch_ws_list(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_ws_q<OP, Qs>(a, n_blocks, stream)) : (void)0), ...);
    return e;
}

}  // namespace

#ifndef GABOR_FORM
#error "compile gabor_ws.hip with -DGABOR_FORM=<FusedOp>"
#endif

template <>
hipError_t ws_form<GABOR_FORM>(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return launch_ws_list<GABOR_FORM, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 52>(a, Q, n_blocks, stream);
    else
        if constexpr (Form<GABOR_FORM>::split)
            return launch_ws_list<GABOR_FORM, 8, 16, 24, 32, 40>(a, Q, n_blocks, stream);
        else
            return launch_ws_list<GABOR_FORM, 8, 16, 24, 32, 40, 48, 56>(a, Q, n_blocks, stream);
}

template <>
hipError_t ws_prepare_form<GABOR_FORM>(int Q)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return prepare_ws_list<GABOR_FORM, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 52>(Q);
    else
        if constexpr (Form<GABOR_FORM>::split)
            return prepare_ws_list<GABOR_FORM, 8, 16, 24, 32, 40>(Q);
        else
            return prepare_ws_list<GABOR_FORM, 8, 16, 24, 32, 40, 48, 56>(Q);
}

// The localized SDFT uses windows of M <= 64 (R <= 32: Q <= 20 in FP32, 24
// in the 16-bit forms).
template <>
hipError_t ws_lsdft_form<GABOR_FORM>(const StreamArgs& a, const LsdftTaps& t, int Q, int n_blocks,
                                     hipStream_t stream)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return launch_ws_lsdft_list<GABOR_FORM, 4, 8, 12, 16, 20>(a, t, Q, n_blocks, stream);
    else
        return launch_ws_lsdft_list<GABOR_FORM, 8, 16, 24>(a, t, Q, n_blocks, stream);
}

static LdsLimit ws_small_limit;

template <>
hipError_t ws_small_form<GABOR_FORM>(const WsTilesArgs* t, hipStream_t stream)
{
    const size_t lds = WsShape<GABOR_FORM, kWsSmallQuarter>::lds_bytes;   // the largest member's
    const hipError_t e = ws_small_limit.ensure((const void*)k_ws_tiles_small<GABOR_FORM>, lds);
    if (e != hipSuccess || !t) return e;
    hipLaunchKernelGGL((k_ws_tiles_small<GABOR_FORM>), dim3(t->n_tiles), dim3(kWThreads), lds, stream, *t);
    return hipGetLastError();
}

template <>
hipError_t ws_tiles_form<GABOR_FORM>(const WsTilesArgs& t, int Q, hipStream_t stream)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return launch_ws_tiles_list<GABOR_FORM, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 52>(t, Q, stream);
    else
        if constexpr (Form<GABOR_FORM>::split)
            return launch_ws_tiles_list<GABOR_FORM, 8, 16, 24, 32, 40>(t, Q, stream);
        else
            return launch_ws_tiles_list<GABOR_FORM, 8, 16, 24, 32, 40, 48, 56>(t, Q, stream);
}

#if GABOR_FORM == 0

size_t ws_lds_bytes(int op, int Q)
{
    if (!ws_supported(op, Q)) return 0;
    const int L = 4 * Q, RING = 16 * (L / 16 + 1), WF = 48 + L;
    const size_t es = op == FUSED_F32 ? 4 : 2;
    const int pad = (int)(16 / es);
    const size_t npl = (op == FUSED_BF16X3 || op == FUSED_F16X3) ? 2 : 1;
    const int per_t = (16 * WF / 2 + kRowThreads - 1) / kRowThreads;
    const int frows = (2 * per_t * kRowThreads + WF - 1) / WF;
    return es * (npl * 2 * (size_t)kWSX * (RING + pad) + 2 * npl * (size_t)frows * (WF + pad));
}

hipError_t launch_ws_tiles(int op, const WsTilesArgs& t, int Q, hipStream_t stream)
{
    if (t.n_tiles <= 0) return hipSuccess;
    if (!ws_supported(op, Q) || !t.images || !t.freqs || !t.tiles || !t.jobs || !t.taps) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return ws_tiles_form<FUSED_F32>(t, Q, stream);
        case FUSED_BF16: return ws_tiles_form<FUSED_BF16>(t, Q, stream);
        case FUSED_BF16X3: return ws_tiles_form<FUSED_BF16X3>(t, Q, stream);
        case FUSED_F16: return ws_tiles_form<FUSED_F16>(t, Q, stream);
        case FUSED_F16X3: return ws_tiles_form<FUSED_F16X3>(t, Q, stream);
    }
    return hipErrorInvalidValue;
}

bool ws_small_quarter(int op, int Q)
{
    return Q <= kWsSmallQuarter && ws_supported(op, Q);
}

hipError_t launch_ws_tiles_small(int op, const WsTilesArgs& t, hipStream_t stream)
{
    if (t.n_tiles <= 0) return hipSuccess;
    if (!t.images || !t.freqs || !t.tiles || !t.jobs || !t.taps) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return ws_small_form<FUSED_F32>(&t, stream);
        case FUSED_BF16: return ws_small_form<FUSED_BF16>(&t, stream);
        case FUSED_BF16X3: return ws_small_form<FUSED_BF16X3>(&t, stream);
        case FUSED_F16: return ws_small_form<FUSED_F16>(&t, stream);
        case FUSED_F16X3: return ws_small_form<FUSED_F16X3>(&t, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_ws_small(int op)
{
    switch (op) {
        case FUSED_F32: return ws_small_form<FUSED_F32>(nullptr, nullptr);
        case FUSED_BF16: return ws_small_form<FUSED_BF16>(nullptr, nullptr);
        case FUSED_BF16X3: return ws_small_form<FUSED_BF16X3>(nullptr, nullptr);
        case FUSED_F16: return ws_small_form<FUSED_F16>(nullptr, nullptr);
        case FUSED_F16X3: return ws_small_form<FUSED_F16X3>(nullptr, nullptr);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_ws(int op, int Q)
{
    if (!ws_supported(op, Q)) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return ws_prepare_form<FUSED_F32>(Q);
        case FUSED_BF16: return ws_prepare_form<FUSED_BF16>(Q);
        case FUSED_BF16X3: return ws_prepare_form<FUSED_BF16X3>(Q);
        case FUSED_F16: return ws_prepare_form<FUSED_F16>(Q);
        case FUSED_F16X3: return ws_prepare_form<FUSED_F16X3>(Q);
    }
    return hipErrorInvalidValue;
}

int ws_quarter(int op, int R)
{
    const int need = 16 + 2 * R;
    return op == FUSED_F32 ? (need + 15) / 16 * 4 : (need + 31) / 32 * 8;
}

int ws_max_quarter(int op)
{
    // Registers without spills (each wave holds one pass's band fragments:
    // FP32 Q = 52 128 + 110 per lane, single 16-bit Q = 56 229, split Q = 40
    // 251; one more step spills) and LDS within 160 KB (FP32 Q = 52 147 KB)
    if (op == FUSED_F32) return 52;
    return op == FUSED_BF16X3 || op == FUSED_F16X3 ? 40 : 56;
}

bool ws_supported(int op, int Q)
{
    if (Q > ws_max_quarter(op)) return false;
    return op == FUSED_F32 ? Q % 4 == 0 : Q % 8 == 0;
}

hipError_t launch_ws_lsdft(int op, const StreamArgs& a, const LsdftTaps& t, int Q, hipStream_t stream)
{
    if (a.n_jobs <= 0) return hipSuccess;
    if (!ws_supported(op, Q) || a.seg_rows <= 0 || a.seg_rows % 16 != 0 || 16 + 2 * a.R > 4 * Q)
        return hipErrorInvalidValue;
    if ((int64_t)a.H * a.W * 8 > (int64_t(1) << 30)) return hipErrorInvalidValue;
    const long long nb = (long long)a.n_xs * a.n_ys * a.n_jobs;
    if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return ws_lsdft_form<FUSED_F32>(a, t, Q, (int)nb, stream);
        case FUSED_BF16: return ws_lsdft_form<FUSED_BF16>(a, t, Q, (int)nb, stream);
        case FUSED_BF16X3: return ws_lsdft_form<FUSED_BF16X3>(a, t, Q, (int)nb, stream);
        case FUSED_F16: return ws_lsdft_form<FUSED_F16>(a, t, Q, (int)nb, stream);
        case FUSED_F16X3: return ws_lsdft_form<FUSED_F16X3>(a, t, Q, (int)nb, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ws(int op, const StreamArgs& a, int Q, hipStream_t stream)
{
    if (a.n_jobs <= 0) return hipSuccess;
    if (!ws_supported(op, Q) || a.seg_rows <= 0 || a.seg_rows % 16 != 0 || 16 + 2 * a.R > 4 * Q)
        return hipErrorInvalidValue;
    if ((int64_t)a.H * a.W * 8 > (int64_t(1) << 30)) return hipErrorInvalidValue;
    if (a.n_images > 1 && (a.img_bstride < 0 || a.out_bstride < 0)) return hipErrorInvalidValue;
    const long long nb = (long long)a.n_xs * a.n_ys * a.n_jobs * (a.n_images > 1 ? a.n_images : 1);
    if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return ws_form<FUSED_F32>(a, Q, (int)nb, stream);
        case FUSED_BF16: return ws_form<FUSED_BF16>(a, Q, (int)nb, stream);
        case FUSED_BF16X3: return ws_form<FUSED_BF16X3>(a, Q, (int)nb, stream);
        case FUSED_F16: return ws_form<FUSED_F16>(a, Q, (int)nb, stream);
        case FUSED_F16X3: return ws_form<FUSED_F16X3>(a, Q, (int)nb, stream);
    }
    return hipErrorInvalidValue;
}
#endif

}  // namespace gabor
