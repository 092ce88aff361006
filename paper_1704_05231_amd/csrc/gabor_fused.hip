// Fused streaming kernel of the Gabor bank (Sec. II, Algorithm 1) on the
// matrix cores.  One workgroup owns one frequency, one horizontal result
// (an orientation theta and, when present, its pi - theta partner, Eq. (13))
// and one 64-column strip of an image row segment.  It walks down the strip
// 16 rows at a time:
//   - the horizontal pass (Eq. (3), (5)-(6)) turns a 16-row image slab into
//     16 new rows of J, kept in an LDS ring of the last L rows;
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
#include "gabor_mfma.h"

namespace gabor {
namespace {

constexpr int kSX = 64;           // strip width: four 16-column blocks, one per wave
constexpr int kThreads = 256;

// JR: J is real (horizontal taps have no sine part); CR: vertical taps have
// no sine part.  Both are compile-time so that no branch separates a
// matrix-core chain from the reads of its result.
// LS: a localized SDFT job (Sec. III): the taps are formed from the window
// weights and twiddles in lt for bins (u, v), and the job also stores
// conj(F_a) and conj(F_b) to the planes out_c, out_d (Eq. (20)).
template <int OP, int Q, bool JR, bool CR, bool LS>
__device__ __forceinline__ void stream_body(const StreamArgs& a, const FusedJob& jb, int job_rest,
                                            const LsdftTaps* lt, int u, int v)
{
    using F = Form<OP>;
    using T = typename F::T;
    using Pack = typename F::Pack;
    using W2 = typename F::W2;
    constexpr bool SPLIT = F::split;
    constexpr int NP = Q / F::PER;           // packs per fragment
    constexpr int L = 4 * Q;                 // contracted length per 16-block
    constexpr int RING = L;                  // J rows held: one band window
    constexpr int PAD = 16 / sizeof(T);
    constexpr int RP = RING + PAD;           // J row pitch (per column)
    constexpr int WF = 48 + L;               // image slab columns
    constexpr int WP = WF + PAD;
    constexpr int NPL = SPLIT ? 2 : 1;       // hi (+ lo) copies
    constexpr int JPLANE = kSX * RP;         // one J component of one copy
    constexpr int SLAB2 = 16 * WF / 2;       // column pairs per slab
    constexpr int PER_T = (SLAB2 + kThreads - 1) / kThreads;
    constexpr int FROWS = (2 * PER_T * kThreads + WF - 1) / WF;
    constexpr int FBUF = FROWS * WP;         // one slab of one copy (+ padding rows)
    static_assert(16 % sizeof(T) == 0 && Q % (16 / sizeof(T)) == 0, "16-byte pieces");
    constexpr bool CENTRE = F::centred && Q >= F::centre_from_q;   // local offset (below)

    extern __shared__ float4 stream_lds4[];
    T* Jst = reinterpret_cast<T*>(stream_lds4);             // [NPL][2 comps][kSX][RP]
    T* Fst = Jst + NPL * 2 * JPLANE;                         // [NPL][FROWS][WP]

    const int xs = job_rest % a.n_xs, ys = job_rest / a.n_xs;
    const int x0 = xs * kSX, yseg = ys * a.seg_rows;
    const int nsteps = (min(a.seg_rows, a.H - yseg) + 15) / 16;
    const int R = a.R;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int o = lane & 15, g = lane >> 4;
    const float* tab = a.taps + jb.tap_off;                  // [4][L + 16]: row c, row d, col c, col d
    constexpr int KT = L + 16;
    // float16 range scales (all exactly 1 for the other forms)
    const float in_s = F::scaled ? a.in_scale : 1.0f, mid_s = F::scaled ? a.mid_scale : 1.0f;
    const float out_s = F::scaled ? a.out_scale : 1.0f;
    const float rt_s = F::scaled ? a.tap_scale[0] : 1.0f, ct_s = F::scaled ? a.tap_scale[1] : 1.0f;
    auto sc = [](float x, float k) { return F::scaled ? x * k : x; };

    // Band fragments: lane (o, g) holds krev[Q g + e - o], e = 0..Q-1
    // (entry m of a table holds krev[m - 16]).
    Pack rch[NP], rcl[NP], rdh[NP], rdl[NP], cch[NP], ccl[NP], cdh[NP], cdl[NP];
    // Forms with the local offset: sums of the four tap sets (unscaled), for
    // the response to a constant (see the local offset below).
    float tsum[4] = {0.f, 0.f, 0.f, 0.f};
    {
        float x0v[Q], x1v[Q], x2v[Q], x3v[Q];
        if constexpr (LS) {
            // Localized SDFT: krev[T] = w[j] exp(-i 2 pi b j / M) at window
            // offset j = T - (R - M/2) (Eq. (17)-(18)), b = u on the
            // horizontal axis and v on the vertical one; the FP64 product of
            // the window weight and the exact twiddle of index b j mod M is
            // rounded once.  The workgroup writes the four sets to the J ring
            // (not yet in use) and every lane reads its band from there.
            float* tl = reinterpret_cast<float*>(stream_lds4);
            for (int i = tid; i < 4 * KT; i += kThreads) {
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
            lds_barrier();
#pragma unroll
            for (int e = 0; e < Q; ++e) {
                const int m = 16 + Q * g + e - o;
                x0v[e] = tl[m];
                x1v[e] = tl[KT + m];
                x2v[e] = tl[2 * KT + m];
                x3v[e] = tl[3 * KT + m];
            }
        } else {
#pragma unroll
            for (int e = 0; e < Q; ++e) {
                const int m = 16 + Q * g + e - o;
                x0v[e] = tab[m];
                x1v[e] = tab[KT + m];
                x2v[e] = tab[2 * KT + m];
                x3v[e] = tab[3 * KT + m];
            }
        }
        if constexpr (CENTRE) {
            // lanes o = 0 (one per lane group) hold krev[0 .. L-1] between
            // them, which covers every nonzero tap
#pragma unroll
            for (int e = 0; e < Q; ++e) {
                tsum[0] += x0v[e];
                tsum[1] += x1v[e];
                tsum[2] += x2v[e];
                tsum[3] += x3v[e];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float v = o == 0 ? tsum[k] : 0.f;
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                tsum[k] = __shfl(v, 0);
            }
        }
#pragma unroll
        for (int e = 0; e < Q; ++e) {
            x0v[e] = sc(x0v[e], rt_s);
            x1v[e] = sc(x1v[e], rt_s);
            x2v[e] = sc(x2v[e], ct_s);
            x3v[e] = sc(x3v[e], ct_s);
        }
        F::template pack<Q>(x0v, rch, rcl);
        F::template pack<Q>(x1v, rdh, rdl);
        F::template pack<Q>(x2v, cch, ccl);
        F::template pack<Q>(x3v, cdh, cdl);
    }

    // ---- image slab staging, by column pairs: rows yseg - R + 16 b + i,
    // columns xs0 + c (lanes past the slab read nothing and write the
    // padding rows).
    const __amdgpu_buffer_rsrc_t img_rsrc =
        make_rsrc(a.img, (uint32_t)(((int64_t)(a.H - 1) * a.stride + a.W) * 4));
    // Per thread and pair k: the folded columns (fixed for the strip), the
    // offset relative to the slab's first row when no row or column folds
    // (rel), and the LDS position.
    // rel4: byte offset from the slab's first row; lanes past the slab read
    // the first element (their values land in padding rows and are never used)
    int col_of[2 * PER_T], lds_at[PER_T], row_of[PER_T];
    uint32_t rel4[2 * PER_T];
    const int xs0 = x0 - R;
    const bool cols_inside = xs0 >= 0 && xs0 + WF <= a.W;
#pragma unroll
    for (int k = 0; k < PER_T; ++k) {
        const int idx = tid + k * kThreads;
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
    // one reflection reaches every folded row when the band is shorter than
    // the image; otherwise the general (division) form
    const bool one_fold = 2 * R + 64 <= a.H;
    // 16 image rows from row0 (folded or zero-extended by the boundary rule)
    // The two cases only form byte offsets; the loads are issued after the
    // branch, so the outstanding-access count is the same on both paths and
    // the compiler need not drain every load and store in flight (the
    // previous step's output stores included) before reusing the registers.
    auto slab_rows = [&](int row0, float (&pre)[2 * PER_T]) {
        uint32_t off[2 * PER_T];
        if (cols_inside && row0 >= 0 && row0 + 16 <= a.H) {
            // interior: no folding, one add per element
            const uint32_t base4 = (uint32_t)row0 * (uint32_t)a.stride * 4u;
#pragma unroll
            for (int k = 0; k < 2 * PER_T; ++k) off[k] = base4 + rel4[k];
        } else {
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
        }
#pragma unroll
        for (int k = 0; k < 2 * PER_T; ++k)
            pre[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img_rsrc, (int)off[k], 0, 0));
    };
    auto slab_load = [&](int b, float (&pre)[2 * PER_T]) { slab_rows(yseg - R + 16 * b, pre); };
    // Local offset (single 16-bit forms; FP32 for R > 56).  By linearity
    // the bank of f equals the bank of f - c plus c times the response to a
    // constant, and that response is (sum of the vertical taps) x (sum of
    // the horizontal taps), conjugated on the horizontal factor for the
    // pi - theta partner, at
    // every pixel and for either boundary rule when c is subtracted from
    // every sample the passes read (zero-extended ones included).  Each
    // workgroup takes c as the mean of the 16 x (64 + L) slab of its strip
    // at the middle rows of the image: J and the image are then rounded to
    // 16 bits without their local mean, which removes the largest part of
    // the rounding error of the low-frequency channels; in FP32 it keeps the
    // accumulators and J near the size of the response, whose peak at
    // omega sigma = pi is about 1 % of the image's mean (below R = 56 FP32
    // meets its bar without it, and the extra registers cost about 4 %).
    // Every segment of a strip takes the same c, so results do not depend on
    // the segment height.  The split forms use c = 0.
    float cs = 0.f;
    auto slab_store = [&](const float (&pre)[2 * PER_T]) {
        T* hi = Fst;
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

    // 16-byte LDS reads straight into operand packs.
    auto frag_get = [&](Pack* dst, const T* src) {
#pragma unroll
        for (int p = 0; p < Q; p += PAD)
            *reinterpret_cast<float4*>(reinterpret_cast<T*>(dst) + p) = *reinterpret_cast<const float4*>(src + p);
    };

    // ---- horizontal pass of J block b (16 rows) for column block w
    auto row_pass = [&](int b) {
        const T* fh = Fst + o * WP + 16 * w + Q * g;
        Pack ah[NP], al[NP];
        frag_get(ah, fh);
        if (SPLIT) frag_get(al, fh + FBUF);
        f4_t re = {0.f, 0.f, 0.f, 0.f}, im = re;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int t = 0; t < F::TERMS; ++t) {
                F::mmat(t, re, ah[p], al[p], rch[p], rcl[p]);
                if constexpr (!JR) F::mmat(t, im, ah[p], al[p], rdh[p], rdl[p]);
            }
        }
        if constexpr (F::drain) f32_mfma_drain(re, im);
        // lane holds J rows 16 b + 4 g + r of column 16 w + o: four
        // consecutive ring entries per component and copy
        const int slot = (16 * b) % RING + 4 * g;
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

    // ---- vertical pass of output rows 16 s .. 16 s + 15, column block w
    const int64_t plane = (int64_t)a.H * a.W;
    const uint32_t plane_bytes = (uint32_t)(plane * 8);
    const __amdgpu_buffer_rsrc_t out_a = make_rsrc(a.out + (int64_t)jb.out_a * plane, plane_bytes);
    const __amdgpu_buffer_rsrc_t out_b = jb.out_b >= 0
        ? make_rsrc(a.out + (int64_t)jb.out_b * plane, plane_bytes)
        : make_rsrc(a.out, 0u);                                 // no partner: every store dropped
    // conjugate fill: planes that receive conj(F_a), conj(F_b)
    const __amdgpu_buffer_rsrc_t out_c = LS && jb.out_c >= 0
        ? make_rsrc(a.out + (int64_t)jb.out_c * plane, plane_bytes) : make_rsrc(a.out, 0u);
    const __amdgpu_buffer_rsrc_t out_d = LS && jb.out_d >= 0
        ? make_rsrc(a.out + (int64_t)jb.out_d * plane, plane_bytes) : make_rsrc(a.out, 0u);
    // Output offsets: a per-lane base plus a wave-uniform row term.  Rows past
    // the segment end are written only in the last step of an odd step
    // count, which happens only where the segment reaches the image bottom
    // (segments are multiples of 32 rows or cover the image), so those rows
    // lie past the plane (at most 31 rows past it: no 32-bit wrap for planes
    // of at most 2^30 bytes) and the range check drops them.  Lanes of
    // columns past the image (last strip only) store at kOutside.
    const uint32_t W8 = (uint32_t)a.W * 8u;
    const int xcol = x0 + 16 * w + o;
    const bool col_live = xcol < a.W;
    const uint32_t lane_off = ((uint32_t)(yseg + 4 * g) * (uint32_t)a.W + (uint32_t)xcol) * 8u;
    // c times the constant responses (hc + i hd)(vc + i vd) and
    // (hc - i hd)(vc + i vd); set once cs is known
    float2 dc_a = make_float2(0.f, 0.f), dc_b = dc_a;
    auto col_pass = [&](int s) {
        Pack bah[NP], bal[NP], bbh[NP], bbl[NP];
        const T* base = Jst + (16 * w + o) * RP;
        int slot = (16 * s + Q * g) % RING;
#pragma unroll
        for (int p = 0; p < Q; p += PAD) {
            const T* src = base + slot;
            *reinterpret_cast<float4*>(reinterpret_cast<T*>(bah) + p) = *reinterpret_cast<const float4*>(src);
            if (SPLIT) *reinterpret_cast<float4*>(reinterpret_cast<T*>(bal) + p) = *reinterpret_cast<const float4*>(src + 2 * JPLANE);
            if constexpr (!JR) {
                *reinterpret_cast<float4*>(reinterpret_cast<T*>(bbh) + p) = *reinterpret_cast<const float4*>(src + JPLANE);
                if (SPLIT) *reinterpret_cast<float4*>(reinterpret_cast<T*>(bbl) + p) = *reinterpret_cast<const float4*>(src + 3 * JPLANE);
            }
            slot += PAD;
            if (slot >= RING) slot -= RING;
        }
        f4_t P1 = {0.f, 0.f, 0.f, 0.f}, P2 = P1, P3 = P1, P4 = P1;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int t = 0; t < F::TERMS; ++t) {
                F::mmat(t, P1, cch[p], ccl[p], bah[p], bal[p]);
                if constexpr (!CR) F::mmat(t, P3, cdh[p], cdl[p], bah[p], bal[p]);
                if constexpr (!JR) {
                    F::mmat(t, P4, cch[p], ccl[p], bbh[p], bbl[p]);
                    if constexpr (!CR) F::mmat(t, P2, cdh[p], cdl[p], bbh[p], bbl[p]);
                }
            }
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
            __builtin_amdgcn_raw_buffer_store_b64(va, out_a, (int)off, 0, 0);
            if constexpr (!JR) __builtin_amdgcn_raw_buffer_store_b64(vb, out_b, (int)off, 0, 0);
            if constexpr (LS) {
                // absent planes have empty resources: their stores are dropped
                va[1] ^= (int)0x80000000;
                vb[1] ^= (int)0x80000000;
                __builtin_amdgcn_raw_buffer_store_b64(va, out_c, (int)off, 0, 0);
                if constexpr (!JR) __builtin_amdgcn_raw_buffer_store_b64(vb, out_d, (int)off, 0, 0);
            }
        }
    };

    // Schedule.  Step b computes J block b (rows 16 b .. 16 b + 15 of the
    // band) from the staged slab, then, once the whole workgroup has written
    // it, output rows 16 s .. 16 s + 15 (s = b - LEAD + 1) from J blocks
    // s .. b, then stages slab b + 1.  Two LDS barriers per step let one
    // slab buffer and a ring of exactly one band window (L rows) serve:
    // the first orders the J writes before the vertical reads and the slab
    // reads before the next slab write; the second orders the vertical reads
    // before the next step overwrites the oldest J block, and the slab write
    // before its reads.  The smaller footprint keeps more workgroups
    // resident per compute unit.  Image slabs travel through two register
    // sets that swap roles every step (no copies, which would wait for loads
    // still in flight); each is fetched two steps before it is staged.  The
    // body has no branch: work past the segment end reads zeros or folded
    // rows and its stores fall outside the output resources.
    constexpr int LEAD = L / 16;
    float pre_a[2 * PER_T], pre_b[2 * PER_T];
    auto lead = [&](int b, float (&stg)[2 * PER_T], float (&fet)[2 * PER_T]) {
        slab_load(b + 2, fet);
        row_pass(b);
        lds_barrier();
        slab_store(stg);
        lds_barrier();
    };
    auto step = [&](int s, float (&stg)[2 * PER_T], float (&fet)[2 * PER_T]) {
        const int b = s + LEAD - 1;
        slab_load(b + 2, fet);
        row_pass(b);
        lds_barrier();
        col_pass(s);
        slab_store(stg);
        lds_barrier();
    };
    slab_load(0, pre_a);
    slab_load(1, pre_b);
    if constexpr (CENTRE) {
        // mean of the strip's middle slab over the live lanes, summed in a
        // fixed order (its registers are free again once c is known)
        float mid[2 * PER_T];
        slab_rows(a.H > 16 ? a.H / 2 - 8 : 0, mid);
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < PER_T; ++k)
            if (tid + k * kThreads < SLAB2) v += mid[2 * k] + mid[2 * k + 1];
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
        // past the localized-SDFT tap table at the start of the ring, which
        // other waves may still be reading
        float* red = reinterpret_cast<float*>(stream_lds4) + 4 * KT;
        if (lane == 0) red[w] = v;
        lds_barrier();
        const float mean = ((red[0] + red[1]) + (red[2] + red[3])) * (1.0f / (16 * WF));
        // rounded to 8 significant bits: any c is exact, and a constant
        // image of such a value then cancels to zero before rounding
        cs = __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, mean) + 0x8000u) & 0xFFFF0000u);
        const float hc = tsum[0], hd = tsum[1], vc = tsum[2], vd = tsum[3];
        // uniform over the workgroup: keep them in scalar registers
        auto uni = [](float x) {
            return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
        };
        cs = uni(cs);
        dc_a = make_float2(uni(cs * (vc * hc - vd * hd)), uni(cs * (vc * hd + vd * hc)));
        dc_b = make_float2(uni(cs * (vc * hc + vd * hd)), uni(cs * (vd * hc - vc * hd)));
    }
    slab_store(pre_a);
    lds_barrier();
    // lead-in: J blocks 0 .. LEAD - 2; slab k sits in pre_a for even k
#pragma unroll
    for (int b = 0; b < LEAD - 1; b += 2) {
        lead(b, pre_b, pre_a);
        if (b + 1 < LEAD - 1) lead(b + 1, pre_a, pre_b);
    }
    float (&m_stg)[2 * PER_T] = (LEAD % 2 == 0) ? pre_a : pre_b;
    float (&m_fet)[2 * PER_T] = (LEAD % 2 == 0) ? pre_b : pre_a;
    for (int s = 0; s < nsteps; s += 2) {
        step(s, m_stg, m_fet);
        step(s + 1, m_fet, m_stg);
    }
}

// Launch conditions the kernel relies on: segments of a multiple of 32 rows
// (or one segment over the whole image), a band that fits the quarter, and
// output planes of at most 2^30 bytes.
inline bool stream_args_ok(const StreamArgs& a, int Q)
{
    if (a.seg_rows <= 0 || a.seg_rows % 16 != 0 || (a.seg_rows % 32 != 0 && a.seg_rows < a.H)) return false;
    if (16 + 2 * a.R > 4 * Q || Q > kStreamMaxQuarter) return false;
    return (int64_t)a.H * a.W * 8 <= (int64_t(1) << 30);
}

template <int OP, int Q>
__global__ __launch_bounds__(kThreads) void k_stream(StreamArgs a)
{
    const int lid = xcd_local_id(blockIdx.x, gridDim.x);
    const FusedJob jb = a.jobs[lid % a.n_jobs];
    const int rest = lid / a.n_jobs;
    // A job whose J and vertical taps are both real (omega = 0) runs the
    // real-J body with zero sine taps.
    if (jb.j_real) stream_body<OP, Q, true, false, false>(a, jb, rest, nullptr, 0, 0);
    else if (jb.c_real) stream_body<OP, Q, false, true, false>(a, jb, rest, nullptr, 0, 0);
    else stream_body<OP, Q, false, false, false>(a, jb, rest, nullptr, 0, 0);
}

// Localized SDFT (Sec. III-A): job (u, v) for u = 0..Mx/2, v = 0..My/2
// computes J_u once (Eq. (18)), F_{u,v} and F_{Mx-u,v} from J_u and its
// conjugate J_{Mx-u} (Eq. (19)), and stores the conjugates to F_{Mx-u,My-v}
// and F_{u,My-v} (Eq. (20)).  Planes are indexed v Mx + u.  Bins u in
// {0, Mx/2} have a real J_u and no partner; v in {0, My/2} real vertical
// taps, whose conjugate outputs coincide with the direct ones.
template <int OP, int Q>
__global__ __launch_bounds__(kThreads) void k_lsdft(StreamArgs a, LsdftTaps t)
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
    if (jb.j_real) stream_body<OP, Q, true, false, true>(a, jb, rest, &t, u, v);
    else if (jb.c_real) stream_body<OP, Q, false, true, true>(a, jb, rest, &t, u, v);
    else stream_body<OP, Q, false, false, true>(a, jb, rest, &t, u, v);
}

// Batch kernel: workgroup b takes tile b of a table in dispatch order
// (decreasing cost, equal-cost runs interleaved for the XCDs), as the
// wave-specialised tile kernel does.  A persistent form (each workgroup
// striding over the table) spilled 34-38 registers at Q = 56 in the split
// forms, where the four-wave kernel already holds 256 + 235-248 per lane.
template <int OP, int Q>
__global__ __launch_bounds__(kThreads) void k_stream_batch(BatchArgs b)
{
    {
        const BatchTile tl = b.tiles[blockIdx.x];
        const BatchImage& im = b.images[tl.image];
        const BatchFreq& fq = b.freqs[tl.freq];
        StreamArgs a{};
        a.img = im.img;
        a.stride = im.stride;
        a.H = im.H;
        a.W = im.W;
        a.boundary = b.boundary;
        a.R = fq.R;
        a.seg_rows = fq.seg_rows;
        a.n_xs = im.n_xs;
        a.jobs = b.jobs;
        a.taps = b.taps;
        a.out = im.out;
        a.in_scale = fq.in_scale;
        a.mid_scale = fq.mid_scale;
        a.out_scale = fq.out_scale;
        a.tap_scale[0] = fq.tap_scale[0];
        a.tap_scale[1] = fq.tap_scale[1];
        const FusedJob jb = b.jobs[tl.job];
        if (jb.j_real) stream_body<OP, Q, true, false, false>(a, jb, tl.rest, nullptr, 0, 0);
        else if (jb.c_real) stream_body<OP, Q, false, true, false>(a, jb, tl.rest, nullptr, 0, 0);
        else stream_body<OP, Q, false, false, false>(a, jb, tl.rest, nullptr, 0, 0);
    }
}

template <int OP, int Q>
hipError_t launch_bq(const BatchArgs& b, hipStream_t stream)
{
    const size_t lds = stream_lds_bytes(OP, Q);
    {
        static LdsLimit lim;
        const hipError_t e = lim.ensure((const void*)k_stream_batch<OP, Q>, lds);
        if (e != hipSuccess) return e;
    }
    if (b.n_tiles <= 0) return hipSuccess;
    const int grid = b.n_tiles;                         // one workgroup per tile
    hipLaunchKernelGGL((k_stream_batch<OP, Q>), dim3(grid), dim3(kThreads), lds, stream, b);
    return hipGetLastError();
}

template <int OP, int... Qs>
hipError_t launch_batch_q(const BatchArgs& b, int Q, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_bq<OP, Qs>(b, stream)) : (void)0), ...);
    return e;
}

template <int OP, int Q>
hipError_t launch_q(const StreamArgs& a, int n_blocks, hipStream_t stream)
{
    const size_t lds = stream_lds_bytes(OP, Q);
    {
        static LdsLimit lim;
        const hipError_t e = lim.ensure((const void*)k_stream<OP, Q>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_stream<OP, Q>), dim3(n_blocks), dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}

template <int OP, int Q>
hipError_t launch_lq(const StreamArgs& a, const LsdftTaps& t, int n_blocks, hipStream_t stream)
{
    const size_t lds = stream_lds_bytes(OP, Q);
    {
        static LdsLimit lim;
        const hipError_t e = lim.ensure((const void*)k_lsdft<OP, Q>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_lsdft<OP, Q>), dim3(n_blocks), dim3(kThreads), lds, stream, a, t);
    return hipGetLastError();
}

// The quarters each form is built for: every R <= 104 for the bank, every
// window M <= 64 (R <= 32) for the localized SDFT.  Quarters above 32 hold
// their band fragments partly in the accumulation registers (one wave per
// SIMD; their LDS footprint allows one workgroup per compute unit anyway).
template <int OP, int... Qs>
hipError_t launch_bank_q(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_q<OP, Qs>(a, n_blocks, stream)) : (void)0), ...);
    return e;
}

template <int OP, int... Qs>
hipError_t launch_lsdft_q(const StreamArgs& a, const LsdftTaps& t, int Q, int n_blocks, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_lq<OP, Qs>(a, t, n_blocks, stream)) : (void)0), ...);
    return e;
}


// ---------------------------------------------------------------------------
// Adjoint on the matrix cores.  For a real loss and G_c = dL/dRe F_c +
// i dL/dIm F_c, dL/df = sum_c Re(G_c * K_c) with the same (Hermitian) Gabor
// kernels as the forward bank.  For a pair theta, pi - theta with horizontal
// taps h = c + i d (and conj(h) for the partner) and vertical taps v:
//   J = h * G_a + conj(h) * G_b,
//   J_re = c * (Ga_re + Gb_re) - d * (Ga_im - Gb_im),
//   J_im = c * (Ga_im + Gb_im) + d * (Ga_re - Gb_re),
//   dL/df += Re(v * J) = v_c * J_re - v_d * J_im,
// which is the streaming kernel's structure with four staged real planes in
// the horizontal pass and the forward's Re F_a in the vertical one.  A
// workgroup owns one job and one 64-column strip segment and writes the
// job's partial plane; a second kernel sums the planes in job order (no
// atomics: the result is deterministic).
template <int Q, bool HR, bool CR>
__device__ __forceinline__ void adj_job(const AdjStreamArgs& a, const FusedJob& jb, int job, int x0, int yseg,
                                        int nsteps)
{
    using F = Form<FUSED_F32>;
    constexpr int L = 4 * Q;
    constexpr int RING = L;
    constexpr int PAD = 4;
    constexpr int RP = RING + PAD;
    constexpr int WF = 48 + L;
    constexpr int WP = WF + PAD;
    constexpr int JPLANE = kSX * RP;
    constexpr int SLAB2 = 16 * WF / 2;
    constexpr int PER_T = (SLAB2 + kThreads - 1) / kThreads;
    constexpr int FROWS = (2 * PER_T * kThreads + WF - 1) / WF;
    constexpr int FBUF = FROWS * WP;
    constexpr int KT = L + 16;
    constexpr int LEAD = L / 16;

    extern __shared__ float4 stream_lds4[];
    float* Jst = reinterpret_cast<float*>(stream_lds4);     // [2 comps][kSX][RP]
    float* Fst = Jst + 2 * JPLANE;                           // [4 planes][FROWS][WP]

    const int R = a.R;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int o = lane & 15, g = lane >> 4;
    const float* tab = a.taps + jb.tap_off;

    float rc[Q], rd[Q], cc[Q], cd[Q];
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        const int m = 16 + Q * g + e - o;
        rc[e] = tab[m];
        rd[e] = tab[KT + m];
        cc[e] = tab[2 * KT + m];
        cd[e] = tab[3 * KT + m];
    }

    // staged planes: S1 = Ga_re + Gb_re, N2 = Gb_im - Ga_im, S2 = Ga_im + Gb_im,
    // D1 = Ga_re - Gb_re; samples outside the image are zero.  Slab positions
    // are output-grid coordinates; the image sits at offset a.off.
    const int64_t plane = (int64_t)a.H * a.W;
    const uint32_t plane_bytes = (uint32_t)(plane * 8);
    const __amdgpu_buffer_rsrc_t ga = make_rsrc(a.G + (int64_t)jb.out_a * plane, plane_bytes);
    const __amdgpu_buffer_rsrc_t gb = jb.out_b >= 0 ? make_rsrc(a.G + (int64_t)jb.out_b * plane, plane_bytes)
                                                    : make_rsrc(a.G, 0u);
    int col_of[2 * PER_T], lds_at[PER_T], row_of[PER_T];
    const int xs0 = x0 - R;
#pragma unroll
    for (int k = 0; k < PER_T; ++k) {
        const int idx = tid + k * kThreads;
        const int e = 2 * idx;
        const int r = e / WF, c = e - r * WF;
        const bool live = idx < SLAB2;
        row_of[k] = r;
        lds_at[k] = r * WP + c;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cx = xs0 + c + h - a.off;
            col_of[2 * k + h] = live && cx >= 0 && cx < a.W ? cx : -1;
        }
    }
    typedef float f2v __attribute__((ext_vector_type(2)));
    auto slab_load = [&](int b, f2v (&pa)[2 * PER_T], f2v (&pb)[2 * PER_T]) {
        const int row0 = yseg - R + 16 * b - a.off;
        uint32_t off[2 * PER_T];
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int yy = row0 + row_of[k];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cx = col_of[2 * k + h];
                off[2 * k + h] = (yy >= 0 && yy < a.H && cx >= 0)
                                     ? (uint32_t)(((int64_t)yy * a.W + cx) * 8) : kOutside;
            }
        }
#pragma unroll
        for (int k = 0; k < 2 * PER_T; ++k) {
            pa[k] = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(ga, (int)off[k], 0, 0));
            pb[k] = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(gb, (int)off[k], 0, 0));
        }
    };
    auto slab_store = [&](const f2v (&pa)[2 * PER_T], const f2v (&pb)[2 * PER_T]) {
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const f2v a0 = pa[2 * k], a1 = pa[2 * k + 1], b0 = pb[2 * k], b1 = pb[2 * k + 1];
            f2v s1, n2, s2, d1;
            s1[0] = a0[0] + b0[0]; s1[1] = a1[0] + b1[0];
            n2[0] = b0[1] - a0[1]; n2[1] = b1[1] - a1[1];
            s2[0] = a0[1] + b0[1]; s2[1] = a1[1] + b1[1];
            d1[0] = a0[0] - b0[0]; d1[1] = a1[0] - b1[0];
            *reinterpret_cast<f2v*>(Fst + lds_at[k]) = s1;
            *reinterpret_cast<f2v*>(Fst + FBUF + lds_at[k]) = n2;
            *reinterpret_cast<f2v*>(Fst + 2 * FBUF + lds_at[k]) = s2;
            *reinterpret_cast<f2v*>(Fst + 3 * FBUF + lds_at[k]) = d1;
        }
    };
    auto frag = [&](float (&dst)[Q], const float* src) {
#pragma unroll
        for (int p = 0; p < Q; p += PAD)
            *reinterpret_cast<float4*>(dst + p) = *reinterpret_cast<const float4*>(src + p);
    };

    // horizontal pass of J block b, column block w
    auto row_pass = [&](int b) {
        const float* fb = Fst + o * WP + 16 * w + Q * g;
        float s1[Q], s2[Q];
        frag(s1, fb);
        frag(s2, fb + 2 * FBUF);
        f4_t re = {0.f, 0.f, 0.f, 0.f}, im = re;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            F::mma1(re, s1[p], 0.f, rc[p], 0.f);
            F::mma1(im, s2[p], 0.f, rc[p], 0.f);
        }
        if constexpr (!HR) {
            float n2[Q], d1[Q];
            frag(n2, fb + FBUF);
            frag(d1, fb + 3 * FBUF);
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                F::mma1(re, n2[p], 0.f, rd[p], 0.f);
                F::mma1(im, d1[p], 0.f, rd[p], 0.f);
            }
        }
        f32_mfma_drain(re, im);
        const int slot = (16 * b) % RING + 4 * g;
        float* ja = Jst + (16 * w + o) * RP + slot;
        *reinterpret_cast<float4*>(ja) = make_float4(re[0], re[1], re[2], re[3]);
        *reinterpret_cast<float4*>(ja + JPLANE) = make_float4(im[0], im[1], im[2], im[3]);
    };

    // partial plane of the job; rows past the segment end are written only
    // in the last step of an odd step count, which happens only where the
    // segment reaches the image bottom, so the range check drops them
    const int64_t plane_o = (int64_t)a.Ho * a.Wo;
    const uint32_t W4 = (uint32_t)a.Wo * 4u;
    const __amdgpu_buffer_rsrc_t part = make_rsrc(a.part + (int64_t)job * plane_o, (uint32_t)(plane_o * 4));
    const int xcol = x0 + 16 * w + o;
    const bool col_live = xcol < a.Wo;      // lanes past the grid store at kOutside
    const uint32_t lane_off = ((uint32_t)(yseg + 4 * g) * (uint32_t)a.Wo + (uint32_t)xcol) * 4u;

    // vertical pass of output rows 16 s .. 16 s + 15
    auto col_pass = [&](int s) {
        float ba[Q], bb[Q];
        const float* base = Jst + (16 * w + o) * RP;
        int slot = (16 * s + Q * g) % RING;
#pragma unroll
        for (int p = 0; p < Q; p += PAD) {
            *reinterpret_cast<float4*>(ba + p) = *reinterpret_cast<const float4*>(base + slot);
            if constexpr (!CR)
                *reinterpret_cast<float4*>(bb + p) = *reinterpret_cast<const float4*>(base + JPLANE + slot);
            slot += PAD;
            if (slot >= RING) slot -= RING;
        }
        f4_t P1 = {0.f, 0.f, 0.f, 0.f}, P2 = P1;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            F::mma1(P1, cc[p], 0.f, ba[p], 0.f);
            if constexpr (!CR) F::mma1(P2, cd[p], 0.f, bb[p], 0.f);
        }
        f32_mfma_drain(P1, P2);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            __builtin_amdgcn_raw_buffer_store_b32(
                __builtin_bit_cast(int, P1[r] - P2[r]), part,
                (int)(col_live ? lane_off + (uint32_t)(16 * s + r) * W4 : kOutside), 0, 0);
    };

    f2v xa[2 * PER_T], xb[2 * PER_T], ya[2 * PER_T], yb[2 * PER_T];
    auto lead = [&](int b, f2v (&sa)[2 * PER_T], f2v (&sb)[2 * PER_T], f2v (&fa)[2 * PER_T],
                    f2v (&fb)[2 * PER_T]) {
        slab_load(b + 2, fa, fb);
        row_pass(b);
        lds_barrier();
        slab_store(sa, sb);
        lds_barrier();
    };
    auto step = [&](int s, f2v (&sa)[2 * PER_T], f2v (&sb)[2 * PER_T], f2v (&fa)[2 * PER_T],
                    f2v (&fb)[2 * PER_T]) {
        const int b = s + LEAD - 1;
        slab_load(b + 2, fa, fb);
        row_pass(b);
        lds_barrier();
        col_pass(s);
        slab_store(sa, sb);
        lds_barrier();
    };
    slab_load(0, xa, xb);
    slab_load(1, ya, yb);
    slab_store(xa, xb);
    lds_barrier();
    // slab k is in (xa, xb) for even k, (ya, yb) for odd k
#pragma unroll
    for (int b = 0; b < LEAD - 1; b += 2) {
        lead(b, ya, yb, xa, xb);
        if (b + 1 < LEAD - 1) lead(b + 1, xa, xb, ya, yb);
    }
    if constexpr (LEAD % 2 == 0) {
        for (int s = 0; s < nsteps; s += 2) {
            step(s, xa, xb, ya, yb);
            step(s + 1, ya, yb, xa, xb);
        }
    } else {
        for (int s = 0; s < nsteps; s += 2) {
            step(s, ya, yb, xa, xb);
            step(s + 1, xa, xb, ya, yb);
        }
    }
}

template <int Q>
__global__ __launch_bounds__(kThreads) void k_adj_stream(AdjStreamArgs a)
{
    int lid = xcd_local_id(blockIdx.x, gridDim.x);
    if (a.n_images > 1) {
        // strided batch: image-major workgroup ids
        const int per = a.n_jobs * a.n_xs * a.n_ys;
        const int b = lid / per;
        lid -= b * per;
        a.G += b * a.g_bstride;
        a.part += b * a.part_bstride;
    }
    const int job = lid % a.n_jobs, rest = lid / a.n_jobs;
    const int xs = rest % a.n_xs, ys = rest / a.n_xs;
    const int x0 = xs * kSX, yseg = ys * a.seg_rows;
    const int nsteps = (min(a.seg_rows, a.Ho - yseg) + 15) / 16;
    const FusedJob jb = a.jobs[job];
    if (jb.j_real) adj_job<Q, true, false>(a, jb, job, x0, yseg, nsteps);
    else if (jb.c_real) adj_job<Q, false, true>(a, jb, job, x0, yseg, nsteps);
    else adj_job<Q, false, false>(a, jb, job, x0, yseg, nsteps);
}

__global__ __launch_bounds__(256) void k_adj_sum(const float* __restrict__ part, int n, int H, int W,
                                                 float* __restrict__ grad, int64_t stride, int64_t part_bstride,
                                                 int64_t grad_bstride)
{
    const int64_t npix = (int64_t)H * W;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npix) return;
    part += blockIdx.y * part_bstride;      // image of a batch
    grad += blockIdx.y * grad_bstride;
    float s = 0.f;
    for (int j = 0; j < n; ++j) s += part[j * npix + i];
    const int64_t y = i / W, x = i - y * W;
    grad[y * stride + x] = s;
}

// Mirror rule: dL/df(q) adds, for every frequency, the extended-grid values
// at all positions u in [-R, n - 1 + R] (per axis) whose fold is q: the
// residues of q and of -q modulo 2(n - 1) (one class when q is 0 or n - 1;
// every u when n = 1).  Fixed order: frequency, row preimage, column
// preimage, job.
__device__ __forceinline__ int fold_first(int u0, int R, int p)
{
    // smallest u = u0 + k p with u >= -R
    int k = (u0 + R) / p;
    return u0 - k * p;
}

__global__ __launch_bounds__(256) void k_adj_fold_sum(AdjFoldArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)a.H * a.W) return;
    a.part += blockIdx.y * a.part_bstride;  // image of a batch
    a.grad += blockIdx.y * a.grad_bstride;
    const int qy = (int)(i / a.W), qx = (int)(i - (int64_t)qy * a.W);
    float s = 0.f;
    for (int f = 0; f < a.n_freq; ++f) {
        const int R = a.f[f].R, Wo = a.W + 2 * R;
        const int64_t plane = (int64_t)(a.H + 2 * R) * Wo;
        const float* base = a.part + a.f[f].base;
        for (int cy = 0; cy < 2; ++cy) {
            int uy, py;
            if (a.H == 1) {
                if (cy) break;
                uy = -R;
                py = 1;
            } else {
                py = 2 * (a.H - 1);
                if (cy && (qy == 0 || qy == a.H - 1)) break;
                uy = fold_first(cy ? py - qy : qy, R, py);
            }
            for (; uy <= a.H - 1 + R; uy += py)
                for (int cx = 0; cx < 2; ++cx) {
                    int ux, px;
                    if (a.W == 1) {
                        if (cx) break;
                        ux = -R;
                        px = 1;
                    } else {
                        px = 2 * (a.W - 1);
                        if (cx && (qx == 0 || qx == a.W - 1)) break;
                        ux = fold_first(cx ? px - qx : qx, R, px);
                    }
                    for (; ux <= a.W - 1 + R; ux += px) {
                        const int64_t e = (int64_t)(uy + R) * Wo + (ux + R);
                        for (int j = 0; j < a.f[f].count; ++j) s += base[j * plane + e];
                    }
                }
        }
    }
    a.grad[(int64_t)qy * a.grad_stride + qx] = s;
}

template <int Q>
hipError_t launch_adj_q(const AdjStreamArgs& a, hipStream_t stream)
{
    const size_t lds = adjoint_stream_lds_bytes(Q);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    {
        static LdsLimit lim;
        const hipError_t e = lim.ensure((const void*)k_adj_stream<Q>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_adj_stream<Q>, dim3(a.n_jobs * a.n_xs * a.n_ys * (a.n_images > 1 ? a.n_images : 1)),
                       dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}

template <int... Qs>
hipError_t launch_adj_stream_q(const AdjStreamArgs& a, int Q, hipStream_t stream)
{
    hipError_t e = hipErrorInvalidValue;
    ((Q == Qs ? (void)(e = launch_adj_q<Qs>(a, stream)) : (void)0), ...);
    return e;
}

}  // namespace

// One object per arithmetic form: this file is compiled once per value of
// GABOR_FORM (a FusedOp), and the form-independent host helpers go with
// form 0.
#ifndef GABOR_FORM
#error "compile gabor_fused.hip with -DGABOR_FORM=<FusedOp>"
#endif

template <>
hipError_t stream_form<GABOR_FORM>(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return launch_bank_q<GABOR_FORM, 4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56>(a, Q, n_blocks, stream);
    else
        return launch_bank_q<GABOR_FORM, 8, 16, 24, 32, 40, 48, 56>(a, Q, n_blocks, stream);
}

template <>
hipError_t lsdft_form<GABOR_FORM>(const StreamArgs& a, const LsdftTaps& t, int Q, int n_blocks,
                                  hipStream_t stream)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return launch_lsdft_q<GABOR_FORM, 4, 8, 12, 16, 20>(a, t, Q, n_blocks, stream);
    else
        return launch_lsdft_q<GABOR_FORM, 8, 16, 24>(a, t, Q, n_blocks, stream);
}

template <>
hipError_t batch_form<GABOR_FORM>(const BatchArgs& b, int Q, hipStream_t stream)
{
    if constexpr (GABOR_FORM == FUSED_F32)
        return launch_batch_q<GABOR_FORM, 4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56>(b, Q, stream);
    else
        return launch_batch_q<GABOR_FORM, 8, 16, 24, 32, 40, 48, 56>(b, Q, stream);
}

#if GABOR_FORM == 0

size_t adjoint_stream_lds_bytes(int Q)
{
    const int L = 4 * Q, WF = 48 + L;
    const int per_t = (16 * WF / 2 + kThreads - 1) / kThreads;
    const int frows = (2 * per_t * kThreads + WF - 1) / WF;
    return 4 * ((size_t)2 * kSX * (L + 4) + (size_t)4 * frows * (WF + 4));
}

hipError_t launch_adjoint_stream(const AdjStreamArgs& a, int Q, hipStream_t stream)
{
    if (a.n_jobs <= 0) return hipSuccess;
    if (!a.G || !a.part || !a.jobs || !a.taps || Q > kAdjStreamMaxQuarter || 16 + 2 * a.R > 4 * Q)
        return hipErrorInvalidValue;
    // the kernel walks the output grid (Ho rows): segments that end above its
    // bottom must hold an even number of 16-row steps
    if (a.seg_rows <= 0 || a.seg_rows % 16 != 0 || (a.seg_rows % 32 != 0 && a.seg_rows < a.Ho)) return hipErrorInvalidValue;
    if ((int64_t)a.H * a.W * 8 > (int64_t(1) << 30) || (int64_t)a.Ho * a.Wo * 4 > (int64_t(1) << 30))
        return hipErrorInvalidValue;
    if (a.Ho < a.H || a.Wo < a.W || a.off < 0 || a.n_xs * kSX < a.Wo || (int64_t)a.n_ys * a.seg_rows < a.Ho)
        return hipErrorInvalidValue;
    if (a.n_images > 1 && (a.g_bstride < 0 || a.part_bstride < 0)) return hipErrorInvalidValue;
    if ((long long)a.n_jobs * a.n_xs * a.n_ys * (a.n_images > 1 ? a.n_images : 1) > 0x7fffffffLL)
        return hipErrorInvalidValue;
    return launch_adj_stream_q<4, 8, 12, 16, 20, 24, 28, 32>(a, Q, stream);
}

hipError_t launch_adjoint_fold_sum(const AdjFoldArgs& a, hipStream_t stream)
{
    const int64_t npix = (int64_t)a.H * a.W;
    if (a.n_freq <= 0 || a.n_freq > kAdjFoldMaxFreq || npix <= 0 || (npix + 255) / 256 > 0x7fffffffLL)
        return hipErrorInvalidValue;
    const int nb = a.n_images > 1 ? a.n_images : 1;
    if (nb > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_fold_sum, dim3((unsigned)((npix + 255) / 256), nb), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_adjoint_sum(const float* part, int n, int H, int W, float* grad, int64_t grad_stride,
                              int n_images, int64_t part_bstride, int64_t grad_bstride, hipStream_t stream)
{
    const int64_t npix = (int64_t)H * W;
    if (n <= 0 || npix <= 0 || (npix + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
    const int nb = n_images > 1 ? n_images : 1;
    if (nb > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_sum, dim3((unsigned)((npix + 255) / 256), nb), dim3(256), 0, stream, part, n, H, W,
                       grad, grad_stride, part_bstride, grad_bstride);
    return hipGetLastError();
}

hipError_t launch_batch(int op, const BatchArgs& b, int Q, hipStream_t stream)
{
    if (b.n_tiles <= 0) return hipSuccess;
    if (Q > kStreamMaxQuarter || !b.images || !b.freqs || !b.tiles || !b.jobs || !b.taps) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return batch_form<FUSED_F32>(b, Q, stream);
        case FUSED_BF16: return batch_form<FUSED_BF16>(b, Q, stream);
        case FUSED_BF16X3: return batch_form<FUSED_BF16X3>(b, Q, stream);
        case FUSED_F16: return batch_form<FUSED_F16>(b, Q, stream);
        case FUSED_F16X3: return batch_form<FUSED_F16X3>(b, Q, stream);
    }
    return hipErrorInvalidValue;
}

int stream_quarter(int op, int R)
{
    const int need = 16 + 2 * R;                         // inputs per 16-block
    if (op == FUSED_F32 && need <= 128) return ((need + 15) / 16) * 4;  // L multiple of 16
    return ((need + 31) / 32) * 8;                       // L multiple of 32
}

size_t stream_lds_bytes(int op, int Q)
{
    const int L = 4 * Q, RING = L, WF = 48 + L;
    const size_t es = op == FUSED_F32 ? 4 : 2;
    const int pad = (int)(16 / es);
    const size_t npl = (op == FUSED_BF16X3 || op == FUSED_F16X3) ? 2 : 1;
    const int per_t = (16 * WF / 2 + kThreads - 1) / kThreads;
    const int frows = (2 * per_t * kThreads + WF - 1) / WF;
    return npl * es * (2 * (size_t)kSX * (RING + pad) + (size_t)frows * (WF + pad));
}

int stream_strip_width() { return kSX; }

hipError_t launch_lsdft(int op, const StreamArgs& a, const LsdftTaps& t, int Q, hipStream_t stream)
{
    if (t.m[0] < 1 || t.m[0] > kLsdftMaxM || t.m[1] < 1 || t.m[1] > kLsdftMaxM) return hipErrorInvalidValue;
    if (a.n_jobs != (t.m[0] / 2 + 1) * (t.m[1] / 2 + 1) || 2 * a.R < t.m[0] - 1 || 2 * a.R < t.m[1] - 1)
        return hipErrorInvalidValue;
    // the wave-specialised kernel where it covers the quarter (every window
    // up to M = 64), else the four-wave one
    if (ws_supported(op, Q)) return launch_ws_lsdft(op, a, t, Q, stream);
    if (!stream_args_ok(a, Q))
        return hipErrorInvalidValue;
    const long long nb = (long long)a.n_xs * a.n_ys * a.n_jobs;
    if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return lsdft_form<FUSED_F32>(a, t, Q, (int)nb, stream);
        case FUSED_BF16: return lsdft_form<FUSED_BF16>(a, t, Q, (int)nb, stream);
        case FUSED_BF16X3: return lsdft_form<FUSED_BF16X3>(a, t, Q, (int)nb, stream);
        case FUSED_F16: return lsdft_form<FUSED_F16>(a, t, Q, (int)nb, stream);
        case FUSED_F16X3: return lsdft_form<FUSED_F16X3>(a, t, Q, (int)nb, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_stream(int op, const StreamArgs& a, int Q, hipStream_t stream)
{
    if (a.n_jobs <= 0) return hipSuccess;
    if (!stream_args_ok(a, Q))
        return hipErrorInvalidValue;
    const long long nb = (long long)a.n_xs * a.n_ys * a.n_jobs;
    if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (op) {
        case FUSED_F32: return stream_form<FUSED_F32>(a, Q, (int)nb, stream);
        case FUSED_BF16: return stream_form<FUSED_BF16>(a, Q, (int)nb, stream);
        case FUSED_BF16X3: return stream_form<FUSED_BF16X3>(a, Q, (int)nb, stream);
        case FUSED_F16: return stream_form<FUSED_F16>(a, Q, (int)nb, stream);
        case FUSED_F16X3: return stream_form<FUSED_F16X3>(a, Q, (int)nb, stream);
    }
    return hipErrorInvalidValue;
}
#endif

}  // namespace gabor
