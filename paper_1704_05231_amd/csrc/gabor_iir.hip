// Recursive-smoother variant of the bank (Sec. II-A): modulate, smooth with
// a third-order recursive Gaussian (a causal pass and its anti-causal
// mirror), demodulate -- Eq. (5)-(6) along x, Eq. (7)-(10) along y, and the
// pi - theta partner from conj(J) (Eq. (13)-(16)).  The cost per sample does
// not depend on sigma.
//
// Every recursion runs down the columns of a plane, one lane per column
// (coalesced across the wave), each line cut into chunks that the waves of a
// workgroup process in parallel (block-parallel linear recursion); the
// horizontal pass therefore works on the transposed image, and writes its
// result back as rows (staged through LDS) or, for long lines, into a
// transposed plane that a transpose turns back.  Each line is extended
// by T samples on both sides by the boundary rule and the recursion starts
// from rest at the far end of the extension; the forward results of the
// whole extended line are kept in a scratch plane for the backward pass.
// Modulation and demodulation use FP32 twiddles of the unfolded coordinate,
// computed in FP64 on the host.
#include <type_traits>

#include "gabor_internal.h"

namespace gabor {
namespace {

constexpr int kTile = 32;

__device__ __forceinline__ int fold_line(int i, int n, int boundary)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (boundary == 0) return -1;
    if (n == 1) return 0;
    const int p = 2 * (n - 1);
    int r = i % p;
    if (r < 0) r += p;
    return r < n ? r : p - r;
}

// in[H][W] (row stride) -> out[W][H], 32 x 32 tiles through LDS
__global__ __launch_bounds__(kTile * 8) void k_transpose_f32(const float* __restrict__ in, int64_t stride, int H, int W,
                                                             float* __restrict__ out)
{
    __shared__ float t[kTile][kTile + 1];
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    for (int j = threadIdx.y; j < kTile; j += blockDim.y) {
        const int y = y0 + j, x = x0 + threadIdx.x;
        if (y < H && x < W) t[j][threadIdx.x] = in[(int64_t)y * stride + x];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < kTile; j += blockDim.y) {
        const int x = x0 + j, y = y0 + threadIdx.x;
        if (x < W && y < H) out[(int64_t)x * H + y] = t[threadIdx.x][j];
    }
}

// plane z of in[z][R][C] -> out[z][C][R]
__global__ __launch_bounds__(kTile * 8) void k_transpose_c64(const float2* __restrict__ in, int R, int C,
                                                             float2* __restrict__ out)
{
    __shared__ float2 t[kTile][kTile + 1];
    const int64_t plane = (int64_t)R * C;
    in += blockIdx.z * plane;
    out += blockIdx.z * plane;
    const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    for (int j = threadIdx.y; j < kTile; j += blockDim.y) {
        const int r = r0 + j, c = c0 + threadIdx.x;
        if (r < R && c < C) t[j][threadIdx.x] = in[(int64_t)r * C + c];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < kTile; j += blockDim.y) {
        const int c = c0 + j, r = r0 + threadIdx.x;
        if (c < C && r < R) out[(int64_t)c * R + r] = t[threadIdx.x][j];
    }
}

// One recursion job per blockIdx.y; 64 columns per workgroup, one column per
// lane, and the extended line of each column cut into kIirChunks chunks, one
// per wave.  A third-order recursion is linear in its state
// s = (w[m], w[m-1], w[m-2]): a chunk of length lc maps an entering state s
// to (its zero-state final state) + A^lc s.  Each direction therefore takes
// three phases: every wave runs its chunk from rest and keeps the final
// state; one wave carries the true entering state across the chunks with
// A^lc; every wave reruns its chunk from that state.  Chunks are aligned to
// the end of the line, so only the first non-empty chunk can be short, and it
// starts the forward pass from rest (its state map is never needed; in the
// backward pass nothing to its left uses it).
__global__ __launch_bounds__(64 * kIirChunks) void k_iir_block(const IirJob* __restrict__ jobs,
                                                               const float2* __restrict__ tw, int boundary,
                                                               float2* __restrict__ out_base)
{
    __shared__ float2 st[kIirChunks][3][64];
    const IirJob jb = jobs[blockIdx.y];
    const int lane = threadIdx.x & 63, chunk = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    const bool live = col < jb.cols;
    const int n = jb.n, T = jb.T, ext = n + 2 * T, lc = jb.lc;
    auto lo_of = [&](int c) { return max(0, ext - (kIirChunks - c) * lc); };
    const int m0 = lo_of(chunk), m1 = lo_of(chunk + 1);
    const float a0 = jb.a[0], a1 = jb.a[1], a2 = jb.a[2], a3 = jb.a[3];
    const float2* twj = tw + jb.tw_off;                   // (cos, sin)(w l), l = -T .. n + T - 1
    float2* scr = jb.scratch + col;
    const int64_t cols = jb.cols;

    // modulated input u = v exp(-i w l) at extended position m
    auto input = [&](int m) {
        const int r = fold_line(m - T, n, boundary);
        float2 v = make_float2(0.f, 0.f);
        if (live && r >= 0) {
            if (jb.in_complex) {
                v = reinterpret_cast<const float2*>(jb.in)[(int64_t)r * jb.in_stride + col];
                if (jb.conj) v.y = -v.y;
            } else {
                v.x = reinterpret_cast<const float*>(jb.in)[(int64_t)r * jb.in_stride + col];
            }
        }
        const float2 t = twj[m];
        return make_float2(v.x * t.x + v.y * t.y, v.y * t.x - v.x * t.y);
    };
    auto rec = [&](float2 u, float2& s1, float2& s2, float2& s3) {
        float2 w;
        w.x = a0 * u.x - a1 * s1.x - a2 * s2.x - a3 * s3.x;
        w.y = a0 * u.y - a1 * s1.y - a2 * s2.y - a3 * s3.y;
        s3 = s2;
        s2 = s1;
        s1 = w;
        return w;
    };
    // carry the entering states across the chunks (one wave); st holds the
    // zero-state final states on entry and the entering states on exit.  In
    // FP64: for sigma of ten and more the poles approach 1 and A^lc has
    // entries of tens with alternating signs that cancel on a smooth state.
    auto carry = [&](bool forward) {
        double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
        const double* P = jb.apow;
        for (int k = 0; k < kIirChunks; ++k) {
            const int c = forward ? k : kIirChunks - 1 - k;
            const float2 z0 = st[c][0][lane], z1 = st[c][1][lane], z2 = st[c][2][lane];
            st[c][0][lane] = make_float2((float)s0r, (float)s0i);
            st[c][1][lane] = make_float2((float)s1r, (float)s1i);
            st[c][2][lane] = make_float2((float)s2r, (float)s2i);
            if (lo_of(c + 1) - lo_of(c) == lc) {
                const double t0r = s0r, t0i = s0i, t1r = s1r, t1i = s1i, t2r = s2r, t2i = s2i;
                s0r = (double)z0.x + P[0] * t0r + P[1] * t1r + P[2] * t2r;
                s0i = (double)z0.y + P[0] * t0i + P[1] * t1i + P[2] * t2i;
                s1r = (double)z1.x + P[3] * t0r + P[4] * t1r + P[5] * t2r;
                s1i = (double)z1.y + P[3] * t0i + P[4] * t1i + P[5] * t2i;
                s2r = (double)z2.x + P[6] * t0r + P[7] * t1r + P[8] * t2r;
                s2i = (double)z2.y + P[6] * t0i + P[7] * t1i + P[8] * t2i;
            } else {
                s0r = z0.x;
                s0i = z0.y;
                s1r = z1.x;
                s1i = z1.y;
                s2r = z2.x;
                s2i = z2.y;
            }
        }
    };

    // ---- forward (causal) pass over the extended line
    float2 w1 = make_float2(0.f, 0.f), w2 = w1, w3 = w1;
    for (int m = m0; m < m1; ++m) rec(input(m), w1, w2, w3);
    st[chunk][0][lane] = w1;
    st[chunk][1][lane] = w2;
    st[chunk][2][lane] = w3;
    __syncthreads();
    if (chunk == 0) carry(true);
    __syncthreads();
    w1 = st[chunk][0][lane];
    w2 = st[chunk][1][lane];
    w3 = st[chunk][2][lane];
    for (int m = m0; m < m1; ++m) {
        const float2 w = rec(input(m), w1, w2, w3);
        if (live) scr[(int64_t)m * cols] = w;
    }
    // ---- backward (anti-causal) pass; each lane reads back only the
    // scratch entries it wrote itself
    __syncthreads();                                      // st is reused
    w1 = w2 = w3 = make_float2(0.f, 0.f);
    for (int m = m1 - 1; m >= m0; --m) rec(live ? scr[(int64_t)m * cols] : make_float2(0.f, 0.f), w1, w2, w3);
    st[chunk][0][lane] = w1;
    st[chunk][1][lane] = w2;
    st[chunk][2][lane] = w3;
    __syncthreads();
    if (chunk == 0) carry(false);
    __syncthreads();
    w1 = st[chunk][0][lane];
    w2 = st[chunk][1][lane];
    w3 = st[chunk][2][lane];
    // demodulate the image samples
    float2* out = (jb.out ? jb.out : out_base + (int64_t)jb.out_plane * n * cols) + col;
    for (int m = m1 - 1; m >= m0; --m) {
        const float2 v = rec(live ? scr[(int64_t)m * cols] : make_float2(0.f, 0.f), w1, w2, w3);
        const int l = m - T;
        if (live && l >= 0 && l < n) {
            const float2 t = twj[m];
            out[(int64_t)l * jb.out_stride] = make_float2(v.x * t.x - v.y * t.y, v.x * t.y + v.y * t.x);
        }
    }
}

// The same recursion with every chunk's samples held in registers (no
// scratch plane): kIirRegChunks = 64 chunks per line, 512 / 64 = 8 columns
// per workgroup, eight chunks per wave (lanes 8 c .. 8 c + 7 take chunk
// 8 w + c); short chunks keep the registers low enough for two workgroups
// per compute unit, so one's loads overlap the other's arithmetic.  Every chunk holds exactly LC samples (the job's lc): the
// line is padded with zeros in front (a recursion from rest over zeros stays
// at rest), so every loop is straight-line code.  The input is read once: after the
// carry, the true forward result of a chunk is its zero-state result plus
// the zero-input response of its entering state (the recursion is linear),
// so nothing is rerun from the input; likewise backward.
constexpr int kIirRegCols = 512 / kIirRegChunks;
template <int LC, bool ROWS>
__global__ __launch_bounds__(512) void k_iir_reg(const IirJob* __restrict__ jobs, const float2* __restrict__ tw,
                                                 int boundary, float2* __restrict__ out_base)
{
    constexpr int CH = kIirRegChunks, NC = kIirRegCols;
    __shared__ double sc[CH][6][NC];                      // carry scan: 3 complex FP64 states per chunk
    __shared__ float2 tws[CH * kIirRegMaxChunk];          // the job's twiddles, staged once
    const IirJob jb = jobs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int cl = lane % NC, chunk = (64 / NC) * (threadIdx.x >> 6) + lane / NC;
    const int xb = blockIdx.x;
    const int col = xb * NC + cl;
    const bool live = col < jb.cols;
    const int n = jb.n, T = jb.T, ext = n + 2 * T;
    constexpr int lc = LC;                                         // the host sets jb.lc = LC
    const int m0 = ext - (CH - chunk) * lc;                        // first sample (< 0: padding)
    const float a0 = jb.a[0], a1 = jb.a[1], a2 = jb.a[2], a3 = jb.a[3];
    // (cos, sin)(w l), l = -T .. n + T - 1, into LDS (ext <= CH * kIirRegMaxChunk)
    for (int i = threadIdx.x; i < ext; i += 512) tws[i] = tw[jb.tw_off + i];

    auto rec = [&](float2 u, float2& s1, float2& s2, float2& s3) {
        float2 w;
        w.x = a0 * u.x - a1 * s1.x - a2 * s2.x - a3 * s3.x;
        w.y = a0 * u.y - a1 * s1.y - a2 * s2.y - a3 * s3.y;
        s3 = s2;
        s2 = s1;
        s1 = w;
        return w;
    };
    auto hom = [&](float2& s1, float2& s2, float2& s3) {       // zero-input step
        float2 w;
        w.x = -a1 * s1.x - a2 * s2.x - a3 * s3.x;
        w.y = -a1 * s1.y - a2 * s2.y - a3 * s3.y;
        s3 = s2;
        s2 = s1;
        s1 = w;
        return w;
    };
    // Entering states across the chunks (FP64, as in k_iir_block), as a
    // parallel scan: chunk c maps its entering state s to z_c + P s (z_c its
    // zero-state final state, P = A^lc), so the true final state is
    // S_c = sum over j <= c of P^(c - j) z_j (forward; mirrored backward).
    // Hillis-Steele over the 64 chunks in six steps, step k adding
    // P^(2^k) times the value 2^k chunks back; then chunk c enters with
    // S_(c - 1) (forward) or S_(c + 1) (backward), zero at the line's end.
    auto carry = [&](bool forward, float2& e1, float2& e2, float2& e3) {
        double z[6] = {e1.x, e1.y, e2.x, e2.y, e3.x, e3.y};
        static_assert(CH == 64, "six scan steps");
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int d = 1 << k;
            const double* P = k == 0 ? jb.apow : jb.apow2[k - 1];
#pragma unroll
            for (int i = 0; i < 6; ++i) sc[chunk][i][cl] = z[i];
            __syncthreads();
            const int src = forward ? chunk - d : chunk + d;
            if (src >= 0 && src < CH) {
                double y[6];
#pragma unroll
                for (int i = 0; i < 6; ++i) y[i] = sc[src][i][cl];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    z[2 * r] += P[3 * r] * y[0] + P[3 * r + 1] * y[2] + P[3 * r + 2] * y[4];
                    z[2 * r + 1] += P[3 * r] * y[1] + P[3 * r + 1] * y[3] + P[3 * r + 2] * y[5];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) sc[chunk][i][cl] = z[i];
        __syncthreads();
        const int src = forward ? chunk - 1 : chunk + 1;
        double y[6] = {0, 0, 0, 0, 0, 0};
        if (src >= 0 && src < CH)
#pragma unroll
            for (int i = 0; i < 6; ++i) y[i] = sc[src][i][cl];
        e1 = make_float2((float)y[0], (float)y[1]);
        e2 = make_float2((float)y[2], (float)y[3]);
        e3 = make_float2((float)y[4], (float)y[5]);
        __syncthreads();                                  // sc is reused
    };

    float2 buf[LC];
    const float2 zero = make_float2(0.f, 0.f);
    // ---- the chunk's input samples.  Source rows follow the boundary rule
    // incrementally: u = m - T walks the line; under the mirror rule its
    // residue q modulo 2(n - 1) folds to q or 2(n - 1) - q.  Every load is
    // issued unconditionally (row clamped, value selected), so they are all
    // in flight together.
    const int p = 2 * (n - 1);
    int u = m0 - T;
    int q = 0;
    if (boundary != 0 && p > 0) {
        q = u % p;
        if (q < 0) q += p;
    }
    const int64_t ccol = live ? col : 0;
    auto load_all = [&](auto complex_in, auto mirror) {
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            int r;
            if constexpr (mirror) r = p > 0 ? (q < n ? q : p - q) : 0;
            else r = (u >= 0 && u < n) ? u : -1;
            const bool ok = live && r >= 0 && u + T >= 0;      // u + T < 0: front padding
            const int64_t at = (int64_t)max(r, 0) * jb.in_stride + ccol;
            if constexpr (complex_in) {
                const float2 v = reinterpret_cast<const float2*>(jb.in)[at];
                buf[k] = make_float2(ok ? v.x : 0.f, ok ? (jb.conj ? -v.y : v.y) : 0.f);
            } else {
                const float v = reinterpret_cast<const float*>(jb.in)[at];
                buf[k] = make_float2(ok ? v : 0.f, 0.f);
            }
            ++u;
            if constexpr (mirror) q = q + 1 == p ? 0 : q + 1;
        }
    };
    using tt = std::true_type;
    using ff = std::false_type;
    if (jb.in_complex) {
        if (boundary != 0) load_all(tt{}, tt{});
        else load_all(tt{}, ff{});
    } else {
        if (boundary != 0) load_all(ff{}, tt{});
        else load_all(ff{}, ff{});
    }
    __syncthreads();                                      // twiddles staged
    // ---- forward (causal): zero-state pass over the modulated inputs
    // u = v exp(-i w l)
    float2 w1 = zero, w2 = zero, w3 = zero;
#pragma unroll
    for (int k = 0; k < LC; ++k) {
            const float2 t = tws[max(m0 + k, 0)], v = buf[k];
            buf[k] = rec(make_float2(v.x * t.x + v.y * t.y, v.y * t.x - v.x * t.y), w1, w2, w3);
        }
    carry(true, w1, w2, w3);
#pragma unroll
    for (int k = 0; k < LC; ++k) {
            const float2 h = hom(w1, w2, w3);
            buf[k].x += h.x;
            buf[k].y += h.y;
        }
    // ---- backward (anti-causal): zero-state pass over the forward results
    w1 = w2 = w3 = zero;
#pragma unroll
    for (int k = LC - 1; k >= 0; --k) buf[k] = rec(buf[k], w1, w2, w3);
    carry(false, w1, w2, w3);
    float2* const base = jb.out ? jb.out : out_base + (int64_t)jb.out_plane * n * jb.cols;
    if constexpr (ROWS) {
        // The lines leave as rows, through the carry buffer (free after the
        // last scan): each round stages CPR chunks of all NC lines, written by
        // the waves that hold them, then wave i stores line i's segment with
        // contiguous lanes.
        constexpr int CAP = (int)(sizeof(sc) / sizeof(float2)) / (NC * LC);   // chunks that fit
        constexpr int CPR = CAP >= 64 ? 64 : CAP >= 32 ? 32 : CAP >= 16 ? 16 : 8;
        static_assert(LC <= kIirRowChunk && NC == 8 && CPR % (64 / NC) == 0 && CH % CPR == 0,
                      "whole waves per round, one line per wave");
        constexpr int SEG = CPR * LC;
        float2* stage = reinterpret_cast<float2*>(&sc[0][0][0]);
#pragma unroll
        for (int k = LC - 1; k >= 0; --k) {
            const float2 h = hom(w1, w2, w3);
            const float2 v = make_float2(buf[k].x + h.x, buf[k].y + h.y);
            const float2 t = tws[max(m0 + k, 0)];
            buf[k] = make_float2(v.x * t.x - v.y * t.y, v.x * t.y + v.y * t.x);
        }
        const int wave = threadIdx.x >> 6;
        for (int r = 0; r < CH / CPR; ++r) {
            const int mstart = ext - (CH - r * CPR) * lc;           // first extended sample of the round
            if (chunk / CPR == r) {
                // every sample of the chunk (padding and extension too: only
                // the image's samples are copied out below)
                float2* st = stage + cl * SEG + (m0 - mstart);
#pragma unroll
                for (int k = 0; k < LC; ++k) st[k] = buf[k];
            }
            __syncthreads();
            const int y = xb * NC + wave;                             // line of this wave
            const int lo = max(0, mstart - T), hi = min(n, mstart + SEG - T);
            if (y < jb.cols) {
                float2* row = base + (int64_t)y * jb.out_stride;
                const float2* src = stage + wave * SEG + (T - mstart);
                for (int l = lo + lane; l < hi; l += 64) row[l] = src[l];
            }
            __syncthreads();
        }
    } else {
        // entering-state response, then demodulate the image samples
        float2* out = base + col;
#pragma unroll
        for (int k = LC - 1; k >= 0; --k) {
            const float2 h = hom(w1, w2, w3);
            const float2 v = make_float2(buf[k].x + h.x, buf[k].y + h.y);
            const int l = m0 + k - T;
            if (live && l >= 0 && l < n) {
                const float2 t = tws[m0 + k];
                out[(int64_t)l * jb.out_stride] = make_float2(v.x * t.x - v.y * t.y, v.x * t.y + v.y * t.x);
            }
        }
    }
}

template <int LC, bool ROWS = false>
hipError_t launch_iir_reg(const IirJob* d_jobs, int n_jobs, int cols, const float2* d_tw, int boundary,
                          float2* d_out, hipStream_t stream)
{
    hipLaunchKernelGGL((k_iir_reg<LC, ROWS>), dim3((cols + kIirRegCols - 1) / kIirRegCols, n_jobs), dim3(512), 0, stream,
                       d_jobs, d_tw, boundary, d_out);
    return hipGetLastError();
}

// One pass: the register kernel when the jobs' chunks (of kIirRegChunks per
// line) fit, else the scratch-plane one (kIirChunks per line).
hipError_t launch_iir_pass(const IirJob* d_jobs, int n_jobs, int cols, int max_lc, bool reg, bool rows,
                           const float2* d_tw, int boundary, float2* d_out, hipStream_t stream)
{
    if (reg && rows) {
        // every job writes its lines as rows (max_lc <= kIirRowChunk)
        switch (max_lc) {
            case 8: return launch_iir_reg<8, true>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 16: return launch_iir_reg<16, true>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 24: return launch_iir_reg<24, true>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 32: return launch_iir_reg<32, true>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 40: return launch_iir_reg<40, true>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 48: return launch_iir_reg<48, true>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
        }
        return hipErrorInvalidValue;
    }
    if (rows) return hipErrorInvalidValue;
    if (reg) {
        // every job of the pass has lc = max_lc, a multiple of 8 from 8 to 64
        switch (max_lc) {
            case 8: return launch_iir_reg<8>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 16: return launch_iir_reg<16>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 24: return launch_iir_reg<24>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 32: return launch_iir_reg<32>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 40: return launch_iir_reg<40>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 48: return launch_iir_reg<48>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 56: return launch_iir_reg<56>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
            case 64: return launch_iir_reg<64>(d_jobs, n_jobs, cols, d_tw, boundary, d_out, stream);
        }
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_iir_block, dim3((cols + 63) / 64, n_jobs), dim3(64 * kIirChunks), 0, stream, d_jobs, d_tw,
                       boundary, d_out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_iir(const float* d_image, int64_t stride, int H, int W, int boundary, float* d_fT,
                      const IirJob* d_hjobs, int n_hjobs, int max_lc_h, bool reg_h, bool rows_h, float2* d_JT, float2* d_J,
                      const IirJob* d_vjobs, int n_vjobs, int max_lc_v, bool reg_v, const float2* d_tw,
                      float2* d_out, hipStream_t stream)
{
    if (n_hjobs <= 0 || n_vjobs <= 0 || n_hjobs > 65535 || n_vjobs > 65535) return hipErrorInvalidValue;
    hipError_t e;
    hipLaunchKernelGGL(k_transpose_f32, dim3((W + kTile - 1) / kTile, (H + kTile - 1) / kTile), dim3(kTile, 8), 0,
                       stream, d_image, stride, H, W, d_fT);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // horizontal pass on the transposed image: lines of length W, H columns
    if ((e = launch_iir_pass(d_hjobs, n_hjobs, H, max_lc_h, reg_h, rows_h, d_tw, boundary, nullptr, stream)) !=
        hipSuccess)
        return e;
    if (!rows_h) {
        hipLaunchKernelGGL(k_transpose_c64, dim3((H + kTile - 1) / kTile, (W + kTile - 1) / kTile, n_hjobs),
                           dim3(kTile, 8), 0, stream, (const float2*)d_JT, W, H, d_J);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // vertical pass: lines of length H, W columns, into the output channels
    return launch_iir_pass(d_vjobs, n_vjobs, W, max_lc_v, reg_v, false, d_tw, boundary, d_out, stream);
}

}  // namespace gabor
