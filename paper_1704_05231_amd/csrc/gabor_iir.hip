// Recursive-smoother variant of the bank (Sec. II-A): modulate, smooth with
// a third-order recursive Gaussian (a causal pass and its anti-causal
// mirror), demodulate -- Eq. (5)-(6) along x, Eq. (7)-(10) along y, and the
// pi - theta partner from conj(J) (Eq. (13)-(16)).  The cost per sample does
// not depend on sigma.
//
// Every recursion runs down the columns of a plane, one lane per column
// (coalesced across the wave), each line cut into chunks that the waves of a
// workgroup process in parallel (block-parallel linear recursion); the
// horizontal pass therefore works on the transposed image and its result is
// transposed back.  Each line is extended
// by T samples on both sides by the boundary rule and the recursion starts
// from rest at the far end of the extension; the forward results of the
// whole extended line are kept in a scratch plane for the backward pass.
// Modulation and demodulation use FP32 twiddles of the unfolded coordinate,
// computed in FP64 on the host.
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

}  // namespace

hipError_t launch_iir(const float* d_image, int64_t stride, int H, int W, int boundary, float* d_fT,
                      const IirJob* d_hjobs, int n_hjobs, float2* d_JT, float2* d_J, const IirJob* d_vjobs, int n_vjobs,
                      const float2* d_tw, float2* d_out, hipStream_t stream)
{
    if (n_hjobs <= 0 || n_vjobs <= 0 || n_hjobs > 65535 || n_vjobs > 65535) return hipErrorInvalidValue;
    hipError_t e;
    hipLaunchKernelGGL(k_transpose_f32, dim3((W + kTile - 1) / kTile, (H + kTile - 1) / kTile), dim3(kTile, 8), 0,
                       stream, d_image, stride, H, W, d_fT);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // horizontal pass on the transposed image: lines of length W, H columns
    hipLaunchKernelGGL(k_iir_block, dim3((H + 63) / 64, n_hjobs), dim3(64 * kIirChunks), 0, stream, d_hjobs, d_tw,
                       boundary, (float2*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_transpose_c64, dim3((H + kTile - 1) / kTile, (W + kTile - 1) / kTile, n_hjobs),
                       dim3(kTile, 8), 0, stream, (const float2*)d_JT, W, H, d_J);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // vertical pass: lines of length H, W columns, into the output channels
    hipLaunchKernelGGL(k_iir_block, dim3((W + 63) / 64, n_vjobs), dim3(64 * kIirChunks), 0, stream, d_vjobs, d_tw,
                       boundary, d_out);
    return hipGetLastError();
}

}  // namespace gabor
