// Recursive-smoother variant of the bank (Sec. II-A): modulate, smooth with
// a third-order recursive Gaussian (a causal pass and its anti-causal
// mirror), demodulate -- Eq. (5)-(6) along x, Eq. (7)-(10) along y, and the
// pi - theta partner from conj(J) (Eq. (13)-(16)).  The cost per sample does
// not depend on sigma.
//
// Every recursion runs down the columns of a plane, one thread per column
// (coalesced across the wave); the horizontal pass therefore works on the
// transposed image and its result is transposed back.  Each line is extended
// by T samples on both sides by the boundary rule and the recursion starts
// from rest at the far end of the extension; the forward results of the
// whole extended line are kept in a scratch plane for the backward pass.
// Modulation and demodulation use FP32 twiddles of the unfolded coordinate,
// computed in FP64 on the host.
#include "gabor_internal.h"

namespace gabor {
namespace {

constexpr int kIirThreads = 64;
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

// One recursion job per blockIdx.y; one column per thread.
__global__ __launch_bounds__(kIirThreads) void k_iir_lines(const IirJob* __restrict__ jobs, const float2* __restrict__ tw,
                                                           int boundary, float2* __restrict__ out_base)
{
    const IirJob jb = jobs[blockIdx.y];
    const int col = blockIdx.x * kIirThreads + threadIdx.x;
    if (col >= jb.cols) return;
    const int n = jb.n, T = jb.T, ext = n + 2 * T;
    const float a0 = jb.a[0], a1 = jb.a[1], a2 = jb.a[2], a3 = jb.a[3];
    const float2* twj = tw + jb.tw_off;                   // (cos, sin)(w l), l = -T .. n + T - 1
    float2* scr = jb.scratch + col;
    // forward (causal) pass over the extended line
    float2 w1 = make_float2(0.f, 0.f), w2 = w1, w3 = w1;
    for (int m = 0; m < ext; ++m) {
        const int r = fold_line(m - T, n, boundary);
        float2 v = make_float2(0.f, 0.f);
        if (r >= 0) {
            if (jb.in_complex) {
                v = reinterpret_cast<const float2*>(jb.in)[(int64_t)r * jb.in_stride + col];
                if (jb.conj) v.y = -v.y;
            } else {
                v.x = reinterpret_cast<const float*>(jb.in)[(int64_t)r * jb.in_stride + col];
            }
        }
        const float2 t = twj[m];
        // u = v exp(-i w l)
        const float ur = v.x * t.x + v.y * t.y, ui = v.y * t.x - v.x * t.y;
        float2 w;
        w.x = a0 * ur - a1 * w1.x - a2 * w2.x - a3 * w3.x;
        w.y = a0 * ui - a1 * w1.y - a2 * w2.y - a3 * w3.y;
        scr[(int64_t)m * jb.cols] = w;
        w3 = w2;
        w2 = w1;
        w1 = w;
    }
    // backward (anti-causal) pass; demodulate the image samples
    float2* out = (jb.out ? jb.out : out_base + (int64_t)jb.out_plane * n * jb.cols) + col;
    float2 v1 = make_float2(0.f, 0.f), v2 = v1, v3 = v1;
    for (int m = ext - 1; m >= 0; --m) {
        const float2 w = scr[(int64_t)m * jb.cols];
        float2 v;
        v.x = a0 * w.x - a1 * v1.x - a2 * v2.x - a3 * v3.x;
        v.y = a0 * w.y - a1 * v1.y - a2 * v2.y - a3 * v3.y;
        v3 = v2;
        v2 = v1;
        v1 = v;
        const int l = m - T;
        if (l >= 0 && l < n) {
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
    hipLaunchKernelGGL(k_iir_lines, dim3((H + kIirThreads - 1) / kIirThreads, n_hjobs), dim3(kIirThreads), 0, stream,
                       d_hjobs, d_tw, boundary, (float2*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_transpose_c64, dim3((H + kTile - 1) / kTile, (W + kTile - 1) / kTile, n_hjobs),
                       dim3(kTile, 8), 0, stream, (const float2*)d_JT, W, H, d_J);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // vertical pass: lines of length H, W columns, into the output channels
    hipLaunchKernelGGL(k_iir_lines, dim3((W + kIirThreads - 1) / kIirThreads, n_vjobs), dim3(kIirThreads), 0, stream,
                       d_vjobs, d_tw, boundary, d_out);
    return hipGetLastError();
}

}  // namespace gabor
