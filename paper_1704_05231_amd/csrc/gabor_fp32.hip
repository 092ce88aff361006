// FP32 vector-ALU kernels of the two-pass Gabor bank (Sec. II, Algorithm 1).
//
// Horizontal pass (Eq. (3), decomposed in Eq. (5)-(6)):
//   J(x, y) = sum_t f(x - t, y) S(t) exp(i w cos(theta) t).
// The paper modulates f by cos/sin(w cos(theta) k), smooths both with the
// real Gaussian S and remodulates.  For an FIR S that sequence is exactly a
// convolution of f with the two real tap sets S(t) cos(w cos(theta) t) and
// S(t) sin(w cos(theta) t): the same two real 1-D passes, with the modulation
// folded into the taps.  Phases are therefore only ever taken of tap offsets
// |t| <= R, never of absolute coordinates.
//
// Vertical pass (Eq. (4), decomposed in Eq. (7)-(10)):
//   F(x, y) = sum_t J(x, y - t) S(t) exp(i w sin(theta) t),
// and for the pi - theta partner (Eq. (13)-(16)) the same taps applied to
// conj(J).  With J = a + ib and taps c + id the four real passes a*c, b*d,
// a*d, b*c give both orientations:
//   F_theta      = (a*c - b*d) + i (a*d + b*c)
//   F_(pi-theta) = (a*c + b*d) + i (a*d - b*c).
//
// Both kernels evaluate the convolutions in correlation order against
// reversed taps krev[T] = k(R - T), T = 0..Kp-1 (zero beyond 2R), so that
// out(z) = sum_T in(z - R + T) krev[T].
#include <algorithm>

#include "gabor_internal.h"

namespace gabor {
namespace {

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

// ---------------------------------------------------------------------------
// Horizontal pass.  One workgroup = one image row segment of blockDim.x * P
// outputs, all NC complex and NR real passes of one frequency.  The row
// segment plus its R-halo is staged once in LDS (boundary rule applied on
// load); each thread keeps P consecutive outputs of every pass in registers
// and slides a (P + U)-sample window over the taps, U taps per step.
// Taps are wave-uniform and come through the scalar cache.
constexpr int kRowP = 4;
constexpr int kRowU = kTapBlock;
constexpr int kRowThreads = 256;

template <int NC, int NR>
__global__ __launch_bounds__(kRowThreads) void k_row_fp32(
    const float* __restrict__ img, int64_t stride, int H, int W, int boundary, int R, int Kp,
    const float* __restrict__ taps, float2* __restrict__ J, int plane0,
    const BatchImage* __restrict__ bimg)
{
    constexpr int P = kRowP, U = kRowU, NT = 2 * NC + NR;
    extern __shared__ float4 row_lds4[];
    float* lds = reinterpret_cast<float*>(row_lds4);
    const int seg = blockDim.x * P;
    const int x0 = blockIdx.x * seg;
    const int y = blockIdx.y;
    if (bimg) {                                   // batched: this block's image
        const BatchImage im = bimg[blockIdx.z];
        img = im.img;
        stride = im.stride;
        H = im.H;
        W = im.W;
        J += im.J_off;
        if (y >= H || x0 >= W) return;
    }
    const float* src = img + (int64_t)y * stride;
    const int nload = seg + Kp;
    for (int i = threadIdx.x; i < nload; i += blockDim.x) {
        const int xx = fold_index(x0 - R + i, W, boundary);
        lds[i] = xx >= 0 ? src[xx] : 0.0f;
    }
    __syncthreads();

    float ar[NC > 0 ? NC : 1][P], ai[NC > 0 ? NC : 1][P], ax[NR > 0 ? NR : 1][P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int c = 0; c < NC; ++c) ar[c][p] = ai[c][p] = 0.0f;
#pragma unroll
        for (int r = 0; r < NR; ++r) ax[r][p] = 0.0f;
    }
    const float* win = lds + threadIdx.x * P;
    for (int T = 0; T < Kp; T += U) {
        float w[P + U];
#pragma unroll
        for (int j = 0; j < P + U; j += 4) {
            const float4 v = *reinterpret_cast<const float4*>(win + T + j);
            w[j] = v.x; w[j + 1] = v.y; w[j + 2] = v.z; w[j + 3] = v.w;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float* tp = taps + (T + u) * NT;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const float tc = tp[2 * c], td = tp[2 * c + 1];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    ar[c][p] = fmaf(w[p + u], tc, ar[c][p]);
                    ai[c][p] = fmaf(w[p + u], td, ai[c][p]);
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const float tr = tp[2 * NC + r];
#pragma unroll
                for (int p = 0; p < P; ++p) ax[r][p] = fmaf(w[p + u], tr, ax[r][p]);
            }
        }
    }

    // Each thread holds P consecutive outputs; storing them directly would
    // make every store instruction write lanes P elements apart (partial
    // lines).  Each plane goes through LDS instead and leaves as contiguous
    // lanes.
    const int64_t plane = (int64_t)H * W;
    float2* dst = J + (int64_t)plane0 * plane + (int64_t)y * W;
    float2* st = reinterpret_cast<float2*>(lds);
#pragma unroll
    for (int q = 0; q < NC + NR; ++q) {
        __syncthreads();                              // the row (or the previous plane) is read
#pragma unroll
        for (int p = 0; p < P; ++p)
            st[threadIdx.x * P + p] = q < NC ? make_float2(ar[q < NC ? q : 0][p], ai[q < NC ? q : 0][p])
                                             : make_float2(ax[q < NC ? 0 : q - NC][p], 0.0f);
        __syncthreads();
        for (int i = threadIdx.x; i < seg; i += blockDim.x) {
            const int x = x0 + i;
            if (x < W) dst[q * plane + x] = st[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Vertical pass.  One workgroup = a TX-column by TY-row output tile of one
// column job.  The J tile plus R-halo rows (boundary rule applied to J, which
// equals the horizontal pass of the extended image) is staged in LDS; each
// thread owns one column and P consecutive rows and slides a window down it.
constexpr int kColTX = 32;
constexpr int kColP = 8;
constexpr int kColThreads = 256;
constexpr int kColGroups = kColThreads / kColTX;   // row groups per tile
constexpr int kColTY = kColP * kColGroups;         // 64 rows
constexpr int kColU = kTapBlock;

template <bool JREAL, bool CREAL>
__device__ __forceinline__ void col_tile(const float2* __restrict__ lds, const float* __restrict__ tp,
                                         int Kp, int lane, int grp, float (&A1)[kColP],
                                         float (&A2)[kColP], float (&A3)[kColP], float (&A4)[kColP])
{
    constexpr int P = kColP, U = kColU;
    for (int T = 0; T < Kp; T += U) {
        float2 w[P + U];
#pragma unroll
        for (int j = 0; j < P + U; ++j) w[j] = lds[(grp * P + T + j) * kColTX + lane];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float c = tp[2 * (T + u)], d = tp[2 * (T + u) + 1];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                A1[p] = fmaf(w[p + u].x, c, A1[p]);
                if (!CREAL) A3[p] = fmaf(w[p + u].x, d, A3[p]);
                if (!JREAL) {
                    A4[p] = fmaf(w[p + u].y, c, A4[p]);
                    if (!CREAL) A2[p] = fmaf(w[p + u].y, d, A2[p]);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kColThreads) void k_col_fp32(
    const float2* __restrict__ J, int H, int W, int boundary, int R, int Kp,
    const ColJob* __restrict__ jobs, int n_jobs, const float* __restrict__ taps, float2* __restrict__ out,
    const BatchImage* __restrict__ bimg)
{
    extern __shared__ float2 col_lds[];
    const ColJob jb = jobs[blockIdx.z % n_jobs];
    const int x0 = blockIdx.x * kColTX, y0 = blockIdx.y * kColTY;
    if (bimg) {                                   // batched: this block's image
        const BatchImage im = bimg[blockIdx.z / n_jobs];
        J += im.J_off;
        out = im.out;
        H = im.H;
        W = im.W;
        if (y0 >= H || x0 >= W) return;
    }
    const int lane = threadIdx.x % kColTX, grp = threadIdx.x / kColTX;
    const int64_t plane = (int64_t)H * W;
    const float2* src = J + (int64_t)jb.plane * plane;
    const int x = x0 + lane;
    const int nrows = kColTY + Kp;
    for (int i = grp; i < nrows; i += kColGroups) {
        const int yy = fold_index(y0 - R + i, H, boundary);
        float2 v = make_float2(0.0f, 0.0f);
        if (yy >= 0 && x < W) v = src[(int64_t)yy * W + x];
        col_lds[i * kColTX + lane] = v;
    }
    __syncthreads();

    float A1[kColP], A2[kColP], A3[kColP], A4[kColP];
#pragma unroll
    for (int p = 0; p < kColP; ++p) A1[p] = A2[p] = A3[p] = A4[p] = 0.0f;
    const float* tp = taps + jb.tap_off;
    if (jb.j_real) {
        if (jb.c_real) col_tile<true, true>(col_lds, tp, Kp, lane, grp, A1, A2, A3, A4);
        else col_tile<true, false>(col_lds, tp, Kp, lane, grp, A1, A2, A3, A4);
    } else {
        if (jb.c_real) col_tile<false, true>(col_lds, tp, Kp, lane, grp, A1, A2, A3, A4);
        else col_tile<false, false>(col_lds, tp, Kp, lane, grp, A1, A2, A3, A4);
    }

    if (x >= W) return;
    float2* oa = out + (int64_t)jb.out_a * plane;
    float2* ob = jb.out_b >= 0 ? out + (int64_t)jb.out_b * plane : nullptr;
#pragma unroll
    for (int p = 0; p < kColP; ++p) {
        const int y = y0 + grp * kColP + p;
        if (y < H) {
            oa[(int64_t)y * W + x] = make_float2(A1[p] - A2[p], A3[p] + A4[p]);
            if (ob) ob[(int64_t)y * W + x] = make_float2(A1[p] + A2[p], A3[p] - A4[p]);
        }
    }
}

template <int NC, int NR>
hipError_t launch_row_t(const float* img, int64_t stride, int H, int W, int boundary,
                        const FreqDesc& fd, const RowGroup& g, const float* d_taps, float2* d_J,
                        hipStream_t stream)
{
    const int need = (W + kRowP - 1) / kRowP;
    int threads = ((need + 63) / 64) * 64;
    if (threads > kRowThreads) threads = kRowThreads;
    const int seg = threads * kRowP;
    dim3 grid((W + seg - 1) / seg, H, 1);
    const size_t lds = sizeof(float) * std::max((size_t)(seg + fd.Kp + 4), (size_t)(2 * seg));
    hipLaunchKernelGGL((k_row_fp32<NC, NR>), grid, dim3(threads), lds, stream, img, stride, H, W,
                       boundary, fd.R, fd.Kp, d_taps + g.tap_off, d_J, g.plane0, (const BatchImage*)nullptr);
    return hipGetLastError();
}

template <int NC, int NR>
hipError_t launch_row_batch_t(const BatchImage* d_imgs, int n_images, int max_h, int max_w, int boundary,
                              const FreqDesc& fd, const RowGroup& g, const float* d_taps, float2* d_J,
                              hipStream_t stream)
{
    const int seg = kRowThreads * kRowP;
    dim3 grid((max_w + seg - 1) / seg, max_h, n_images);
    const size_t lds = sizeof(float) * std::max((size_t)(seg + fd.Kp + 4), (size_t)(2 * seg));
    hipLaunchKernelGGL((k_row_fp32<NC, NR>), grid, dim3(kRowThreads), lds, stream, (const float*)nullptr,
                       (int64_t)0, 0, 0, boundary, fd.R, fd.Kp, d_taps + g.tap_off, d_J, g.plane0, d_imgs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_row_fp32(const float* img, int64_t stride, int H, int W, int boundary,
                           const FreqDesc& fd, const RowGroup& g, const float* d_taps,
                           float2* d_J, hipStream_t stream)
{
#define GABOR_ROW_CASE(NC, NR) \
    if (g.n_cplx == NC && g.n_real == NR) return launch_row_t<NC, NR>(img, stride, H, W, boundary, fd, g, d_taps, d_J, stream);
    GABOR_ROW_CASE(0, 1) GABOR_ROW_CASE(1, 0) GABOR_ROW_CASE(1, 1) GABOR_ROW_CASE(2, 0)
    GABOR_ROW_CASE(2, 1) GABOR_ROW_CASE(3, 0) GABOR_ROW_CASE(3, 1) GABOR_ROW_CASE(4, 0)
    GABOR_ROW_CASE(4, 1) GABOR_ROW_CASE(5, 0) GABOR_ROW_CASE(5, 1) GABOR_ROW_CASE(6, 0)
    GABOR_ROW_CASE(6, 1)
#undef GABOR_ROW_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_fp32_batch(const BatchImage* d_imgs, int n_images, int max_h, int max_w, int boundary,
                                 const FreqDesc& fd, const RowGroup& g, const float* d_taps, float2* d_J,
                                 hipStream_t stream)
{
    if (n_images <= 0 || n_images > 65535 || max_h > 65535) return hipErrorInvalidValue;
#define GABOR_ROW_CASE(NC, NR) \
    if (g.n_cplx == NC && g.n_real == NR) return launch_row_batch_t<NC, NR>(d_imgs, n_images, max_h, max_w, boundary, fd, g, d_taps, d_J, stream);
    GABOR_ROW_CASE(0, 1) GABOR_ROW_CASE(1, 0) GABOR_ROW_CASE(1, 1) GABOR_ROW_CASE(2, 0)
    GABOR_ROW_CASE(2, 1) GABOR_ROW_CASE(3, 0) GABOR_ROW_CASE(3, 1) GABOR_ROW_CASE(4, 0)
    GABOR_ROW_CASE(4, 1) GABOR_ROW_CASE(5, 0) GABOR_ROW_CASE(5, 1) GABOR_ROW_CASE(6, 0)
    GABOR_ROW_CASE(6, 1)
#undef GABOR_ROW_CASE
    return hipErrorInvalidValue;
}

// one limit for k_col_fp32, shared by both of its launchers
static LdsLimit g_col_lim;

hipError_t launch_col_fp32_batch(const BatchImage* d_imgs, int n_images, int max_h, int max_w, int boundary,
                                 const FreqDesc& fd, const ColJob* d_jobs, int n_jobs, const float* d_taps,
                                 float2* d_J, hipStream_t stream)
{
    if (n_jobs <= 0) return hipSuccess;
    if (n_images <= 0 || (long long)n_jobs * n_images > 65535) return hipErrorInvalidValue;
    const size_t lds = sizeof(float2) * (size_t)(kColTY + fd.Kp) * kColTX;
    {
        const hipError_t e = g_col_lim.ensure((const void*)k_col_fp32, lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((max_w + kColTX - 1) / kColTX, (max_h + kColTY - 1) / kColTY, n_jobs * n_images);
    hipLaunchKernelGGL(k_col_fp32, grid, dim3(kColThreads), lds, stream, (const float2*)d_J, 0, 0, boundary,
                       fd.R, fd.Kp, d_jobs, n_jobs, d_taps, (float2*)nullptr, d_imgs);
    return hipGetLastError();
}

hipError_t launch_col_fp32(const float2* d_J, int H, int W, int boundary, const FreqDesc& fd,
                           const ColJob* d_jobs, int n_jobs, const float* d_taps, float2* d_out,
                           hipStream_t stream)
{
    if (n_jobs <= 0) return hipSuccess;
    const size_t lds = sizeof(float2) * (size_t)(kColTY + fd.Kp) * kColTX;
    {
        const hipError_t e = g_col_lim.ensure((const void*)k_col_fp32, lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((W + kColTX - 1) / kColTX, (H + kColTY - 1) / kColTY, n_jobs);
    hipLaunchKernelGGL(k_col_fp32, grid, dim3(kColThreads), lds, stream, d_J, H, W, boundary,
                       fd.R, fd.Kp, d_jobs, n_jobs, d_taps, d_out, (const BatchImage*)nullptr);
    return hipGetLastError();
}

}  // namespace gabor
