// Adjoint of the Gabor bank on the vector ALU: the gradient of a real loss
// with respect to the image, given its gradient with respect to every output
// channel.
//
// Eq. (1) is F_c = f * K_c with K_c(t) = S(t_x) S(t_y) exp(i w (t_x cos(theta)
// + t_y sin(theta))).  For a real loss and G_c = dL/dRe F_c + i dL/dIm F_c,
//   dL/df(q) = sum_c sum_p Re(conj(G_c(p)) K_c(p - q)) = sum_c Re((G_c * K_c)(q)),
// because the Gabor kernel is Hermitian, K_c(-t) = conj(K_c(t)).  The adjoint
// is therefore the same separable bank applied to the complex G_c, keeping
// the real part and summing over channels.  Both 1-D passes reuse the
// forward's reversed taps krev[T] = k(R - T).
//
// Horizontal pass (one per forward horizontal result): with row taps c + id,
//   theta alone:          J = G_a * k
//   theta, pi - theta:    J = G_a * k + G_b * conj(k)        (Eq. (13))
// Both are two real signal pairs against c and d:
//   Re J = A * c + B * d,   Im J = C * c + D * d,
//   alone:  A = Re G_a, B = -Im G_a, C = Im G_a, D = Re G_a,
//   pair:   A = Re(G_a + G_b), B = Im(G_b - G_a), C = Im(G_a + G_b), D = Re(G_a - G_b).
// Vertical pass (one per horizontal result): Re(J * k_y) = Re J * c - Im J * d,
// accumulated over every job of the launch in registers and written once.
//
// Both passes can run on a grid extended by `off` on every side (J planes
// [H][W + 2 off], output [H + 2 off][W + 2 off], pixel (y, x) at image
// position (y - off, x - off), G zero outside the image): with off = R this
// is the adjoint on the mirror rule's extended image, whose positions the
// caller then folds back onto the pixels they mirror.
#include "gabor_internal.h"

namespace gabor {
namespace {

constexpr int kAdjRowP = 4;
constexpr int kAdjRowThreads = 256;
constexpr int kAdjColTX = 32, kAdjColTY = 64, kAdjColP = 8;

__global__ __launch_bounds__(kAdjRowThreads) void k_adj_row(
    const float2* __restrict__ G, int H, int W, int off, const AdjJob* __restrict__ jobs,
    const float* __restrict__ taps, float2* __restrict__ J)
{
    const int Wo = W + 2 * off;
    constexpr int P = kAdjRowP;
    extern __shared__ float4 adj_row_lds4[];
    const AdjJob jb = jobs[blockIdx.z];
    const int R = jb.R, Kp = jb.Kp;
    const int seg = kAdjRowThreads * P;
    const int x0 = blockIdx.x * seg, y = blockIdx.y;
    const int n = seg + Kp;                                  // staged samples x0 - R .. x0 - R + n - 1
    float* sA = reinterpret_cast<float*>(adj_row_lds4);
    float* sB = sA + n;
    float* sC = sB + n;
    float* sD = sC + n;
    const int64_t plane = (int64_t)H * W;
    const float2* ga = G + (int64_t)jb.out_a * plane + (int64_t)y * W;
    const float2* gb = jb.out_b >= 0 ? G + (int64_t)jb.out_b * plane + (int64_t)y * W : nullptr;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int xx = x0 - off - R + i;
        float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
        if (xx >= 0 && xx < W) {
            a = ga[xx];
            if (gb) b = gb[xx];
        }
        if (gb) {
            sA[i] = a.x + b.x;
            sB[i] = b.y - a.y;
            sC[i] = a.y + b.y;
            sD[i] = a.x - b.x;
        } else {
            sA[i] = a.x;
            sB[i] = -a.y;
            sC[i] = a.y;
            sD[i] = a.x;
        }
    }
    __syncthreads();

    const float* tc = taps + jb.tap_off;                     // row c
    const float* td = tc + Kp;                               // row d
    float re[P], im[P];
#pragma unroll
    for (int p = 0; p < P; ++p) re[p] = im[p] = 0.f;
    const int base = threadIdx.x * P;
    // Sliding register window: U taps per step over P + U staged samples of
    // each signal (16-byte LDS reads; Kp and the segment are multiples of 4).
    constexpr int U = kTapBlock;
    auto win = [&](const float* sig, int T, float (&w)[P + U]) {
#pragma unroll
        for (int j = 0; j < P + U; j += 4) {
            const float4 v = *reinterpret_cast<const float4*>(sig + base + T + j);
            w[j] = v.x; w[j + 1] = v.y; w[j + 2] = v.z; w[j + 3] = v.w;
        }
    };
    if (jb.j_real) {
        for (int T = 0; T < Kp; T += U) {
            float wa[P + U], wc[P + U];
            win(sA, T, wa);
            win(sC, T, wc);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float c = tc[T + u];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    re[p] = fmaf(wa[p + u], c, re[p]);
                    im[p] = fmaf(wc[p + u], c, im[p]);
                }
            }
        }
    } else {
        for (int T = 0; T < Kp; T += U) {
            float wa[P + U], wb[P + U], wc[P + U], wd[P + U];
            win(sA, T, wa);
            win(sB, T, wb);
            win(sC, T, wc);
            win(sD, T, wd);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float c = tc[T + u], d = td[T + u];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    re[p] = fmaf(wa[p + u], c, fmaf(wb[p + u], d, re[p]));
                    im[p] = fmaf(wc[p + u], c, fmaf(wd[p + u], d, im[p]));
                }
            }
        }
    }
    float2* dst = J + (int64_t)blockIdx.z * H * Wo + (int64_t)y * Wo;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int x = x0 + base + p;
        if (x < Wo) dst[x] = make_float2(re[p], im[p]);
    }
}

__global__ __launch_bounds__(kAdjColTX * (kAdjColTY / kAdjColP)) void k_adj_col(
    const float2* __restrict__ J, int H, int W, int off, const AdjJob* __restrict__ jobs, int n_jobs,
    const float* __restrict__ taps, float* __restrict__ grad, int64_t grad_stride)
{
    constexpr int TX = kAdjColTX, TY = kAdjColTY, P = kAdjColP;
    extern __shared__ float4 adj_col_lds4[];
    float2* tile = reinterpret_cast<float2*>(adj_col_lds4);  // [TY + Kp][TX]
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int x = x0 + tx;
    const int Ho = H + 2 * off, Wo = W + 2 * off;
    const int64_t plane = (int64_t)H * Wo;
    float acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.f;
    for (int j = 0; j < n_jobs; ++j) {
        const AdjJob jb = jobs[j];
        const int R = jb.R, Kp = jb.Kp;
        const float2* src = J + (int64_t)j * plane;
        const int rows = TY + Kp;
        __syncthreads();                                     // previous job's reads are done
        for (int i = threadIdx.x; i < rows * TX; i += blockDim.x) {
            const int r = i / TX, cx = i % TX;
            const int yy = y0 - off - R + r, xx = x0 + cx;
            tile[i] = (yy >= 0 && yy < H && xx < Wo) ? src[(int64_t)yy * Wo + xx] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const float* tc = taps + jb.tap_off + 2 * Kp;        // col c
        const float* td = tc + Kp;                           // col d
        const float2* col = tile + (ty * P) * TX + tx;
        // Sliding register window down the column: U taps per step.
        constexpr int U = kTapBlock;
        if (jb.c_real) {
            for (int T = 0; T < Kp; T += U) {
                float w[P + U];
#pragma unroll
                for (int j = 0; j < P + U; ++j) w[j] = col[(T + j) * TX].x;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const float c = tc[T + u];
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[p] = fmaf(w[p + u], c, acc[p]);
                }
            }
        } else {
            for (int T = 0; T < Kp; T += U) {
                float2 w[P + U];
#pragma unroll
                for (int j = 0; j < P + U; ++j) w[j] = col[(T + j) * TX];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const float c = tc[T + u], d = td[T + u];
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[p] = fmaf(w[p + u].x, c, fmaf(-w[p + u].y, d, acc[p]));
                }
            }
        }
    }
    if (x < Wo) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int y = y0 + ty * P + p;
            if (y < Ho) grad[(int64_t)y * grad_stride + x] = acc[p];
        }
    }
}

}  // namespace

size_t adj_row_lds_bytes(int max_kp) { return 4 * sizeof(float) * (size_t)(kAdjRowThreads * kAdjRowP + max_kp); }
size_t adj_col_lds_bytes(int max_kp) { return sizeof(float2) * (size_t)(kAdjColTY + max_kp) * kAdjColTX; }

hipError_t launch_adjoint(const float2* d_G, int H, int W, int off, const AdjJob* d_jobs, int n_jobs,
                          int max_kp, const float* d_taps, float2* d_J, float* d_grad, int64_t grad_stride,
                          hipStream_t stream)
{
    if (n_jobs <= 0 || n_jobs > 65535 || H > 65535 || off < 0) return hipErrorInvalidValue;
    const int Ho = H + 2 * off, Wo = W + 2 * off;
    if (grad_stride < Wo) return hipErrorInvalidValue;
    const size_t row_lds = adj_row_lds_bytes(max_kp), col_lds = adj_col_lds_bytes(max_kp);
    if (row_lds > 160 * 1024 || col_lds > 160 * 1024) return hipErrorInvalidValue;
    static LdsLimit row_lim, col_lim;
    hipError_t e;
    if ((e = row_lim.ensure((const void*)k_adj_row, row_lds)) != hipSuccess) return e;
    if ((e = col_lim.ensure((const void*)k_adj_col, col_lds)) != hipSuccess) return e;
    const int seg = kAdjRowThreads * kAdjRowP;
    hipLaunchKernelGGL(k_adj_row, dim3((Wo + seg - 1) / seg, H, n_jobs), dim3(kAdjRowThreads), row_lds, stream,
                       d_G, H, W, off, d_jobs, d_taps, d_J);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_col, dim3((Wo + kAdjColTX - 1) / kAdjColTX, (Ho + kAdjColTY - 1) / kAdjColTY),
                       dim3(kAdjColTX * (kAdjColTY / kAdjColP)), col_lds, stream,
                       (const float2*)d_J, H, W, off, d_jobs, n_jobs, d_taps, d_grad, grad_stride);
    return hipGetLastError();
}

}  // namespace gabor
