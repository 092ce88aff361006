// libgabor host side of the localized sliding DFT (Sec. III-A): argument
// checks, the window weights and twiddles of Eq. (17)-(18) in FP64, and the
// single launch of the fused kernel in its localized-SDFT form.
//
// The horizontal pass of bin u is the 1-D transform J_u of Eq. (18) with the
// window weights folded into the taps; J_{Mx-u} = conj(J_u) for a real image
// (Eq. (19)), so only u <= Mx/2 is filtered.  The vertical pass of bin v runs
// over J_u and conj(J_u) for v <= My/2, and the remaining bins are the
// conjugates of computed ones (Eq. (20)).  Every table lives in the launch
// arguments: nothing is allocated.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/libgabor.h"
#include "gabor_internal.h"

using namespace gabor;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

int fused_op_of(gabor_precision p)
{
    switch (p) {
        case GABOR_PREC_FP32: return FUSED_F32;
        case GABOR_PREC_BF16_SPLIT: return FUSED_BF16X3;
        case GABOR_PREC_FP16_SPLIT: return FUSED_F16X3;
        case GABOR_PREC_BF16: return FUSED_BF16;
        case GABOR_PREC_FP16: return FUSED_F16;
    }
    return -1;
}

// Window weights of offsets j = 0..M-1 (centre M/2, unit sum) and the
// twiddles cos, sin(2 pi k / M).  Quarter turns are exact, and the second
// half of the table mirrors the first so that tw(M - k) = conj(tw(k)) holds
// bit for bit.
void axis_tables(int M, double sigma, double* win, double* twc, double* tws)
{
    const int h = M / 2;
    double sum = 0.0;
    for (int j = 0; j < M; ++j) {
        const double t = (double)(h - j);
        win[j] = std::exp(-t * t / (2.0 * sigma * sigma));
        sum += win[j];
    }
    for (int j = 0; j < M; ++j) win[j] /= sum;
    for (int k = 0; k <= M / 2; ++k) {
        double c, s;
        if ((4 * k) % M == 0) {
            static const double qc[4] = {1.0, 0.0, -1.0, 0.0}, qs[4] = {0.0, 1.0, 0.0, -1.0};
            c = qc[(4 * k / M) % 4];
            s = qs[(4 * k / M) % 4];
        } else {
            const double a = 2.0 * kPi * (double)k / (double)M;
            c = std::cos(a);
            s = std::sin(a);
        }
        twc[k] = c;
        tws[k] = s;
        if (k > 0 && M - k != k) {
            twc[M - k] = c;
            tws[M - k] = -s;
        }
    }
}

}  // namespace

extern "C" gabor_status lsdft_work(int32_t height, int32_t width, int32_t m_y, int32_t m_x,
                                   int64_t* real_macs, int64_t* bytes)
{
    if (height <= 0 || width <= 0 || m_y <= 0 || m_x <= 0) return GABOR_ERR_INVALID_ARG;
    const int64_t npix = (int64_t)height * width;
    int64_t macs = 0;
    for (int u = 0; u <= m_x / 2; ++u) {
        const bool jr = u == 0 || 2 * u == m_x;
        macs += (jr ? 1 : 2) * (int64_t)m_x;                       // horizontal pass of J_u
        for (int v = 0; v <= m_y / 2; ++v) {
            const bool cr = v == 0 || 2 * v == m_y;
            macs += (int64_t)(jr ? 1 : 2) * (cr ? 1 : 2) * m_y;     // vertical pass of J_u (and conj)
        }
    }
    if (real_macs) *real_macs = macs * npix;
    if (bytes) *bytes = 4 * npix + 8 * (int64_t)m_y * m_x * npix;
    return GABOR_OK;
}

extern "C" gabor_status lsdft_apply(const float* d_image, int32_t height, int32_t width,
                                    int64_t row_stride_elems, int32_t m_y, int32_t m_x, double sigma,
                                    gabor_boundary boundary, gabor_precision precision, void* d_out,
                                    void* hip_stream)
{
    if (!d_image || !d_out) return GABOR_ERR_INVALID_ARG;
    if (height <= 0 || width <= 0 || m_y <= 0 || m_x <= 0) return GABOR_ERR_INVALID_ARG;
    if (row_stride_elems < width) return GABOR_ERR_INVALID_ARG;
    if (!std::isfinite(sigma) || !(sigma > 0.0)) return GABOR_ERR_INVALID_ARG;
    if (boundary != GABOR_BOUNDARY_ZERO && boundary != GABOR_BOUNDARY_MIRROR) return GABOR_ERR_INVALID_ARG;
    const int op = fused_op_of(precision);
    if (op < 0) return GABOR_ERR_INVALID_ARG;
    // Limits of this build: tables in the launch arguments (M <= 64), 32-bit
    // buffer offsets within the image and within each output plane (2^30
    // bytes: 2^27 pixels).
    if (m_y > kLsdftMaxM || m_x > kLsdftMaxM) return GABOR_ERR_UNSUPPORTED;
    const int64_t npix = (int64_t)height * width;
    if (npix > (int64_t(1) << 27) || height > 65535) return GABOR_ERR_UNSUPPORTED;
    if ((int64_t)(height - 1) * row_stride_elems + width >= (int64_t(1) << 30)) return GABOR_ERR_UNSUPPORTED;

    LsdftTaps t;
    std::memset(&t, 0, sizeof(t));
    t.m[0] = m_x;
    t.m[1] = m_y;
    axis_tables(m_x, sigma, t.win[0], t.tw[0][0], t.tw[0][1]);
    axis_tables(m_y, sigma, t.win[1], t.tw[1][0], t.tw[1][1]);

    // One radius covers both windows: offsets run from -M/2 to M - 1 - M/2.
    const int R = std::max(m_x / 2, m_y / 2);
    const int Q = stream_quarter(op, R);
    StreamArgs a{};
    a.img = d_image;
    a.stride = row_stride_elems;
    a.H = height;
    a.W = width;
    a.boundary = boundary;
    a.R = R;
    a.seg_rows = std::max(128, 16 * Q);
    if (a.seg_rows > height) a.seg_rows = (height + 15) / 16 * 16;
    a.n_xs = (width + stream_strip_width() - 1) / stream_strip_width();
    a.n_ys = (height + a.seg_rows - 1) / a.seg_rows;
    a.n_jobs = (m_x / 2 + 1) * (m_y / 2 + 1);
    a.jobs = nullptr;
    a.taps = nullptr;
    a.out = (float2*)d_out;
    a.in_scale = a.mid_scale = a.out_scale = a.tap_scale[0] = a.tap_scale[1] = 1.0f;
    if (op == FUSED_F16 || op == FUSED_F16X3) {
        // float16 range: image scaled by 2^8, each axis' taps by the power of
        // two that brings its largest window weight to [2^13, 2^14).
        const double wx = *std::max_element(t.win[0], t.win[0] + m_x);
        const double wy = *std::max_element(t.win[1], t.win[1] + m_y);
        const float tx = std::ldexp(1.0f, 13 - (int)std::floor(std::log2(wx)));
        const float ty = std::ldexp(1.0f, 13 - (int)std::floor(std::log2(wy)));
        a.in_scale = 256.0f;
        a.tap_scale[0] = tx;
        a.tap_scale[1] = ty;
        a.mid_scale = 1.0f / tx;
        a.out_scale = 1.0f / (256.0f * ty);
    }
    if ((int64_t)a.n_xs * a.n_ys * a.n_jobs > 0x7fffffffLL) return GABOR_ERR_UNSUPPORTED;
    return launch_lsdft(op, a, t, Q, (hipStream_t)hip_stream) == hipSuccess ? GABOR_OK : GABOR_ERR_DEVICE;
}
