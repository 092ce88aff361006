// Internal declarations shared by the libgabor host code and its HIP kernels.
// Nothing here is part of the public C ABI (include/libgabor.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace gabor {

// Dynamic-LDS limit of one kernel, raised once per device and size: the
// attribute persists, and setting it before every launch costs a driver call
// on the host (a noticeable part of an apply's submission time).
struct LdsLimit {
    static constexpr int kDevices = 64;
    std::atomic<int> bytes[kDevices] = {};
    hipError_t ensure(const void* fn, size_t need)
    {
        if (need <= 64 * 1024) return hipSuccess;
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices)
            return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
        if (bytes[dev].load(std::memory_order_acquire) >= (int)need) return hipSuccess;
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
        if (e == hipSuccess) {
            int cur = bytes[dev].load(std::memory_order_relaxed);
            while (cur < (int)need && !bytes[dev].compare_exchange_weak(cur, (int)need, std::memory_order_acq_rel)) {
            }
        }
        return e;
    }
};

// Tap blocks: every tap table is zero-padded to a multiple of this many taps.
constexpr int kTapBlock = 4;

// One vertical pass (Eq. (4)) over one horizontal result J.  It produces
// F_a = J * k and, when out_b >= 0, F_b = conj(J) * k (the pi - theta
// orientation, Eq. (15)-(16)), where k(t) = S(t) exp(i w sin(theta) t).
struct ColJob {
    int32_t freq;      // frequency index (selects R and the taps)
    int32_t plane;     // J plane in the workspace
    int32_t out_a;     // output channel index i*N + n
    int32_t out_b;     // partner channel or -1
    int32_t j_real;    // J is real (w cos(theta) == 0)
    int32_t c_real;    // column taps are real (w sin(theta) == 0)
    int32_t tap_off;   // offset of this job's [Kp][2] (c, d) taps in the tap table
    int32_t pad_;
};

// Launch parameters of one horizontal-pass group: all horizontal passes of
// one frequency that read the same image rows.
struct RowGroup {
    int32_t freq;
    int32_t n_cplx;    // complex-J passes (taps c, d)
    int32_t n_real;    // real-J passes (taps c only), 0 or 1
    int32_t tap_off;   // offset of the [Kp][2*n_cplx + n_real] taps
    int32_t plane0;    // first J plane; passes write plane0 .. plane0+n-1
};

struct FreqDesc {
    int32_t R;         // truncation radius
    int32_t K;         // 2R + 1
    int32_t Kp;        // K padded to a multiple of kTapBlock
};

// Fused streaming matrix-core kernel (gabor_fused.hip): one horizontal
// result and its vertical pass per workgroup over a 64-column strip, J held
// in an LDS ring.
enum FusedOp { FUSED_F32 = 0, FUSED_BF16 = 1, FUSED_BF16X3 = 2, FUSED_F16 = 3, FUSED_F16X3 = 4 };
constexpr int kStreamMaxQuarter = 56;   // contracted length L = 4Q <= 224: R <= 104

struct FusedJob {
    int32_t out_a;     // output plane of F = J * k
    int32_t out_b;     // output plane of conj(J) * k (pi - theta, or M - u) or -1
    int32_t out_c;     // plane that receives conj(F_a) or -1 (conjugate fill)
    int32_t out_d;     // plane that receives conj(F_b) or -1
    int32_t j_real;    // horizontal taps have no sine part
    int32_t c_real;    // vertical taps have no sine part
    int32_t tap_off;   // [4][L+16] zero-padded reversed taps: row c, row d, col c, col d
    int32_t pad_;
};

struct StreamArgs {
    const float* img;
    int64_t stride;
    int32_t H, W, boundary, R;
    int32_t seg_rows;          // rows per strip segment (multiple of 16)
    int32_t n_xs, n_ys, n_jobs;
    const FusedJob* jobs;
    const float* taps;
    float2* out;
    float in_scale;            // image scale before conversion (16-bit range)
    float mid_scale;           // J scale after the horizontal pass
    float out_scale;           // output scale after the vertical pass
    float tap_scale[2];        // horizontal, vertical tap scales
    // Images of one strided batch (wave-specialised kernel only; 1 and 0
    // elsewhere): image b reads img + b * img_bstride and writes
    // out + b * out_bstride.
    int32_t n_images;
    int64_t img_bstride, out_bstride;
};

// Adjoint on the matrix cores: one launch per fused frequency (FP32), one
// workgroup per (job, 64-column strip, row segment), each job writing its
// own partial plane; the planes are then summed in job order.  The partial
// planes cover an output grid Ho x Wo whose pixel (y, x) is image position
// (y - off, x - off): the image itself for the zero boundary, the image
// extended by R on every side for the mirror rule, whose sum then adds each
// extended position into the pixel it folds to.
struct AdjStreamArgs {
    const float2* G;           // dL/dF planes [O N][H][W], complex64
    float* part;               // partial planes of this frequency's jobs [n_jobs][Ho][Wo]
    int32_t H, W;              // image
    int32_t Ho, Wo, off;       // output grid of the partial planes
    int32_t R, seg_rows, n_xs, n_ys, n_jobs;
    const FusedJob* jobs;      // this frequency's jobs
    const float* taps;         // reversed taps, fused-kernel layout [4][4Q + 16]
    // strided batch: image b reads G + b * g_bstride, writes part + b * part_bstride
    int32_t n_images;
    int64_t g_bstride, part_bstride;
};
constexpr int kAdjStreamMaxQuarter = 32;   // R <= 56
size_t adjoint_stream_lds_bytes(int Q);
hipError_t launch_adjoint_stream(const AdjStreamArgs& a, int Q, hipStream_t stream);
// zero boundary: dL/df[y][x] = sum over the n planes [H][W] of part, in plane
// order; image b of a batch of n_images sums part + b * part_bstride into
// grad + b * grad_bstride
hipError_t launch_adjoint_sum(const float* part, int n, int H, int W, float* grad, int64_t grad_stride,
                              int n_images, int64_t part_bstride, int64_t grad_bstride, hipStream_t stream);
// mirror rule: per frequency, planes [count][H + 2R][W + 2R] from element base
struct AdjFoldFreq {
    int64_t base;
    int32_t R, count;
};
constexpr int kAdjFoldMaxFreq = 32;
struct AdjFoldArgs {
    const float* part;
    float* grad;
    int64_t grad_stride;
    int32_t H, W, n_freq, n_images;
    int64_t part_bstride, grad_bstride;   // per image of a batch
    AdjFoldFreq f[kAdjFoldMaxFreq];
};
hipError_t launch_adjoint_fold_sum(const AdjFoldArgs& a, hipStream_t stream);

// Batched bank (one launch per operand quarter): images of any size up to
// the plan's, each tile one (image, job, strip segment).
struct BatchImage {
    const float* img;
    float2* out;               // [O][N][H][W] of this image
    int64_t stride;
    int64_t J_off;             // first element of its J planes (two-pass frequencies)
    int32_t H, W, n_xs, pad_;
};
struct BatchFreq {
    int32_t R, seg_rows;
    float in_scale, mid_scale, out_scale, tap_scale[2];
    int32_t q;                 // operand quarter (contracted length 4q)
};
struct BatchTile {
    int32_t image, job, freq;  // job indexes the plan's fused job table
    int32_t rest;              // strip + segment * n_xs of the image
};
struct BatchArgs {
    const BatchImage* images;
    const BatchFreq* freqs;
    const BatchTile* tiles;
    const FusedJob* jobs;
    const float* taps;
    int32_t n_tiles, boundary;
};
// Launches the four-wave batch kernel of one form and quarter, one
// workgroup per tile.
hipError_t launch_batch(int op, const BatchArgs& b, int Q, hipStream_t stream);

// Localized SDFT taps, passed by value as a kernel argument (no device
// tables): axis 0 is x (the horizontal pass), axis 1 is y.
constexpr int kLsdftMaxM = 64;
struct LsdftTaps {
    int32_t m[2];                      // window size Mx, My
    double win[2][kLsdftMaxM];         // Gaussian window weights of offsets j = 0..M-1, unit sum
    double tw[2][2][kLsdftMaxM];       // cos, sin of 2 pi k / M, k = 0..M-1 (exact at quarter turns)
};

// Wave-specialised streaming kernel (gabor_ws.hip): the same jobs and
// results as launch_stream, eight waves per workgroup (four on the
// horizontal pass, four on the vertical one), quarters up to
// ws_max_quarter(op) (FP32 52, single 16-bit 56, split 40), segments of any
// multiple of 16 rows.
int ws_max_quarter(int op);
bool ws_supported(int op, int Q);
// Q for radius R on the wave-specialised kernel: L = 4Q >= 16 + 2R, a
// multiple of 16 (FP32) or 32 (16-bit forms) whatever R.
int ws_quarter(int op, int R);
hipError_t launch_ws(int op, const StreamArgs& a, int Q, hipStream_t stream);
// The localized SDFT on the wave-specialised kernel (the same jobs and
// results as launch_lsdft's four-wave kernel).
hipError_t launch_ws_lsdft(int op, const StreamArgs& a, const LsdftTaps& t, int Q, hipStream_t stream);
// Raises the dynamic-LDS limits of the wave-specialised kernels of (op, Q)
// once, outside any graph capture (plan creation).
hipError_t prepare_ws(int op, int Q);
size_t ws_lds_bytes(int op, int Q);

// The same kernel over a tile table (batches): workgroup b takes tile b,
// every tile of one quarter Q; tiles sorted by decreasing cost.
struct WsTilesArgs {
    const BatchImage* images;
    const BatchFreq* freqs;
    const BatchTile* tiles;
    const FusedJob* jobs;
    const float* taps;
    int32_t n_tiles, boundary;
};
hipError_t launch_ws_tiles(int op, const WsTilesArgs& t, int Q, hipStream_t stream);
// The small quarters (Q <= kWsSmallQuarter) in one launch: each workgroup
// runs its tile's quarter; registers and LDS are the largest member's.
constexpr int kWsSmallQuarter = 16;
bool ws_small_quarter(int op, int Q);
hipError_t launch_ws_tiles_small(int op, const WsTilesArgs& t, hipStream_t stream);
hipError_t prepare_ws_small(int op);

int stream_quarter(int op, int R);             // Q for radius R (L = 4Q >= 16 + 2R)
size_t stream_lds_bytes(int op, int Q);
int stream_strip_width();
hipError_t launch_stream(int op, const StreamArgs& a, int Q, hipStream_t stream);
hipError_t launch_lsdft(int op, const StreamArgs& a, const LsdftTaps& t, int Q, hipStream_t stream);

// Per-form launchers (one object per form); Q outside the built set returns
// hipErrorInvalidValue.
template <int OP> hipError_t stream_form(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream);
template <int OP> hipError_t lsdft_form(const StreamArgs& a, const LsdftTaps& t, int Q, int n_blocks,
                                        hipStream_t stream);
template <int OP> hipError_t batch_form(const BatchArgs& b, int Q, hipStream_t stream);
template <int OP> hipError_t ws_form(const StreamArgs& a, int Q, int n_blocks, hipStream_t stream);
template <int OP> hipError_t ws_tiles_form(const WsTilesArgs& t, int Q, hipStream_t stream);
template <int OP> hipError_t ws_prepare_form(int Q);
template <int OP> hipError_t ws_lsdft_form(const StreamArgs& a, const LsdftTaps& t, int Q, int n_blocks,
                                           hipStream_t stream);
template <int OP> hipError_t ws_small_form(const WsTilesArgs* t, hipStream_t stream);   // t null: prepare only
#define GABOR_DECLARE_FORM(OP)                                                                   \
    template <> hipError_t stream_form<OP>(const StreamArgs&, int, int, hipStream_t);            \
    template <> hipError_t ws_form<OP>(const StreamArgs&, int, int, hipStream_t);                \
    template <> hipError_t ws_tiles_form<OP>(const WsTilesArgs&, int, hipStream_t);              \
    template <> hipError_t ws_prepare_form<OP>(int);                                              \
    template <> hipError_t ws_lsdft_form<OP>(const StreamArgs&, const LsdftTaps&, int, int, hipStream_t); \
    template <> hipError_t ws_small_form<OP>(const WsTilesArgs*, hipStream_t);                    \
    template <> hipError_t lsdft_form<OP>(const StreamArgs&, const LsdftTaps&, int, int, hipStream_t); \
    template <> hipError_t batch_form<OP>(const BatchArgs&, int, hipStream_t);
GABOR_DECLARE_FORM(FUSED_F32)
GABOR_DECLARE_FORM(FUSED_BF16)
GABOR_DECLARE_FORM(FUSED_BF16X3)
GABOR_DECLARE_FORM(FUSED_F16)
GABOR_DECLARE_FORM(FUSED_F16X3)
#undef GABOR_DECLARE_FORM

// One horizontal result of the bank as seen by the adjoint (zero boundary):
// the channels it feeds and its tap sets.
struct AdjJob {
    int32_t R, Kp;     // radius and padded tap count of its frequency
    int32_t out_a;     // channel i*N + n
    int32_t out_b;     // pi - theta partner channel or -1
    int32_t j_real;    // horizontal taps have no sine part
    int32_t c_real;    // vertical taps have no sine part
    int32_t tap_off;   // [4][Kp] reversed taps k(R - T): row c, row d, col c, col d
    int32_t pad_;
};

size_t adj_row_lds_bytes(int max_kp);
size_t adj_col_lds_bytes(int max_kp);
// Horizontal adjoint pass of every job into d_J ([n_jobs][H][Wo]), then the
// vertical pass summed over the jobs into d_grad, an Ho x Wo grid whose
// pixel (y, x) is image position (y - off, x - off) with Ho = H + 2 off and
// Wo = W + 2 off (gabor_adjoint.hip).  off = 0 gives the zero boundary's
// gradient itself; the mirror rule takes off = R and folds the grid.
hipError_t launch_adjoint(const float2* d_G, int H, int W, int off, const AdjJob* d_jobs, int n_jobs,
                          int max_kp, const float* d_taps, float2* d_J, float* d_grad, int64_t grad_stride,
                          hipStream_t stream);

// Recursive-smoother variant (gabor_iir.hip): one recursion job runs a
// causal and an anti-causal third-order recursion down every column of a
// plane of n rows (lines extended by T rows on both sides by the boundary
// rule), with modulation by exp(-i w l) before and demodulation by
// exp(i w l) after, twiddles (cos, sin)(w l) at tw[tw_off + l + T].
// Chunks per line of the block-parallel recursion (one wave each).
constexpr int kIirChunks = 16;
struct IirJob {
    const void* in;            // float [n][in_stride] or float2 [n][in_stride]
    float2* scratch;           // [n + 2T][cols] forward results (scratch-plane kernel)
    float2* out;               // [n][out_stride], or null: out_base plane out_plane
    int64_t in_stride, out_stride;
    int32_t in_complex, conj;  // input type; conjugate a complex input
    int32_t n, cols, T, tw_off, out_plane;
    int32_t out_rows;          // line c's outputs go to row c of the output (register kernel, lc <= kIirRowChunk)
    int32_t lc;                // chunk length: ceil((n + 2T) / chunks per line)
    float a[4];                // w[m] = a0 u[m] - a1 w[m-1] - a2 w[m-2] - a3 w[m-3]
    double apow[9];            // A^lc, row-major, A = [[-a1, -a2, -a3], [1, 0, 0], [0, 1, 0]]
    double apow2[5][9];        // (A^lc)^(2^k), k = 1..5 (the register kernel's parallel carry)
};
// The register-resident recursion cuts each line into kIirRegChunks chunks
// of at most kIirRegMaxChunk samples (lines of up to 4096 extended samples);
// longer lines keep their forward results in a scratch plane (kIirChunks
// chunks per line).
constexpr int kIirRegChunks = 64;
constexpr int kIirRegMaxChunk = 64;
// Longest chunk with which the register kernel can write its lines as rows
// (staged through its 24 KB carry buffer, eight chunks of each line at a time).
constexpr int kIirRowChunk = 48;
// Transpose, horizontal jobs (on the transposed image, into d_J planes [H][W]
// directly when their jobs write rows, else into d_JT planes [W][H] and
// transposed back into d_J), vertical jobs (into the output channels of
// d_out).  max_lc_h / max_lc_v: the longest chunk of each pass's jobs;
// reg_h / reg_v: the pass's jobs are chunked for the register kernel (else
// for the scratch-plane one); rows_h: the horizontal jobs write rows.
hipError_t launch_iir(const float* d_image, int64_t stride, int H, int W, int boundary, float* d_fT,
                      const IirJob* d_hjobs, int n_hjobs, int max_lc_h, bool reg_h, bool rows_h, float2* d_JT, float2* d_J,
                      const IirJob* d_vjobs, int n_vjobs, int max_lc_v, bool reg_v, const float2* d_tw,
                      float2* d_out, hipStream_t stream);

// Launchers (defined in gabor_fp32.hip).  They return the status of the
// launch (hipGetLastError after enqueue).
hipError_t launch_row_fp32(const float* img, int64_t stride, int H, int W, int boundary,
                           const FreqDesc& fd, const RowGroup& g, const float* d_taps,
                           float2* d_J, hipStream_t stream);

hipError_t launch_col_fp32(const float2* d_J, int H, int W, int boundary, const FreqDesc& fd,
                           const ColJob* d_jobs, int n_jobs, const float* d_taps,
                           float2* d_out, hipStream_t stream);

// The same kernels over every image of a batch in one launch each: grid z
// selects the image (and the job), H and W are the largest extents, and
// blocks outside an image return at once.  Each image's J planes start at
// its J_off in d_J; its outputs at its own pointer.
hipError_t launch_row_fp32_batch(const BatchImage* d_imgs, int n_images, int max_h, int max_w, int boundary,
                                 const FreqDesc& fd, const RowGroup& g, const float* d_taps, float2* d_J,
                                 hipStream_t stream);
hipError_t launch_col_fp32_batch(const BatchImage* d_imgs, int n_images, int max_h, int max_w, int boundary,
                                 const FreqDesc& fd, const ColJob* d_jobs, int n_jobs, const float* d_taps,
                                 float2* d_J, hipStream_t stream);

}  // namespace gabor
