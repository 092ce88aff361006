/*
 * libgabor -- 2-D complex Gabor filter bank by kernel decomposition, and the
 * Gaussian-windowed 2-D localized sliding DFT, on AMD Instinct MI355X (gfx950).
 *
 * Method: Um, Kim & Min, "Fast 2-D Complex Gabor Filter with Kernel
 * Decomposition" (arXiv 1704.05231).  The bank output of Eq. (1)-(2) is
 * computed as a horizontal 1-D Gabor pass J (Eq. (3)) followed by a vertical
 * 1-D Gabor pass (Eq. (4)); the horizontal result of orientation theta is
 * reused, conjugated, for pi - theta (Eq. (13)-(16)); Algorithm 1 is the bank
 * schedule.  The localized SDFT is Eq. (17)-(18) computed the same way
 * (Eq. (19)-(26), Algorithm 2); its box-window special case, the
 * conventional SDFT, is also computed by the circular-shift recursion.
 *
 * Conventions shared by every entry point:
 *   - Images are single-channel FP32, row-major, H rows by W columns, with a
 *     row stride in elements (>= W).  x is the column, y the row, 0-based.
 *   - Outputs are complex64, interleaved (re, im) pairs of float, dense
 *     row-major planes of H x W complex values, fully overwritten.
 *   - All image and output pointers are DEVICE pointers owned by the caller;
 *     input and output must not overlap.  Host arrays (omega, sigma, theta)
 *     are read during the call only.
 *   - Eq. (1) is a convolution: the kernel is evaluated at (x-k, y-l), so an
 *     impulse reproduces the kernel itself.
 *   - The Gaussian factor S (G(x,y) = S(x) S(y), Sec. II) is sampled at
 *     integer offsets |t| <= R with R = floor(radius_sigmas * sigma + 0.5),
 *     and normalised to unit sum over those taps (the paper fixes neither
 *     the support nor the normalisation; this is the exact FIR the paper
 *     calls lossless in Sec. IV-B).
 *   - Every call is asynchronous on the given HIP stream (hipStream_t passed
 *     as void*; NULL = the default stream).  Argument checks run on the host
 *     before anything is enqueued; a rejected call writes nothing.  Device
 *     faults surface at the caller's next synchronisation of the stream.
 *   - No call throws; every call returns a gabor_status.
 */
#ifndef LIBGABOR_H
#define LIBGABOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gabor_plan_s* gabor_plan;

typedef enum gabor_status {
    GABOR_OK = 0,
    GABOR_ERR_INVALID_ARG = 1,   /* a null pointer, a size <= 0, sigma <= 0,
                                    a non-finite parameter, stride < W, a bad
                                    enum value, a plan/image size mismatch */
    GABOR_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
    GABOR_ERR_DEVICE = 3,        /* a HIP runtime call or launch failed */
    GABOR_ERR_UNSUPPORTED = 4    /* valid arguments this build cannot run */
} gabor_status;

typedef enum gabor_boundary {
    GABOR_BOUNDARY_ZERO = 0,   /* f = 0 outside the image */
    GABOR_BOUNDARY_MIRROR = 1  /* whole-sample mirror f(-1) = f(1), folded
                                  repeatedly with period 2(n-1); n = 1 gives a
                                  constant extension */
} gabor_boundary;

typedef enum gabor_precision {
    GABOR_PREC_FP32 = 0,        /* FP32 products, FP32 accumulation */
    GABOR_PREC_BF16_SPLIT = 1,  /* matrix cores: operands split hi+lo in
                                   bfloat16, three products, FP32 accumulation */
    GABOR_PREC_FP16_SPLIT = 2,  /* as above with float16 operands; the image
                                   is scaled by 2^8 so that the lo parts stay
                                   normal, so |f| must stay below 128: larger
                                   pixel values overflow float16 and give
                                   Inf/NaN outputs, which no status reports */
    GABOR_PREC_BF16 = 3,        /* matrix cores: one bfloat16 product */
    GABOR_PREC_FP16 = 4         /* matrix cores: one float16 product; the
                                   same |f| < 128 input range as FP16_SPLIT */
} gabor_precision;

/* Human-readable name of a status code (static storage, never NULL). */
const char* gabor_status_string(gabor_status status);

/*
 * gabor_bank_plan -- prepare the bank of Algorithm 1 (Sec. II-B) for images
 * of height x width.
 *
 *   out            receives the plan handle (set to NULL on failure).
 *   n_freq         O >= 1 frequencies; omega[O] in radians per pixel
 *                  (omega = 2 pi / lambda, Eq. (2)); sigma[O] > 0 in pixels,
 *                  one Gaussian scale per frequency (the set Sigma of
 *                  Algorithm 1).
 *   n_orient       N >= 1 orientations; theta[N] in radians, or NULL for
 *                  theta_k = k pi / N, k = 0..N-1 (Sec. II-B).  Orientations
 *                  whose sum is pi share one horizontal pass (Eq. (13));
 *                  unpaired orientations are computed on their own.
 *   radius_sigmas  truncation of S in units of sigma (3.0 gives R = 3 sigma).
 *   boundary       rule for samples outside the image.
 *   precision      arithmetic of the Gaussian contractions.  Frequencies the
 *                  fused kernel cannot take (R > 104, or planes of more than
 *                  2^27 pixels) run the FP32 two-pass kernels whatever the
 *                  precision.
 *   hip_stream     stream used to upload the plan's tables.
 *
 * The plan owns device memory for its tap tables and any intermediate
 * workspace; it is freed by gabor_bank_destroy.  One plan serves one stream
 * at a time.
 */
gabor_status gabor_bank_plan(gabor_plan* out, int32_t height, int32_t width,
                             int32_t n_freq, const double* omega, const double* sigma,
                             int32_t n_orient, const double* theta,
                             double radius_sigmas, gabor_boundary boundary,
                             gabor_precision precision, void* hip_stream);

/*
 * gabor_bank_plan_iir -- the same bank with the paper's recursive smoother
 * (Sec. II-A): each 1-D pass modulates by exp(-i w t), smooths with the
 * third-order recursive Gaussian of van Vliet, Young and Verbeek (ICPR
 * 1998; a causal pass and its anti-causal mirror, poles scaled so that the
 * impulse response has variance sigma^2), and demodulates; the pi - theta
 * partner reuses conj(J).  The cost per pixel does not depend on sigma; the
 * result approximates Eq. (1) with the untruncated Gaussian (about 30 dB
 * signal-to-error ratio), it is not the truncated FIR of gabor_bank_plan.
 * Lines are extended by ceil(6 sigma) + 3 samples by the boundary rule.
 * Arguments as for gabor_bank_plan (no truncation radius; FP32 arithmetic
 * with FP64-reduced twiddles).  sigma below 0.5 returns
 * GABOR_ERR_UNSUPPORTED.  The plan is applied with gabor_bank_apply; the
 * adjoint and batches are not available for it (GABOR_ERR_UNSUPPORTED) and
 * autotuning does nothing.
 */
gabor_status gabor_bank_plan_iir(gabor_plan* out, int32_t height, int32_t width,
                                 int32_t n_freq, const double* omega, const double* sigma,
                                 int32_t n_orient, const double* theta,
                                 gabor_boundary boundary, void* hip_stream);

/*
 * gabor_bank_apply -- run the bank on one image.
 *
 *   d_image           device FP32 image, height x width of the plan, row
 *                     stride row_stride_elems (>= width).
 *   d_out             device complex64 output, layout [O][N][H][W] (frequency
 *                     major, then orientation in the order given to the
 *                     plan), O*N*H*W*8 bytes, fully overwritten.
 */
gabor_status gabor_bank_apply(gabor_plan plan, const float* d_image,
                              int64_t row_stride_elems, void* d_out, void* hip_stream);

/*
 * gabor_bank_apply_adjoint -- gradient of a real loss L with respect to the
 * image, given its gradient with respect to every bank output (the adjoint
 * of gabor_bank_apply; derived from Eq. (1)).
 *
 *   d_grad_out        device complex64 [O][N][H][W], the plan's output
 *                     layout; element c holds dL/dRe F_c + i dL/dIm F_c (the
 *                     convention of PyTorch's complex gradients).
 *   d_grad_image      device FP32 [H][W] with row stride
 *                     grad_row_stride_elems (>= width), fully overwritten with
 *                       dL/df(q) = sum_c sum_p Re(conj(G_c(p)) K_c(p - q)),
 *                     i.e. sum_c Re((G_c * K_c)(q)): the Gabor kernel is
 *                     Hermitian, so the adjoint is the same bank applied to
 *                     the complex gradients, real part summed over channels.
 *                     Under the mirror rule the sum runs over every position
 *                     p - t whose fold is q (the transpose of the fold).
 *
 * Each frequency that runs in the fused kernel with R <= 56 takes the
 * matrix cores (one partial plane per horizontal result); every other
 * frequency takes the vector-ALU kernels (one partial plane).  The planes
 * cover the image (zero boundary) or the image extended by the frequency's R
 * (mirror rule), and a last launch sums them in a fixed order, folding the
 * extended positions under the mirror rule.  A zero-boundary plan with no
 * matrix-core frequency writes dL/df straight from the vector kernels.
 * Mirror plans of more than 32 frequencies and recursive-smoother plans
 * return GABOR_ERR_UNSUPPORTED.  The arithmetic is FP32 whatever the plan's
 * precision, and the result is deterministic.  The first call on a plan
 * allocates its adjoint workspace (4 bytes per partial-plane pixel, plus 8
 * bytes per pixel of (W + 2R) wide rows per horizontal result of a
 * vector-ALU frequency; or 8 bytes per pixel per horizontal result when the
 * vector kernels write dL/df straight), which the plan keeps until
 * destroyed; later calls allocate nothing.
 */
gabor_status gabor_bank_apply_adjoint(gabor_plan plan, const void* d_grad_out, float* d_grad_image,
                                      int64_t grad_row_stride_elems, void* hip_stream);

/*
 * gabor_bank_apply_batched -- gabor_bank_apply over n_images images of the
 * plan's size (Eq. (1) per image), in one launch per frequency when every
 * frequency runs in the wave-specialised fused kernel (else one
 * gabor_bank_apply per image, in order, on the stream).
 *
 *   d_images            device FP32; image b starts at d_images + b *
 *                       image_stride_elems (>= (H - 1) * row_stride_elems + W
 *                       when n_images > 1), rows row_stride_elems apart.
 *   d_out               device complex64 [n_images][O][N][H][W], fully
 *                       overwritten.
 *
 * n_images = 0 does nothing.  Results are bit-identical to gabor_bank_apply
 * on each image.  Nothing is allocated; the plan serves one stream at a
 * time.  Profiling names these launches <kernel>_r<R>_x<n_images>.
 */
gabor_status gabor_bank_apply_batched(gabor_plan plan, const float* d_images, int32_t n_images,
                                      int64_t image_stride_elems, int64_t row_stride_elems, void* d_out,
                                      void* hip_stream);

/*
 * gabor_bank_apply_adjoint_batched -- gabor_bank_apply_adjoint over
 * n_images images (the adjoint of gabor_bank_apply_batched).
 *
 *   d_grad_out          device complex64 [n_images][O][N][H][W].
 *   d_grad_images       device FP32; image b's gradient starts at
 *                       d_grad_images + b * grad_image_stride_elems (>= (H - 1)
 *                       * grad_row_stride_elems + W when n_images > 1), rows
 *                       grad_row_stride_elems apart; fully overwritten.
 *
 * The matrix-core frequencies take every image of a group in one launch, and
 * one launch sums each group; groups hold as many images as fit a 1 GiB
 * workspace (at least one).  The plan's adjoint workspace grows to one
 * group's size at the first call that needs it (after synchronising the
 * stream when an older, smaller one is replaced), so a call that allocates
 * cannot be captured in a HIP graph; once grown, calls allocate nothing.
 * Results are bit-identical to gabor_bank_apply_adjoint on each image.
 * n_images = 0 does nothing.
 */
gabor_status gabor_bank_apply_adjoint_batched(gabor_plan plan, const void* d_grad_out, int32_t n_images,
                                              float* d_grad_images, int64_t grad_image_stride_elems,
                                              int64_t grad_row_stride_elems, void* hip_stream);

/*
 * gabor_bank_apply_adjoint_noalloc -- gabor_bank_apply_adjoint for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, same
 * kernels and bit-identical results, but the workspace comes from a fixed
 * array of 64 MiB that the library holds on each GPU it runs on (until the
 * process ends) instead of memory the plan allocates; the call allocates
 * nothing.  The workspace a plan needs is that of gabor_bank_apply_adjoint
 * (4 bytes per partial-plane pixel: horizontal results x (H + 2R) x (W + 2R)
 * summed over the matrix-core frequencies, one such plane per vector-ALU
 * frequency, R = 0 under the zero boundary, plus the vector kernels'
 * complex rows); a plan that needs more than 64 MiB returns
 * GABOR_ERR_UNSUPPORTED before anything is enqueued.  Every call on
 * one GPU shares that GPU's array, so calls whose executions overlap on one
 * GPU (different streams, or different host threads) race and give wrong
 * results; serialise them.  The first call on a device looks up the array's
 * device address.  Plan profiling (gabor_profile_enable) does not time these
 * launches.
 */
gabor_status gabor_bank_apply_adjoint_noalloc(gabor_plan plan, const void* d_grad_out, float* d_grad_image,
                                              int64_t grad_row_stride_elems, void* hip_stream);

/*
 * Batched bank: many images of uneven sizes through one plan.
 *
 * gabor_batch_create binds n_images device images (d_images[i], heights[i]
 * x widths[i], row stride row_strides[i] >= widths[i]; every image no larger
 * than the plan's height x width) to device outputs d_outs[i], complex64
 * [O][N][heights[i]][widths[i]].  The host arrays are read during the call
 * only; the batch keeps the pointers and owns a device tile table (one tile
 * per image, horizontal result and strip segment).  The plan must outlive
 * the batch; a batch shares its plan's streams and workspace, so the two are
 * not used concurrently.
 *
 * gabor_batch_apply runs Algorithm 1 on every bound image: one launch per
 * operand size of the fused kernel, each over the tiles of all images in
 * decreasing order of cost, plus FP32 two-pass launches over all images for
 * frequencies
 * outside the fused kernel's range (R > 104, or planes of more than 2^27
 * pixels; their intermediate planes live in a batch-owned workspace allocated
 * by gabor_batch_create).  It allocates and copies nothing, so it may be
 * captured in a HIP graph and replayed; the images are read and the outputs
 * written at each replay.
 */
typedef struct gabor_batch_s* gabor_batch;

gabor_status gabor_batch_create(gabor_batch* out, gabor_plan plan, int32_t n_images,
                                const float* const* d_images, const int32_t* heights,
                                const int32_t* widths, const int64_t* row_strides,
                                void* const* d_outs, void* hip_stream);
gabor_status gabor_batch_apply(gabor_batch batch, void* hip_stream);
/* Number of launches and of tiles of a batch (either may be NULL). */
gabor_status gabor_batch_info(gabor_batch batch, int32_t* n_launches, int64_t* n_tiles);
/* Release a batch's tile table.  NULL is accepted (no-op). */
gabor_status gabor_batch_destroy(gabor_batch batch);

/* Release a plan and its device memory.  NULL is accepted (no-op). */
gabor_status gabor_bank_destroy(gabor_plan plan);

/*
 * lsdft_apply -- Gaussian-windowed 2-D localized sliding DFT of one image
 * (Sec. III-A, Eq. (17)-(18)), computed by the separable passes of
 * Eq. (19)-(26) (Algorithm 2):
 *
 *   F_{u,v}(x,y) = sum_{j<Mx} sum_{i<My} f(x - Mx/2 + j, y - My/2 + i)
 *                  w_x(j) w_y(i) exp(-i 2 pi (u j / Mx + v i / My))
 *
 * for every pixel and every bin u = 0..m_x-1, v = 0..m_y-1 (M/2 rounds down).
 * The window is the sampled Gaussian w(j) = exp(-(M/2 - j)^2 / (2 sigma^2))
 * over its M offsets, normalised to unit sum per axis.  The horizontal pass
 * runs for u <= Mx/2 only, since J_{Mx-u} = conj(J_u) for a real input; the
 * vertical pass runs for v <= My/2 over J_u and conj(J_u), which gives both
 * F_{u,v} and F_{Mx-u,v} (Eq. (19)); the bins with v > My/2 are stored as
 * the conjugates F_{Mx-u,My-v} = conj(F_{u,v}) (Eq. (20)).  Every bin plane
 * is written exactly once.  Twiddles are the FP64 values of
 * 2 pi k / M at k = u j mod M, exact at quarter turns.
 *
 *   d_image           device FP32 image, height x width, row stride
 *                     row_stride_elems (>= width).
 *   m_y, m_x          window rows and columns, 1 .. 64 each (larger windows
 *                     return GABOR_ERR_UNSUPPORTED).
 *   sigma             Gaussian window scale in pixels (> 0, finite).
 *   boundary          rule for samples outside the image.
 *   precision         arithmetic of the contractions (as for the bank).
 *   d_out             device complex64 output, layout [m_y][m_x][H][W]
 *                     (plane v * m_x + u), m_y*m_x*H*W*8 bytes, fully
 *                     overwritten.
 *
 * One kernel launch on hip_stream; the call allocates nothing (the window
 * and twiddle tables travel as launch arguments), so it may be captured in
 * a HIP graph.  Images of more than 2^27 pixels, or whose row span reaches
 * 2^30 elements, return GABOR_ERR_UNSUPPORTED.
 */
gabor_status lsdft_apply(const float* d_image, int32_t height, int32_t width,
                         int64_t row_stride_elems, int32_t m_y, int32_t m_x, double sigma,
                         gabor_boundary boundary, gabor_precision precision, void* d_out,
                         void* hip_stream);

/*
 * sdft_box_apply -- box-window 2-D sliding DFT of one image by the
 * circular-shift recursion (Sec. I; Eq. (17) with a uniform window, the
 * conventional SDFT the paper builds on):
 *
 *   F_{u,v}(x,y) = 1/(Mx My) sum_{j<Mx} sum_{i<My} f(x - Mx/2 + j, y - My/2 + i)
 *                  exp(-i 2 pi (u j / Mx + v i / My))
 *
 * for every pixel and bin u = 0..m_x-1, v = 0..m_y-1 (M/2 rounds down).  With
 * C_v(m) the My-point DFT of column m over the window rows, moving the window
 * one column right gives
 *   F(x+1) = exp(i 2 pi u / Mx) (F(x) + (C_v(x - Mx/2 + Mx) - C_v(x - Mx/2)) / Mx).
 * The column DFTs are direct FP64 sums; the recursion state is FP64 and is
 * re-anchored by a direct FP64 window sum every 8 columns, so the only
 * single-precision step is the final rounding to complex64.  Bins with
 * 0 < v < My/2 give their conjugate partners (Mx-u mod Mx, My-v).  Same
 * output as lsdft_apply with an infinite sigma.
 *
 *   d_image           device FP32 image, height x width, row stride
 *                     row_stride_elems (>= width).
 *   m_y, m_x          window rows and columns, 1 .. 64 each.
 *   boundary          rule for samples outside the image.
 *   d_out             device complex64 output, layout [m_y][m_x][H][W]
 *                     (plane v * m_x + u), m_y*m_x*H*W*8 bytes, fully
 *                     overwritten; 8-byte aligned (16-byte aligned with an
 *                     even width selects two-column stores).
 *
 * One kernel launch on hip_stream; nothing is allocated (twiddle tables
 * travel as launch arguments), so it may be captured in a HIP graph.
 * Widths above 8192 (the row of FP64 column DFTs lives in on-chip memory),
 * heights above 65535 or windows above 64 return GABOR_ERR_UNSUPPORTED.
 */
gabor_status sdft_box_apply(const float* d_image, int32_t height, int32_t width,
                            int64_t row_stride_elems, int32_t m_y, int32_t m_x,
                            gabor_boundary boundary, void* d_out, void* hip_stream);

/*
 * lsdft_work -- algorithmic work of one lsdft_apply (host arithmetic only):
 * real multiply-adds counted as M taps per real 1-D pass per pixel over the
 * computed bins, and bytes as one read of the image plus one write of every
 * output.  Either output pointer may be NULL.
 */
gabor_status lsdft_work(int32_t height, int32_t width, int32_t m_y, int32_t m_x,
                        int64_t* real_macs, int64_t* bytes);

/*
 * Autotuning (schedule only; results do not depend on it).  Each frequency
 * on the fused kernel streams strip segments of seg_rows image rows per
 * workgroup (a multiple of 32, or the whole image height; each segment
 * recomputes a lead-in of about 2R rows of the horizontal pass).  gabor_bank_autotune times every candidate
 * segment height per fused frequency on the caller's image and output
 * buffers (d_out is overwritten) and keeps the fastest median of `reps`
 * timed launches; it then times whole applies (median over `reps` bursts of
 * 8 back-to-back applies) with every height scaled by 1, 2 and 4 (the
 * frequencies run concurrently), keeps the fastest, and
 * refines it by coordinate descent on the whole apply (each frequency's
 * height retimed with the others fixed, two passes).  When the plan has
 * two or more distinct small operand sizes on the wave-specialised kernel
 * (quarters Q <= 16, i.e. radii up to 24: 16 + 2R <= 64), it repeats the whole-apply tuning with the
 * grouping option flipped and keeps that option only if the apply gets at
 * least 1 % faster.  It synchronises hip_stream.  get/set copy the chosen heights
 * (n = number of frequencies; 0 for frequencies on the two-pass kernels) so
 * that a caller can cache them; set rejects heights below the image height
 * that are not positive multiples of 32, and replaces every height of at
 * least the image height by the image height rounded up to a multiple of
 * 16 (one segment per strip).  Batches created afterwards use the new
 * heights.
 */
gabor_status gabor_bank_autotune(gabor_plan plan, const float* d_image, int64_t row_stride_elems,
                                 void* d_out, int32_t reps, void* hip_stream);
gabor_status gabor_bank_get_tuning(gabor_plan plan, int32_t* seg_rows, int32_t capacity, int32_t* n);
gabor_status gabor_bank_set_tuning(gabor_plan plan, const int32_t* seg_rows, int32_t n);

/*
 * Grouping option (schedule only; results are bit-identical either way).
 * An apply and a batch launch the fused frequencies once per operand size
 * (quarter Q, contracted length 4Q), the launches running concurrently on
 * the caller's and the plan's streams.  With group_small = 1 every tile of
 * the small quarters (Q <= 16) goes into one launch instead, sorted by
 * decreasing cost, whose workgroups each run their tile's quarter: fewer
 * concurrent launches to fork and join, at the registers and LDS of the
 * largest member.  Default 0; gabor_bank_autotune may set it.  set accepts
 * 0 or 1 (else GABOR_ERR_INVALID_ARG) and drops the plan's cached apply
 * graphs when the option changes; batches created afterwards follow it.
 */
gabor_status gabor_bank_get_grouping(gabor_plan plan, int32_t* group_small);
gabor_status gabor_bank_set_grouping(gabor_plan plan, int32_t group_small);

typedef struct gabor_plan_info {
    int32_t height, width, n_freq, n_orient;
    int32_t max_radius;          /* largest R over the frequencies */
    int32_t n_row_passes;        /* horizontal passes per image (after reuse) */
    int32_t n_col_passes;        /* vertical passes per image */
    int32_t precision;           /* gabor_precision of the plan */
    int64_t workspace_bytes;     /* device memory held by the plan */
    int64_t real_macs;           /* real multiply-adds of one apply, counted as
                                    K taps per real 1-D pass per pixel */
    int64_t row_real_macs;       /* ... of which in horizontal passes */
    int64_t col_real_macs;       /* ... of which in vertical passes */
} gabor_plan_info;

/* Describe a plan (sizes, reuse, algorithmic work). */
gabor_status gabor_bank_plan_info(gabor_plan plan, gabor_plan_info* info);

/*
 * Per-kernel timing (tracing hook; not part of the paper's method).
 *
 * gabor_profile_enable(plan, 1) clears the counters and makes every later
 * apply on the plan bracket each kernel launch with a pair of HIP events
 * recorded on the launch stream; gabor_profile_enable(plan, 0) stops it.
 * gabor_profile_read waits for the recorded events, folds them into
 * per-kernel totals and copies up to `capacity` entries into `stats`
 * (n_stats receives the number of kernels seen).  Host pointers.
 */
typedef struct gabor_kernel_stat {
    char name[32];       /* kernel and radius, e.g. "stream_bf16x3_r48" */
    int64_t launches;    /* launches timed */
    double total_ms;     /* sum of event-measured launch durations */
    int64_t real_macs;   /* algorithmic real multiply-adds of one launch
                            (K taps per real 1-D pass per pixel) */
    int64_t bytes;       /* algorithmic memory bytes of one launch: what its
                            inputs and outputs must move at least once */
} gabor_kernel_stat;

gabor_status gabor_profile_enable(gabor_plan plan, int32_t enable);
gabor_status gabor_profile_read(gabor_plan plan, gabor_kernel_stat* stats, int32_t capacity,
                                int32_t* n_stats);

#ifdef __cplusplus
}
#endif

#endif /* LIBGABOR_H */
