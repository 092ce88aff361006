/*
 * FP64 reference oracle for the 2-D complex Gabor filter bank and the
 * Gaussian-windowed 2-D localized sliding DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow, direct arithmetic used
 * to check the GPU library.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may build, load or call it.  It shares no code,
 * header, table or constant with the GPU path, and the GPU path never calls it.
 *
 * Every function evaluates the paper's defining sums literally, in double
 * precision, with no separable decomposition, no reuse between orientations
 * and no reordering beyond the order the sums are written in:
 *
 *   Gabor bank   -- Eq. (1) with the kernel of Eq. (2), Sec. II:
 *       F(x,y) = sum_{k,l} f(k,l) C(x-k, y-l) G(x-k, y-l),
 *       C(x,y) = exp(i w (x cos t + y sin t)),  G(x,y) = S(x) S(y).
 *     Written over the kernel offset (dx,dy) = (x-k, y-l), |dx|,|dy| <= R.
 *   Localized SDFT -- Eq. (17) with the basis of Eq. (18), Sec. III-A.
 *   Gradient     -- d/df of L = mean |F|^2 over every bank output, from the
 *     chain rule applied to Eq. (1) (Sec. II); zero boundary only.
 *   Recursive variant -- the paper's decomposition with a recursive
 *     Gaussian smoother (an approximation of Eq. (1)), written out step by
 *     step in the paper's order; see oracle_gabor_bank_iir.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *   - Eq. (1) is a convolution: the kernel is evaluated at (x-k, y-l).
 *   - x is the column index, y the row index, both 0-based; the image is
 *     row-major with a row stride.
 *   - S is the sampled Gaussian exp(-t^2 / (2 sigma^2)) normalised to unit sum
 *     over the realised taps |t| <= R, with R = floor(radius_sigmas*sigma+0.5).
 *   - Outside the image f is either 0 (ZERO) or the whole-sample mirror
 *     f(-1) = f(1), folded repeatedly with period 2(n-1) (MIRROR).
 *   - LSDFT: the M-sample window of output x holds m = x - floor(M/2) + j,
 *     j = 0..M-1; the phase origin is x^ = x - floor(M/2) (equal to x - M/2
 *     for the even M the paper uses), so the basis phase is -w0*u*j; the
 *     Gaussian is centred at x and normalised over the M window taps.
 *
 * Parity pins: see tests/test_oracle_pins.py (impulse, constant-image closed
 * form, linearity, conjugate symmetries, Gaussian-blur special case, the
 * paper's own decomposition, FFT of the windowed patch, brute force).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_BAD_ARG 1
#define ORACLE_NO_MEM 2

#define BOUNDARY_ZERO 0
#define BOUNDARY_MIRROR 1

static const double kPi = 3.14159265358979323846264338327950288;

/* Maps an integer coordinate onto the image line of length n.  Returns -1
 * where the ZERO rule makes the sample vanish. */
static int64_t oracle_fold(int64_t i, int64_t n, int boundary)
{
    if (i >= 0 && i < n) return i;
    if (boundary == BOUNDARY_ZERO) return -1;
    if (n == 1) return 0;
    int64_t p = 2 * (n - 1);
    int64_t r = i % p;
    if (r < 0) r += p;
    return r < n ? r : p - r;
}

static double oracle_pixel(const float* img, int64_t stride, int H, int W,
                           int64_t col, int64_t row, int boundary)
{
    int64_t c = oracle_fold(col, W, boundary);
    int64_t r = oracle_fold(row, H, boundary);
    if (c < 0 || r < 0) return 0.0;
    return (double)img[r * stride + c];
}

int oracle_radius(double sigma, double radius_sigmas)
{
    return (int)floor(radius_sigmas * sigma + 0.5);
}

/* Sampled isotropic-Gaussian factor S(t), t = -R..R, unit sum (Sec. II,
 * G(x,y) = S(x) S(y)). */
int oracle_gaussian_taps(double sigma, int R, double* taps)
{
    if (!(sigma > 0.0) || R < 0 || !taps) return ORACLE_BAD_ARG;
    double sum = 0.0;
    for (int t = -R; t <= R; ++t) {
        taps[t + R] = exp(-(double)t * (double)t / (2.0 * sigma * sigma));
        sum += taps[t + R];
    }
    for (int t = 0; t < 2 * R + 1; ++t) taps[t] /= sum;
    return ORACLE_OK;
}

/* Complex kernel of one bank channel, Eq. (1)-(2): entry [dy+R][dx+R] holds
 * S(dx) S(dy) exp(i w (dx cos t + dy sin t)), interleaved (re, im). */
static double* oracle_channel_kernel(double omega, double sigma, double theta, int R)
{
    int K = 2 * R + 1;
    double* s = (double*)malloc(sizeof(double) * K);
    double* k = (double*)malloc(sizeof(double) * 2 * K * K);
    if (!s || !k) { free(s); free(k); return NULL; }
    oracle_gaussian_taps(sigma, R, s);
    double ct = cos(theta), st = sin(theta);
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            double g = s[dx + R] * s[dy + R];
            double ph = omega * ((double)dx * ct + (double)dy * st);
            k[2 * ((dy + R) * K + (dx + R)) + 0] = g * cos(ph);
            k[2 * ((dy + R) * K + (dx + R)) + 1] = g * sin(ph);
        }
    free(s);
    return k;
}

static int oracle_check_bank(const float* img, int H, int W, int64_t stride, int O,
                             const double* omega, const double* sigma, int N,
                             double radius_sigmas, int boundary)
{
    if (!img || H <= 0 || W <= 0 || stride < W || O <= 0 || N <= 0) return ORACLE_BAD_ARG;
    if (!omega || !sigma || !(radius_sigmas >= 0.0)) return ORACLE_BAD_ARG;
    if (boundary != BOUNDARY_ZERO && boundary != BOUNDARY_MIRROR) return ORACLE_BAD_ARG;
    for (int i = 0; i < O; ++i)
        if (!(sigma[i] > 0.0) || !isfinite(omega[i]) || !isfinite(sigma[i])) return ORACLE_BAD_ARG;
    return ORACLE_OK;
}

static double oracle_theta(const double* theta, int k, int N)
{
    return theta ? theta[k] : kPi * (double)k / (double)N;
}

/* One output of Eq. (1) for one channel kernel. */
static void oracle_eq1_point(const float* img, int64_t stride, int H, int W, int boundary,
                             const double* kern, int R, int64_t x, int64_t y,
                             double* re, double* im)
{
    int K = 2 * R + 1;
    double sr = 0.0, si = 0.0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            double f = oracle_pixel(img, stride, H, W, x - dx, y - dy, boundary);
            const double* c = kern + 2 * ((dy + R) * K + (dx + R));
            sr += f * c[0];
            si += f * c[1];
        }
    *re = sr;
    *im = si;
}

/* Whole bank: out is complex128 interleaved, layout [O][N][H][W].
 * theta == NULL selects theta_k = k pi / N. */
int oracle_gabor_bank(const float* img, int H, int W, int64_t stride,
                      int O, const double* omega, const double* sigma,
                      int N, const double* theta, double radius_sigmas, int boundary,
                      double* out, int n_threads)
{
    int rc = oracle_check_bank(img, H, W, stride, O, omega, sigma, N, radius_sigmas, boundary);
    if (rc || !out) return rc ? rc : ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int i = 0; i < O; ++i)
        for (int k = 0; k < N; ++k) {
            int R = oracle_radius(sigma[i], radius_sigmas);
            double* kern = oracle_channel_kernel(omega[i], sigma[i], oracle_theta(theta, k, N), R);
            if (!kern) return ORACLE_NO_MEM;
            double* plane = out + 2 * ((int64_t)(i * N + k) * H * W);
#pragma omp parallel for schedule(dynamic, 1)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    double* o = plane + 2 * ((int64_t)y * W + x);
                    oracle_eq1_point(img, stride, H, W, boundary, kern, R, x, y, &o[0], &o[1]);
                }
            free(kern);
        }
    return ORACLE_OK;
}

/* Bank outputs at n_pts sample pixels (xs[p], ys[p]); out is complex128
 * interleaved, layout [n_pts][O][N]. */
int oracle_gabor_bank_points(const float* img, int H, int W, int64_t stride,
                             int O, const double* omega, const double* sigma,
                             int N, const double* theta, double radius_sigmas, int boundary,
                             int64_t n_pts, const int32_t* xs, const int32_t* ys,
                             double* out, int n_threads)
{
    int rc = oracle_check_bank(img, H, W, stride, O, omega, sigma, N, radius_sigmas, boundary);
    if (rc || !out || n_pts < 0 || (n_pts > 0 && (!xs || !ys))) return rc ? rc : ORACLE_BAD_ARG;
    for (int64_t p = 0; p < n_pts; ++p)
        if (xs[p] < 0 || xs[p] >= W || ys[p] < 0 || ys[p] >= H) return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int i = 0; i < O; ++i)
        for (int k = 0; k < N; ++k) {
            int R = oracle_radius(sigma[i], radius_sigmas);
            double* kern = oracle_channel_kernel(omega[i], sigma[i], oracle_theta(theta, k, N), R);
            if (!kern) return ORACLE_NO_MEM;
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t p = 0; p < n_pts; ++p) {
                double* o = out + 2 * (p * O * N + (int64_t)i * N + k);
                oracle_eq1_point(img, stride, H, W, boundary, kern, R, xs[p], ys[p], &o[0], &o[1]);
            }
            free(kern);
        }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Localized sliding DFT, Eq. (17)-(18), Sec. III-A.
 *   F_{u,v}(x,y) = sum_{n,m} f(m,n) exp(i(w0x u (x^-m) + w0y v (y^-n))) G(x-m, y-n)
 * over the My x Mx window; w0x = 2 pi / Mx, w0y = 2 pi / My.  Output bins
 * u = 0..Mx-1, v = 0..My-1; out is complex128 interleaved [My][Mx][H][W]
 * (full grid) or [n_pts][My][Mx] (points).
 */
static int oracle_window_taps(double sigma, int M, double* s)
{
    /* s[j] = S(x - m) for m = x - floor(M/2) + j, i.e. offset floor(M/2) - j */
    int h = M / 2;
    double sum = 0.0;
    for (int j = 0; j < M; ++j) {
        double t = (double)(h - j);
        s[j] = exp(-t * t / (2.0 * sigma * sigma));
        sum += s[j];
    }
    for (int j = 0; j < M; ++j) s[j] /= sum;
    return ORACLE_OK;
}

static void oracle_eq17_point(const float* img, int64_t stride, int H, int W, int boundary,
                              int My, int Mx, const double* sx, const double* sy,
                              int64_t x, int64_t y, double* o /* [My][Mx][2], stride ostr */,
                              int64_t ostr)
{
    int hx = Mx / 2, hy = My / 2;
    double w0x = 2.0 * kPi / (double)Mx, w0y = 2.0 * kPi / (double)My;
    for (int v = 0; v < My; ++v)
        for (int u = 0; u < Mx; ++u) {
            double sr = 0.0, si = 0.0;
            for (int i = 0; i < My; ++i)
                for (int j = 0; j < Mx; ++j) {
                    int64_t m = x - hx + j, n = y - hy + i;
                    double f = oracle_pixel(img, stride, H, W, m, n, boundary);
                    /* x^ - m = (x - floor(Mx/2)) - m = -j, likewise for y */
                    double ph = w0x * (double)u * (double)(-j) + w0y * (double)v * (double)(-i);
                    double g = sx[j] * sy[i];
                    sr += f * g * cos(ph);
                    si += f * g * sin(ph);
                }
            double* d = o + 2 * ((int64_t)(v * Mx + u) * ostr);
            d[0] = sr;
            d[1] = si;
        }
}

static int oracle_check_lsdft(const float* img, int H, int W, int64_t stride, int My, int Mx,
                              double sigma, int boundary)
{
    if (!img || H <= 0 || W <= 0 || stride < W || My <= 0 || Mx <= 0) return ORACLE_BAD_ARG;
    if (!(sigma > 0.0) || !isfinite(sigma)) return ORACLE_BAD_ARG;
    if (boundary != BOUNDARY_ZERO && boundary != BOUNDARY_MIRROR) return ORACLE_BAD_ARG;
    return ORACLE_OK;
}

int oracle_lsdft(const float* img, int H, int W, int64_t stride, int My, int Mx,
                 double sigma, int boundary, double* out, int n_threads)
{
    int rc = oracle_check_lsdft(img, H, W, stride, My, Mx, sigma, boundary);
    if (rc || !out) return rc ? rc : ORACLE_BAD_ARG;
    double* sx = (double*)malloc(sizeof(double) * Mx);
    double* sy = (double*)malloc(sizeof(double) * My);
    if (!sx || !sy) { free(sx); free(sy); return ORACLE_NO_MEM; }
    oracle_window_taps(sigma, Mx, sx);
    oracle_window_taps(sigma, My, sy);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int64_t plane = (int64_t)H * W;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            oracle_eq17_point(img, stride, H, W, boundary, My, Mx, sx, sy, x, y,
                              out + 2 * ((int64_t)y * W + x), plane);
    free(sx);
    free(sy);
    return ORACLE_OK;
}

int oracle_lsdft_points(const float* img, int H, int W, int64_t stride, int My, int Mx,
                        double sigma, int boundary, int64_t n_pts, const int32_t* xs,
                        const int32_t* ys, double* out, int n_threads)
{
    int rc = oracle_check_lsdft(img, H, W, stride, My, Mx, sigma, boundary);
    if (rc || !out || n_pts < 0 || (n_pts > 0 && (!xs || !ys))) return rc ? rc : ORACLE_BAD_ARG;
    for (int64_t p = 0; p < n_pts; ++p)
        if (xs[p] < 0 || xs[p] >= W || ys[p] < 0 || ys[p] >= H) return ORACLE_BAD_ARG;
    double* sx = (double*)malloc(sizeof(double) * Mx);
    double* sy = (double*)malloc(sizeof(double) * My);
    if (!sx || !sy) { free(sx); free(sy); return ORACLE_NO_MEM; }
    oracle_window_taps(sigma, Mx, sx);
    oracle_window_taps(sigma, My, sy);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_pts; ++p)
        oracle_eq17_point(img, stride, H, W, boundary, My, Mx, sx, sy, xs[p], ys[p],
                          out + 2 * (p * (int64_t)My * Mx), 1);
    free(sx);
    free(sy);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Gradient of L = (1/n) sum_c sum_{x,y} |F_c(x,y)|^2, n = O*N*H*W, with
 * respect to the pixel f(px,py), ZERO boundary.  From Eq. (1),
 * dF_c(x,y)/df(px,py) = K_c(x-px, y-py), so
 *   dL/df(p) = (2/n) sum_c sum_{x,y} Re( conj(F_c(x,y)) K_c(x-px, y-py) ).
 * F_c is evaluated by Eq. (1) at every output within R of p.
 * out[p] is the gradient at (xs[p], ys[p]).
 */
int oracle_gabor_grad_points(const float* img, int H, int W, int64_t stride,
                             int O, const double* omega, const double* sigma,
                             int N, const double* theta, double radius_sigmas,
                             int64_t n_pts, const int32_t* xs, const int32_t* ys,
                             double* out, int n_threads)
{
    int rc = oracle_check_bank(img, H, W, stride, O, omega, sigma, N, radius_sigmas, BOUNDARY_ZERO);
    if (rc || !out || n_pts < 0 || (n_pts > 0 && (!xs || !ys))) return rc ? rc : ORACLE_BAD_ARG;
    for (int64_t p = 0; p < n_pts; ++p)
        if (xs[p] < 0 || xs[p] >= W || ys[p] < 0 || ys[p] >= H) return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    double n_out = (double)O * (double)N * (double)H * (double)W;
    for (int64_t p = 0; p < n_pts; ++p) out[p] = 0.0;
    for (int i = 0; i < O; ++i)
        for (int k = 0; k < N; ++k) {
            int R = oracle_radius(sigma[i], radius_sigmas);
            int K = 2 * R + 1;
            double* kern = oracle_channel_kernel(omega[i], sigma[i], oracle_theta(theta, k, N), R);
            if (!kern) return ORACLE_NO_MEM;
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t p = 0; p < n_pts; ++p) {
                double acc = 0.0;
                for (int64_t y = ys[p] - R; y <= ys[p] + R; ++y)
                    for (int64_t x = xs[p] - R; x <= xs[p] + R; ++x) {
                        if (x < 0 || x >= W || y < 0 || y >= H) continue;
                        double fr, fi;
                        oracle_eq1_point(img, stride, H, W, BOUNDARY_ZERO, kern, R, x, y, &fr, &fi);
                        const double* c = kern + 2 * ((y - ys[p] + R) * K + (x - xs[p] + R));
                        /* Re(conj(F) * K) = Fr*Kr + Fi*Ki */
                        acc += fr * c[0] + fi * c[1];
                    }
                out[p] += 2.0 * acc / n_out;
            }
            free(kern);
        }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Recursive (IIR) variant of the bank, Sec. II-A: the paper modulates the
 * signal (Eq. (5)-(6) horizontally, Eq. (7)-(10) vertically), smooths with a
 * recursive Gaussian filter whose cost per sample does not depend on sigma,
 * and demodulates.  The smoother is the third-order recursive Gaussian of
 * van Vliet, Young and Verbeek (ICPR 1998), which the paper adopts: a causal
 * pass with poles 1/d and its anti-causal mirror, where d are the poles of
 * the sigma = 2 design,
 *   d1, d1* = 1.40098 +- 1.00236 i,   d3 = 1.85132,
 * scaled to d^(1/q) with q chosen so that the variance of the cascade,
 *   sum over the three poles of 2 d / (d - 1)^2,
 * equals sigma^2 (bisection on q).  With (1 - z^-1/d1)(1 - z^-1/d1*)
 * (1 - z^-1/d3) = 1 + a1 z^-1 + a2 z^-2 + a3 z^-3 and a0 = 1 + a1 + a2 + a3
 * (unit DC gain):
 *   forward  w[n] = a0 u[n] - a1 w[n-1] - a2 w[n-2] - a3 w[n-3]
 *   backward v[n] = a0 w[n] - a1 v[n+1] - a2 v[n+2] - a3 v[n+3]
 * Each line is extended by T = ceil(6 sigma) + 3 samples on both sides by
 * the boundary rule (the recursion starts from rest at the far end of the
 * extension); modulation uses the unfolded coordinate.  Per channel:
 *   J(x,y) = exp(i wc x) IIR_x[ f_ext(k,y) exp(-i wc k) ](x)
 *   F(x,y) = exp(i ws y) IIR_y[ J_ext(x,l) exp(-i ws l) ](y)
 * with wc = w cos(theta), ws = w sin(theta); J_ext folds rows of J (the
 * horizontal pass acts on each row alone).  The result approximates Eq. (1)
 * with the untruncated Gaussian; it is judged against the direct sum by its
 * signal-to-error ratio, and this function is the exact (FP64) reference for
 * the GPU implementation of the same recursion.
 */
static double oracle_iir_variance(double q)
{
    const double dr = 1.40098, di = 1.00236, d3 = 1.85132;
    /* d^(1/q) for the complex pole: modulus^(1/q), argument / q */
    double mod = pow(sqrt(dr * dr + di * di), 1.0 / q), arg = atan2(di, dr) / q;
    double cr = mod * cos(arg), ci = mod * sin(arg);
    /* 2 d / (d - 1)^2 for d = cr + i ci, twice its real part for the pair */
    double er = cr - 1.0, ei = ci;
    double den_r = er * er - ei * ei, den_i = 2.0 * er * ei;     /* (d - 1)^2 */
    double den2 = den_r * den_r + den_i * den_i;
    double re = (2.0 * cr * den_r + 2.0 * ci * den_i) / den2;    /* Re 2d/(d-1)^2 */
    double p3 = pow(d3, 1.0 / q);
    return 2.0 * re + 2.0 * p3 / ((p3 - 1.0) * (p3 - 1.0));
}

int oracle_iir_coeffs(double sigma, double* a /* [4]: a0..a3 */)
{
    if (!(sigma >= 0.5) || !isfinite(sigma) || !a) return ORACLE_BAD_ARG;
    double lo = 1e-3, hi = 1e4;
    for (int it = 0; it < 200; ++it) {
        double mid = sqrt(lo * hi);
        if (oracle_iir_variance(mid) < sigma * sigma) lo = mid; else hi = mid;
    }
    double q = sqrt(lo * hi);
    const double dr = 1.40098, di = 1.00236, d3 = 1.85132;
    double mod = pow(sqrt(dr * dr + di * di), 1.0 / q), arg = atan2(di, dr) / q;
    /* 1/d for the pair: (1/mod) e^{-i arg}; real pole 1/d3^(1/q) */
    double pr = cos(arg) / mod, pi_ = -sin(arg) / mod, p3 = 1.0 / pow(d3, 1.0 / q);
    /* (1 - p z^-1)(1 - p* z^-1) = 1 - 2 Re p z^-1 + |p|^2 z^-2, times (1 - p3 z^-1) */
    double c1 = -2.0 * pr, c2 = pr * pr + pi_ * pi_;
    a[1] = c1 - p3;
    a[2] = c2 - c1 * p3;
    a[3] = -c2 * p3;
    a[0] = 1.0 + a[1] + a[2] + a[3];
    return ORACLE_OK;
}

int oracle_iir_extension(double sigma)
{
    return (int)ceil(6.0 * sigma) + 3;
}

/* In place on n complex samples (re, im interleaved): forward then backward
 * recursion, each from rest. */
static void oracle_iir_line(double* z, int64_t n, const double* a)
{
    for (int c = 0; c < 2; ++c) {
        double w1 = 0.0, w2 = 0.0, w3 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double w = a[0] * z[2 * i + c] - a[1] * w1 - a[2] * w2 - a[3] * w3;
            z[2 * i + c] = w;
            w3 = w2; w2 = w1; w1 = w;
        }
        w1 = w2 = w3 = 0.0;
        for (int64_t i = n - 1; i >= 0; --i) {
            double v = a[0] * z[2 * i + c] - a[1] * w1 - a[2] * w2 - a[3] * w3;
            z[2 * i + c] = v;
            w3 = w2; w2 = w1; w1 = v;
        }
    }
}

int oracle_gabor_bank_iir(const float* img, int H, int W, int64_t stride,
                          int O, const double* omega, const double* sigma,
                          int N, const double* theta, int boundary,
                          double* out /* complex128 [O][N][H][W] */, int n_threads)
{
    int rc = oracle_check_bank(img, H, W, stride, O, omega, sigma, N, 0.0, boundary);
    if (rc || !out) return rc ? rc : ORACLE_BAD_ARG;
    for (int i = 0; i < O; ++i)
        if (!(sigma[i] >= 0.5)) return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int64_t plane = (int64_t)H * W;
    double* J = (double*)malloc(sizeof(double) * 2 * plane);
    if (!J) return ORACLE_NO_MEM;
    for (int i = 0; i < O; ++i) {
        double b[4];
        oracle_iir_coeffs(sigma[i], b);
        int64_t T = oracle_iir_extension(sigma[i]);
        for (int k = 0; k < N; ++k) {
            double th = oracle_theta(theta, k, N);
            double wc = omega[i] * cos(th), ws = omega[i] * sin(th);
            int bad = 0;
            /* horizontal: rows */
#pragma omp parallel for schedule(dynamic, 4)
            for (int y = 0; y < H; ++y) {
                int64_t n = W + 2 * T;
                double* z = (double*)malloc(sizeof(double) * 2 * n);
                if (!z) { bad = 1; continue; }
                for (int64_t m = 0; m < n; ++m) {
                    int64_t kx = m - T;
                    double f = oracle_pixel(img, stride, H, W, kx, y, boundary);
                    z[2 * m] = f * cos(wc * (double)kx);
                    z[2 * m + 1] = -f * sin(wc * (double)kx);
                }
                oracle_iir_line(z, n, b);
                for (int x = 0; x < W; ++x) {
                    double re = z[2 * (x + T)], im = z[2 * (x + T) + 1];
                    double c = cos(wc * (double)x), s = sin(wc * (double)x);
                    J[2 * ((int64_t)y * W + x)] = re * c - im * s;
                    J[2 * ((int64_t)y * W + x) + 1] = re * s + im * c;
                }
                free(z);
            }
            if (bad) { free(J); return ORACLE_NO_MEM; }
            /* vertical: columns */
            double* F = out + 2 * ((int64_t)i * N + k) * plane;
#pragma omp parallel for schedule(dynamic, 4)
            for (int x = 0; x < W; ++x) {
                int64_t n = H + 2 * T;
                double* z = (double*)malloc(sizeof(double) * 2 * n);
                if (!z) { bad = 1; continue; }
                for (int64_t m = 0; m < n; ++m) {
                    int64_t ly = m - T;
                    int64_t r = oracle_fold(ly, H, boundary);
                    double jr = 0.0, ji = 0.0;
                    if (r >= 0) { jr = J[2 * (r * W + x)]; ji = J[2 * (r * W + x) + 1]; }
                    double c = cos(ws * (double)ly), s = sin(ws * (double)ly);
                    z[2 * m] = jr * c + ji * s;           /* J exp(-i ws l) */
                    z[2 * m + 1] = ji * c - jr * s;
                }
                oracle_iir_line(z, n, b);
                for (int y = 0; y < H; ++y) {
                    double re = z[2 * (y + T)], im = z[2 * (y + T) + 1];
                    double c = cos(ws * (double)y), s = sin(ws * (double)y);
                    F[2 * ((int64_t)y * W + x)] = re * c - im * s;
                    F[2 * ((int64_t)y * W + x) + 1] = re * s + im * c;
                }
                free(z);
            }
            if (bad) { free(J); return ORACLE_NO_MEM; }
        }
    }
    free(J);
    return ORACLE_OK;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
