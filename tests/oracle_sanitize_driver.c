/* Test infrastructure: exercises every exported oracle routine on small
 * inputs (both boundary rules, ragged shapes, one-row and one-column images,
 * lines shorter than the extension) and on invalid arguments, for a build
 * of the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py).  Exits non-zero on an unexpected status;
 * the sanitizers abort on a memory or undefined-behaviour error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_radius(double sigma, double radius_sigmas);
int oracle_gaussian_taps(double sigma, int R, double* taps);
int oracle_gabor_bank(const float* img, int H, int W, int64_t stride, int O, const double* omega,
                      const double* sigma, int N, const double* theta, double radius_sigmas, int boundary,
                      double* out, int n_threads);
int oracle_gabor_bank_points(const float* img, int H, int W, int64_t stride, int O, const double* omega,
                             const double* sigma, int N, const double* theta, double radius_sigmas, int boundary,
                             int64_t n_pts, const int32_t* xs, const int32_t* ys, double* out, int n_threads);
int oracle_lsdft(const float* img, int H, int W, int64_t stride, int My, int Mx, double sigma, int boundary,
                 double* out, int n_threads);
int oracle_lsdft_points(const float* img, int H, int W, int64_t stride, int My, int Mx, double sigma,
                        int boundary, int64_t n_pts, const int32_t* xs, const int32_t* ys, double* out,
                        int n_threads);
int oracle_gabor_grad_points(const float* img, int H, int W, int64_t stride, int O, const double* omega,
                             const double* sigma, int N, const double* theta, double radius_sigmas,
                             int64_t n_pts, const int32_t* xs, const int32_t* ys, double* out, int n_threads);
int oracle_iir_coeffs(double sigma, double* a);
int oracle_iir_extension(double sigma);
int oracle_gabor_bank_iir(const float* img, int H, int W, int64_t stride, int O, const double* omega,
                          const double* sigma, int N, const double* theta, int boundary, double* out,
                          int n_threads);

static int failures = 0;

static void expect(int got, int want, const char* what)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, got, want);
        ++failures;
    }
}

static float* image(int H, int W, int64_t stride, unsigned seed)
{
    float* img = malloc(sizeof(float) * (size_t)((H - 1) * stride + W));
    for (int64_t i = 0; i < (H - 1) * stride + W; ++i) {
        seed = seed * 1664525u + 1013904223u;
        img[i] = (float)(seed >> 8) / 16777216.0f;
    }
    return img;
}

static int finite_all(const double* v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    const int shapes[][3] = {{9, 11, 13}, {1, 17, 17}, {14, 1, 3}, {5, 6, 6}, {23, 19, 20}};
    const double omega[2] = {0.9, 2.0}, sigma[2] = {1.5, 3.0}, theta[3] = {0.0, 0.7, 3.14159265358979 - 0.7};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s) {
        const int H = shapes[s][0], W = shapes[s][1];
        const int64_t stride = shapes[s][2];
        float* img = image(H, W, stride, 7u + (unsigned)s);
        for (int boundary = 0; boundary < 2; ++boundary) {
            const int64_t n_out = 2 * 2 * 4 * (int64_t)H * W;
            double* out = malloc(sizeof(double) * (size_t)n_out);
            expect(oracle_gabor_bank(img, H, W, stride, 2, omega, sigma, 4, NULL, 3.0, boundary, out, 1), 0, "bank");
            if (!finite_all(out, n_out)) { fprintf(stderr, "bank: non-finite output\n"); ++failures; }
            free(out);
            double* out3 = malloc(sizeof(double) * (size_t)(2 * 2 * 3 * (int64_t)H * W));
            expect(oracle_gabor_bank(img, H, W, stride, 2, omega, sigma, 3, theta, 2.5, boundary, out3, 1), 0,
                   "bank, given orientations");
            free(out3);
            const int32_t xs[3] = {0, W - 1, W / 2}, ys[3] = {H - 1, 0, H / 2};
            double pts[2 * 3 * 2 * 4];
            expect(oracle_gabor_bank_points(img, H, W, stride, 2, omega, sigma, 4, NULL, 3.0, boundary, 3, xs, ys,
                                            pts, 1), 0, "bank points");
            const int64_t n_ls = 2 * 5 * 4 * (int64_t)H * W;
            double* ls = malloc(sizeof(double) * (size_t)n_ls);
            expect(oracle_lsdft(img, H, W, stride, 5, 4, 1.7, boundary, ls, 1), 0, "lsdft");
            if (!finite_all(ls, n_ls)) { fprintf(stderr, "lsdft: non-finite output\n"); ++failures; }
            free(ls);
            double lpts[2 * 3 * 5 * 4];
            expect(oracle_lsdft_points(img, H, W, stride, 5, 4, 1.7, boundary, 3, xs, ys, lpts, 1), 0, "lsdft points");
            double* iir = malloc(sizeof(double) * (size_t)(2 * 2 * 4 * (int64_t)H * W));
            expect(oracle_gabor_bank_iir(img, H, W, stride, 2, omega, sigma, 4, NULL, boundary, iir, 1), 0, "iir bank");
            free(iir);
            if (boundary == 0) {
                double g[3];
                expect(oracle_gabor_grad_points(img, H, W, stride, 2, omega, sigma, 4, NULL, 3.0, 3, xs, ys, g, 1), 0,
                       "gradient points");
            }
        }
        free(img);
    }
    /* invalid arguments: an error status, never a crash */
    float* img = image(4, 4, 4, 3u);
    double out[2 * 4 * 4 * 4], a[4], taps[7];
    const int32_t bad_x[1] = {4}, ok_y[1] = {0};
    expect(oracle_gabor_bank(NULL, 4, 4, 4, 1, omega, sigma, 4, NULL, 3.0, 0, out, 1), 1, "bank, null image");
    expect(oracle_gabor_bank(img, 4, 4, 3, 1, omega, sigma, 4, NULL, 3.0, 0, out, 1), 1, "bank, short stride");
    expect(oracle_gabor_bank(img, 4, 4, 4, 1, omega, sigma, 4, NULL, 3.0, 5, out, 1), 1, "bank, bad boundary");
    expect(oracle_gabor_bank_points(img, 4, 4, 4, 1, omega, sigma, 4, NULL, 3.0, 0, 1, bad_x, ok_y, out, 1), 1,
           "bank points, pixel outside");
    expect(oracle_lsdft(img, 4, 4, 4, 0, 4, 1.0, 0, out, 1), 1, "lsdft, empty window");
    expect(oracle_gaussian_taps(-1.0, 3, taps), 1, "taps, negative sigma");
    expect(oracle_iir_coeffs(0.0, a), 1, "iir coefficients, zero sigma");
    expect(oracle_gaussian_taps(2.0, 3, taps), 0, "taps");
    expect(oracle_iir_coeffs(4.0, a), 0, "iir coefficients");
    if (oracle_radius(2.0, 3.0) != 6 || oracle_iir_extension(4.0) <= 0) {
        fprintf(stderr, "radius or extension out of range\n");
        ++failures;
    }
    free(img);
    if (failures) {
        fprintf(stderr, "%d unexpected results\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
