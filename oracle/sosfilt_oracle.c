/*
 * FP64 CPU oracle for cascaded second-order-section (biquad) filtering.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP path.
 *
 * What it computes is the plain definition of the cascade (Section II):
 *   y = F_K o ... o F_1 (x),
 *   F_k:  y_k[n] = b0 x_k[n] + b1 x_k[n-1] + b2 x_k[n-2]
 *                  - a1 y_k[n-1] - a2 y_k[n-2],
 * with x_1 = x, x_k = y_{k-1}, y = y_K (eq. complex_second_order).  A row
 * with a0 != 1 is first divided by a0 (the SOS convention in which the
 * denominator is [a0, a1, a2]).  The recurrence is run sample by sample in
 * direct form I, which is forward substitution of the banded Toeplitz system
 * A y = B x + B_- x_-1 - A_- y_-1 (Section III, eq.
 * recursive_equation_block_form).  Every multiply and add is a separate
 * rounding step: build with -ffp-contract=off and without fast-math.
 *
 * The adjoint (reverse-mode derivative of L = sum_n g[n] y[n]) follows from
 * the same matrix form: with A and B the section's lower-triangular banded
 * Toeplitz matrices, y = A^{-1} B u gives dL/du = B^T A^{-T} g.  Per section:
 *   mu = A^{-T} lambda   (anti-causal: mu[n] = lambda[n] - a1 mu[n+1] - a2 mu[n+2])
 *   dL/db_i =  sum_n mu[n] u[n-i],   dL/da_i = -sum_n mu[n] y[n-i]
 *   lambda_prev = B^T mu (lambda_prev[n] = b0 mu[n] + b1 mu[n+1] + b2 mu[n+2])
 * and the a0 column follows by the chain rule through the normalisation.
 *
 * State layout (when given): per section four values
 *   [x_k[-2], x_k[-1], y_k[-2], y_k[-1]]
 * i.e. the initial (zi) or final (zf) values of the delay lines of DF1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Normalised coefficients of one section: b0 b1 b2 a1 a2 (a0 divided out). */
static int norm_row(const double *row, double out[5]) {
    double a0 = row[3];
    if (a0 == 0.0) return -1;
    out[0] = row[0] / a0;
    out[1] = row[1] / a0;
    out[2] = row[2] / a0;
    out[3] = row[4] / a0;
    out[4] = row[5] / a0;
    return 0;
}

/* Forward cascade in FP64.  x and y may alias (in-place filtering). */
int oracle_sosfilt_f64(const double *x, int64_t n, const double *sos, int32_t K,
                       const double *zi, double *y, double *zf) {
    if (n < 0 || K < 1) return -1;
    if (y != x && n > 0) memmove(y, x, (size_t)n * sizeof(double));
    for (int32_t k = 0; k < K; ++k) {
        double c[5];
        if (norm_row(sos + 6 * k, c)) return -2;
        double x2 = 0.0, x1 = 0.0, y2 = 0.0, y1 = 0.0;
        if (zi) { x2 = zi[4 * k]; x1 = zi[4 * k + 1]; y2 = zi[4 * k + 2]; y1 = zi[4 * k + 3]; }
        for (int64_t i = 0; i < n; ++i) {
            double xi = y[i];
            double acc = c[0] * xi;
            acc = acc + c[1] * x1;
            acc = acc + c[2] * x2;
            acc = acc - c[3] * y1;
            acc = acc - c[4] * y2;
            x2 = x1; x1 = xi;
            y2 = y1; y1 = acc;
            y[i] = acc;
        }
        if (zf) { zf[4 * k] = x2; zf[4 * k + 1] = x1; zf[4 * k + 2] = y2; zf[4 * k + 3] = y1; }
    }
    return 0;
}

/* Same definition with FP32 inputs promoted to double and FP64 output. */
int oracle_sosfilt_f32in(const float *x, int64_t n, const double *sos, int32_t K,
                         double *y) {
    if (n < 0) return -1;
    for (int64_t i = 0; i < n; ++i) y[i] = (double)x[i];
    return oracle_sosfilt_f64(y, n, sos, K, NULL, y, NULL);
}

/* Same definition evaluated in x87 extended precision (long double), used to
 * measure the FP64 oracle's own rounding error. */
int oracle_sosfilt_ld(const double *x, int64_t n, const double *sos, int32_t K,
                      double *y) {
    if (n < 0 || K < 1) return -1;
    long double *w = (long double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(long double));
    if (!w) return -3;
    for (int64_t i = 0; i < n; ++i) w[i] = (long double)x[i];
    for (int32_t k = 0; k < K; ++k) {
        const double *row = sos + 6 * k;
        long double a0 = row[3];
        if (a0 == 0.0L) { free(w); return -2; }
        long double b0 = row[0] / a0, b1 = row[1] / a0, b2 = row[2] / a0;
        long double a1 = row[4] / a0, a2 = row[5] / a0;
        long double x2 = 0, x1 = 0, y2 = 0, y1 = 0;
        for (int64_t i = 0; i < n; ++i) {
            long double xi = w[i];
            long double acc = b0 * xi + b1 * x1 + b2 * x2 - a1 * y1 - a2 * y2;
            x2 = x1; x1 = xi; y2 = y1; y1 = acc;
            w[i] = acc;
        }
    }
    for (int64_t i = 0; i < n; ++i) y[i] = (double)w[i];
    free(w);
    return 0;
}

/* Plain sequential cascade evaluated entirely in FP32: the accuracy that a
 * straightforward single-precision implementation reaches on a given draw
 * (coefficients rounded to float once, after normalisation). */
int oracle_sosfilt_f32arith(const float *x, int64_t n, const double *sos, int32_t K,
                            float *y) {
    if (n < 0 || K < 1) return -1;
    if (y != x && n > 0) memmove(y, x, (size_t)n * sizeof(float));
    for (int32_t k = 0; k < K; ++k) {
        double c[5];
        if (norm_row(sos + 6 * k, c)) return -2;
        float b0 = (float)c[0], b1 = (float)c[1], b2 = (float)c[2];
        float a1 = (float)c[3], a2 = (float)c[4];
        float x2 = 0.f, x1 = 0.f, y2 = 0.f, y1 = 0.f;
        for (int64_t i = 0; i < n; ++i) {
            float xi = y[i];
            float acc = b0 * xi;
            acc = acc + b1 * x1;
            acc = acc + b2 * x2;
            acc = acc - a1 * y1;
            acc = acc - a2 * y2;
            x2 = x1; x1 = xi; y2 = y1; y1 = acc;
            y[i] = acc;
        }
    }
    return 0;
}

/* Adjoint of the zero-initial-state cascade for L = sum_n gy[n] y[n].
 * Outputs gx[n] = dL/dx[n] and gsos[K][6] = dL/d(b0 b1 b2 a0 a1 a2) of the
 * rows as given (before normalisation). */
#define NAME oracle_sosfilt_backward_f64
#define REAL double
#include "backward_impl.h"
#undef NAME
#undef REAL

/* The same adjoint in x86 extended precision (long double), rounded to FP64
 * at the end: the arbiter where two FP64 results differ by more than their
 * own rounding. */
#define NAME oracle_sosfilt_backward_ld
#define REAL long double
#include "backward_impl.h"
#undef NAME
#undef REAL
