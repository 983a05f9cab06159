/*
 * Adjoint of the FP64 oracle cascade, written once for an arithmetic type.
 * TEST INFRASTRUCTURE ONLY; included by sosfilt_oracle.c with NAME (the
 * exported function) and REAL (the arithmetic type: double for the oracle
 * adjoint, long double for the extended-precision arbiter) defined.
 * Coefficients are normalised in FP64 as in the forward oracle; inputs and
 * outputs are FP64.  The derivation is in sosfilt_oracle.c's header.
 */
int NAME(const double *x, int64_t n, const double *sos,
         int32_t K, const double *gy, double *gx, double *gsos) {
    if (n < 0 || K < 1) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    /* sig[k] = input of section k (k = 0..K-1); sig[K] = output of the cascade */
    REAL *sig = (REAL *)malloc(nn * (size_t)(K + 1) * sizeof(REAL));
    REAL *lam = (REAL *)malloc(nn * sizeof(REAL));
    REAL *mu = (REAL *)malloc(nn * sizeof(REAL));
    if (!sig || !lam || !mu) { free(sig); free(lam); free(mu); return -3; }
    for (int64_t i = 0; i < n; ++i) sig[i] = x[i];
    double c[64][5];
    if (K > 64) { free(sig); free(lam); free(mu); return -1; }
    for (int32_t k = 0; k < K; ++k) {
        if (norm_row(sos + 6 * k, c[k])) { free(sig); free(lam); free(mu); return -2; }
        const REAL *u = sig + (size_t)k * nn;
        REAL *w = sig + (size_t)(k + 1) * nn;
        REAL x2 = 0, x1 = 0, y2 = 0, y1 = 0;
        for (int64_t i = 0; i < n; ++i) {
            REAL acc = (REAL)c[k][0] * u[i];
            acc = acc + c[k][1] * x1;
            acc = acc + c[k][2] * x2;
            acc = acc - c[k][3] * y1;
            acc = acc - c[k][4] * y2;
            x2 = x1; x1 = u[i]; y2 = y1; y1 = acc;
            w[i] = acc;
        }
    }
    for (int64_t i = 0; i < n; ++i) lam[i] = gy[i];
    for (int32_t k = K - 1; k >= 0; --k) {
        const REAL *u = sig + (size_t)k * nn;
        const REAL *w = sig + (size_t)(k + 1) * nn;
        REAL b0 = c[k][0], b1 = c[k][1], b2 = c[k][2], a1 = c[k][3], a2 = c[k][4];
        /* mu = A^{-T} lambda */
        REAL m1 = 0.0, m2 = 0.0; /* mu[n+1], mu[n+2] */
        for (int64_t i = n - 1; i >= 0; --i) {
            REAL v = lam[i];
            v = v - a1 * m1;
            v = v - a2 * m2;
            mu[i] = v;
            m2 = m1; m1 = v;
        }
        REAL gb[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
        for (int64_t i = 0; i < n; ++i) {
            gb[0] += mu[i] * u[i];
            if (i >= 1) { gb[1] += mu[i] * u[i - 1]; ga[1] -= mu[i] * w[i - 1]; }
            if (i >= 2) { gb[2] += mu[i] * u[i - 2]; ga[2] -= mu[i] * w[i - 2]; }
        }
        /* chain rule through the division by a0 */
        const double *row = sos + 6 * k;
        REAL a0 = row[3];
        double *g = gsos + 6 * k;
        g[0] = (double)(gb[0] / a0); g[1] = (double)(gb[1] / a0); g[2] = (double)(gb[2] / a0);
        g[4] = (double)(ga[1] / a0); g[5] = (double)(ga[2] / a0);
        g[3] = (double)(-(gb[0] * b0 + gb[1] * b1 + gb[2] * b2 + ga[1] * a1 + ga[2] * a2) / a0);
        /* lambda_prev = B^T mu */
        for (int64_t i = 0; i < n; ++i) {
            REAL v = b0 * mu[i];
            if (i + 1 < n) v = v + b1 * mu[i + 1];
            if (i + 2 < n) v = v + b2 * mu[i + 2];
            lam[i] = v;
        }
    }
    for (int64_t i = 0; i < n; ++i) gx[i] = (double)lam[i];
    free(sig); free(lam); free(mu);
    return 0;
}
