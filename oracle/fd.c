/*
 * Frequent Directions with an exact or a randomized shrink, FP64.
 * TEST INFRASTRUCTURE ONLY.
 *
 * Exact shrink: Sec. 2.3 "Frequent Directions" and Algorithm "AeroSketch:
 * Update" (its FD reduce): when the 2*ell-row buffer is full, take its SVD, subtract
 * the ell-th largest squared singular value from every squared singular value
 * (clamped at zero) and keep Sigma' V^T, which has at least ell+1 zero rows.
 *
 * Randomized shrink: the SVD of the full buffer is replaced by Algorithm
 * "Simultaneous Iteration" (Sec. 2.2) applied to the buffer C (2*ell x d):
 *   sketch      K = (C C^T)^q C Omega   (Omega d x k Gaussian),
 *               computed as K <- C C^T QR(K), q times (same span; the
 *               orthonormal basis between steps keeps the small directions
 *               in floating point)
 *   range       Q = QR(K)
 *   projection  M = Q^T C C^T Q
 *   core        M = U Sigma^2 U^T
 *   lift        Z = Q U
 * and the FD shrink is taken with the estimated singular values and the rows
 * z_i^T C / sigma_i as right singular vectors.  The test matrix sits on the
 * d side (Omega d x k) so that the result depends only on C^T C and Omega.
 *
 * Query: the final step of Algorithm "AeroSketch: Query" (eigen-decomposition
 * and a shrink by the ell-th eigenvalue), non-destructive.
 * Merge: Lemma "Decomposability": stacking sketches of disjoint row sets and
 * sketching the stack keeps the errors additive.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

struct o_fd {
    int d, ell, mode, k, q;
    uint64_t seed, stream;
    double* C;      /* 2*ell x d buffer */
    int64_t r;      /* filled rows */
    int64_t shrinks;
};

static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

int o_shrink_exact(double* X, int m, int d, int ld, int ell) {
    double* sigma = dalloc(m);
    int rc = o_jacobi_rows(X, m, d, ld, sigma);
    if (rc) { free(sigma); return rc; }
    double delta = (m >= ell) ? sigma[ell - 1] * sigma[ell - 1] : 0.0;
    for (int i = 0; i < m; ++i) {
        double f = 0.0;
        if (i < ell && sigma[i] > 0.0) {
            double t = sigma[i] * sigma[i] - delta;
            f = (t > 0.0) ? sqrt(t) / sigma[i] : 0.0;
        }
        for (int t = 0; t < d; ++t) X[(int64_t)i * ld + t] *= f;
    }
    free(sigma);
    return 0;
}

/* y = A x with A (m x n, lda) */
static void matvec(const double* A, int m, int n, int lda, const double* x, double* y) {
    for (int i = 0; i < m; ++i) {
        double s = 0;
        for (int j = 0; j < n; ++j) s += A[(int64_t)i * lda + j] * x[j];
        y[i] = s;
    }
}

int o_shrink_rand(double* X, int m, int d, int ld, int ell, int k, int q,
                  uint64_t seed, uint64_t stream, uint64_t b) {
    if (k < 1 || k > m || k > d) return -1;
    double* Om = dalloc((int64_t)d * k);
    double* K = dalloc((int64_t)m * k);
    double* T = dalloc((int64_t)d * k);
    double* Q = dalloc((int64_t)m * k);
    double* V = dalloc((int64_t)d * k);     /* C^T Q */
    double* M = dalloc((int64_t)k * k);
    double* U = dalloc((int64_t)k * k);
    double* w = dalloc(k);
    double* Z = dalloc((int64_t)m * k);
    double* Bn = dalloc((int64_t)m * d);
    int rc = 0;
    /* Omega ~ N(0,1)^{d x k} from the counter stream of shrink b */
    o_omega(seed, stream, b, 0, d, k, Om);
    /* sketch: K = C Omega, then q times K <- C (C^T K) */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0;
            for (int t = 0; t < d; ++t) s += X[(int64_t)i * ld + t] * Om[(int64_t)t * k + j];
            K[(int64_t)i * k + j] = s;
        }
    for (int it = 0; it < q; ++it) {
        /* re-orthonormalise before each power step: the span is that of
         * (C C^T)^q C Omega, without the loss of small directions that
         * repeated products cause in floating point */
        rc = o_qr_householder(K, m, k, Q);
        if (rc) goto out;
        for (int t = 0; t < d; ++t)
            for (int j = 0; j < k; ++j) {
                double s = 0;
                for (int i = 0; i < m; ++i) s += X[(int64_t)i * ld + t] * Q[(int64_t)i * k + j];
                T[(int64_t)t * k + j] = s;
            }
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < k; ++j) {
                double s = 0;
                for (int t = 0; t < d; ++t) s += X[(int64_t)i * ld + t] * T[(int64_t)t * k + j];
                K[(int64_t)i * k + j] = s;
            }
    }
    /* range: Q = QR(K) */
    rc = o_qr_householder(K, m, k, Q);
    if (rc) goto out;
    /* projection: M = Q^T C C^T Q = V^T V with V = C^T Q */
    for (int t = 0; t < d; ++t)
        for (int j = 0; j < k; ++j) {
            double s = 0;
            for (int i = 0; i < m; ++i) s += X[(int64_t)i * ld + t] * Q[(int64_t)i * k + j];
            V[(int64_t)t * k + j] = s;
        }
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
            double s = 0;
            for (int t = 0; t < d; ++t) s += V[(int64_t)t * k + a] * V[(int64_t)t * k + c];
            M[(int64_t)a * k + c] = s;
        }
    /* core: eigen-decomposition of M (sigma_hat^2 = w) */
    rc = o_sym_eig(M, k, w, U);
    if (rc) goto out;
    /* lift: Z = Q U */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0;
            for (int c = 0; c < k; ++c) s += Q[(int64_t)i * k + c] * U[(int64_t)c * k + j];
            Z[(int64_t)i * k + j] = s;
        }
    /* FD shrink with the estimates: row i = sqrt(max(w_i - w_ell, 0)) / sqrt(w_i) * z_i^T C */
    {
        double delta = (k >= ell) ? fmax(w[ell - 1], 0.0) : 0.0;
        int keep = (k < ell) ? k : ell;
        for (int i = 0; i < keep; ++i) {
            double wi = w[i];
            double f = (wi > 0.0 && wi - delta > 0.0) ? sqrt(wi - delta) / sqrt(wi) : 0.0;
            for (int t = 0; t < d; ++t) {
                double s = 0;
                for (int r = 0; r < m; ++r) s += Z[(int64_t)r * k + i] * X[(int64_t)r * ld + t];
                Bn[(int64_t)i * d + t] = f * s;
            }
        }
        for (int i = 0; i < m; ++i)
            for (int t = 0; t < d; ++t)
                X[(int64_t)i * ld + t] = (i < keep) ? Bn[(int64_t)i * d + t] : 0.0;
    }
out:
    free(Om); free(K); free(T); free(Q); free(V); free(M); free(U); free(w); free(Z); free(Bn);
    return rc;
}

o_fd* o_fd_create(int d, int ell, int mode, int k, int q, uint64_t seed, uint64_t stream) {
    if (d < 1 || ell < 1 || (mode != O_EXACT && mode != O_RAND) || q < 0) return NULL;
    if (mode == O_RAND) {
        if (k < 1) k = ell;
        if (k > 2 * ell) k = 2 * ell;
        if (k > d) k = d;
    }
    o_fd* s = (o_fd*)calloc(1, sizeof(o_fd));
    s->d = d; s->ell = ell; s->mode = mode; s->k = k; s->q = q;
    s->seed = seed; s->stream = stream;
    s->C = dalloc((int64_t)2 * ell * d);
    return s;
}

void o_fd_destroy(o_fd* s) {
    if (!s) return;
    free(s->C);
    free(s);
}

static int fd_shrink(o_fd* s) {
    int rc;
    if (s->mode == O_EXACT)
        rc = o_shrink_exact(s->C, 2 * s->ell, s->d, s->d, s->ell);
    else
        rc = o_shrink_rand(s->C, 2 * s->ell, s->d, s->d, s->ell, s->k, s->q, s->seed, s->stream,
                           (uint64_t)s->shrinks);
    if (rc) return rc;
    /* rows ell-1 .. 2*ell-1 are zero now; the fill pointer is ell-1 */
    for (int64_t i = s->ell - 1; i < 2 * s->ell; ++i)
        memset(s->C + i * s->d, 0, sizeof(double) * (size_t)s->d);
    s->r = s->ell - 1;
    s->shrinks += 1;
    return 0;
}

int o_fd_update(o_fd* s, const double* rows, int64_t n, int64_t ld) {
    if (!s || n < 0 || ld < s->d) return -1;
    for (int64_t i = 0; i < n; ++i) {
        memcpy(s->C + s->r * s->d, rows + i * ld, sizeof(double) * (size_t)s->d);
        s->r += 1;
        if (s->r == 2 * s->ell) {
            int rc = fd_shrink(s);
            if (rc) return rc;
        }
    }
    return 0;
}

int o_fd_query(const o_fd* s, double* out) {
    int64_t r = s->r;
    double* X = dalloc(r * s->d);
    memcpy(X, s->C, sizeof(double) * (size_t)(r * s->d));
    if (r >= s->ell) {
        int rc = o_shrink_exact(X, (int)r, s->d, s->d, s->ell);
        if (rc) { free(X); return rc; }
    }
    memset(out, 0, sizeof(double) * (size_t)s->ell * (size_t)s->d);
    int64_t keep = (r < s->ell) ? r : s->ell;
    memcpy(out, X, sizeof(double) * (size_t)(keep * s->d));
    free(X);
    return 0;
}

int64_t o_fd_buffer(const o_fd* s, double* out) {
    memcpy(out, s->C, sizeof(double) * (size_t)(s->r * s->d));
    return s->r;
}
int64_t o_fd_fill(const o_fd* s) { return s->r; }
int64_t o_fd_shrinks(const o_fd* s) { return s->shrinks; }

int o_fd_merge(o_fd* dst, const o_fd* src) {
    if (!dst || !src || dst->d != src->d) return -1;
    double* B = dalloc((int64_t)src->ell * src->d);
    int rc = o_fd_query(src, B);
    if (rc) { free(B); return rc; }
    int64_t nz = (src->r >= src->ell) ? src->ell - 1 : src->r;
    rc = o_fd_update(dst, B, nz, src->d);
    free(B);
    return rc;
}

double o_power_iteration(const double* C, int m, int d, int ld, const double* x0, int steps,
                         double* v) {
    double* x = dalloc(d);
    double* y = dalloc(m);
    double nrm = 0;
    for (int t = 0; t < d; ++t) { x[t] = x0[t]; nrm += x[t] * x[t]; }
    nrm = sqrt(nrm);
    if (nrm > 0) for (int t = 0; t < d; ++t) x[t] /= nrm;
    for (int it = 0; it < steps; ++it) {
        /* x <- C^T C x / |C^T C x| */
        matvec(C, m, d, ld, x, y);
        for (int t = 0; t < d; ++t) {
            double s = 0;
            for (int i = 0; i < m; ++i) s += C[(int64_t)i * ld + t] * y[i];
            x[t] = s;
        }
        nrm = 0;
        for (int t = 0; t < d; ++t) nrm += x[t] * x[t];
        nrm = sqrt(nrm);
        if (nrm == 0) break;
        for (int t = 0; t < d; ++t) x[t] /= nrm;
    }
    matvec(C, m, d, ld, x, y);
    double rq = 0;
    for (int i = 0; i < m; ++i) rq += y[i] * y[i];
    if (v) memcpy(v, x, sizeof(double) * (size_t)d);
    free(x);
    free(y);
    return rq;
}
