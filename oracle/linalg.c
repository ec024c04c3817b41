/*
 * Dense FP64 building blocks of the oracle: one-sided Jacobi SVD on rows,
 * cyclic Jacobi symmetric eigen-decomposition, Householder QR.
 * TEST INFRASTRUCTURE ONLY -- deliberately plain loops, no blocking.
 *
 * The paper treats SVD, eigen-decomposition and QR as black boxes (Sec. 2.2,
 * the QR and eigen steps of Algorithm "Simultaneous Iteration"; Sec. 2.3 FD;
 * the eigen step of Algorithm "AeroSketch: Query").  These are the textbook algorithms
 * (Hestenes 1958; Jacobi/Rutishauser; Householder), see Golub & Van Loan,
 * "Matrix Computations", Sec. 8.5 (Jacobi) and 5.2 (Householder QR).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define JACOBI_MAX_SWEEPS 60

/* Rotation that makes rows i and j orthogonal: (alpha, beta, gamma) are
 * |x_i|^2, |x_j|^2, <x_i, x_j>.  Returns 0 if the pair is already orthogonal
 * to working precision. */
static int row_rotation(double alpha, double beta, double gamma, double tiny, double* c,
                        double* s) {
    if (gamma == 0.0) return 0;
    /* a row whose squared norm is below tiny is numerically zero */
    if (alpha <= tiny || beta <= tiny) return 0;
    if (fabs(gamma) <= 1e-15 * sqrt(alpha * beta)) return 0;
    double zeta = (beta - alpha) / (2.0 * gamma);
    double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = *c * t;
    return 1;
}

int o_jacobi_rows(double* X, int m, int d, int ld, double* sigma) {
    if (m < 0 || d < 0 || ld < d) return -1;
    double total = 0;
    for (int i = 0; i < m; ++i)
        for (int t = 0; t < d; ++t) total += X[(int64_t)i * ld + t] * X[(int64_t)i * ld + t];
    const double tiny = 1e-30 * total + 1e-300;
    int converged = 0;
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS && !converged; ++sweep) {
        int rotated = 0;
        for (int i = 0; i < m - 1; ++i) {
            for (int j = i + 1; j < m; ++j) {
                double* xi = X + (int64_t)i * ld;
                double* xj = X + (int64_t)j * ld;
                double a = 0, b = 0, g = 0;
                for (int t = 0; t < d; ++t) {
                    a += xi[t] * xi[t];
                    b += xj[t] * xj[t];
                    g += xi[t] * xj[t];
                }
                double c, s;
                if (!row_rotation(a, b, g, tiny, &c, &s)) continue;
                rotated = 1;
                for (int t = 0; t < d; ++t) {
                    double u = xi[t], v = xj[t];
                    xi[t] = c * u - s * v;
                    xj[t] = s * u + c * v;
                }
            }
        }
        if (!rotated) converged = 1;
    }
    if (!converged) return -2;
    /* norms, then a stable insertion sort of rows by norm, descending */
    double* tmp = (double*)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
    for (int i = 0; i < m; ++i) {
        double a = 0;
        for (int t = 0; t < d; ++t) a += X[(int64_t)i * ld + t] * X[(int64_t)i * ld + t];
        sigma[i] = sqrt(a);
    }
    for (int i = 1; i < m; ++i) {
        double key = sigma[i];
        memcpy(tmp, X + (int64_t)i * ld, sizeof(double) * (size_t)d);
        int j = i - 1;
        while (j >= 0 && sigma[j] < key) {
            sigma[j + 1] = sigma[j];
            memcpy(X + (int64_t)(j + 1) * ld, X + (int64_t)j * ld, sizeof(double) * (size_t)d);
            --j;
        }
        sigma[j + 1] = key;
        memcpy(X + (int64_t)(j + 1) * ld, tmp, sizeof(double) * (size_t)d);
    }
    free(tmp);
    return 0;
}

int o_sym_eig(double* A, int n, double* w, double* V) {
    if (n < 0) return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(int64_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    double frob = 0;
    for (int64_t e = 0; e < (int64_t)n * n; ++e) frob += A[e] * A[e];
    frob = sqrt(frob);
    const double floor_abs = 1e-300 + 1e-17 * frob;
    int converged = 0;
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS && !converged; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(int64_t)p * n + q];
                double app = A[(int64_t)p * n + p];
                double aqq = A[(int64_t)q * n + q];
                if (fabs(apq) <= floor_abs) continue;
                if (fabs(apq) <= 1e-15 * sqrt(fabs(app * aqq))) continue;
                rotated = 1;
                /* Golub & Van Loan Alg. 8.5.1 (symmetric Schur): zero A[p][q]. */
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- J^T A J with J = I except J_pp = J_qq = c, J_pq = s, J_qp = -s */
                for (int k = 0; k < n; ++k) {
                    double akp = A[(int64_t)k * n + p], akq = A[(int64_t)k * n + q];
                    A[(int64_t)k * n + p] = c * akp - s * akq;
                    A[(int64_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[(int64_t)p * n + k], aqk = A[(int64_t)q * n + k];
                    A[(int64_t)p * n + k] = c * apk - s * aqk;
                    A[(int64_t)q * n + k] = s * apk + c * aqk;
                }
                A[(int64_t)p * n + q] = 0.0;
                A[(int64_t)q * n + p] = 0.0;
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(int64_t)k * n + p], vkq = V[(int64_t)k * n + q];
                    V[(int64_t)k * n + p] = c * vkp - s * vkq;
                    V[(int64_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
        if (!rotated) converged = 1;
    }
    if (!converged) return -2;
    for (int i = 0; i < n; ++i) w[i] = A[(int64_t)i * n + i];
    /* selection sort, descending, moving eigenvector columns along */
    for (int i = 0; i < n; ++i) {
        int best = i;
        for (int j = i + 1; j < n; ++j)
            if (w[j] > w[best]) best = j;
        if (best != i) {
            double t = w[i]; w[i] = w[best]; w[best] = t;
            for (int k = 0; k < n; ++k) {
                double u = V[(int64_t)k * n + i];
                V[(int64_t)k * n + i] = V[(int64_t)k * n + best];
                V[(int64_t)k * n + best] = u;
            }
        }
    }
    return 0;
}

int o_qr_householder(const double* K, int m, int k, double* Q) {
    if (m < k || k < 0) return -1;
    double* R = (double*)malloc(sizeof(double) * (size_t)m * (size_t)(k > 0 ? k : 1));
    double* vs = (double*)malloc(sizeof(double) * (size_t)m * (size_t)(k > 0 ? k : 1));
    double* beta = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    memcpy(R, K, sizeof(double) * (size_t)m * (size_t)k);
    for (int j = 0; j < k; ++j) {
        /* Householder vector v for column j below the diagonal */
        double* v = vs + (int64_t)j * m;
        double norm = 0;
        for (int i = j; i < m; ++i) norm += R[(int64_t)i * k + j] * R[(int64_t)i * k + j];
        norm = sqrt(norm);
        for (int i = 0; i < m; ++i) v[i] = 0;
        if (norm == 0.0) {
            /* zero column: use e_j so Q stays orthonormal (completion) */
            v[j] = 1.0;
            beta[j] = 0.0;
            continue;
        }
        double x0 = R[(int64_t)j * k + j];
        double alpha = (x0 >= 0) ? -norm : norm;
        v[j] = x0 - alpha;
        for (int i = j + 1; i < m; ++i) v[i] = R[(int64_t)i * k + j];
        double vv = 0;
        for (int i = j; i < m; ++i) vv += v[i] * v[i];
        beta[j] = (vv > 0) ? 2.0 / vv : 0.0;
        /* R <- (I - beta v v^T) R for columns j..k-1 */
        for (int c = j; c < k; ++c) {
            double dot = 0;
            for (int i = j; i < m; ++i) dot += v[i] * R[(int64_t)i * k + c];
            dot *= beta[j];
            for (int i = j; i < m; ++i) R[(int64_t)i * k + c] -= dot * v[i];
        }
    }
    /* Q = H_0 H_1 ... H_{k-1} [I_k; 0], applied right to left */
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < k; ++c) Q[(int64_t)i * k + c] = (i == c) ? 1.0 : 0.0;
    for (int j = k - 1; j >= 0; --j) {
        const double* v = vs + (int64_t)j * m;
        if (beta[j] == 0.0) continue;
        for (int c = 0; c < k; ++c) {
            double dot = 0;
            for (int i = j; i < m; ++i) dot += v[i] * Q[(int64_t)i * k + c];
            dot *= beta[j];
            for (int i = j; i < m; ++i) Q[(int64_t)i * k + c] -= dot * v[i];
        }
    }
    free(R);
    free(vs);
    free(beta);
    return 0;
}
