/*
 * AeroSketchCOD: approximate matrix multiplication over a sliding window
 * (Algorithm "AeroSketchCOD Framework", Sec. 4.2; Theorem "sw-amm", proof in
 * the appendix "Proof of Theorem sw-amm").  TEST INFRASTRUCTURE ONLY --
 * plain FP64 loops.
 *
 * Two streams of column vectors x_i (d_x) and y_i (d_y) arrive together.
 * One level with dump threshold theta keeps buffers A (2 ell x d_x) and
 * B (2 ell x d_y) whose rows are sketch vectors (the product that matters is
 * M = A^T B, d_x x d_y, approximating the window's X Y^T), and a queue of
 * snapshots (Z, Z^T M', M' H, H, s, t).  Per pair (timestamp i = 1, 2, ...):
 *   1. snapshots with t + N <= i leave the queue;
 *   2. x_i, y_i are appended to A, B; when the buffers hold 2 ell rows the
 *      co-occurring-directions reduce replaces them (below);
 *   3. power iteration on M' = A'^T B' in R^{d_y} (x <- M'^T M' x,
 *      ceil(log2 d_y) + 1 normalised steps, start vector from Philox counter
 *      (coordinate, 0, i, 0x100)) estimates sigma_1(M')^2;
 *   4. if sigma_1 >= theta / 2: for k = 2, 4, ... (capped at
 *      min(ell, d_x, d_y, rows)): Z' = simul_iter(M', k) (left directions,
 *      test matrix in R^{d_x}, counter word 3 = 0x200 + step) and
 *      [H', S] = simul_iter(M'^T, k) (right directions, test matrix in
 *      R^{d_y}, counter word 3 = 0x400 + step); when S_k < theta (or k is
 *      the cap) the k' leading directions with S >= theta are dumped:
 *      snapshot (Z, Z^T M', M' H, H) with Z = Z'[:, :k'], H = H'[:, :k'],
 *      then A <- A' - A' Z Z^T, B <- B' - B' H H^T.
 * Query: M_W = A^T B + sum over the queue of Z (Z^T M') + (M' H) H^T
 * - Z (Z^T M' H) H^T; its SVD U S V^T gives A* = U sqrt(max(S - s_ell, 0))
 * and B* = V sqrt(max(S - s_ell, 0)) (ell columns each).
 *
 * The co-occurring-directions reduce (the COD publication the paper cites
 * for the sketch of a pair of matrices) factors A~^T = Q_x R_x and
 * B~^T = Q_y R_y, takes the SVD U S V^T of R_x R_y^T and keeps
 * A'^T = Q_x U sqrt(max(S - s_ell, 0)), B'^T = Q_y V sqrt(max(S - s_ell, 0)).
 * Since Q_x U S V^T Q_y^T is the SVD of the product A~^T B~, the reduce
 * equals that plain definition: the product's SVD, shrunk by its ell-th
 * singular value, split evenly between the two factors.  The oracle
 * computes it that way (one-sided Jacobi SVD of the product).
 *
 * Readings where the listing is silent or loose:
 *   - rows: A and B hold sketch vectors as rows, so the listing's A'_i B'_i^T
 *     is the d_x x d_y product A'^T B';
 *   - the reduce runs when the buffers reach 2 ell rows and leaves ell - 1
 *     rows (the (ell)-th shrunk value is zero), as for the FD reduce;
 *   - the test sigma_1 >= theta / 2 compares the singular value (the square
 *     root of the power-iteration estimate), and the dump counts singular
 *     values (square roots of simul_iter's estimates) >= theta, taking them
 *     from the second call, on M'^T, as the listing does;
 *   - the doubling dumps at the cap even if every estimate reaches theta;
 *   - power-iteration steps: ceil(log2 d_y) + 1, the rule of the appendix
 *     for the d-dimensional case;
 *   - one level with theta given (the listing's Initialize takes theta);
 *   - Philox key (seed, stream); the simul_iter test matrices and the start
 *     vector use the row timestamp i as counter word 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    int xi;
    double *Z, *ZM, *MH, *H; /* dx x xi, xi x dy, dx x xi, dy x xi */
    int64_t s, t;
} csnap;

struct o_cod {
    int dx, dy, ell, q;
    uint64_t seed, stream;
    int64_t N;
    double theta;
    double *A, *B; /* 2 ell x dx, 2 ell x dy */
    int64_t r, T, reduces, nsi, dumps, dirs, last_t;
    csnap* sn;
    int64_t head, nsn, cap; /* live snapshots sn[head .. nsn) */
};

static double* calloc_d(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

o_cod* o_cod_create(int dx, int dy, int ell, int64_t N, double theta, int q, uint64_t seed, uint64_t stream) {
    if (dx < 1 || dy < 1 || ell < 2 || N < 1 || !(theta > 0.0) || q < 0) return NULL;
    o_cod* c = (o_cod*)calloc(1, sizeof(o_cod));
    c->dx = dx; c->dy = dy; c->ell = ell; c->q = q; c->seed = seed; c->stream = stream;
    c->N = N; c->theta = theta;
    c->A = calloc_d((int64_t)2 * ell * dx);
    c->B = calloc_d((int64_t)2 * ell * dy);
    return c;
}

static void snap_free(csnap* s) { free(s->Z); free(s->ZM); free(s->MH); free(s->H); }

void o_cod_destroy(o_cod* c) {
    if (!c) return;
    for (int64_t e = c->head; e < c->nsn; ++e) snap_free(&c->sn[e]);
    free(c->sn); free(c->A); free(c->B); free(c);
}

/* M = A^T B over r rows (dx x dy). */
static void product(const double* A, const double* B, int64_t r, int dx, int dy, double* M) {
    memset(M, 0, sizeof(double) * (size_t)dx * dy);
    for (int64_t i = 0; i < r; ++i)
        for (int a = 0; a < dx; ++a) {
            const double xa = A[i * dx + a];
            if (xa == 0.0) continue;
            for (int b = 0; b < dy; ++b) M[(int64_t)a * dy + b] += xa * B[i * dy + b];
        }
}

/* Thin SVD of G (m x n) by one-sided Jacobi on the columns of G (m >= n) or
 * of G^T: U (m x p), s (p, descending), V (n x p), p = min(m, n). */
static int svd_jacobi(const double* G, int m, int n, double* U, double* s, double* V) {
    const int tr = m < n;
    const int mm = tr ? n : m, nn = tr ? m : n; /* work on W (mm x nn), mm >= nn */
    double* W = calloc_d((int64_t)mm * nn);
    double* R = calloc_d((int64_t)nn * nn);
    for (int i = 0; i < mm; ++i)
        for (int j = 0; j < nn; ++j) W[(int64_t)i * nn + j] = tr ? G[(int64_t)j * n + i] : G[(int64_t)i * n + j];
    for (int j = 0; j < nn; ++j) R[(int64_t)j * nn + j] = 1.0;
    int converged = 0;
    for (int sweep = 0; sweep < 80 && !converged; ++sweep) {
        converged = 1;
        for (int p = 0; p < nn - 1; ++p)
            for (int q = p + 1; q < nn; ++q) {
                double a = 0, b = 0, g = 0;
                for (int i = 0; i < mm; ++i) {
                    const double wp = W[(int64_t)i * nn + p], wq = W[(int64_t)i * nn + q];
                    a += wp * wp; b += wq * wq; g += wp * wq;
                }
                if (fabs(g) <= 1e-15 * sqrt(a * b) || g == 0.0) continue;
                converged = 0;
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < mm; ++i) {
                    const double wp = W[(int64_t)i * nn + p], wq = W[(int64_t)i * nn + q];
                    W[(int64_t)i * nn + p] = cs * wp - sn * wq;
                    W[(int64_t)i * nn + q] = sn * wp + cs * wq;
                }
                for (int i = 0; i < nn; ++i) {
                    const double rp = R[(int64_t)i * nn + p], rq = R[(int64_t)i * nn + q];
                    R[(int64_t)i * nn + p] = cs * rp - sn * rq;
                    R[(int64_t)i * nn + q] = sn * rp + cs * rq;
                }
            }
    }
    /* column norms, sorted descending */
    double* nrm = calloc_d(nn);
    int* ord = (int*)calloc((size_t)nn, sizeof(int));
    for (int j = 0; j < nn; ++j) {
        double a = 0;
        for (int i = 0; i < mm; ++i) a += W[(int64_t)i * nn + j] * W[(int64_t)i * nn + j];
        nrm[j] = sqrt(a);
        ord[j] = j;
    }
    for (int i = 1; i < nn; ++i) {
        const int v = ord[i];
        int j = i - 1;
        while (j >= 0 && nrm[ord[j]] < nrm[v]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = v;
    }
    /* W = Uw S, G (or G^T) = W R^T: columns of W / s are the left vectors of
     * the worked matrix, columns of R its right vectors */
    for (int c = 0; c < nn; ++c) {
        const int j = ord[c];
        s[c] = nrm[j];
        const double inv = nrm[j] > 0 ? 1.0 / nrm[j] : 0.0;
        double* Lw = tr ? V : U; /* left vectors of the worked matrix */
        double* Rw = tr ? U : V; /* its right vectors */
        for (int i = 0; i < mm; ++i) Lw[(int64_t)i * nn + c] = W[(int64_t)i * nn + j] * inv;
        for (int i = 0; i < nn; ++i) Rw[(int64_t)i * nn + c] = R[(int64_t)i * nn + j];
    }
    free(W); free(R); free(nrm); free(ord);
    return converged ? 0 : -2;
}

/* The co-occurring-directions reduce of buffers A~ (r x dx), B~ (r x dy):
 * the SVD U S V^T of A~^T B~; rows c < ell - 1 become sqrt(S_c - S_ell) U_c^T
 * and sqrt(S_c - S_ell) V_c^T, the rest zero. */
int o_cod_reduce(double* A, double* B, int64_t r, int dx, int dy, int ell) {
    const int p = dx < dy ? dx : dy;
    double* M = calloc_d((int64_t)dx * dy);
    double* U = calloc_d((int64_t)dx * p);
    double* V = calloc_d((int64_t)dy * p);
    double* s = calloc_d(p);
    product(A, B, r, dx, dy, M);
    int rc = svd_jacobi(M, dx, dy, U, s, V);
    if (rc == 0) {
        const double delta = (p >= ell) ? s[ell - 1] : 0.0;
        memset(A, 0, sizeof(double) * (size_t)r * dx);
        memset(B, 0, sizeof(double) * (size_t)r * dy);
        for (int c = 0; c < ell && c < p && c < r; ++c) {
            const double w = s[c] - delta;
            if (!(w > 0.0)) continue;
            const double f = sqrt(w);
            for (int a = 0; a < dx; ++a) A[(int64_t)c * dx + a] = f * U[(int64_t)a * p + c];
            for (int b = 0; b < dy; ++b) B[(int64_t)c * dy + b] = f * V[(int64_t)b * p + c];
        }
    }
    free(M); free(U); free(V); free(s);
    return rc;
}

/* The dump step on the current buffers for the pair with timestamp i. */
static int cod_dump(o_cod* c, int64_t i) {
    const int dx = c->dx, dy = c->dy, ell = c->ell;
    const int64_t r = c->r;
    double* M = calloc_d((int64_t)dx * dy);
    double* Mt = calloc_d((int64_t)dy * dx);
    product(c->A, c->B, r, dx, dy, M);
    for (int a = 0; a < dx; ++a)
        for (int b = 0; b < dy; ++b) Mt[(int64_t)b * dx + a] = M[(int64_t)a * dy + b];
    int rc = 0;
    /* power iteration in R^{dy} on M^T M */
    const int steps = (int)ceil(log2((double)dy)) + 1;
    double* x0 = calloc_d(dy);
    o_omega(c->seed, c->stream, (uint64_t)i, 0x100u, dy, 1, x0);
    const double s1 = sqrt(o_power_iteration(M, dx, dy, dy, x0, steps, NULL));
    free(x0);
    if (s1 >= c->theta / 2.0) {
        int kmax = ell;
        if (kmax > dx) kmax = dx;
        if (kmax > dy) kmax = dy;
        if (kmax > (int)r) kmax = (int)r;
        int nsteps = kmax > 1 ? (int)ceil(log2((double)kmax)) : 1;
        if (nsteps < 1) nsteps = 1;
        for (int s = 1; s <= nsteps && kmax >= 1 && rc == 0; ++s) {
            int k = 1 << s;
            if (k > kmax) k = kmax;
            double* Zp = calloc_d((int64_t)dx * k);
            double* Hp = calloc_d((int64_t)dy * k);
            double* ez = calloc_d(k);
            double* eh = calloc_d(k);
            /* left directions: simul_iter on A = M (C = M^T, dy x dx, test matrix in R^{dx}) */
            rc = o_simul_iter(Mt, dy, dx, k, c->q, c->seed, c->stream, (uint64_t)i, 0x200u + (uint64_t)s, Zp, ez);
            /* right directions and the estimates: simul_iter on M^T (C = M, dx x dy) */
            if (rc == 0)
                rc = o_simul_iter(M, dx, dy, k, c->q, c->seed, c->stream, (uint64_t)i, 0x400u + (uint64_t)s, Hp, eh);
            c->nsi += 2;
            int done = 0;
            if (rc == 0 && (!(sqrt(fmax(eh[k - 1], 0.0)) >= c->theta) || k == kmax)) {
                int xi = 0;
                while (xi < k && sqrt(fmax(eh[xi], 0.0)) >= c->theta) ++xi;
                if (xi > 0) {
                    csnap sn;
                    sn.xi = xi;
                    sn.Z = calloc_d((int64_t)dx * xi);
                    sn.H = calloc_d((int64_t)dy * xi);
                    sn.ZM = calloc_d((int64_t)xi * dy);
                    sn.MH = calloc_d((int64_t)dx * xi);
                    for (int a = 0; a < dx; ++a)
                        for (int e = 0; e < xi; ++e) sn.Z[(int64_t)a * xi + e] = Zp[(int64_t)a * k + e];
                    for (int b = 0; b < dy; ++b)
                        for (int e = 0; e < xi; ++e) sn.H[(int64_t)b * xi + e] = Hp[(int64_t)b * k + e];
                    for (int e = 0; e < xi; ++e)
                        for (int b = 0; b < dy; ++b) {
                            double acc = 0;
                            for (int a = 0; a < dx; ++a) acc += sn.Z[(int64_t)a * xi + e] * M[(int64_t)a * dy + b];
                            sn.ZM[(int64_t)e * dy + b] = acc;
                        }
                    for (int a = 0; a < dx; ++a)
                        for (int e = 0; e < xi; ++e) {
                            double acc = 0;
                            for (int b = 0; b < dy; ++b) acc += M[(int64_t)a * dy + b] * sn.H[(int64_t)b * xi + e];
                            sn.MH[(int64_t)a * xi + e] = acc;
                        }
                    sn.s = c->last_t + 1;
                    sn.t = i;
                    c->last_t = i;
                    if (c->nsn == c->cap) {
                        c->cap = c->cap ? 2 * c->cap : 16;
                        c->sn = (csnap*)realloc(c->sn, sizeof(csnap) * (size_t)c->cap);
                    }
                    c->sn[c->nsn++] = sn;
                    c->dumps += 1;
                    c->dirs += xi;
                    /* A <- A' - A' Z Z^T, B <- B' - B' H H^T */
                    for (int64_t rr = 0; rr < r; ++rr) {
                        double* ar = c->A + rr * dx;
                        double* br = c->B + rr * dy;
                        /* the projections use the pre-update rows: form them first */
                        double* az = calloc_d(xi);
                        double* bh = calloc_d(xi);
                        for (int e = 0; e < xi; ++e) {
                            for (int a = 0; a < dx; ++a) az[e] += ar[a] * sn.Z[(int64_t)a * xi + e];
                            for (int b = 0; b < dy; ++b) bh[e] += br[b] * sn.H[(int64_t)b * xi + e];
                        }
                        for (int e = 0; e < xi; ++e) {
                            for (int a = 0; a < dx; ++a) ar[a] -= az[e] * sn.Z[(int64_t)a * xi + e];
                            for (int b = 0; b < dy; ++b) br[b] -= bh[e] * sn.H[(int64_t)b * xi + e];
                        }
                        free(az); free(bh);
                    }
                }
                done = 1;
            }
            free(Zp); free(Hp); free(ez); free(eh);
            if (done) break;
        }
    }
    free(M); free(Mt);
    return rc;
}

static int cod_pair(o_cod* c, const double* x, const double* y) {
    const int dx = c->dx, dy = c->dy, ell = c->ell;
    const int64_t i = c->T + 1;
    c->T = i;
    while (c->head < c->nsn && c->sn[c->head].t + c->N <= i) snap_free(&c->sn[c->head++]);
    memcpy(c->A + c->r * dx, x, sizeof(double) * (size_t)dx);
    memcpy(c->B + c->r * dy, y, sizeof(double) * (size_t)dy);
    c->r += 1;
    if (c->r == 2 * ell) {
        int rc = o_cod_reduce(c->A, c->B, c->r, dx, dy, ell);
        if (rc) return rc;
        c->r = ell - 1;
        c->reduces += 1;
    }
    return cod_dump(c, i);
}

int o_cod_update(o_cod* c, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n) {
    if (!c || n < 0 || ldx < c->dx || ldy < c->dy || (n > 0 && (!X || !Y))) return -1;
    for (int64_t e = 0; e < n; ++e) {
        int rc = cod_pair(c, X + e * ldx, Y + e * ldy);
        if (rc) return rc;
    }
    return 0;
}

/* The restored product M_W (dx x dy) of the query, before its shrink. */
int o_cod_product(const o_cod* c, double* MW) {
    if (!c || !MW) return -1;
    const int dx = c->dx, dy = c->dy;
    product(c->A, c->B, c->r, dx, dy, MW);
    for (int64_t e = c->head; e < c->nsn; ++e) {
        const csnap* s = &c->sn[e];
        const int xi = s->xi;
        double* ZMH = calloc_d((int64_t)xi * xi); /* Z^T M' H */
        for (int a = 0; a < xi; ++a)
            for (int b = 0; b < xi; ++b) {
                double acc = 0;
                for (int u = 0; u < dx; ++u) acc += s->Z[(int64_t)u * xi + a] * s->MH[(int64_t)u * xi + b];
                ZMH[(int64_t)a * xi + b] = acc;
            }
        for (int a = 0; a < dx; ++a)
            for (int b = 0; b < dy; ++b) {
                double acc = 0;
                for (int e2 = 0; e2 < xi; ++e2)
                    acc += s->Z[(int64_t)a * xi + e2] * s->ZM[(int64_t)e2 * dy + b] +
                           s->MH[(int64_t)a * xi + e2] * s->H[(int64_t)b * xi + e2];
                double sub = 0;
                for (int p = 0; p < xi; ++p) {
                    double t = 0; /* (Z^T M' H H^T)[p][b] */
                    for (int q = 0; q < xi; ++q) t += ZMH[(int64_t)p * xi + q] * s->H[(int64_t)b * xi + q];
                    sub += s->Z[(int64_t)a * xi + p] * t;
                }
                MW[(int64_t)a * dy + b] += acc - sub;
            }
        free(ZMH);
    }
    return 0;
}

/* Query: A* (dx x ell) and B* (dy x ell), columns sqrt(max(S_c - S_ell, 0))
 * times the singular vectors of M_W (S_ell = 0 when min(dx, dy) < ell). */
int o_cod_query(const o_cod* c, double* Aout, double* Bout) {
    if (!c || !Aout || !Bout) return -1;
    const int dx = c->dx, dy = c->dy, ell = c->ell, p = dx < dy ? dx : dy;
    double* M = calloc_d((int64_t)dx * dy);
    double* U = calloc_d((int64_t)dx * p);
    double* V = calloc_d((int64_t)dy * p);
    double* s = calloc_d(p);
    o_cod_product(c, M);
    int rc = svd_jacobi(M, dx, dy, U, s, V);
    if (rc == 0) {
        memset(Aout, 0, sizeof(double) * (size_t)dx * ell);
        memset(Bout, 0, sizeof(double) * (size_t)dy * ell);
        const double delta = (p >= ell) ? s[ell - 1] : 0.0;
        for (int col = 0; col < ell && col < p; ++col) {
            const double w = s[col] - delta;
            const double f = w > 0 ? sqrt(w) : 0.0;
            for (int a = 0; a < dx; ++a) Aout[(int64_t)a * ell + col] = f * U[(int64_t)a * p + col];
            for (int b = 0; b < dy; ++b) Bout[(int64_t)b * ell + col] = f * V[(int64_t)b * p + col];
        }
    }
    free(M); free(U); free(V); free(s);
    return rc;
}

/* [0] snapshots dumped [1] dumped directions [2] buffer rows [3] reduces
 * [4] simul_iter calls [5] snapshots in the queue [6] current time T. */
int o_cod_stats(const o_cod* c, int64_t* st) {
    if (!c || !st) return -1;
    st[0] = c->dumps; st[1] = c->dirs; st[2] = c->r; st[3] = c->reduces;
    st[4] = c->nsi; st[5] = c->nsn - c->head; st[6] = c->T;
    return 0;
}

/* Buffers (r rows each); returns r. */
int o_cod_buffers(const o_cod* c, double* A, double* B) {
    if (!c) return -1;
    if (A) memcpy(A, c->A, sizeof(double) * (size_t)c->r * c->dx);
    if (B) memcpy(B, c->B, sizeof(double) * (size_t)c->r * c->dy);
    return (int)c->r;
}

/* Live snapshot e (oldest first): meta = {xi, s, t}; Z (dx x xi), ZM
 * (xi x dy), MH (dx x xi), H (dy x xi); outputs may be NULL. */
int o_cod_snapshot(const o_cod* c, int64_t e, int64_t* meta, double* Z, double* ZM, double* MH, double* H) {
    if (!c || e < 0 || c->head + e >= c->nsn) return -1;
    const csnap* s = &c->sn[c->head + e];
    if (meta) { meta[0] = s->xi; meta[1] = s->s; meta[2] = s->t; }
    if (Z) memcpy(Z, s->Z, sizeof(double) * (size_t)c->dx * s->xi);
    if (ZM) memcpy(ZM, s->ZM, sizeof(double) * (size_t)s->xi * c->dy);
    if (MH) memcpy(MH, s->MH, sizeof(double) * (size_t)c->dx * s->xi);
    if (H) memcpy(H, s->H, sizeof(double) * (size_t)c->dy * s->xi);
    return 0;
}
