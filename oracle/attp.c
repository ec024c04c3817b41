/*
 * ATTP persistent sketch: Algorithm "ATTP Sketch using AeroSketch" (Sec. 4.1,
 * Theorem "ATTP"; proof in the appendix "Proof of Theorem ATTP").
 * TEST INFRASTRUCTURE ONLY -- plain FP64 loops.
 *
 * One AeroSketch (Algorithm "AeroSketch: Initialize / Update / Query") whose
 * dump threshold follows the stream: before the update of row a_i the
 * threshold becomes theta_i = eps ||A_i||_F^2 (eps = 2 / ell), where
 * ||A_i||_F^2 is the running sum of squared row norms.  The snapshots are
 * never expired, so the sketch of any earlier time t is the restore of the
 * snapshots taken at times <= t.
 *
 * Per row (timestamp i = 1, 2, ...): insert into the 2 ell x d buffer; FD
 * reduce when it is full (exact SVD, or the simul_iter shrink with
 * k = min(ell, d) keyed (seed, 64 stream + 1) and the shrink count); then the
 * dump step of Algorithm "AeroSketch: Update" at theta_i (o_aero_dump with
 * level 0: the same random counters as level 0 of the window).
 *
 * Readings where the paper is silent:
 *   - Query(t) is AeroSketch.Query(0, t).  The residual C_t of a past time is
 *     not kept, so for t < T the restored matrix is the snapshot sum alone
 *     (the proof bounds the part left out, ||C_t^T C_t||, by 4 theta_t);
 *     at the current time t = T the residual C_T^T C_T is added as in the
 *     query's first line.
 *   - The query's final step is the shrink by the ell-th eigenvalue of the
 *     restored d x d matrix (ell rows out; the ell-th eigenvalue is 0 when
 *     d < ell).
 *   - The squared norms are summed in row order, each row's in coordinate
 *     order, in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    int xi;
    double* Z; /* d x xi */
    double* W; /* xi x d */
    int64_t s, t;
} asnap;

struct o_attp {
    int d, ell, q, fd_mode;
    uint64_t seed, stream;
    double* C; /* 2 ell x d */
    int64_t r, T, shrinks, ndirs, nsi, last_t;
    double fro2, theta;
    int amp_r, amp_s; /* probability amplification of the dump step (1, 0: off) */
    asnap* sn;
    int64_t nsn, cap;
};

static double* aalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

o_attp* o_attp_create(int d, int ell, int q, uint64_t seed, uint64_t stream, int fd_mode) {
    if (d < 1 || ell < 2 || q < 0 || (fd_mode != O_EXACT && fd_mode != O_RAND)) return NULL;
    o_attp* a = (o_attp*)calloc(1, sizeof(o_attp));
    a->d = d; a->ell = ell; a->q = q; a->fd_mode = fd_mode; a->seed = seed; a->stream = stream;
    a->C = aalloc((int64_t)2 * ell * d);
    a->amp_r = 1;
    a->amp_s = 0;
    return a;
}

int o_attp_set_amplify(o_attp* a, int r, int s) {
    if (!a || r < 1 || r > 16 || s < 0 || s > 16) return -1;
    a->amp_r = r;
    a->amp_s = s;
    return 0;
}

void o_attp_destroy(o_attp* a) {
    if (!a) return;
    for (int64_t e = 0; e < a->nsn; ++e) { free(a->sn[e].Z); free(a->sn[e].W); }
    free(a->sn);
    free(a->C);
    free(a);
}

/* Algorithm "ATTP Sketch": Update(a_i). */
static int attp_row(o_attp* a, const double* row) {
    const int d = a->d, ell = a->ell;
    const int64_t i = a->T + 1;
    a->T = i;
    double nrm = 0.0;
    for (int t = 0; t < d; ++t) nrm += row[t] * row[t];
    a->fro2 += nrm;
    a->theta = (2.0 / ell) * a->fro2;
    /* AeroSketch.Update: insert, FD reduce when full */
    memcpy(a->C + a->r * d, row, sizeof(double) * (size_t)d);
    a->r += 1;
    if (a->r == 2 * ell) {
        int rc;
        if (a->fd_mode == O_EXACT)
            rc = o_shrink_exact(a->C, 2 * ell, d, d, ell);
        else
            rc = o_shrink_rand(a->C, 2 * ell, d, d, ell, ell < d ? ell : d, a->q, a->seed, a->stream * 64u + 1u,
                               (uint64_t)a->shrinks);
        if (rc) return rc;
        for (int64_t e = ell - 1; e < 2 * ell; ++e) memset(a->C + e * d, 0, sizeof(double) * (size_t)d);
        a->r = ell - 1;
        a->shrinks += 1;
    }
    /* the dump step at theta_i */
    double* Z = aalloc((int64_t)d * ell);
    double* W = aalloc((int64_t)ell * d);
    int xi = 0, nsi = 0;
    double pi = 0.0;
    int rc = o_aero_dump_amp(d, ell, a->q, a->seed, a->stream, 0, a->theta, a->C, a->r, i, Z, W, &xi, &nsi, &pi,
                             a->amp_r, a->amp_s, NULL, NULL);
    a->nsi += nsi;
    if (rc == 0 && xi > 0) {
        if (a->nsn == a->cap) {
            a->cap = a->cap ? 2 * a->cap : 16;
            a->sn = (asnap*)realloc(a->sn, sizeof(asnap) * (size_t)a->cap);
        }
        asnap* s = &a->sn[a->nsn++];
        s->xi = xi;
        s->Z = aalloc((int64_t)d * xi);
        s->W = aalloc((int64_t)xi * d);
        for (int t = 0; t < d; ++t)
            for (int c = 0; c < xi; ++c) s->Z[(int64_t)t * xi + c] = Z[(int64_t)t * ell + c];
        memcpy(s->W, W, sizeof(double) * (size_t)xi * d);
        s->s = a->last_t + 1;
        s->t = i;
        a->last_t = i;
        a->ndirs += xi;
    }
    free(Z);
    free(W);
    return rc;
}

int o_attp_update(o_attp* a, const double* rows, int64_t n, int64_t ld) {
    if (!a || n < 0 || ld < a->d) return -1;
    for (int64_t e = 0; e < n; ++e) {
        int rc = attp_row(a, rows + e * ld);
        if (rc) return rc;
    }
    return 0;
}

/* The restored matrix of AeroSketch.Query(0, t): the restore
 * Z W + W^T Z^T - Z (W Z) Z^T of every snapshot with timestamp <= t, plus
 * C_T^T C_T when t is the current time. */
int o_attp_gram_at(const o_attp* a, int64_t t, double* G) {
    if (!a || !G || t < 0 || t > a->T) return -1;
    const int d = a->d;
    memset(G, 0, sizeof(double) * (size_t)d * d);
    if (t == a->T)
        for (int64_t rr = 0; rr < a->r; ++rr)
            for (int x = 0; x < d; ++x)
                for (int y = 0; y < d; ++y) G[(int64_t)x * d + y] += a->C[rr * d + x] * a->C[rr * d + y];
    for (int64_t e = 0; e < a->nsn; ++e) {
        const asnap* s = &a->sn[e];
        if (s->t > t) continue;
        const int xi = s->xi;
        double* WZ = aalloc((int64_t)xi * xi);
        for (int p = 0; p < xi; ++p)
            for (int c = 0; c < xi; ++c) {
                double acc = 0.0;
                for (int u = 0; u < d; ++u) acc += s->W[(int64_t)p * d + u] * s->Z[(int64_t)u * xi + c];
                WZ[(int64_t)p * xi + c] = acc;
            }
        for (int x = 0; x < d; ++x)
            for (int y = 0; y < d; ++y) {
                double acc = 0.0;
                for (int c = 0; c < xi; ++c)
                    acc += s->Z[(int64_t)x * xi + c] * s->W[(int64_t)c * d + y] +
                           s->W[(int64_t)c * d + x] * s->Z[(int64_t)y * xi + c];
                double sub = 0.0;
                for (int p = 0; p < xi; ++p) {
                    double zc = 0.0; /* (W Z Z^T)[p][y] */
                    for (int c = 0; c < xi; ++c) zc += WZ[(int64_t)p * xi + c] * s->Z[(int64_t)y * xi + c];
                    sub += s->Z[(int64_t)x * xi + p] * zc;
                }
                G[(int64_t)x * d + y] += acc - sub;
            }
        free(WZ);
    }
    return 0;
}

/* ell x d sketch of A_t: the restored matrix shrunk by its ell-th eigenvalue
 * (Algorithm "AeroSketch: Query", last two lines). */
int o_attp_query_at(const o_attp* a, int64_t t, double* out) {
    if (!a || !out || t < 0 || t > a->T) return -1;
    const int d = a->d, ell = a->ell;
    double* G = aalloc((int64_t)d * d);
    double* V = aalloc((int64_t)d * d);
    double* lam = aalloc(d);
    int rc = o_attp_gram_at(a, t, G);
    if (rc == 0) rc = o_sym_eig(G, d, lam, V);
    if (rc == 0) {
        memset(out, 0, sizeof(double) * (size_t)ell * d);
        const double lell = (d >= ell) ? lam[ell - 1] : 0.0;
        const int top = d < ell ? d : ell;
        for (int c = 0; c < top; ++c) {
            double f = lam[c] - lell;
            f = f > 0.0 ? sqrt(f) : 0.0;
            for (int u = 0; u < d; ++u) out[(int64_t)c * d + u] = f * V[(int64_t)u * d + c];
        }
    }
    free(G); free(V); free(lam);
    return rc;
}

int o_attp_stats(const o_attp* a, int64_t* st) {
    if (!a || !st) return -1;
    st[0] = a->nsn; st[1] = a->ndirs; st[2] = a->r; st[3] = a->shrinks; st[4] = a->nsi; st[5] = a->T;
    return 0;
}

double o_attp_theta(const o_attp* a) { return a ? a->theta : -1.0; }

int o_attp_snapshot(const o_attp* a, int64_t e, int64_t* meta, double* Z, double* W) {
    if (!a || e < 0 || e >= a->nsn || !meta) return -1;
    const asnap* s = &a->sn[e];
    meta[0] = s->xi; meta[1] = s->s; meta[2] = s->t;
    if (Z) memcpy(Z, s->Z, sizeof(double) * (size_t)a->d * s->xi);
    if (W) memcpy(W, s->W, sizeof(double) * (size_t)s->xi * a->d);
    return 0;
}

int o_attp_buffer(const o_attp* a, double* C) {
    if (!a || !C) return -1;
    memcpy(C, a->C, sizeof(double) * (size_t)a->r * a->d);
    return (int)a->r;
}
