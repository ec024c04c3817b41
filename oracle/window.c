/*
 * ML-AeroSketch: the sliding-window sketch of Algorithm "ML-AeroSketch",
 * built from Algorithm "AeroSketch: Initialize / Update / Query".
 * TEST INFRASTRUCTURE ONLY -- plain FP64 loops.
 *
 * Per level j (theta_j = 2^j * eps * N, eps = 2/ell, Algorithm "ML-AeroSketch"
 * Initialize) and per arriving row a_i (timestamp i = 1, 2, ...):
 *   - pop queue heads while the queue is longer than 8/eps or the head's
 *     timestamp has left the window;
 *   - a row with |a|^2 >= theta is stored raw in the queue;
 *   - otherwise AeroSketch.Update: insert; FD reduce with an exact SVD when
 *     the buffer is full; power iteration on C'^T C' (ceil(log2 d)+1 steps);
 *     if the estimate reaches theta/2, simul_iter with k = 2, 4, ... until the
 *     k-th estimate falls below theta, dump the xi directions whose estimate
 *     reaches theta as a snapshot (Z, Z^T C'^T C') and remove them from C'.
 * Query: restore B = C^T C + sum over in-window snapshots of
 *   Z W + W^T Z^T - Z (W Z) Z^T  (the restore of Algorithm "AeroSketch: Query"),
 * eigen-decompose, shrink by the ell-th eigenvalue, then FD over that sketch
 * stacked with the in-window raw rows.
 *
 * Readings where the paper is silent:
 *   - simul_iter's test matrix is on the d side: K = (C'^T C')^q C'^T (C' Omega)
 *     with Omega (d x k) Gaussian, so the snapshot depends only on C'^T C'.
 *   - if every k up to min(ell, d) keeps its k-th estimate >= theta, the
 *     directions with estimate >= theta are still dumped at k = min(ell, d).
 *   - s of a new entry is the previous entry's t + 1 (0 + 1 for the first).
 *   - a level is valid for a query when no entry with t inside the window was
 *     dropped by the length cap; the smallest valid level is used (the last
 *     level if none is valid).
 *   - the FD over the stacked rows is one exact shrink of the whole stack.
 *   - the FD reduce of Algorithm "AeroSketch: Update" is the exact
 *     SVD shrink or, with fd_mode O_RAND, the simul_iter shrink of the
 *     persistent sketch (k = min(ell, d)), keyed per level.
 *   - random streams: power-iteration start vector of level j at time i uses
 *     counter (coordinate, 0, i, 0x100 + j); simul_iter's Omega at doubling
 *     step s uses counter (row, column/4, i, 0x200 + 32 j + s).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    int kind;        /* 0 dump, 1 raw row */
    int xi;          /* dumped directions (kind 0) */
    double* Z;       /* d x xi (kind 0) */
    double* W;       /* xi x d (kind 0) */
    double* a;       /* d (kind 1) */
    int64_t s, t;
} wentry;

typedef struct {
    double theta;
    double* C;       /* 2*ell x d */
    int64_t r;
    wentry* q;       /* ring buffer */
    int64_t head, len, capq;
    int64_t last_t, dropped_t;
    int64_t ndumps, nraw, ndirs, shrinks, nsi;
} wlevel;

struct o_win {
    int d, ell, L, q, fd_mode;
    int amp_r, amp_s; /* probability amplification of the dump step (1, 0: off) */
    int64_t N, T;
    uint64_t seed, stream;
    wlevel* lv;
};

static double* walloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static void entry_free(wentry* e) {
    free(e->Z); free(e->W); free(e->a);
    memset(e, 0, sizeof(*e));
}

o_win* o_win_create(int d, int ell, int64_t N, double R, int q, uint64_t seed, uint64_t stream) {
    return o_win_create2(d, ell, N, R, q, seed, stream, O_EXACT);
}

o_win* o_win_create2(int d, int ell, int64_t N, double R, int q, uint64_t seed, uint64_t stream,
                     int fd_mode) {
    if (d < 1 || ell < 2 || N < 1 || !(R >= 1.0) || q < 0) return NULL;
    if (fd_mode != O_EXACT && fd_mode != O_RAND) return NULL;
    o_win* w = (o_win*)calloc(1, sizeof(o_win));
    w->d = d; w->ell = ell; w->N = N; w->q = q; w->seed = seed; w->stream = stream;
    w->fd_mode = fd_mode;
    w->amp_r = 1;
    w->amp_s = 0;
    int L = (int)ceil(log2(R));
    if (L < 1) L = 1;
    w->L = L;
    double eps = 2.0 / ell;
    w->lv = (wlevel*)calloc((size_t)L, sizeof(wlevel));
    for (int j = 0; j < L; ++j) {
        wlevel* l = &w->lv[j];
        l->theta = ldexp(1.0, j) * eps * (double)N;
        l->C = walloc((int64_t)2 * ell * d);
        l->capq = 4 * (int64_t)ell + 2;
        l->q = (wentry*)calloc((size_t)l->capq, sizeof(wentry));
    }
    return w;
}

int o_win_set_amplify(o_win* w, int r, int s) {
    if (!w || r < 1 || r > 16 || s < 0 || s > 16) return -1;
    w->amp_r = r;
    w->amp_s = s;
    return 0;
}

void o_win_destroy(o_win* w) {
    if (!w) return;
    for (int j = 0; j < w->L; ++j) {
        wlevel* l = &w->lv[j];
        for (int64_t e = 0; e < l->len; ++e) entry_free(&l->q[(l->head + e) % l->capq]);
        free(l->q);
        free(l->C);
    }
    free(w->lv);
    free(w);
}

static wentry* qat(wlevel* l, int64_t e) { return &l->q[(l->head + e) % l->capq]; }

static void qpop(wlevel* l) {
    entry_free(qat(l, 0));
    l->head = (l->head + 1) % l->capq;
    l->len -= 1;
}

static wentry* qpush(wlevel* l) {
    wentry* e = qat(l, l->len);
    l->len += 1;
    return e;
}

/* Expiry and length cap, Algorithm "ML-AeroSketch" Update, first loop. */
static void expire(o_win* w, wlevel* l, int64_t i) {
    const int64_t cap = 4 * (int64_t)w->ell; /* 8 / eps with eps = 2 / ell */
    while (l->len > 0 && (l->len > cap || qat(l, 0)->t <= i - w->N)) {
        wentry* h = qat(l, 0);
        if (h->t > i - w->N && h->t > l->dropped_t) l->dropped_t = h->t;
        qpop(l);
    }
}

/* Parameters of one level's dump step; amp_r > 1 or amp_s > 0 turns on the
 * probability amplification of Algorithm "Probability Amplification". */
typedef struct {
    int d, ell, q;
    uint64_t seed, stream;
    int amp_r, amp_s;
    double* amp_c; /* optional: the r candidate estimates of the last amplified step */
    int* amp_h;    /* optional: the candidate kept there */
} dump_par;

/* simul_iter on A = C'^T (reading: Omega on the d side), returns Z' (d x k)
 * and the estimates w (descending). */
static int simul_iter_window(const dump_par* w, const double* C, int64_t r, int k, uint64_t ts,
                             uint64_t tag, double* Zp, double* est) {
    const int d = w->d;
    double* Om = walloc((int64_t)d * k);
    double* Y = walloc(r * k);
    double* K = walloc((int64_t)d * k);
    double* Q = walloc((int64_t)d * k);
    double* CQ = walloc(r * k);
    double* M = walloc((int64_t)k * k);
    double* U = walloc((int64_t)k * k);
    int rc;
    o_omega(w->seed, w->stream, ts, tag, d, k, Om);
    /* K = (C^T C)^{q+1} Omega, as q+1 products with C^T C, with the
     * basis re-orthonormalised before every product after the first */
    memcpy(K, Om, sizeof(double) * (size_t)d * k);
    for (int it = 0; it <= w->q; ++it) {
        if (it > 0) {
            rc = o_qr_householder(K, d, k, Q);
            if (rc) goto out;
            memcpy(K, Q, sizeof(double) * (size_t)d * k);
        }
        for (int64_t i = 0; i < r; ++i)
            for (int j = 0; j < k; ++j) {
                double s = 0;
                for (int t = 0; t < d; ++t) s += C[i * d + t] * K[(int64_t)t * k + j];
                Y[i * k + j] = s;
            }
        for (int t = 0; t < d; ++t)
            for (int j = 0; j < k; ++j) {
                double s = 0;
                for (int64_t i = 0; i < r; ++i) s += C[i * d + t] * Y[i * k + j];
                K[(int64_t)t * k + j] = s;
            }
    }
    rc = o_qr_householder(K, d, k, Q);
    if (rc) goto out;
    for (int64_t i = 0; i < r; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0;
            for (int t = 0; t < d; ++t) s += C[i * d + t] * Q[(int64_t)t * k + j];
            CQ[i * k + j] = s;
        }
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
            double s = 0;
            for (int64_t i = 0; i < r; ++i) s += CQ[i * k + a] * CQ[i * k + c];
            M[(int64_t)a * k + c] = s;
        }
    rc = o_sym_eig(M, k, est, U);
    if (rc) goto out;
    for (int t = 0; t < d; ++t)
        for (int j = 0; j < k; ++j) {
            double s = 0;
            for (int c = 0; c < k; ++c) s += Q[(int64_t)t * k + c] * U[(int64_t)c * k + j];
            Zp[(int64_t)t * k + j] = s;
        }
out:
    free(Om); free(Y); free(K); free(Q); free(CQ); free(M); free(U);
    return rc;
}

int o_simul_iter(const double* C, int64_t r, int d, int k, int q, uint64_t seed, uint64_t stream, uint64_t ts,
                 uint64_t tag, double* Z, double* est) {
    if (!C || !Z || !est || r < 1 || d < 1 || k < 1 || k > d || q < 0) return -1;
    dump_par par = {d, k, q, seed, stream, 1, 0, NULL, NULL};
    return simul_iter_window(&par, C, r, k, ts, tag, Z, est);
}

/* Algorithm "Probability Amplification" in place of the simul_iter call of
 * doubling step s (k columns): r independent simul_iters, candidate h with
 * Omega counter (row, column/4, i, 0x200 + 32 j + s + 0x1000 h) (h = 0 is the
 * plain call); for each, xi_h = the count of leading estimates >= theta,
 * Z_h = its first xi_h columns, and the residual R_h = C - C Z_h Z_h^T; then
 * s power iterations on R_h (start vectors from counter (coordinate, 0, i,
 * 0x100000 + 0x10000 g + 0x1000 h + 32 j + s), ceil(log2 d) + 1 steps each),
 * c_h^2 = the largest of their estimates; the candidate with the smallest
 * c_h (the first on ties) becomes [Z', estimates].
 * Readings: the squared estimates are compared (same order as c_h); xi_h
 * counts leading estimates as the dump itself does. */
static int simul_iter_amplified(const dump_par* w, int j, int s, const double* C, int64_t r, int k,
                                double theta, uint64_t i, double* Zp, double* est) {
    const int d = w->d;
    const int steps = (int)ceil(log2((double)d)) + 1;
    double* Zh = walloc((int64_t)d * k);
    double* eh = walloc(k);
    double* R = walloc(r * d);
    double* x0 = walloc(d);
    double best = 0.0;
    int besth = -1, rc = 0;
    for (int h = 0; h < w->amp_r; ++h) {
        rc = simul_iter_window(w, C, r, k, i, 0x200u + 32u * (uint64_t)j + (uint64_t)s + 0x1000u * (uint64_t)h,
                               Zh, eh);
        if (rc) break;
        int xi = 0;
        while (xi < k && eh[xi] >= theta) ++xi;
        /* R_h = C - C Z_h Z_h^T */
        for (int64_t rr = 0; rr < r; ++rr) {
            for (int t = 0; t < d; ++t) R[rr * d + t] = C[rr * d + t];
            for (int c = 0; c < xi; ++c) {
                double cz = 0.0;
                for (int t = 0; t < d; ++t) cz += C[rr * d + t] * Zh[(int64_t)t * k + c];
                for (int t = 0; t < d; ++t) R[rr * d + t] -= cz * Zh[(int64_t)t * k + c];
            }
        }
        double ch = 0.0;
        for (int g = 0; g < w->amp_s; ++g) {
            o_omega(w->seed, w->stream, i,
                    0x100000u + 0x10000u * (uint64_t)g + 0x1000u * (uint64_t)h + 32u * (uint64_t)j + (uint64_t)s, d,
                    1, x0);
            const double e = o_power_iteration(R, (int)r, d, d, x0, steps, NULL);
            if (e > ch) ch = e;
        }
        if (w->amp_c && h < 16) w->amp_c[h] = ch;
        if (besth < 0 || ch < best) {
            best = ch;
            besth = h;
            memcpy(Zp, Zh, sizeof(double) * (size_t)d * k);
            memcpy(est, eh, sizeof(double) * (size_t)k);
        }
    }
    if (w->amp_h) *w->amp_h = besth;
    free(Zh); free(eh); free(R); free(x0);
    return rc;
}

/* The dump step of Algorithm "AeroSketch: Update" on the level buffer C
 * (r x d, after the FD reduce) for the row with timestamp i at level j:
 * power iteration on C^T C with ceil(log2 d) + 1 steps (start vector from
 * Philox counter (coordinate, 0, i, 0x100 + j)); if its estimate reaches
 * theta / 2, simul_iter with k = 2, 4, ... (capped at min(ell, d, r)) until the
 * k-th estimate falls below theta or k reaches the cap; the xi leading
 * directions whose estimate reaches theta form the snapshot Z (d x xi, the
 * first xi of the ell columns of Z) and W = Z^T C^T C (the first xi rows of
 * W), and C becomes C - C Z Z^T.  *pi: the power-iteration estimate; *nsi:
 * simul_iter calls. */
static int aero_dump(const dump_par* w, int j, double theta, double* C, int64_t r, int64_t i, double* Zout,
                     double* Wout, int* xi_out, int* nsi, double* pi) {
    const int d = w->d, ell = w->ell;
    *xi_out = 0;
    *nsi = 0;
    int steps = (int)ceil(log2((double)d)) + 1;
    double* x0 = walloc(d);
    o_omega(w->seed, w->stream, (uint64_t)i, 0x100u + (uint64_t)j, d, 1, x0);
    double s1 = o_power_iteration(C, (int)r, d, d, x0, steps, NULL);
    free(x0);
    *pi = s1;
    if (!(s1 >= theta / 2.0)) return 0;
    int kmax = (ell < d) ? ell : d;
    if (kmax > (int)r) kmax = (int)r;
    if (kmax < 1) return 0;
    int nsteps = (int)ceil(log2((double)kmax));
    if (nsteps < 1) nsteps = 1;
    for (int s = 1; s <= nsteps; ++s) {
        int k = 1 << s;
        if (k > kmax) k = kmax;
        double* Zp = walloc((int64_t)d * k);
        double* est = walloc(k);
        const int amplified = w->amp_r > 1 || w->amp_s > 0;
        int rc = amplified ? simul_iter_amplified(w, j, s, C, r, k, theta, (uint64_t)i, Zp, est)
                           : simul_iter_window(w, C, r, k, (uint64_t)i, 0x200u + 32u * (uint64_t)j + (uint64_t)s, Zp, est);
        *nsi += amplified ? w->amp_r : 1;
        if (rc) { free(Zp); free(est); return rc; }
        if (est[k - 1] < theta || k == kmax) {
            int xi = 0;
            while (xi < k && est[xi] >= theta) ++xi;
            if (xi > 0) {
                for (int t = 0; t < d; ++t)
                    for (int c = 0; c < xi; ++c) Zout[(int64_t)t * ell + c] = Zp[(int64_t)t * k + c];
                /* CZ = C' Z (r x xi); W = (C'Z)^T C' */
                double* CZ = walloc(r * xi);
                for (int64_t rr = 0; rr < r; ++rr)
                    for (int c = 0; c < xi; ++c) {
                        double acc = 0;
                        for (int t = 0; t < d; ++t) acc += C[rr * d + t] * Zout[(int64_t)t * ell + c];
                        CZ[rr * xi + c] = acc;
                    }
                for (int c = 0; c < xi; ++c)
                    for (int t = 0; t < d; ++t) {
                        double acc = 0;
                        for (int64_t rr = 0; rr < r; ++rr) acc += CZ[rr * xi + c] * C[rr * d + t];
                        Wout[(int64_t)c * d + t] = acc;
                    }
                /* C <- C' - C' Z Z^T */
                for (int64_t rr = 0; rr < r; ++rr)
                    for (int t = 0; t < d; ++t) {
                        double acc = 0;
                        for (int c = 0; c < xi; ++c) acc += CZ[rr * xi + c] * Zout[(int64_t)t * ell + c];
                        C[rr * d + t] -= acc;
                    }
                free(CZ);
            }
            *xi_out = xi;
            free(Zp); free(est);
            break;
        }
        free(Zp); free(est);
    }
    return 0;
}

int o_aero_dump(int d, int ell, int q, uint64_t seed, uint64_t stream, int level, double theta, double* C,
                int64_t r, int64_t i, double* Z, double* W, int* xi, int* nsi, double* pi) {
    return o_aero_dump_amp(d, ell, q, seed, stream, level, theta, C, r, i, Z, W, xi, nsi, pi, 1, 0, NULL, NULL);
}

int o_aero_dump_amp(int d, int ell, int q, uint64_t seed, uint64_t stream, int level, double theta, double* C,
                    int64_t r, int64_t i, double* Z, double* W, int* xi, int* nsi, double* pi, int amp_r, int amp_s,
                    double* amp_c, int* amp_h) {
    if (d < 1 || ell < 2 || q < 0 || r < 0 || !C || !Z || !W || !xi || !nsi || !pi) return -1;
    if (amp_r < 1 || amp_r > 16 || amp_s < 0 || amp_s > 16) return -1;
    dump_par par = {d, ell, q, seed, stream, amp_r, amp_s, amp_c, amp_h};
    return aero_dump(&par, level, theta, C, r, i, Z, W, xi, nsi, pi);
}

/* Algorithm "AeroSketch: Update" for one level. */
static int level_update(o_win* w, int j, const double* a, int64_t i) {
    wlevel* l = &w->lv[j];
    const int d = w->d, ell = w->ell;
    memcpy(l->C + l->r * d, a, sizeof(double) * (size_t)d);
    l->r += 1;
    if (l->r == 2 * ell) {
        /* FD reduce: exact SVD, or simul_iter with k = min(ell, d)
         * keyed by (seed, 64 stream + j + 1) and the level's shrink count */
        int rc;
        if (w->fd_mode == O_EXACT)
            rc = o_shrink_exact(l->C, 2 * ell, d, d, ell);
        else
            rc = o_shrink_rand(l->C, 2 * ell, d, d, ell, ell < d ? ell : d, w->q, w->seed,
                               w->stream * 64u + (uint64_t)j + 1u, (uint64_t)l->shrinks);
        if (rc) return rc;
        for (int64_t e = ell - 1; e < 2 * ell; ++e) memset(l->C + e * d, 0, sizeof(double) * (size_t)d);
        l->r = ell - 1;
        l->shrinks += 1;
    }
    double* Z = walloc((int64_t)d * ell);
    double* W = walloc((int64_t)ell * d);
    int xi = 0, nsi = 0;
    double pi = 0.0;
    dump_par par = {d, ell, w->q, w->seed, w->stream, w->amp_r, w->amp_s, NULL, NULL};
    int rc = aero_dump(&par, j, l->theta, l->C, l->r, i, Z, W, &xi, &nsi, &pi);
    l->nsi += nsi;
    if (rc == 0 && xi > 0) {
        wentry* e = qpush(l);
        e->kind = 0;
        e->xi = xi;
        e->Z = walloc((int64_t)d * xi);
        e->W = walloc((int64_t)xi * d);
        for (int t = 0; t < d; ++t)
            for (int c = 0; c < xi; ++c) e->Z[(int64_t)t * xi + c] = Z[(int64_t)t * ell + c];
        memcpy(e->W, W, sizeof(double) * (size_t)xi * d);
        e->s = l->last_t + 1;
        e->t = i;
        l->last_t = i;
        l->ndumps += 1;
        l->ndirs += xi;
    }
    free(Z); free(W);
    return rc;
}

int o_win_update(o_win* w, const double* rows, int64_t n, int64_t ld) {
    if (!w || n < 0 || ld < w->d) return -1;
    const int d = w->d;
    for (int64_t e = 0; e < n; ++e) {
        const double* a = rows + e * ld;
        int64_t i = w->T + 1;
        w->T = i;
        double nrm = 0;
        for (int t = 0; t < d; ++t) nrm += a[t] * a[t];
        for (int j = 0; j < w->L; ++j) {
            wlevel* l = &w->lv[j];
            expire(w, l, i);
            if (nrm >= l->theta) {
                wentry* en = qpush(l);
                en->kind = 1;
                en->a = walloc(d);
                memcpy(en->a, a, sizeof(double) * (size_t)d);
                en->s = l->last_t + 1;
                en->t = i;
                l->last_t = i;
                l->nraw += 1;
            } else {
                int rc = level_update(w, j, a, i);
                if (rc) return rc;
            }
        }
    }
    return 0;
}

int o_win_advance(o_win* w, int64_t t_now) {
    if (!w || t_now < w->T) return -1;
    w->T = t_now;
    for (int j = 0; j < w->L; ++j) {
        wlevel* l = &w->lv[j];
        while (l->len > 0 && qat(l, 0)->t <= t_now - w->N) qpop(l);
    }
    return 0;
}

int o_win_levels(const o_win* w) { return w->L; }

int o_win_stats(const o_win* w, int level, int64_t* st) {
    if (!w || level < 0 || level >= w->L) return -1;
    const wlevel* l = &w->lv[level];
    st[0] = l->ndumps; st[1] = l->nraw; st[2] = l->ndirs; st[3] = l->r; st[4] = l->len; st[5] = l->shrinks;
    return 0;
}

/* B_T of the restore in Algorithm "AeroSketch: Query" for a level, window (T-N, T]. */
static void level_restore(const o_win* w, int j, double* G) {
    const wlevel* l = &w->lv[j];
    const int d = w->d;
    const int64_t lb = w->T - w->N, ub = w->T;
    memset(G, 0, sizeof(double) * (size_t)d * d);
    for (int64_t rr = 0; rr < l->r; ++rr)
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) G[(int64_t)a * d + b] += l->C[rr * d + a] * l->C[rr * d + b];
    for (int64_t e = 0; e < l->len; ++e) {
        const wentry* en = &l->q[(l->head + e) % l->capq];
        if (en->kind != 0 || !(lb < en->t && en->t <= ub)) continue;
        const int xi = en->xi;
        double* WZ = walloc((int64_t)xi * xi);
        for (int a = 0; a < xi; ++a)
            for (int b = 0; b < xi; ++b) {
                double s = 0;
                for (int t = 0; t < d; ++t) s += en->W[(int64_t)a * d + t] * en->Z[(int64_t)t * xi + b];
                WZ[(int64_t)a * xi + b] = s;
            }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double s = 0;
                for (int c = 0; c < xi; ++c)
                    s += en->Z[(int64_t)a * xi + c] * en->W[(int64_t)c * d + b] +
                         en->W[(int64_t)c * d + a] * en->Z[(int64_t)b * xi + c];
                double s2 = 0;
                for (int c = 0; c < xi; ++c) {
                    double zc = 0; /* (W Z Z^T)[c][b] */
                    for (int e2 = 0; e2 < xi; ++e2) zc += WZ[(int64_t)c * xi + e2] * en->Z[(int64_t)b * xi + e2];
                    s2 += en->Z[(int64_t)a * xi + c] * zc;
                }
                G[(int64_t)a * d + b] += s - s2;
            }
        free(WZ);
    }
}

int o_win_level_gram(const o_win* w, int level, double* G) {
    if (!w || level < 0 || level >= w->L) return -1;
    const int d = w->d;
    level_restore(w, level, G);
    const wlevel* l = &w->lv[level];
    for (int64_t e = 0; e < l->len; ++e) {
        const wentry* en = &l->q[(l->head + e) % l->capq];
        if (en->kind != 1 || !(w->T - w->N < en->t && en->t <= w->T)) continue;
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) G[(int64_t)a * d + b] += en->a[a] * en->a[b];
    }
    return 0;
}

int o_win_query(const o_win* w, double* out, int* level_out) {
    const int d = w->d, ell = w->ell;
    int j = w->L - 1;
    for (int c = 0; c < w->L; ++c)
        if (w->lv[c].dropped_t <= w->T - w->N) { j = c; break; }
    if (level_out) *level_out = j;
    const wlevel* l = &w->lv[j];
    double* G = walloc((int64_t)d * d);
    double* V = walloc((int64_t)d * d);
    double* lam = walloc(d);
    level_restore(w, j, G);
    int rc = o_sym_eig(G, d, lam, V);
    if (rc) { free(G); free(V); free(lam); return rc; }
    double lell = (d >= ell) ? lam[ell - 1] : 0.0;
    int64_t nraw = 0;
    for (int64_t e = 0; e < l->len; ++e) {
        const wentry* en = &l->q[(l->head + e) % l->capq];
        if (en->kind == 1 && w->T - w->N < en->t && en->t <= w->T) ++nraw;
    }
    int64_t m = ell + nraw;
    double* X = walloc(m * d);
    int top = (d < ell) ? d : ell;
    for (int i = 0; i < top; ++i) {
        double f = lam[i] - lell;
        f = (f > 0) ? sqrt(f) : 0.0;
        for (int t = 0; t < d; ++t) X[(int64_t)i * d + t] = f * V[(int64_t)t * d + i];
    }
    int64_t row = ell;
    for (int64_t e = 0; e < l->len; ++e) {
        const wentry* en = &l->q[(l->head + e) % l->capq];
        if (en->kind == 1 && w->T - w->N < en->t && en->t <= w->T) {
            memcpy(X + row * d, en->a, sizeof(double) * (size_t)d);
            ++row;
        }
    }
    if (m >= ell) rc = o_shrink_exact(X, (int)m, d, d, ell);
    memcpy(out, X, sizeof(double) * (size_t)ell * d);
    free(G); free(V); free(lam); free(X);
    return rc;
}

int o_win_counters(const o_win* w, int level, int64_t* st) {
    if (!w || level < 0 || level >= w->L) return -1;
    const wlevel* l = &w->lv[level];
    st[0] = l->ndumps; st[1] = l->nraw; st[2] = l->ndirs; st[3] = l->r; st[4] = l->len; st[5] = l->shrinks;
    st[6] = l->nsi; st[7] = l->dropped_t;
    return 0;
}

int o_win_entry(const o_win* w, int level, int64_t e, int64_t* meta, double* Z, double* W, double* a) {
    if (!w || level < 0 || level >= w->L) return -1;
    const wlevel* l = &w->lv[level];
    if (e < 0 || e >= l->len) return -1;
    const wentry* en = &l->q[(l->head + e) % l->capq];
    meta[0] = en->kind; meta[1] = en->xi; meta[2] = en->s; meta[3] = en->t;
    if (en->kind == 0) {
        if (Z) memcpy(Z, en->Z, sizeof(double) * (size_t)w->d * en->xi);
        if (W) memcpy(W, en->W, sizeof(double) * (size_t)en->xi * w->d);
    } else if (a) {
        memcpy(a, en->a, sizeof(double) * (size_t)w->d);
    }
    return 0;
}

int o_win_buffer(const o_win* w, int level, double* C) {
    if (!w || level < 0 || level >= w->L) return -1;
    const wlevel* l = &w->lv[level];
    memcpy(C, l->C, sizeof(double) * (size_t)l->r * w->d);
    return (int)l->r;
}
