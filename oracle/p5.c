/*
 * P5: continuous tracking of a distributed matrix sketch (Algorithm "P5",
 * Sec. 4.3; Theorem "dist", proof in the appendix "Proof of Theorem dist").
 * TEST INFRASTRUCTURE ONLY -- plain FP64 loops.
 *
 * m sites and one coordinator; a message is delivered at once.  Site j keeps
 * a counter F_j, its copy Fhat_j of the last broadcast value, and one
 * AeroSketch (2 ell x d FD buffer and the dump step of Algorithm
 * "AeroSketch: Update") whose threshold is theta_j = (eps / m) Fhat_j,
 * eps = 2 / ell.
 * The coordinator keeps Fhat, the count of counter messages since its last
 * broadcast, and the d x d matrix B.
 *
 * Rows arrive one at a time, each at one site.  For row a at site j (the
 * site's own timestamp i counts its rows):
 *   1. F_j += |a|^2.  If F_j >= (eps / m) Fhat_j, the site sends F_j:
 *      Fhat += F_j, the message is counted, F_j = 0; at the m-th message
 *      since the last broadcast the coordinator broadcasts Fhat and every
 *      site k sets Fhat_k = Fhat (theta_k = (eps / m) Fhat).
 *   2. The site's AeroSketch update at theta_j: insert a, FD reduce when the
 *      buffer is full (exact SVD or the simul_iter shrink), then the dump
 *      step; a snapshot (Z, W = Z^T C'^T C') goes to the coordinator, which
 *      adds its restore Z W + W^T Z^T - Z (W Z) Z^T to B.
 * Query: the eigen-decomposition of B, shrunk by its ell-th eigenvalue
 * (ell rows), as the last two lines of the coordinator's Query.
 *
 * Readings where the listing is silent or at odds with the proof:
 *   - delivery is instantaneous and in order: the broadcast that a row's
 *     counter message triggers reaches every site before that row's sketch
 *     update;
 *   - eps = 2 / ell, as for the sliding window and ATTP;
 *   - the site's dump threshold: the listing sets theta = eps Fhat, but the
 *     proof bounds each site's error by (eps / m) ||A||_F^2 through Theorem
 *     "ATTP", which needs the site's threshold at (eps / m) Fhat -- the
 *     threshold of the site's counter messages; with eps Fhat the total
 *     error reaches m times the bound (0.44 ||A||_F^2 against eps = 0.25 on
 *     a 4-site stream at ell = 8), so theta_j = (eps / m) Fhat_j is taken;
 *   - while theta_j = 0 (before the first broadcast of a positive Fhat) the
 *     dump step would send every direction of a buffer whose earlier rows
 *     are zero residuals: the site sends the row itself (the coordinator
 *     adds a^T a) and leaves its buffer as it is, so that no decision rests
 *     on the rounding noise of a zero residual; a zero row sends nothing;
 *   - site j's AeroSketch is keyed as an ATTP sketch with stream word
 *     4096 stream + j (FD reduce keyed (seed, 64 (4096 stream + j) + 1) and
 *     the reduce count; dump counters of level 0 with the site's timestamp),
 *     so m <= 4096;
 *   - communication is counted in words: 1 per counter message, m per
 *     broadcast, d per row sent as it is, 2 d per dumped direction (a column
 *     of Z and a row of Z^T C'^T C').
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    double* C; /* 2 ell x d */
    int64_t r, T, shrinks, snaps, dirs, raw, nsi;
    double F, Fhat;
} p5site;

struct o_p5 {
    int d, ell, m, q, fd_mode, amp_r, amp_s;
    uint64_t seed, stream;
    p5site* s;
    double Fhat;
    int64_t nmsg, T;
    int64_t fmsgs, bcasts, smsgs, dirs, raws, words;
    double* B; /* d x d */
};

static double* palloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

o_p5* o_p5_create(int d, int ell, int m, int q, uint64_t seed, uint64_t stream, int fd_mode) {
    if (d < 1 || ell < 2 || m < 1 || m > 4096 || q < 0 || (fd_mode != O_EXACT && fd_mode != O_RAND)) return NULL;
    o_p5* p = (o_p5*)calloc(1, sizeof(o_p5));
    p->d = d; p->ell = ell; p->m = m; p->q = q; p->fd_mode = fd_mode;
    p->seed = seed; p->stream = stream;
    p->amp_r = 1;
    p->amp_s = 0;
    p->s = (p5site*)calloc((size_t)m, sizeof(p5site));
    for (int j = 0; j < m; ++j) p->s[j].C = palloc((int64_t)2 * ell * d);
    p->B = palloc((int64_t)d * d);
    return p;
}

int o_p5_set_amplify(o_p5* p, int r, int s) {
    if (!p || r < 1 || r > 16 || s < 0 || s > 16) return -1;
    p->amp_r = r;
    p->amp_s = s;
    return 0;
}

void o_p5_destroy(o_p5* p) {
    if (!p) return;
    for (int j = 0; j < p->m; ++j) free(p->s[j].C);
    free(p->s);
    free(p->B);
    free(p);
}

/* Coordinator, on a snapshot (Z d x xi, W xi x d):
 * B += Z W + W^T Z^T - Z (W Z) Z^T. */
static void coord_restore(o_p5* p, const double* Z, int ldz, const double* W, int xi) {
    const int d = p->d;
    double* WZ = palloc((int64_t)xi * xi);
    for (int a = 0; a < xi; ++a)
        for (int c = 0; c < xi; ++c) {
            double acc = 0.0;
            for (int u = 0; u < d; ++u) acc += W[(int64_t)a * d + u] * Z[(int64_t)u * ldz + c];
            WZ[(int64_t)a * xi + c] = acc;
        }
    for (int x = 0; x < d; ++x)
        for (int y = 0; y < d; ++y) {
            double acc = 0.0;
            for (int c = 0; c < xi; ++c)
                acc += Z[(int64_t)x * ldz + c] * W[(int64_t)c * d + y] + W[(int64_t)c * d + x] * Z[(int64_t)y * ldz + c];
            double sub = 0.0;
            for (int a = 0; a < xi; ++a) {
                double t = 0.0; /* (W Z Z^T)[a][y] */
                for (int c = 0; c < xi; ++c) t += WZ[(int64_t)a * xi + c] * Z[(int64_t)y * ldz + c];
                sub += Z[(int64_t)x * ldz + a] * t;
            }
            p->B[(int64_t)x * d + y] += acc - sub;
        }
    free(WZ);
}

/* Algorithm "P5": Update(a) at site j, then the coordinator's Receive_Update
 * for the messages it sends. */
static int p5_row(o_p5* p, int j, const double* a) {
    const int d = p->d, ell = p->ell, m = p->m;
    const double eps = 2.0 / ell;
    p5site* s = &p->s[j];
    const int64_t i = s->T + 1;
    s->T = i;
    p->T += 1;
    double nrm = 0.0;
    for (int t = 0; t < d; ++t) nrm += a[t] * a[t];
    s->F += nrm;
    if (s->F >= (eps / m) * s->Fhat) {
        p->Fhat += s->F;
        s->F = 0.0;
        p->fmsgs += 1;
        p->words += 1;
        p->nmsg += 1;
        if (p->nmsg >= m) {
            p->nmsg = 0;
            p->bcasts += 1;
            p->words += m;
            for (int k = 0; k < m; ++k) p->s[k].Fhat = p->Fhat;
        }
    }
    const double theta = (eps / m) * s->Fhat;
    if (theta == 0.0) {
        /* the row itself goes to the coordinator: B += a^T a */
        if (nrm > 0.0) {
            for (int x = 0; x < d; ++x)
                for (int y = 0; y < d; ++y) p->B[(int64_t)x * d + y] += a[x] * a[y];
            s->raw += 1;
            p->raws += 1;
            p->words += d;
        }
        return 0;
    }
    const uint64_t sid = p->stream * 4096u + (uint64_t)j;
    /* AeroSketch.Update: insert, FD reduce when full */
    memcpy(s->C + s->r * d, a, sizeof(double) * (size_t)d);
    s->r += 1;
    if (s->r == 2 * ell) {
        int rc;
        if (p->fd_mode == O_EXACT)
            rc = o_shrink_exact(s->C, 2 * ell, d, d, ell);
        else
            rc = o_shrink_rand(s->C, 2 * ell, d, d, ell, ell < d ? ell : d, p->q, p->seed, sid * 64u + 1u,
                               (uint64_t)s->shrinks);
        if (rc) return rc;
        for (int64_t e = ell - 1; e < 2 * ell; ++e) memset(s->C + e * d, 0, sizeof(double) * (size_t)d);
        s->r = ell - 1;
        s->shrinks += 1;
    }
    /* the dump step at theta_j; a snapshot goes to the coordinator */
    double* Z = palloc((int64_t)d * ell);
    double* W = palloc((int64_t)ell * d);
    int xi = 0, nsi = 0;
    double pi = 0.0;
    int rc = o_aero_dump_amp(d, ell, p->q, p->seed, sid, 0, theta, s->C, s->r, i, Z, W, &xi, &nsi, &pi, p->amp_r,
                             p->amp_s, NULL, NULL);
    s->nsi += nsi;
    if (rc == 0 && xi > 0) {
        coord_restore(p, Z, ell, W, xi);
        s->snaps += 1;
        s->dirs += xi;
        p->smsgs += 1;
        p->dirs += xi;
        p->words += 2 * (int64_t)d * xi;
    }
    free(Z);
    free(W);
    return rc;
}

int o_p5_update(o_p5* p, const int32_t* site, const double* rows, int64_t n, int64_t ld) {
    if (!p || n < 0 || ld < p->d || (n > 0 && (!site || !rows))) return -1;
    for (int64_t e = 0; e < n; ++e)
        if (site[e] < 0 || site[e] >= p->m) return -1;
    for (int64_t e = 0; e < n; ++e) {
        int rc = p5_row(p, site[e], rows + e * ld);
        if (rc) return rc;
    }
    return 0;
}

/* The coordinator's B (d x d). */
int o_p5_gram(const o_p5* p, double* G) {
    if (!p || !G) return -1;
    memcpy(G, p->B, sizeof(double) * (size_t)p->d * p->d);
    return 0;
}

/* Coordinator's Query: ell rows sqrt(max(lambda_c - lambda_ell, 0)) v_c^T
 * of B's eigen-decomposition (the ell-th eigenvalue is 0 when d < ell). */
int o_p5_query(const o_p5* p, double* out) {
    if (!p || !out) return -1;
    const int d = p->d, ell = p->ell;
    double* G = palloc((int64_t)d * d);
    double* V = palloc((int64_t)d * d);
    double* lam = palloc(d);
    memcpy(G, p->B, sizeof(double) * (size_t)d * d);
    int rc = o_sym_eig(G, d, lam, V);
    if (rc == 0) {
        memset(out, 0, sizeof(double) * (size_t)ell * d);
        const double lell = (d >= ell) ? lam[ell - 1] : 0.0;
        const int top = d < ell ? d : ell;
        for (int c = 0; c < top; ++c) {
            const double w = lam[c] - lell;
            const double sc = w > 0.0 ? sqrt(w) : 0.0;
            for (int t = 0; t < d; ++t) out[(int64_t)c * d + t] = sc * V[(int64_t)t * d + c];
        }
    }
    free(G); free(V); free(lam);
    return rc;
}

/* [0] counter messages, [1] broadcasts, [2] snapshot messages, [3] dumped
 * directions, [4] rows sent as they are, [5] words sent, [6] FD reduces
 * over all sites, [7] rows seen. */
int o_p5_stats(const o_p5* p, int64_t* st) {
    if (!p || !st) return -1;
    int64_t red = 0;
    for (int j = 0; j < p->m; ++j) red += p->s[j].shrinks;
    st[0] = p->fmsgs; st[1] = p->bcasts; st[2] = p->smsgs; st[3] = p->dirs;
    st[4] = p->raws; st[5] = p->words; st[6] = red; st[7] = p->T;
    return 0;
}

double o_p5_fhat(const o_p5* p) { return p ? p->Fhat : NAN; }

/* Site j: [0] F_j, [1] Fhat_j, [2] theta_j; counters [0] rows, [1] buffer
 * rows, [2] FD reduces, [3] snapshots, [4] directions, [5] rows sent as they
 * are, [6] simul_iter calls.  C (optional): the buffer rows (2 ell x d). */
int o_p5_site(const o_p5* p, int j, double* f3, int64_t* st, double* C) {
    if (!p || j < 0 || j >= p->m) return -1;
    const p5site* s = &p->s[j];
    if (f3) { f3[0] = s->F; f3[1] = s->Fhat; f3[2] = (2.0 / p->ell) / p->m * s->Fhat; }
    if (st) {
        st[0] = s->T; st[1] = s->r; st[2] = s->shrinks; st[3] = s->snaps;
        st[4] = s->dirs; st[5] = s->raw; st[6] = s->nsi;
    }
    if (C) memcpy(C, s->C, sizeof(double) * (size_t)s->r * p->d);
    return 0;
}
