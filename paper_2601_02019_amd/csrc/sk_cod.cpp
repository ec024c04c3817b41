// sk_cod.cpp -- approximate matrix multiplication over a sliding window:
// Algorithm "AeroSketchCOD Framework" (Sec. 4.2) on the GPU, behind the same
// C ABI.
//
// One level with dump threshold theta.  The buffers A (2 ell x d_x) and
// B (2 ell x d_y) are FP64 rows; everything the method decides depends only
// on their product M = A^T B, which is never formed: every product with M or
// M^T is two skinny products with A and B.
//
//   - The co-occurring-directions reduce (the product's SVD shrunk by its
//     ell-th singular value, split evenly between the factors) works in the
//     2 ell-dimensional row space: G_x = A A^T = W_x L_x W_x^T and
//     G_y = B B^T = W_y L_y W_y^T (tridiagonal eigen-solver), K = R_x R_y^T
//     with R_x = L_x^{1/2} W_x^T (the R of a QR of A^T), the SVD of K from
//     the eigen-decomposition K^T K = V S^2 V^T, and the new rows
//     A' = diag(sqrt(s^)/s) V^T K^T L_x^{-1/2} W_x^T A and
//     B' = diag(sqrt(s^)) V^T L_y^{-1/2} W_y^T B, s^ = max(s - s_ell, 0);
//     eigenvalues of a Gram (here and in the query) at or below 1e-13 of the
//     largest are taken as zero: their rounding, about n eps of the largest,
//     decides them (singular values below 3e-7 of the largest).
//   - The power iteration on M^T M runs in the row space too (k_cod_pi).
//   - simul_iter on M and on M^T with the test matrices of the oracle's
//     counters; CholeskyQR for the orthonormalisations.
//   - Snapshots (Z^T, Z^T M, (M H)^T, H^T as rows) in a growing ring; the
//     query restores them with the block mask of the window engine and
//     shrinks the d_x x d_y product through the eigen-decomposition of
//     M M^T (or M^T M, the smaller side).
#include <algorithm>
#include <cmath>
#include <deque>

#include "sk_internal.h"
#include "sk_window.h"

namespace {

struct CodEntry {
    int xi;
    int64_t s, t, slot;
};

const double kDropTol = 1e-13;

}  // namespace

struct CodState {
    int dx = 0, dy = 0, ell = 0, q = 1, n2 = 0, kmax = 0, pn = 0;
    int64_t N = 0, T = 0, ldx = 0, ldy = 0, r = 0, last_t = 0;
    double theta = 0.0;
    uint64_t seed = 0, stream = 0;
    int64_t reduces = 0, dumps = 0, dirs = 0, nsi = 0;
    int par = 0;
    double *A[2] = {nullptr, nullptr}, *B[2] = {nullptr, nullptr};
    // reduce scratch (n2 x n2)
    double *Gx = nullptr, *Gy = nullptr, *Wx = nullptr, *Wy = nullptr, *Sx = nullptr, *Sy = nullptr;
    double *Px = nullptr, *Py = nullptr, *K = nullptr, *KK = nullptr, *V = nullptr, *T1 = nullptr, *T2 = nullptr;
    double *lx = nullptr, *ly = nullptr, *lk = nullptr, *e1 = nullptr, *e2 = nullptr;
    // simul_iter scratch
    double *Om = nullptr, *Yd = nullptr, *Tr = nullptr, *Z = nullptr, *H = nullptr;
    double *Wk = nullptr, *Xk = nullptr, *Mk = nullptr, *Uk = nullptr, *lam = nullptr, *w1 = nullptr, *w2 = nullptr;
    // power iteration: the kept Grams A A^T and B B^T (n2 x n2, complete for
    // the first g_rows rows of buffer pair g_par; g_rows < 0 after a dump),
    // u = B x0 with |x0|^2 in ub[n2], the pass descriptors (device, pinned)
    double *Gkx = nullptr, *Gky = nullptr, *ua = nullptr, *ub = nullptr, *pi_out = nullptr;
    double* rs[4] = {nullptr, nullptr, nullptr, nullptr};  // row-space simul_iter iterates (n2 x kmax)
    double* s_last = nullptr;                             // the rs buffer holding the last call's S
    GramPiDesc* gdd = nullptr;
    GramPiDesc* gdh = nullptr;
    int64_t g_rows = -1;
    int g_par = -1;
    double* h_small = nullptr;  // pinned: estimates / power-iteration result
    hipEvent_t done = nullptr;  // polled by the per-pair waits
    int32_t* info = nullptr;
    // snapshot ring: directions as rows
    double *Zs = nullptr, *ZMs = nullptr, *MHs = nullptr, *Hs = nullptr;
    int64_t cap = 0, tail = 0;
    std::deque<CodEntry> q_;
    // query scratch
    double *Mw = nullptr, *Gq = nullptr, *Uq = nullptr, *lq = nullptr, *eq1 = nullptr, *eq2 = nullptr;
    double *Aq = nullptr, *Bq = nullptr, *Tq = nullptr, *S = nullptr, *T3 = nullptr;
    int32_t* ent = nullptr;
    int chunk = 1024;
    double* gpart = nullptr;
    int64_t gpart_cap = 0;
};

#define C_TRY(expr)                                                                      \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess) return h->device_fail(std::string("cod: ") + #expr + ": " + \
                                                    hipGetErrorString(_e));              \
    } while (0)

// Waits for the stream by polling an event recorded on it (the per-pair
// decisions wait on short GPU stages, where a polled wait returns sooner).
static hipError_t wait_stream(sketch_t h) {
    hipError_t e = hipEventRecord(h->cod->done, h->stream);
    while (e == hipSuccess) {
        e = hipEventQuery(h->cod->done);
        if (e == hipErrorNotReady) e = hipSuccess;
        else break;
    }
    return e;
}

static GemmDesc cg(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C, int ldc, int M,
                   int N, int K, double alpha = 1.0, double beta = 0.0) {
    GemmDesc g{};
    g.A = A;
    g.B = B;
    g.C = C;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = lda;
    g.ldb = ldb;
    g.ldc = ldc;
    g.ta = ta;
    g.tb = tb;
    g.alpha = alpha;
    g.beta = beta;
    return g;
}

// One FP64 product; products with few output tiles and a long K are cut
// along K into chunks of >= 64, about 128 workgroups per product (the cut
// depends on the shape alone, partials summed in order).
static sk_status gemm(sketch_t h, const GemmDesc& g0) {
    if (g0.M <= 0 || g0.N <= 0) return SK_OK;
    CodState* c = h->cod;
    GemmDesc g = g0;
    const int64_t tiles = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64);
    if (g.K <= 0) return h->device_fail("cod: product with an empty inner dimension");
    if (tiles < 64 && g.K >= 256) {
        int ns = (int)std::min<int64_t>(g.K / 64, std::max<int64_t>(2, 128 / tiles));
        const int kc = (int)round_up((g.K + ns - 1) / ns, 16);
        ns = (g.K + kc - 1) / kc;
        if (ns > 1 && (int64_t)ns * g.M * g.N <= c->gpart_cap) {
            g.part = c->gpart;
            g.nsplit = ns;
            g.kchunk = kc;
            C_TRY(launch_gemm_split(g, h->stream));
            return SK_OK;
        }
    }
    C_TRY(launch_gemm1(g, h->stream));
    return SK_OK;
}

// Symmetric eigen-decomposition of A (n x n, ld lda): X eigenvectors
// (columns, ld ldx), lam descending.
static sk_status eig(sketch_t h, const double* A, int lda, double* X, int ldx, double* lam, int n, double* wk1,
                     double* wk2) {
    SmallDesc sd{};
    sd.A = A;
    sd.lda = lda;
    sd.X = X;
    sd.ldx = ldx;
    sd.lam = lam;
    sd.n = n;
    sd.work = wk1;
    sd.work2 = wk2;
    sd.info = h->cod->info;
    hipError_t e = eig_solver_jacobi() ? launch_jacobi1(sd, h->stream) : launch_tri_eig1(sd, h->stream);
    if (e != hipSuccess) return h->device_fail(std::string("cod eigen-solve: ") + hipGetErrorString(e));
    return SK_OK;
}

// Algorithm "Simultaneous Iteration" for the left directions of M = A^T B
// (left = true: directions and test matrix in R^{d_x}) or its right ones
// (left = false: in R^{d_y}).  The oracle's form: simul_iter on the matrix
// C^T with C = M^T (left) or C = M (right), test matrix Omega (d x k) on C's
// column side, q re-orthonormalised power steps, Rayleigh-Ritz.  With P the
// buffer applied first (A left, B right), R the other, C v = R^T (P v), and
// the kept Grams G_P = P P^T, G_R = R R^T, the iterate K is carried as
// K = P^T S with S (r x k) in the row space: C^T C K = P^T (G_R G_P S),
// K^T K = S^T G_P S, K X^T = P^T (S X^T), (C K)^T (C K) = S^T G_P G_R G_P S.
// In exact arithmetic these are the d-side steps; only P Omega and the final
// K U = P^T (S U) read a buffer.  Leaves the directions (d x k, ld kmax) in
// out and, with wait, the k eigenvalue estimates (squared singular values) in
// h_small once the stream is done (without wait nothing is read back and the
// call returns after queueing).  The kept Grams must be complete.
static sk_status simul_iter(sketch_t h, bool left, int k, int64_t ts, uint64_t tag, double* out, bool wait,
                            bool dirs) {
    CodState* c = h->cod;
    const int kl = c->kmax, r = (int)c->r, ld = c->n2;
    const double* P = left ? c->A[c->par] : c->B[c->par];
    const int ldp = (int)(left ? c->ldx : c->ldy);
    const int d = left ? c->dx : c->dy;
    const double* GP = left ? c->Gkx : c->Gky;
    const double* GR = left ? c->Gky : c->Gkx;
    sk_status rc;
    MatGenDesc m{};
    m.M = c->Om;
    m.rows = d;
    m.cols = k;
    m.ld = kl;
    m.seed = c->seed;
    m.stream = c->stream;
    m.c2 = (uint64_t)ts;
    m.c3 = tag;
    C_TRY(launch_philox_mat1(m, h->stream));
    double* S = c->rs[0];
    double* S2 = c->rs[1];
    double* GS = c->rs[2];
    double* V = c->rs[3];
    // the first power step: K = C^T C Omega = P^T (G_R (P Omega))
    if ((rc = gemm(h, cg(P, ldp, false, c->Om, kl, false, V, kl, r, k, d)))) return rc;
    if ((rc = gemm(h, cg(GR, ld, false, V, kl, false, S, kl, r, k, r)))) return rc;
    // CholeskyQR passes on K = P^T S: W = S^T G_P S, X = chol(W)^-1, S <- S X^T
    auto cholqr_rows = [&](int passes) -> sk_status {
        for (int p = 0; p < passes; ++p) {
            sk_status e;
            if ((e = gemm(h, cg(GP, ld, false, S, kl, false, GS, kl, r, k, r)))) return e;
            if ((e = gemm(h, cg(S, kl, true, GS, kl, false, c->Wk, kl, k, k, r)))) return e;
            SmallDesc sd{};
            sd.A = c->Wk;
            sd.lda = kl;
            sd.X = c->Xk;
            sd.ldx = kl;
            sd.n = k;
            sd.work = c->w1;
            C_TRY(launch_cholinv1(sd, h->stream));
            if ((e = gemm(h, cg(S, kl, false, c->Xk, kl, true, S2, kl, r, k, k)))) return e;
            std::swap(S, S2);
        }
        return SK_OK;
    };
    for (int it = 1; it <= c->q; ++it) {
        if ((rc = cholqr_rows(1))) return rc;
        // K <- C^T C K: S <- G_R G_P S
        if ((rc = gemm(h, cg(GP, ld, false, S, kl, false, GS, kl, r, k, r)))) return rc;
        if ((rc = gemm(h, cg(GR, ld, false, GS, kl, false, S2, kl, r, k, r)))) return rc;
        std::swap(S, S2);
    }
    if ((rc = cholqr_rows(2))) return rc;  // K = P^T S has orthonormal columns
    // M_k = (C K)^T (C K) = (G_P S)^T G_R (G_P S)
    if ((rc = gemm(h, cg(GP, ld, false, S, kl, false, GS, kl, r, k, r)))) return rc;
    if ((rc = gemm(h, cg(GR, ld, false, GS, kl, false, V, kl, r, k, r)))) return rc;
    if ((rc = gemm(h, cg(GS, kl, true, V, kl, false, c->Mk, kl, k, k, r)))) return rc;
    if ((rc = eig(h, c->Mk, kl, c->Uk, kl, c->lam, k, c->w1, c->w2))) return rc;
    // directions K U = P^T (S U), now or (dirs false) by directions_of_last
    c->s_last = S;
    if (dirs) {
        if ((rc = gemm(h, cg(S, kl, false, c->Uk, kl, false, S2, kl, r, k, k)))) return rc;
        if ((rc = gemm(h, cg(P, ldp, true, S2, kl, false, out, kl, d, k, r)))) return rc;
    }
    if (wait) {
        C_TRY(hipMemcpyAsync(c->h_small, c->lam, sizeof(double) * (size_t)k, hipMemcpyDeviceToHost, h->stream));
        C_TRY(wait_stream(h));
    }
    c->nsi += 1;
    return SK_OK;
}

// The directions K U = P^T (S U) of the last simul_iter call (made with
// dirs = false), from its S and U, before another call reuses them.
static sk_status directions_of_last(sketch_t h, bool left, int k, double* out) {
    CodState* c = h->cod;
    const int kl = c->kmax, r = (int)c->r;
    const double* P = left ? c->A[c->par] : c->B[c->par];
    const int ldp = (int)(left ? c->ldx : c->ldy);
    const int d = left ? c->dx : c->dy;
    double* T = c->s_last == c->rs[0] ? c->rs[1] : c->rs[0];
    sk_status rc;
    if ((rc = gemm(h, cg(c->s_last, kl, false, c->Uk, kl, false, T, kl, r, k, k)))) return rc;
    return gemm(h, cg(P, ldp, true, T, kl, false, out, kl, d, k, r));
}

// The co-occurring-directions reduce of the full buffers (2 ell rows) into
// the other pair of buffers; leaves ell - 1 rows.
static sk_status reduce(sketch_t h) {
    CodState* c = h->cod;
    const int n = c->n2, ld = c->n2, ell = c->ell;
    const double* A = c->A[c->par];
    const double* B = c->B[c->par];
    double* A2 = c->A[c->par ^ 1];
    double* B2 = c->B[c->par ^ 1];
    const int lx = (int)c->ldx, ly = (int)c->ldy;
    sk_status rc;
    if ((rc = gemm(h, cg(A, lx, false, A, lx, true, c->Gx, ld, n, n, c->dx)))) return rc;
    if ((rc = gemm(h, cg(B, ly, false, B, ly, true, c->Gy, ld, n, n, c->dy)))) return rc;
    if ((rc = eig(h, c->Gx, ld, c->Wx, ld, c->lx, n, c->e1, c->e2))) return rc;
    if ((rc = eig(h, c->Gy, ld, c->Wy, ld, c->ly, n, c->e1, c->e2))) return rc;
    // S = W L^{1/2}, P = W L^{-1/2} (dropped columns zero)
    C_TRY(launch_cod_scale(c->Wx, ld, c->Sx, ld, n, n, c->lx, n, COD_SQRT, kDropTol, ell, h->stream));
    C_TRY(launch_cod_scale(c->Wy, ld, c->Sy, ld, n, n, c->ly, n, COD_SQRT, kDropTol, ell, h->stream));
    C_TRY(launch_cod_scale(c->Wx, ld, c->Px, ld, n, n, c->lx, n, COD_INVSQRT, kDropTol, ell, h->stream));
    C_TRY(launch_cod_scale(c->Wy, ld, c->Py, ld, n, n, c->ly, n, COD_INVSQRT, kDropTol, ell, h->stream));
    // K = R_x R_y^T = S_x^T S_y; K^T K = V s^2 V^T
    if ((rc = gemm(h, cg(c->Sx, ld, true, c->Sy, ld, false, c->K, ld, n, n, n)))) return rc;
    if ((rc = gemm(h, cg(c->K, ld, true, c->K, ld, false, c->KK, ld, n, n, n)))) return rc;
    if ((rc = eig(h, c->KK, ld, c->V, ld, c->lk, n, c->e1, c->e2))) return rc;
    // A'^T = A^T P_x K V diag(sqrt(s^)/s): T1 = K V (n x n), T2 = P_x T1, scaled
    if ((rc = gemm(h, cg(c->K, ld, false, c->V, ld, false, c->T1, ld, n, n, n)))) return rc;
    if ((rc = gemm(h, cg(c->Px, ld, false, c->T1, ld, false, c->T2, ld, n, n, n)))) return rc;
    C_TRY(launch_cod_scale(c->T2, ld, c->T1, ld, n, ell, c->lk, n, COD_SHRINK_GAIN, kDropTol, ell, h->stream));
    if ((rc = gemm(h, cg(c->T1, ld, true, A, lx, false, A2, lx, ell - 1, c->dx, n)))) return rc;
    // B'^T = B^T P_y V diag(sqrt(s^))
    C_TRY(launch_cod_scale(c->V, ld, c->T1, ld, n, ell, c->lk, n, COD_SHRINK_SQRT, kDropTol, ell, h->stream));
    if ((rc = gemm(h, cg(c->Py, ld, false, c->T1, ld, false, c->T2, ld, n, ell, n)))) return rc;
    if ((rc = gemm(h, cg(c->T2, ld, true, B, ly, false, B2, ly, ell - 1, c->dy, n)))) return rc;
    c->par ^= 1;
    c->r = ell - 1;
    c->reduces += 1;
    return SK_OK;
}

static sk_status grow_ring(sketch_t h, int64_t need) {
    CodState* c = h->cod;
    // the live entries move to the front of a fresh ring; it grows only when
    // they fill more than half of it
    const int64_t ncap = std::max<int64_t>(c->cap, 2 * need);
    double* nb[4] = {nullptr, nullptr, nullptr, nullptr};
    double* ob[4] = {c->Zs, c->ZMs, c->MHs, c->Hs};
    const int64_t lds[4] = {c->ldx, c->ldy, c->ldx, c->ldy};
    C_TRY(hipStreamSynchronize(h->stream));
    for (int b = 0; b < 4; ++b) C_TRY(hipMalloc((void**)&nb[b], sizeof(double) * (size_t)ncap * lds[b]));
    // live entries packed to the front, oldest first
    int64_t at = 0;
    for (CodEntry& e : c->q_) {
        for (int b = 0; b < 4; ++b)
            C_TRY(hipMemcpyAsync(nb[b] + at * lds[b], ob[b] + e.slot * lds[b], sizeof(double) * (size_t)e.xi * lds[b],
                                 hipMemcpyDeviceToDevice, h->stream));
        e.slot = at;
        at += e.xi;
    }
    C_TRY(hipStreamSynchronize(h->stream));
    for (int b = 0; b < 4; ++b) h->replace_alloc(ob[b], nb[b], sizeof(double) * (size_t)(ncap - c->cap) * lds[b]);
    c->Zs = nb[0];
    c->ZMs = nb[1];
    c->MHs = nb[2];
    c->Hs = nb[3];
    c->cap = ncap;
    c->tail = at;
    return SK_OK;
}

// Snapshot of the first xi directions of Z (d_x x kmax) and H (d_y x kmax),
// then A <- A - (A Z) Z^T, B <- B - (B H) H^T.
static sk_status dump(sketch_t h, int xi, int64_t ts) {
    CodState* c = h->cod;
    const int kl = c->kmax, r = (int)c->r;
    double* A = c->A[c->par];
    double* B = c->B[c->par];
    const int lx = (int)c->ldx, ly = (int)c->ldy;
    if (c->tail + xi > c->cap) {
        int64_t live = 0;
        for (const CodEntry& e : c->q_) live += e.xi;
        sk_status rc = grow_ring(h, live + xi);
        if (rc) return rc;
    }
    const int64_t slot = c->tail;
    c->tail += xi;
    sk_status rc;
    // AZ = A Z (r x xi) in Tr, BH = B H (r x xi) in Yd
    if ((rc = gemm(h, cg(A, lx, false, c->Z, kl, false, c->Tr, kl, r, xi, c->dx)))) return rc;
    if ((rc = gemm(h, cg(B, ly, false, c->H, kl, false, c->Yd, kl, r, xi, c->dy)))) return rc;
    // Z^T M = (A Z)^T B ; (M H)^T = (B H)^T A
    if ((rc = gemm(h, cg(c->Tr, kl, true, B, ly, false, c->ZMs + slot * c->ldy, ly, xi, c->dy, r)))) return rc;
    if ((rc = gemm(h, cg(c->Yd, kl, true, A, lx, false, c->MHs + slot * c->ldx, lx, xi, c->dx, r)))) return rc;
    C_TRY(launch_transpose(c->Z, kl, c->Zs + slot * c->ldx, c->ldx, c->dx, xi, h->stream));
    C_TRY(launch_transpose(c->H, kl, c->Hs + slot * c->ldy, c->ldy, c->dy, xi, h->stream));
    if ((rc = gemm(h, cg(c->Tr, kl, false, c->Z, kl, true, A, lx, r, c->dx, xi, -1.0, 1.0)))) return rc;
    if ((rc = gemm(h, cg(c->Yd, kl, false, c->H, kl, true, B, ly, r, c->dy, xi, -1.0, 1.0)))) return rc;
    CodEntry e{};
    e.xi = xi;
    e.s = c->last_t + 1;
    e.t = ts;
    e.slot = slot;
    c->q_.push_back(e);
    c->last_t = ts;
    c->g_rows = -1;  // the residual rewrote both buffers
    c->dumps += 1;
    c->dirs += xi;
    return SK_OK;
}

// The dump step for the pair with timestamp i.
static sk_status dump_step(sketch_t h, int64_t i) {
    CodState* c = h->cod;
    const int r = (int)c->r, ld = c->n2;
    const double* A = c->A[c->par];
    const double* B = c->B[c->par];
    const int lx = (int)c->ldx, ly = (int)c->ldy;
    sk_status rc;
    // power iteration in the row space.  The kept Grams gain the new pair's
    // row and column in one pass over the buffers, which also forms
    // u0 = B x0 and |x0|^2 (x0: normal 0 of the Philox block at counter
    // (t, 0, i, 0x100) for coordinate t); after a reduce (the other buffer
    // pair) or a dump they are recomputed first.
    const bool same = c->g_rows >= 0 && c->g_par == c->par;
    const bool inc = same && c->g_rows == r - 1;
    if (!inc && !(same && c->g_rows == r)) {
        if ((rc = gemm(h, cg(A, lx, false, A, lx, true, c->Gkx, ld, r, r, c->dx)))) return rc;
        if ((rc = gemm(h, cg(B, ly, false, B, ly, true, c->Gky, ld, r, r, c->dy)))) return rc;
    }
    GramPiDesc* gd = c->gdh;
    for (int s = 0; s < 2; ++s) {
        GramPiDesc& g = gd[s];
        g = GramPiDesc{};
        g.C = s == 0 ? B : A;
        g.G = s == 0 ? c->Gky : c->Gkx;
        g.u = s == 0 ? c->ub : c->ua;
        g.ldc = s == 0 ? ly : lx;
        g.d = s == 0 ? c->dy : c->dx;
        g.r = (s == 0 || inc) ? r : 0;  // A's pass only extends its Gram
        g.grow = inc ? r - 1 : -1;
        g.ldg = ld;
        g.seed = c->seed;
        g.stream = c->stream;
        g.c2 = (uint64_t)i;
        g.c3 = 0x100u;
    }
    C_TRY(hipMemcpyAsync(c->gdd, c->gdh, 2 * sizeof(GramPiDesc), hipMemcpyHostToDevice, h->stream));
    C_TRY(launch_win_gemv(c->gdd, 2, r, std::max(c->dx, c->dy), h->stream));
    c->g_rows = r;
    c->g_par = c->par;
    const int steps = (int)std::ceil(std::log2((double)c->dy)) + 1;
    C_TRY(launch_cod_pi(c->Gkx, c->Gky, ld, c->ub, c->ub + ld, r, steps, c->pi_out, h->stream));
    C_TRY(hipMemcpyAsync(c->h_small, c->pi_out, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    C_TRY(wait_stream(h));
    const double s1 = std::sqrt(std::max(c->h_small[0], 0.0));
    if (!(s1 >= c->theta / 2.0)) return SK_OK;
    int kmax = std::min(std::min(c->ell, c->dx), std::min(c->dy, r));
    int nsteps = kmax > 1 ? (int)std::ceil(std::log2((double)kmax)) : 1;
    if (nsteps < 1) nsteps = 1;
    for (int s = 1; s <= nsteps && kmax >= 1; ++s) {
        int k = 1 << s;
        if (k > kmax) k = kmax;
        // Each step makes a left and a right simul_iter call with their own
        // Philox counters; only the right call's estimates decide, and the
        // left call's directions are used only by a dump at this step.  So
        // the left call runs only before a dump (its values do not depend on
        // the order of the two calls); a step that does not dump elides it
        // and still counts it, so the call count is the algorithm's.
        if ((rc = simul_iter(h, false, k, i, 0x400u + (uint64_t)s, c->H, true, false))) return rc;
        const double* est = c->h_small;  // the right call's estimates
        const bool stop = !(std::sqrt(std::max(est[k - 1], 0.0)) >= c->theta) || k == kmax;
        int xi = 0;
        if (stop)
            while (xi < k && std::sqrt(std::max(est[xi], 0.0)) >= c->theta) ++xi;
        if (xi > 0) {
            if ((rc = directions_of_last(h, false, k, c->H))) return rc;
            if ((rc = simul_iter(h, true, k, i, 0x200u + (uint64_t)s, c->Z, false, true))) return rc;
            if ((rc = dump(h, xi, i))) return rc;
        } else {
            c->nsi += 1;
        }
        if (stop) break;
    }
    return SK_OK;
}

sk_status cod_create(sketch_t h) {
    const sketch_config& cfg = h->cfg;
    CodState* c = new CodState();
    h->cod = c;
    c->dx = cfg.d;
    c->dy = cfg.d_y;
    c->ell = cfg.ell;
    c->q = cfg.q;
    c->n2 = 2 * cfg.ell;
    c->kmax = std::min(cfg.ell, std::min(cfg.d, cfg.d_y));
    c->N = cfg.window_N;
    c->theta = cfg.theta;
    c->seed = cfg.seed;
    c->stream = cfg.stream_id;
    c->ldx = round_up(cfg.d, 64);
    c->ldy = round_up(cfg.d_y, 64);
    h->ld = c->ldx;
    c->pn = std::min(c->dx, c->dy);
    const int n = c->n2, kl = c->kmax, dmax = std::max(c->dx, c->dy), pn = c->pn;
    auto A = [&](double** p, size_t cnt) { return h->dalloc((void**)p, sizeof(double) * (cnt ? cnt : 1)); };
    for (int b = 0; b < 2; ++b) {
        C_TRY(A(&c->A[b], (size_t)n * c->ldx));
        C_TRY(A(&c->B[b], (size_t)n * c->ldy));
    }
    // eigen-solver work: padded to 32, squared
    const size_t wn = (size_t)round_up(n, 32) * round_up(n, 32), wk = (size_t)round_up(kl, 32) * round_up(kl, 32),
                 wq = (size_t)round_up(pn, 32) * round_up(pn, 32);
    for (double** p : {&c->Gx, &c->Gy, &c->Wx, &c->Wy, &c->Sx, &c->Sy, &c->Px, &c->Py, &c->K, &c->KK, &c->V, &c->T1,
                       &c->T2})
        C_TRY(A(p, (size_t)n * n));
    for (double** p : {&c->e1, &c->e2}) C_TRY(A(p, wn));
    for (double** p : {&c->lx, &c->ly, &c->lk}) C_TRY(A(p, (size_t)n));
    for (double** p : {&c->Om, &c->Yd, &c->Z, &c->H}) C_TRY(A(p, (size_t)dmax * kl));
    C_TRY(A(&c->Tr, (size_t)n * kl));
    for (double** p : {&c->Wk, &c->Xk, &c->Mk, &c->Uk}) C_TRY(A(p, (size_t)kl * kl));
    for (double** p : {&c->w1, &c->w2}) C_TRY(A(p, wk));
    C_TRY(A(&c->lam, (size_t)kl));
    for (double** p : {&c->Gkx, &c->Gky}) C_TRY(A(p, (size_t)n * n));
    for (double** p : {&c->ua, &c->ub}) C_TRY(A(p, (size_t)n + 1));
    for (double*& p : c->rs) C_TRY(A(&p, (size_t)n * kl));
    C_TRY(A(&c->pi_out, 1));
    C_TRY(h->dalloc((void**)&c->gdd, 2 * sizeof(GramPiDesc)));
    C_TRY(h->dalloc((void**)&c->info, 64));
    C_TRY(hipMemset(c->info, 0, 64));
    c->cap = 8 * (int64_t)c->ell;
    C_TRY(A(&c->Zs, (size_t)c->cap * c->ldx));
    C_TRY(A(&c->ZMs, (size_t)c->cap * c->ldy));
    C_TRY(A(&c->MHs, (size_t)c->cap * c->ldx));
    C_TRY(A(&c->Hs, (size_t)c->cap * c->ldy));
    C_TRY(A(&c->Mw, (size_t)c->dx * c->dy));
    for (double** p : {&c->Gq, &c->Uq}) C_TRY(A(p, (size_t)pn * pn));
    for (double** p : {&c->eq1, &c->eq2}) C_TRY(A(p, wq));
    C_TRY(A(&c->lq, (size_t)pn));
    C_TRY(A(&c->Aq, (size_t)c->dx * c->ell));
    C_TRY(A(&c->Bq, (size_t)c->dy * c->ell));
    C_TRY(A(&c->Tq, (size_t)pn * c->ell));
    C_TRY(A(&c->S, (size_t)c->chunk * c->chunk));
    C_TRY(A(&c->T3, (size_t)c->dx * c->chunk));
    C_TRY(h->dalloc((void**)&c->ent, sizeof(int32_t) * (size_t)c->chunk));
    c->gpart_cap = (int64_t)1 << 21;
    C_TRY(A(&c->gpart, (size_t)c->gpart_cap));
    C_TRY(hipHostMalloc((void**)&c->h_small, sizeof(double) * (size_t)std::max(kl, 1), hipHostMallocDefault));
    C_TRY(hipHostMalloc((void**)&c->gdh, 2 * sizeof(GramPiDesc), hipHostMallocDefault));
    C_TRY(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
    return SK_OK;
}

void cod_destroy(sketch_t h) {
    CodState* c = h->cod;
    if (!c) return;
    if (c->h_small) (void)hipHostFree(c->h_small);
    if (c->gdh) (void)hipHostFree(c->gdh);
    if (c->done) (void)hipEventDestroy(c->done);
    delete c;
    h->cod = nullptr;
}

sk_status cod_update_impl(sketch_t h, const char* X, int64_t ldx, const char* Y, int64_t ldy, int64_t n, int dtype) {
    CodState* c = h->cod;
    const int64_t es = dtype_size(dtype);
    sk_status rc;
    for (int64_t e = 0; e < n; ++e) {
        const int64_t i = c->T + 1;
        c->T = i;
        while (!c->q_.empty() && c->q_.front().t + c->N <= i) c->q_.pop_front();
        if (c->q_.empty()) c->tail = 0;
        C_TRY(launch_rows_to_f64(X + e * ldx * es, ldx, dtype, c->A[c->par] + c->r * c->ldx, c->ldx, 1, c->dx,
                                 h->stream));
        C_TRY(launch_rows_to_f64(Y + e * ldy * es, ldy, dtype, c->B[c->par] + c->r * c->ldy, c->ldy, 1, c->dy,
                                 h->stream));
        c->r += 1;
        if (c->r == c->n2 && (rc = reduce(h))) return rc;
        if ((rc = dump_step(h, i))) return rc;
    }
    C_TRY(hipStreamSynchronize(h->stream));
    int32_t inf[2] = {0, 0};
    C_TRY(hipMemcpy(inf, c->info, sizeof(inf), hipMemcpyDeviceToHost));
    if (inf[0] != 0) return h->device_fail("cod: eigen-solver did not converge");
    return SK_OK;
}

sk_status cod_product_impl(sketch_t h, double* M) {
    CodState* c = h->cod;
    const int dx = c->dx, dy = c->dy, lx = (int)c->ldx, ly = (int)c->ldy, r = (int)c->r;
    sk_status rc;
    if (r > 0) {
        if ((rc = gemm(h, cg(c->A[c->par], lx, true, c->B[c->par], ly, false, M, dy, dx, dy, r)))) return rc;
    } else {
        C_TRY(hipMemsetAsync(M, 0, sizeof(double) * (size_t)dx * dy, h->stream));
    }
    // snapshot restores in chunks of consecutive ring rows:
    // M += Zs^T ZMs + MHs^T Hs - Zs^T (mask(Zs MHs^T)) Hs
    std::vector<const CodEntry*> es;
    for (const CodEntry& e : c->q_) es.push_back(&e);
    size_t a = 0;
    std::vector<int32_t> ent;
    while (a < es.size()) {
        const int64_t s0 = es[a]->slot;
        int D = 0;
        ent.clear();
        size_t b = a;
        while (b < es.size() && es[b]->slot == s0 + D && D + es[b]->xi <= c->chunk) {
            for (int x = 0; x < es[b]->xi; ++x) ent.push_back((int32_t)b);
            D += es[b]->xi;
            ++b;
        }
        const double* Zs = c->Zs + s0 * c->ldx;
        const double* ZMs = c->ZMs + s0 * c->ldy;
        const double* MHs = c->MHs + s0 * c->ldx;
        const double* Hs = c->Hs + s0 * c->ldy;
        C_TRY(hipMemcpyAsync(c->ent, ent.data(), sizeof(int32_t) * ent.size(), hipMemcpyHostToDevice, h->stream));
        if ((rc = gemm(h, cg(Zs, lx, true, ZMs, ly, false, M, dy, dx, dy, D, 1.0, 1.0)))) return rc;
        if ((rc = gemm(h, cg(MHs, lx, true, Hs, ly, false, M, dy, dx, dy, D, 1.0, 1.0)))) return rc;
        if ((rc = gemm(h, cg(Zs, lx, false, MHs, lx, true, c->S, c->chunk, D, D, dx)))) return rc;
        C_TRY(launch_blockmask(c->S, c->chunk, D, c->ent, h->stream));
        if ((rc = gemm(h, cg(Zs, lx, true, c->S, c->chunk, false, c->T3, c->chunk, dx, D, D)))) return rc;
        if ((rc = gemm(h, cg(c->T3, c->chunk, false, Hs, ly, false, M, dy, dx, dy, D, -1.0, 1.0)))) return rc;
        C_TRY(hipStreamSynchronize(h->stream));  // the host entry list is reused
        a = b;
    }
    return SK_OK;
}

sk_status cod_query_impl(sketch_t h, const double** Aout, const double** Bout) {
    CodState* c = h->cod;
    const int dx = c->dx, dy = c->dy, ell = c->ell, pn = c->pn;
    sk_status rc;
    if ((rc = cod_product_impl(h, c->Mw))) return rc;
    // SVD of M_W through the eigen-decomposition of its smaller Gram
    const bool xs = dx <= dy;
    // G = M M^T (dx x dx) or M^T M (dy x dy)
    if ((rc = gemm(h, cg(c->Mw, dy, !xs, c->Mw, dy, xs, c->Gq, pn, pn, pn, xs ? dy : dx)))) return rc;
    if ((rc = eig(h, c->Gq, pn, c->Uq, pn, c->lq, pn, c->eq1, c->eq2))) return rc;
    // the small side: columns sqrt(s^); the other side: M^T U diag(sqrt(s^)/s) (or M V ...)
    double* small = xs ? c->Aq : c->Bq;
    double* other = xs ? c->Bq : c->Aq;
    const int nother = xs ? dy : dx;
    C_TRY(launch_cod_scale(c->Uq, pn, small, ell, pn, std::min(ell, pn), c->lq, pn, COD_SHRINK_SQRT, kDropTol, ell,
                           h->stream));
    C_TRY(launch_cod_scale(c->Uq, pn, c->Tq, ell, pn, std::min(ell, pn), c->lq, pn, COD_SHRINK_GAIN, kDropTol, ell,
                           h->stream));
    if (pn < ell) {
        // columns beyond the rank are zero
        C_TRY(hipMemsetAsync(c->Aq, 0, sizeof(double) * (size_t)dx * ell, h->stream));
        C_TRY(hipMemsetAsync(c->Bq, 0, sizeof(double) * (size_t)dy * ell, h->stream));
        C_TRY(launch_cod_scale(c->Uq, pn, small, ell, pn, pn, c->lq, pn, COD_SHRINK_SQRT, kDropTol, ell, h->stream));
    }
    if ((rc = gemm(h, cg(c->Mw, dy, xs, c->Tq, ell, false, other, ell, nother, std::min(ell, pn), pn)))) return rc;
    C_TRY(hipStreamSynchronize(h->stream));
    int32_t inf[2] = {0, 0};
    C_TRY(hipMemcpy(inf, c->info, sizeof(inf), hipMemcpyDeviceToHost));
    if (inf[0] != 0) return h->device_fail("cod: eigen-solver did not converge");
    *Aout = c->Aq;
    *Bout = c->Bq;
    return SK_OK;
}

void cod_stats(sketch_t h, int64_t* st) {
    const CodState* c = h->cod;
    st[0] = c->dumps;
    st[1] = 0;
    st[2] = c->dirs;
    st[3] = c->r;
    st[4] = (int64_t)c->q_.size();
    st[5] = c->reduces;
}

int64_t cod_time(sketch_t h) { return h->cod->T; }
const int32_t* cod_info_ptr(sketch_t h) { return h->cod->info; }
