/*
 * oracle.h -- plain, slow, FP64 CPU reference for the Frequent-Directions
 * (FD) shrink and its randomized variant.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source with the GPU path.
 *
 * Paper: "Near-Optimal Time Matrix Sketch Framework for Persistent, Sliding
 * Window, and Distributed Streams" (arXiv 2601.02019).
 *   - FD buffer and shrink: Sec. 2.3 "Frequent Directions".
 *   - Randomized factorisation: Sec. 2.2, Algorithm "Simultaneous Iteration"
 *     (simul_iter).
 *   - Power iteration: Sec. 2.2, Algorithm "Power Iteration".
 *   - Update loop with the FD reduce: Algorithm "AeroSketch: Update".
 *   - Query with the final shrink: Algorithm "AeroSketch: Query".
 *   - Sliding window: Algorithm "ML-AeroSketch".
 *   - Merge: Lemma "Decomposability" (appendix, proof of the P5 theorem).
 *   - Persistent (at-the-time) sketch: Algorithm "ATTP Sketch using
 *     AeroSketch" (Sec. 4.1).
 *
 * Conventions: every matrix is row-major FP64 with an explicit leading
 * dimension; every function returns 0 on success and a negative code on a
 * bad argument or non-convergence.
 */
#ifndef SKETCH_ORACLE_H
#define SKETCH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based random numbers (Philox4x64-10, Salmon et al. SC'11) -- */
void o_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* Four standard normals from one Philox block by the Box-Muller transform. */
void o_gauss4(uint64_t seed, uint64_t stream, const uint64_t ctr[4], double out[4]);
/* Omega[i][j] (d x k, row-major) for shrink number b: counter (i, j/4, b, tag). */
void o_omega(uint64_t seed, uint64_t stream, uint64_t b, uint64_t tag,
             int d, int k, double* omega);

/* ---- dense linear algebra --------------------------------------------- */
/* One-sided (Hestenes) Jacobi on the m rows of X (m x d, ld): rows are
 * rotated until mutually orthogonal, then sorted by norm (descending);
 * sigma[i] = norm of row i. */
int o_jacobi_rows(double* X, int m, int d, int ld, double* sigma);
/* Cyclic two-sided Jacobi eigen-decomposition of symmetric A (n x n).
 * w: eigenvalues descending; V (n x n): eigenvectors in columns. A is
 * destroyed. */
int o_sym_eig(double* A, int n, double* w, double* V);
/* Householder QR of K (m x k, m >= k): Q (m x k) with orthonormal columns
 * spanning range(K) (completed arbitrarily if K is rank deficient). */
int o_qr_householder(const double* K, int m, int k, double* Q);

/* ---- Frequent Directions state machine --------------------------------- */
typedef struct o_fd o_fd;
enum { O_EXACT = 0, O_RAND = 1 };
/* mode O_EXACT: FD with an exact SVD in every shrink.
 * mode O_RAND : the SVD replaced by simul_iter on the buffer with target rank
 *               k and q power steps, Omega drawn from Philox(seed, stream). */
o_fd* o_fd_create(int d, int ell, int mode, int k, int q,
                  uint64_t seed, uint64_t stream);
void o_fd_destroy(o_fd* s);
int o_fd_update(o_fd* s, const double* rows, int64_t n, int64_t ld);
/* ell x d sketch: f_ell of the buffer rows (non-destructive). */
int o_fd_query(const o_fd* s, double* out);
/* Raw buffer rows [0, r) into out (r x d); returns r. */
int64_t o_fd_buffer(const o_fd* s, double* out);
int64_t o_fd_fill(const o_fd* s);
int64_t o_fd_shrinks(const o_fd* s);
/* dst absorbs the non-zero rows of src's queried sketch as ordinary rows. */
int o_fd_merge(o_fd* dst, const o_fd* src);
/* One shrink of an m-row buffer X in place, exposed for tests. */
int o_shrink_exact(double* X, int m, int d, int ld, int ell);
int o_shrink_rand(double* X, int m, int d, int ld, int ell, int k, int q,
                  uint64_t seed, uint64_t stream, uint64_t b);

/* ---- power iteration (Algorithm "Power Iteration") on C^T C ------------ */
/* C is m x d. x0 is the start vector (length d, need not be normalised).
 * Returns the Rayleigh quotient after `steps` steps; v receives the vector. */
double o_power_iteration(const double* C, int m, int d, int ld,
                         const double* x0, int steps, double* v);

/* ---- sliding window: ML-AeroSketch ------------------------------------- */
typedef struct o_win o_win;
/* d, ell (eps = 2/ell), window N, R (bound on squared row norms; L =
 * max(1, ceil(log2 R)) levels), q power steps of simul_iter. */
o_win* o_win_create(int d, int ell, int64_t N, double R, int q,
                    uint64_t seed, uint64_t stream);
/* The same with the FD reduce chosen: O_EXACT or O_RAND (simul_iter shrink,
 * k = min(ell, d), q power steps, Philox key (seed, 64 stream + level + 1)). */
o_win* o_win_create2(int d, int ell, int64_t N, double R, int q, uint64_t seed, uint64_t stream,
                     int fd_mode);
void o_win_destroy(o_win* w);
int o_win_update(o_win* w, const double* rows, int64_t n, int64_t ld);
/* Move time forward to t_now without rows (expires old entries). */
int o_win_advance(o_win* w, int64_t t_now);
/* ell x d sketch of the window (T-N, T]. level_out: the level used. */
int o_win_query(const o_win* w, double* out, int* level_out);
int o_win_levels(const o_win* w);
/* Diagnostics of one level: counts of dumps, raw rows, dumped directions,
 * residual rows and queue length. */
int o_win_stats(const o_win* w, int level, int64_t* stats /* [6] */);
/* Gram of the level's restored matrix B_T (d x d): the restore of Algorithm
 * "AeroSketch: Query" over the in-window snapshots, with the in-window raw
 * rows added. */
int o_win_level_gram(const o_win* w, int level, double* G);
/* Counters of one level: the six of o_win_stats, then [6] simul_iter calls
 * and [7] the largest in-window timestamp dropped by the length cap. */
int o_win_counters(const o_win* w, int level, int64_t* st /* [8] */);
/* Queue entry e (0 = oldest) of a level: meta = {kind (0 snapshot, 1 raw
 * row), xi, s, t}; Z (d x xi), W (xi x d) of a snapshot or a (d) of a raw
 * row are copied where the pointer is non-NULL. */
int o_win_entry(const o_win* w, int level, int64_t e, int64_t* meta /* [4] */, double* Z, double* W,
                double* a);
/* The level's residual buffer rows (r x d) into C; returns r. */
int o_win_buffer(const o_win* w, int level, double* C);
/* The dump step of Algorithm "AeroSketch: Update" on a level buffer C (r x d,
 * row-major, ld d), as the window runs it for the row with timestamp i at
 * level `level` with threshold theta: power iteration on C^T C (ceil(log2 d)
 * + 1 steps); if its estimate (*pi) reaches theta / 2, simul_iter with
 * k = 2, 4, ... up to min(ell, d, r) until the k-th estimate falls below
 * theta (*nsi calls); the *xi directions whose estimate reaches theta are the
 * snapshot: Z (d x ell, first *xi columns), W = Z^T C^T C (ell x d, first *xi
 * rows), and C becomes C - C Z Z^T. */
int o_aero_dump(int d, int ell, int q, uint64_t seed, uint64_t stream, int level, double theta, double* C,
                int64_t r, int64_t i, double* Z, double* W, int* xi, int* nsi, double* pi);
/* The same with Algorithm "Probability Amplification" in place of each
 * simul_iter call: amp_r candidates (1..16), amp_s power iterations on each
 * candidate's residual (0..16); amp_r = 1, amp_s = 0 is o_aero_dump.  amp_c
 * (amp_r doubles, optional) receives the candidates' squared estimates c_h^2
 * of the last amplified step, amp_h (optional) the candidate kept there. */
int o_aero_dump_amp(int d, int ell, int q, uint64_t seed, uint64_t stream, int level, double theta, double* C,
                    int64_t r, int64_t i, double* Z, double* W, int* xi, int* nsi, double* pi, int amp_r, int amp_s,
                    double* amp_c, int* amp_h);
int o_win_set_amplify(o_win* w, int r, int s);
/* Algorithm "Simultaneous Iteration" on A = C^T (C: r x d, row stride d),
 * test matrix on the d side from counter (row, column/4, ts, tag), q power
 * steps re-orthonormalised: Z (d x k) = Q U, est (k, descending) the
 * eigenvalues of Q^T C^T C Q (squared singular-value estimates of C). */
int o_simul_iter(const double* C, int64_t r, int d, int k, int q, uint64_t seed, uint64_t stream, uint64_t ts,
                 uint64_t tag, double* Z, double* est);

/* ---- ATTP persistent sketch (Algorithm "ATTP Sketch using AeroSketch") --
 * One AeroSketch whose dump threshold is theta_i = eps ||A_i||_F^2 (eps =
 * 2 / ell) at row i; snapshots are kept for ever, so the sketch of any time
 * t <= T can be queried.  fd_mode as for the window (level 0's key). */
typedef struct o_attp o_attp;
o_attp* o_attp_create(int d, int ell, int q, uint64_t seed, uint64_t stream, int fd_mode);
int o_attp_set_amplify(o_attp* a, int r, int s);
void o_attp_destroy(o_attp* a);
int o_attp_update(o_attp* a, const double* rows, int64_t n, int64_t ld);
/* d x d restored matrix of time t: the restore of every snapshot with
 * timestamp <= t, plus the residual's Gram when t is the current time T. */
int o_attp_gram_at(const o_attp* a, int64_t t, double* G);
/* ell x d sketch of A_t (the restored matrix shrunk by its ell-th eigenvalue). */
int o_attp_query_at(const o_attp* a, int64_t t, double* out);
/* [0] snapshots [1] dumped directions [2] residual rows [3] FD reduces
 * [4] simul_iter calls [5] current time T. */
int o_attp_stats(const o_attp* a, int64_t* st /* [6] */);
/* Threshold used for the last row (eps ||A_T||_F^2). */
double o_attp_theta(const o_attp* a);
/* Snapshot e (oldest first): meta = {xi, s, t}; Z (d x xi), W (xi x d). */
int o_attp_snapshot(const o_attp* a, int64_t e, int64_t* meta /* [3] */, double* Z, double* W);
/* The residual rows (r x d) into C; returns r. */
int o_attp_buffer(const o_attp* a, double* C);

/* ---- P5: continuous distributed tracking (Algorithm "P5") --------------
 * m sites (1..4096), each with a counter F_j and an AeroSketch at threshold
 * (eps / m) Fhat_j (eps = 2 / ell); a coordinator with Fhat, broadcasts every m
 * counter messages, and B += the restore of every snapshot a site dumps.
 * site[e] names the site of row e; rows are taken in order. */
typedef struct o_p5 o_p5;
o_p5* o_p5_create(int d, int ell, int m, int q, uint64_t seed, uint64_t stream, int fd_mode);
int o_p5_set_amplify(o_p5* p, int r, int s);
void o_p5_destroy(o_p5* p);
int o_p5_update(o_p5* p, const int32_t* site, const double* rows, int64_t n, int64_t ld);
/* The coordinator's B (d x d). */
int o_p5_gram(const o_p5* p, double* G);
/* ell x d: B shrunk by its ell-th eigenvalue. */
int o_p5_query(const o_p5* p, double* out);
/* [0] counter messages [1] broadcasts [2] snapshot messages [3] dumped
 * directions [4] rows sent as they are [5] words sent [6] FD reduces
 * [7] rows seen. */
int o_p5_stats(const o_p5* p, int64_t* st /* [8] */);
double o_p5_fhat(const o_p5* p);
/* ---- AeroSketchCOD: approximate matrix multiplication over a sliding
 * window (Algorithm "AeroSketchCOD Framework"), one level with threshold
 * theta; the co-occurring-directions reduce is the SVD of A~^T B~ shrunk by
 * its ell-th singular value and split evenly between the factors. */
typedef struct o_cod o_cod;
o_cod* o_cod_create(int dx, int dy, int ell, int64_t N, double theta, int q, uint64_t seed, uint64_t stream);
void o_cod_destroy(o_cod* c);
/* n pairs: X (n x dx, ldx), Y (n x dy, ldy). */
int o_cod_update(o_cod* c, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n);
/* The restored window product M_W (dx x dy) before the query's shrink. */
int o_cod_product(const o_cod* c, double* MW);
/* A* (dx x ell), B* (dy x ell). */
int o_cod_query(const o_cod* c, double* Aout, double* Bout);
/* [0] snapshots [1] directions [2] buffer rows [3] reduces [4] simul_iter
 * calls [5] snapshots in the queue [6] T. */
int o_cod_stats(const o_cod* c, int64_t* st /* [7] */);
int o_cod_buffers(const o_cod* c, double* A, double* B);
int o_cod_snapshot(const o_cod* c, int64_t e, int64_t* meta, double* Z, double* ZM, double* MH, double* H);
/* The reduce alone, in place on r rows (r <= 2 ell). */
int o_cod_reduce(double* A, double* B, int64_t r, int dx, int dy, int ell);

/* Site j: f3 = {F_j, Fhat_j, theta_j}; st = {rows, buffer rows, FD reduces,
 * snapshots, directions, rows sent as they are, simul_iter calls}; C: the
 * buffer rows.  Any output may be NULL. */
int o_p5_site(const o_p5* p, int j, double* f3, int64_t* st /* [7] */, double* C);

#ifdef __cplusplus
}
#endif
#endif
