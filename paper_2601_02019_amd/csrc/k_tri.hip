// k_tri.hip -- symmetric eigen-decomposition of the shrink's core (the eigen
// step of Algorithm "Simultaneous Iteration" on the k x k Rayleigh-Ritz
// matrix; the exact FD shrink's eigen-decomposition of the 2 ell x 2 ell
// buffer Gram, Sec. 2.3), in four kernels:
//
//   1. k_tri_reduce / k_tri_reduce_blk: Householder tridiagonalisation
//      A = Q T Q^T on one workgroup per problem (A in LDS when it fits; else
//      in the global work matrix, which stays in L2, blocked by 32-column
//      panels for n <= 256).  Orders from trix_min_n() up run instead on
//      ceil(n / 16) workgroups (k_tri_reduce_x in k_trix.hip);
//   2. k_tri_eigval: eigenvalues of T by multisection on Sturm counts to
//      absolute accuracy eps ||T||, the spectrum split by index over up to
//      64 workgroups per problem;
//   3. k_tri_eig: eigenvectors of T by a twisted factorisation at each
//      eigenvalue (the forward and backward pivots of T - lambda I meet at
//      the index where the twist is smallest; the vector follows from one
//      pass each way), one eigenvector per thread;
//   4. k_tri_back: U = Q Z, one wavefront per strip of NS columns of Z with
//      each column's rows held in registers, applying the reflectors from
//      the last to the first.
//
// Eigenvectors from step 3 are accurate to eps ||T|| / gap.  Within clusters
// of close eigenvalues the vectors are made orthogonal by Gram-Schmidt, with
// other twist indices where they coincide; more than 8 equal eigenvalues, or
// a vector that is not finite, send the problem to the Jacobi method.  Every
// reduction has a fixed order: results repeat bit for bit.
#include "k_jacobi_body.h"
#include "sk_device.h"
#include "sk_kernels.h"

namespace sk {

constexpr int TRI_NMAX = 512;

// Static LDS of the solver (small enough that a 128 x 128 FP64 matrix fits
// the dynamic LDS next to it).  w holds e_i^2 between the tridiagonalisation
// and the back-transformation.
struct TriShared {
    double d[TRI_NMAX], e[TRI_NMAX];
    double v[TRI_NMAX], w[TRI_NMAX];
    double red[32];
    double y[1024];
    int flag, ncl;
};

// a / b from the hardware reciprocal refined by two Newton steps and a
// residual correction (a few ulp; the recurrences below are backward stable
// under relative perturbations of that size).
__device__ __forceinline__ double tri_div(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    r = fma(r, fma(-b, r, 1.0), r);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

// Number of eigenvalues of T (d, e2) below x (the count of a matrix within
// a few ulp of T: one Newton step on the reciprocal is enough).
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
    for (int i = 1; i < n; ++i) {
        double r = __builtin_amdgcn_rcp(q);
        r = fma(r, fma(-q, r, 1.0), r);
        q = (d[i] - x) - e2[i - 1] * r;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Eigenvector of T (d, e, e2 = e^2) for the eigenvalue x by a twisted
// factorisation: forward pivots D+ go to Pp[i * sp], backward pivots D- to
// Pm[i * sm]; the twist is the index with the rank-th smallest |gamma_i|
// (rank 0: the smallest; larger ranks give independent vectors inside a
// cluster); the normalised vector goes to Z[i * sz], which may alias Pp.
// Returns false when the vector is not finite.
__device__ bool twisted_vec(const double* d, const double* e, const double* e2, int n, double x, double pivmin,
                            double* Pp, int64_t sp, double* Pm, int64_t sm, int rank, double* Z, int64_t sz) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    Pp[0] = q;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - tri_div(e2[i - 1], q);
        if (fabs(q) < pivmin) q = -pivmin;
        Pp[(int64_t)i * sp] = q;
    }
    double qb = d[n - 1] - x;
    if (fabs(qb) < pivmin) qb = -pivmin;
    Pm[(int64_t)(n - 1) * sm] = qb;
    int r = n - 1;
    double gbest = fabs(Pp[(int64_t)(n - 1) * sp] + qb - (d[n - 1] - x));
    // the stored pivots are read in batches of 8 ahead of the recurrence
    for (int i0 = n - 2; i0 >= 0; i0 -= 8) {
        double pp[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pp[u] = Pp[(int64_t)max(i0 - u, 0) * sp];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 - u;
            if (i < 0) break;
            qb = (d[i] - x) - tri_div(e2[i], qb);
            if (fabs(qb) < pivmin) qb = -pivmin;
            Pm[(int64_t)i * sm] = qb;
            const double g = fabs(pp[u] + qb - (d[i] - x));
            if (g < gbest) {
                gbest = g;
                r = i;
            }
        }
    }
    if (rank > 0) {  // the rank-th smallest |gamma|: rank + 1 passes with exclusion
        int used[8];
        int nu = 0;
        for (int pass = 0; pass <= rank && pass < 8; ++pass) {
            int best = -1;
            double bg = 0.0;
            for (int i = 0; i < n; ++i) {
                bool skip = false;
                for (int u = 0; u < nu; ++u) skip |= used[u] == i;
                if (skip) continue;
                const double g = fabs(Pp[(int64_t)i * sp] + Pm[(int64_t)i * sm] - (d[i] - x));
                if (best < 0 || g < bg) {
                    bg = g;
                    best = i;
                }
            }
            used[nu++] = best;
            r = best;
        }
    }
    // z_r = 1; upwards with the forward pivots, downwards with the backward ones
    double z = 1.0, nrm2 = 1.0;
    for (int i0 = r - 1; i0 >= 0; i0 -= 8) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pv[u] = Pp[(int64_t)max(i0 - u, 0) * sp];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 - u;
            if (i < 0) break;
            z = -tri_div(e[i], pv[u]) * z;
            Z[(int64_t)i * sz] = z;
            nrm2 = fma(z, z, nrm2);
        }
    }
    Z[(int64_t)r * sz] = 1.0;
    z = 1.0;
    for (int i0 = r + 1; i0 < n; i0 += 8) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pv[u] = Pm[(int64_t)min(i0 + u, n - 1) * sm];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u;
            if (i >= n) break;
            z = -tri_div(e[i - 1], pv[u]) * z;
            Z[(int64_t)i * sz] = z;
            nrm2 = fma(z, z, nrm2);
        }
    }
    if (!(nrm2 < 1e300)) return false;
    const double inv = 1.0 / sqrt(nrm2);
#pragma unroll 8
    for (int i = 0; i < n; ++i) Z[(int64_t)i * sz] *= inv;
    return true;
}

// Householder reduction of the symmetric n x n matrix (Ain, symmetrised) to
// tridiagonal form T = Q^T A Q.  Output: the reflectors in W (row j holds v_j
// beyond the super-diagonal, v_j[j + 1] = 1 implied, W[j][j] = tau_j), the
// diagonal of T in row 0 of U and its off-diagonal in row 1 (read back by the
// eigenpair kernel before it writes U).  lds: dynamic LDS of lds_doubles.
//
//  * n (n + 1) <= lds_doubles: A in LDS (row stride n + 1), unblocked;
//  * n <= 256: A in W, blocked by panels of TRI_NB columns (below);
//  * otherwise A in W, unblocked.
constexpr int TRI_NB = 32;
typedef __attribute__((address_space(1))) double gdouble;

// Lane exchanges inside rows of 16 lanes by DPP (no trip through the LDS
// crossbar): CTRL 0xB1 / 0x4E swap lanes 1 and 2 apart within quads, 0x141
// mirrors each half-row, 0x140 each row.
template <int CTRL>
__device__ __forceinline__ double tri_dpp(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over each quad, every lane of the quad getting the same value (the
// same operations as exchanges with lane ^ 1, then lane ^ 2).
__device__ __forceinline__ double tri_quad_sum(double x) {
    x += tri_dpp<0xB1>(x);
    x += tri_dpp<0x4E>(x);
    return x;
}

// Sum over each row of 16 lanes: after the quad sums every quad is uniform,
// so the half-row and row mirrors pair quads as lane ^ 4 and lane ^ 8 would.
__device__ __forceinline__ double tri_row_sum(double x) {
    x = tri_quad_sum(x);
    x += tri_dpp<0x141>(x);
    x += tri_dpp<0x140>(x);
    return x;
}

__device__ __forceinline__ double tri_wave_sum(double x) {
    x = tri_row_sum(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

__device__ __forceinline__ void tri_reduce_unblk_body(const double* Ain, int ldin, int n, double* W, double* U, int lu,
                                                double* lds, int lds_doubles) {
    __shared__ TriShared S;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    const bool inl = (n + 1) * n <= lds_doubles;
    const int la = inl ? n + 1 : n;
    double* A = inl ? lds : W;

    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - i * n;
        A[(int64_t)i * la + j] = 0.5 * (Ain[(int64_t)i * ldin + j] + Ain[(int64_t)j * ldin + i]);
    }
    __syncthreads();

    // ---- 1. tridiagonalisation: four barriers per column
    if (wave == 0) {  // |x|^2 of the first column below its first entry
        double acc = 0.0;
        for (int k = 2 + lane; k < n; k += 64) acc = fma(A[k], A[k], acc);
        acc = tri_wave_sum(acc);
        if (lane == 0) S.red[1] = acc;
    }
    __syncthreads();
    for (int j = 0; j + 1 < n; ++j) {
        const int L = n - j - 1;
        double* row = A + (int64_t)j * la + j + 1;   // row j right of the diagonal = column j below it
        double* A22 = A + (int64_t)(j + 1) * la + j + 1;
        const double xn2 = S.red[1];
        const double alpha = row[0];
        double beta = alpha, tau = 0.0, scal = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (tid == 0) {
            S.d[j] = A[(int64_t)j * la + j];
            S.e[j] = beta;
            A[(int64_t)j * la + j] = tau;
        }
        double K = 0.0;
        if (tau != 0.0) {
            for (int i = tid; i < L; i += nth) {  // v (v_0 = 1) in LDS and in row j
                const double vi = (i == 0) ? 1.0 : row[i] * scal;
                S.v[i] = vi;
                if (i > 0) row[i] = vi;
            }
            __syncthreads();
            // p = tau A22 v and the products p_i v_i
            if (inl && 4 * L <= nth) {  // four lanes per row
                const int i = tid >> 2, sub = tid & 3;
                double acc = 0.0;
                if (i < L)
                    for (int k = sub; k < L; k += 4) acc = fma(A22[(int64_t)i * la + k], S.v[k], acc);
                acc = tri_quad_sum(acc);
                if (i < L && sub == 0) {
                    S.w[i] = tau * acc;
                    S.y[i] = tau * acc * S.v[i];
                }
            } else {  // one wave per row
                for (int i = wave; i < L; i += nw) {
                    const double* Ai = A22 + (int64_t)i * la;
                    double acc = 0.0;
                    for (int k = lane; k < L; k += 64) acc = fma(Ai[k], S.v[k], acc);
                    acc = tri_wave_sum(acc);
                    if (lane == 0) {
                        S.w[i] = tau * acc;
                        S.y[i] = tau * acc * S.v[i];
                    }
                }
            }
            __syncthreads();
            if (wave == 0) {  // K = tau / 2 (p . v)
                double acc = 0.0;
                for (int i = lane; i < L; i += 64) acc += S.y[i];
                acc = tri_wave_sum(acc);
                if (lane == 0) S.red[0] = 0.5 * tau * acc;
            }
            __syncthreads();
            K = S.red[0];
            // A22 -= v w^T + w v^T with w = p - K v; wave 0 also sums the squares
            // of the next column below its first entry (row 0 of A22, k >= 2)
            double nx = 0.0;
            // a lane's columns k = lane + 64 c are the same on every row: their
            // v_k and w_k stay in registers (L <= 511: c < 8)
            double vk[8], wk[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int k = lane + 64 * c;
                vk[c] = k < L ? S.v[k] : 0.0;
                wk[c] = k < L ? fma(-K, vk[c], S.w[k]) : 0.0;
            }
            for (int i = wave; i < L; i += nw) {
                const double vi = S.v[i], wi = fma(-K, vi, S.w[i]);
                double* Ai = A22 + (int64_t)i * la;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int k = lane + 64 * c;
                    if (k < L) {
                        const double a = Ai[k] - (vi * wk[c] + wi * vk[c]);
                        Ai[k] = a;
                        if (i == 0 && k >= 2) nx = fma(a, a, nx);
                    }
                }
            }
            if (wave == 0) {
                nx = tri_wave_sum(nx);
                if (lane == 0) S.red[1] = nx;
            }
        } else if (wave == 0) {  // no reflection: the next column as it stands
            double acc = 0.0;
            for (int k = 2 + lane; k < L; k += 64) acc = fma(A22[k], A22[k], acc);
            acc = tri_wave_sum(acc);
            if (lane == 0) S.red[1] = acc;
        }
        __syncthreads();
    }
    if (tid == 0) {
        S.d[n - 1] = A[(int64_t)(n - 1) * la + n - 1];
        A[(int64_t)(n - 1) * la + n - 1] = 0.0;
    }
    __syncthreads();
    if (inl)  // the reflectors (ld n) for the back-transformation
        for (int e = tid; e < n * n; e += nth) {
            const int i = e / n, k = e - i * n;
            W[e] = lds[(int64_t)i * la + k];
        }
    for (int i = tid; i < n; i += nth) {
        U[i] = S.d[i];
        if (i + 1 < n) U[lu + i] = S.e[i];
    }
}

// The blocked reduction (A in W, 128 < n <= 256, 1024 threads); a kernel of
// its own so that its product loop keeps its loads in registers.
//
// Within a panel of TRI_NB columns the matrix is not updated: column j uses
// the panel-start matrix minus sum_{c<jc} (v_c w_c^T + w_c v_c^T), with the
// panel's vectors in LDS, and after the panel its 2 TRI_NB vectors update the
// trailing matrix at once.  Nothing is stored to global memory inside a panel
// (a barrier would wait for the stores): the reflectors go to W with the
// update.  Four barriers per column:
//   X  effective column j and |x|^2 (4 lanes per entry);
//   Y  W^T v, V^T v (16 lanes per product), then A22 v (lanes along columns,
//      waves along row stripes, batches of independent loads);
//   P  p = tau (A22 v - V W^T v - W V^T v) and p . v (4 lanes per entry);
//   S  v and w = p - (tau/2)(p . v) v into the panel.
// v_i = x_i * scal is recomputed from x where needed (same rounding).  The
// product leaves row j + 1 (panel-start) in d[j + 1 ..], the part of d not
// yet written, for the next column.  The panel vectors are stored entry-major
// (row g holds entry g of every vector), so a lane's walk over the vectors
// has constant offsets.
struct TriBlkShared {
    double d[256], e[256], v[256];
    double y[1024];
    double red[32];
};

constexpr int TRI_NBP = TRI_NB + 1;  // row stride of the panel (bank spread)

// Dynamic LDS (doubles) of the blocked reduction at size n: the panels, 128
// scalars, and 16 rows of slack that the products with v may read (and
// discard) past the last row.
__host__ __device__ constexpr int tri_blk_lds(int n) { return 2 * n * TRI_NBP + 128 + 16 * TRI_NBP; }

// Product of a panel vector with v on 16 lanes: rows part + 16 t, t < T, of
// which those past the column (16 t >= rem) are read and discarded.
template <int T>
__device__ __forceinline__ double tri_vdot(const double* P, const double* vp, int rem, bool first, double scal) {
    double ds = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const bool in = 16 * t < rem;
        const double pt = P[16 * t * TRI_NBP], vt = vp[16 * t];
        const double vi = in ? ((first && t == 0) ? 1.0 : vt * scal) : 0.0;
        ds = fma(in ? pt : 0.0, vi, ds);
    }
    return ds;
}
__device__ __forceinline__ double tri_vdot_n(int T, const double* P, const double* vp, int rem, bool first,
                                             double scal) {
    switch (T) {
        case 1: return tri_vdot<1>(P, vp, rem, first, scal);
        case 2: return tri_vdot<2>(P, vp, rem, first, scal);
        case 3: return tri_vdot<3>(P, vp, rem, first, scal);
        case 4: return tri_vdot<4>(P, vp, rem, first, scal);
        case 5: return tri_vdot<5>(P, vp, rem, first, scal);
        case 6: return tri_vdot<6>(P, vp, rem, first, scal);
        case 7: return tri_vdot<7>(P, vp, rem, first, scal);
        case 8: return tri_vdot<8>(P, vp, rem, first, scal);
        case 9: return tri_vdot<9>(P, vp, rem, first, scal);
        case 10: return tri_vdot<10>(P, vp, rem, first, scal);
        case 11: return tri_vdot<11>(P, vp, rem, first, scal);
        case 12: return tri_vdot<12>(P, vp, rem, first, scal);
        case 13: return tri_vdot<13>(P, vp, rem, first, scal);
        case 14: return tri_vdot<14>(P, vp, rem, first, scal);
        case 15: return tri_vdot<15>(P, vp, rem, first, scal);
        default: return tri_vdot<16>(P, vp, rem, first, scal);
    }
}

__device__ __forceinline__ bool tri_blocked(int n, int blk_ok) { return blk_ok && n > 128 && n <= 256; }

__device__ __forceinline__ void tri_reduce_blk_body(const double* Ain, int ldin, int n, double* W, double* U, int lu,
                                                    double* lds) {
    __shared__ TriBlkShared S;
    constexpr int NW = 16;  // wavefronts (1024 threads)
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - i * n;
        W[(int64_t)i * n + j] = 0.5 * (Ain[(int64_t)i * ldin + j] + Ain[(int64_t)j * ldin + i]);
    }
    double* Vt = lds;                  // [n][TRI_NBP], zero outside each vector's range
    double* Wt = lds + n * TRI_NBP;    // [n][TRI_NBP]
    double* pan = lds + 2 * n * TRI_NBP;
    double* dW = pan;                  // W^T v (zero beyond the panel's columns so far)
    double* dV = pan + TRI_NB;         // V^T v
    double* taus = pan + 64;
    gdouble* Ag = (gdouble*)W;
    const int quad = tid >> 2, q = tid & 3;
    bool row_ok = false;  // d[j ..] holds row j of the panel-start matrix
    __syncthreads();
    for (int j0 = 0; j0 + 1 < n; j0 += TRI_NB) {
        const int jb = min(TRI_NB, n - 1 - j0);
        for (int e = tid; e < 2 * n * TRI_NBP + 2 * TRI_NB; e += nth) lds[e] = 0.0;
        __syncthreads();
        for (int jc = 0; jc < jb; ++jc) {
            const int j = j0 + jc, L = n - j - 1;
            const bool pre = jc > 0 && row_ok;
            // X: entry quad of column j below the diagonal (quad 255: the
            // diagonal; L <= 254 whenever jc > 0); lane q takes the vectors
            // c = q (mod 4)
            {
                const bool diag = quad == 255;
                const bool act = quad < L || diag;
                const int g = diag ? j : j + 1 + (act ? quad : 0);
                const double* vg = Vt + g * TRI_NBP + q;
                const double* wg = Wt + g * TRI_NBP + q;
                const double* vj = Vt + j * TRI_NBP + q;
                const double* wj = Wt + j * TRI_NBP + q;
                double sub = 0.0;
                const int tmax = (jc - q + 3) >> 2;  // vectors c = q + 4 t < jc
#pragma unroll
                for (int t = 0; t < TRI_NB / 4; ++t)
                    if (t < tmax) sub += vg[4 * t] * wj[4 * t] + wg[4 * t] * vj[4 * t];
                sub = tri_quad_sum(sub);
                double x2 = 0.0;
                if (act && q == 0) {
                    const double a = pre ? S.d[g] : (double)Ag[j * n + g];
                    const double x = a - sub;
                    if (diag) {
                        pan[97] = x;
                    } else {
                        S.v[quad] = x;
                        if (quad == 0) pan[96] = x;
                        else x2 = x * x;
                    }
                }
                x2 = tri_wave_sum(x2);
                if (lane == 0) S.red[wave] = x2;
            }
            __syncthreads();
            double xn2 = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) xn2 += S.red[w];
            const double alpha = pan[96];
            double beta = alpha, tau = 0.0, scal = 0.0;
            if (xn2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            row_ok = tau != 0.0;
            if (tid == 0) {
                S.d[j] = pan[97];
                S.e[j] = beta;
                taus[jc] = tau;
            }
            if (tau != 0.0) {
                // Y: products of v with the panel vectors (slot c < 32: w_c,
                // 32 + c: v_c; 16 lanes each, rows j + 1 + part + 16 t)
                {
                    const int slot = tid >> 4, part = tid & 15, cc = slot & 31;
                    const double* P = (slot < 32 ? Wt : Vt) + (j + 1 + part) * TRI_NBP + cc;
                    const double* vp = S.v + part;
                    const int rem = L - part;  // rows t with 16 t < rem
                    double ds = 0.0;
                    if (cc < jc) ds = tri_vdot_n((L + 15) >> 4, P, vp, rem, part == 0, scal);
                    ds = tri_row_sum(ds);
                    if (part == 0 && cc < jc) pan[slot] = ds;
                }
                const int cb = (L + 63) >> 6, nst = NW / cb, Lp = cb << 6;
                if (wave < cb * nst) {
                    const int st = wave / cb, k = ((wave - st * cb) << 6) + lane;
                    double acc = 0.0;
                    if (k < L) {
                        const gdouble* colp = Ag + (j + 1) * n + j + 1 + k;
                        const int step = nst * n;
                        int i = st;
                        constexpr int B = 16;
                        for (; i + (B - 1) * nst < L; i += B * nst) {
                            const gdouble* p0 = colp + i * n;
                            double av[B];
#pragma unroll
                            for (int u = 0; u < B; ++u) av[u] = p0[u * step];
                            if (i == 0) S.d[j + 1 + k] = av[0];
#pragma unroll
                            for (int u = 0; u < B; ++u) {
                                const int r = i + u * nst;
                                acc = fma(av[u], r == 0 ? 1.0 : S.v[r] * scal, acc);
                            }
                        }
                        for (; i < L; i += nst) {
                            const double a = colp[i * n];
                            if (i == 0) S.d[j + 1 + k] = a;
                            acc = fma(a, i == 0 ? 1.0 : S.v[i] * scal, acc);
                        }
                    }
                    S.y[st * Lp + k] = acc;
                }
                __syncthreads();
                // P: entry quad; lane q takes the stripes and vectors = q (mod 4)
                const bool act = quad < L;
                const int ic = act ? quad : 0, g = j + 1 + ic;
                double pp = 0.0;
                {
                    const double* yp = S.y + q * Lp + ic;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (q + 4 * t < nst) pp += yp[4 * t * Lp];
                    const double* vg = Vt + g * TRI_NBP + q;
                    const double* wg = Wt + g * TRI_NBP + q;
                    const int tmax = (jc - q + 3) >> 2;
#pragma unroll
                    for (int t = 0; t < TRI_NB / 4; ++t)
                        if (t < tmax) pp -= vg[4 * t] * dW[q + 4 * t] + wg[4 * t] * dV[q + 4 * t];
                }
                pp = tri_quad_sum(pp);
                const double vi = act ? (quad == 0 ? 1.0 : S.v[quad] * scal) : 0.0;
                const double pi = tau * pp;
                double pv = (act && q == 0) ? pi * vi : 0.0;
                pv = tri_wave_sum(pv);
                if (lane == 0) S.red[16 + wave] = pv;
                __syncthreads();
                // S: w = p - K v, K = tau / 2 (p . v)
                double pvs = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) pvs += S.red[16 + w];
                const double K = 0.5 * tau * pvs;
                if (act && q == 0) {
                    Vt[g * TRI_NBP + jc] = vi;
                    Wt[g * TRI_NBP + jc] = fma(-K, vi, pi);
                }
            }
            __syncthreads();
        }
        // reflectors to W; trailing matrix (rows and columns >= j0 + jb)
        // -= V W^T + W V^T in 4 x 4 tiles
        for (int e = tid; e < jb * n; e += nth) {
            const int cc = e / n, g = e - cc * n, j = j0 + cc;
            if (g == j) Ag[j * n + j] = taus[cc];
            else if (g > j + 1) Ag[j * n + g] = Vt[g * TRI_NBP + cc];
        }
        const int t0 = j0 + jb, Lt = n - t0;
        const int nt = (Lt + 3) / 4;
        for (int tile = tid; tile < nt * nt; tile += nth) {
            const int ti = tile / nt, tk = tile - ti * nt;
            const int i0 = t0 + 4 * ti, k0 = t0 + 4 * tk;
            const double* vr[4];
            const double* wr[4];
            const double* vc[4];
            const double* wc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ii = min(i0 + u, n - 1), kk = min(k0 + u, n - 1);
                vr[u] = Vt + ii * TRI_NBP;
                wr[u] = Wt + ii * TRI_NBP;
                vc[u] = Vt + kk * TRI_NBP;
                wc[u] = Wt + kk * TRI_NBP;
            }
            double acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
            for (int cc = 0; cc < jb; ++cc) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = fma(vr[a][cc], wc[b][cc], fma(wr[a][cc], vc[b][cc], acc[a][b]));
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (i0 + a < n && k0 + b < n) Ag[(i0 + a) * n + k0 + b] -= acc[a][b];
        }
        __syncthreads();
    }
    if (tid == 0) {
        S.d[n - 1] = W[(int64_t)(n - 1) * n + n - 1];
        W[(int64_t)(n - 1) * n + n - 1] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += nth) {
        U[i] = S.d[i];
        if (i + 1 < n) U[lu + i] = S.e[i];
    }
}

// Gershgorin bounds of T widened by the bisection tolerance, its norm and
// the pivot floor (the same values in every kernel that calls this).
struct TriBounds {
    double gl, gu, tnorm, pivmin;
};
__device__ __forceinline__ TriBounds tri_bounds(const double* d, const double* e, int n) {
    double emax2 = 0.0;
    for (int i = 0; i + 1 < n; ++i) emax2 = fmax(emax2, e[i] * e[i]);
    double gl = 1e308, gu = -1e308;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        gl = fmin(gl, d[i] - r);
        gu = fmax(gu, d[i] + r);
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    gl -= 2.0 * eps * tnorm + 2.0 * pivmin;
    gu += 2.0 * eps * tnorm + 2.0 * pivmin;
    return {gl, gu, tnorm, pivmin};
}

// The same bounds from the lanes of one wavefront (min and max are exact, so
// the values equal tri_bounds' bit for bit).
__device__ __forceinline__ TriBounds tri_bounds_wave(const double* d, const double* e, int n) {
    const int lane = threadIdx.x & 63;
    double emax2 = 0.0, gl = 1e308, gu = -1e308;
    for (int i = lane; i < n; i += 64) {
        if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        gl = fmin(gl, d[i] - r);
        gu = fmax(gu, d[i] + r);
    }
    for (int o = 32; o > 0; o >>= 1) {
        emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
        gl = fmin(gl, __shfl_xor(gl, o, 64));
        gu = fmax(gu, __shfl_xor(gu, o, 64));
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    gl -= 2.0 * eps * tnorm + 2.0 * pivmin;
    gu += 2.0 * eps * tnorm + 2.0 * pivmin;
    return {gl, gu, tnorm, pivmin};
}

// Eigenvalues k0 .. k1-1 (k-th largest) of T (d, e2 = e^2) into lam[k] by
// multisection: tpe threads (contiguous lanes) per eigenvalue count at the
// tpe interior points that cut the interval into tpe + 1 parts; the first
// point with more than m eigenvalues below it bounds the next interval.
// Every thread of the workgroup must call it.
#ifndef TRI_BISECT_LANES
#define TRI_BISECT_LANES 768
#endif
__device__ __forceinline__ void tri_bisect(const double* d, const double* e2, int n, const TriBounds& tb, int k0,
                                           int k1, double* lam) {
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int cnt = k1 - k0;
    const double eps = 2.220446049250313e-16;
    int tpe = 1;  // tpe * cnt <= lanes: one eigenvalue per group of lanes
    const int lanes = cnt < n ? nth : min(nth, TRI_BISECT_LANES);
    while (tpe < 32 && tpe * 2 * cnt <= lanes) tpe *= 2;
    const int sub = lane % tpe, k = k0 + tid / tpe;
    const unsigned long long gmask = (1ull << tpe) - 1ull;
    const bool act = k < k1;
    const int m = n - 1 - (act ? k : 0);  // k-th largest = ascending index n - 1 - k
    double lo = tb.gl, hi = tb.gu;
    for (int it = 0; it < 200; ++it) {
        const double tol = fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), eps * tb.tnorm) + tb.pivmin;
        const bool more = act && hi - lo > tol;
        if (!__any(more)) break;  // wave-uniform: every ballot sees whole groups
        const double h = (hi - lo) / (double)(tpe + 1);
        bool gt = false;
        if (more) gt = sturm_count(d, e2, n, lo + h * (double)(sub + 1), tb.pivmin) > m;
        const unsigned long long bal = (__ballot(gt) >> (lane - sub)) & gmask;
        if (more) {
            const int sidx = bal ? __ffsll((long long)bal) - 1 : tpe;  // part holding eigenvalue m
            const double nhi = (sidx < tpe) ? lo + h * (double)(sidx + 1) : hi;
            const double nlo = (sidx > 0) ? lo + h * (double)sidx : lo;
            lo = nlo;
            hi = nhi;
        }
    }
    if (act && sub == 0) lam[k] = 0.5 * (lo + hi);
}

// Eigenpairs of the tridiagonal T left by the reduction (diagonal in row 0
// of U, off-diagonal in row 1) into lam (descending) and U (eigenvectors of
// T; the back-transformation applies Q).  On clusters it cannot separate,
// the problem is solved again from Ain by the Jacobi method (info[2] counts
// these; Dm[0] = 1 then tells the back-transformation to skip).
// Dm: n x n global scratch.
__device__ __forceinline__ void tri_eig_body(const double* Ain, int ldin, int n, double* W, double* Dm, double* U,
                                             int lu, double* lam, int* info, int have_lam) {
    __shared__ TriShared S;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    for (int i = tid; i < n; i += nth) {
        S.d[i] = U[i];
        if (i + 1 < n) S.e[i] = U[lu + i];
    }
    if (tid == 0) S.flag = 0;
    __syncthreads();

    // ---- 2. eigenvalues by bisection (unless computed already)
    double* e2 = S.w;
    for (int i = tid; i + 1 < n; i += nth) e2[i] = S.e[i] * S.e[i];
    TriBounds tb = tri_bounds(S.d, S.e, n);
    const double tnorm = tb.tnorm, pivmin = tb.pivmin;
    __syncthreads();
    if (!have_lam) tri_bisect(S.d, e2, n, tb, 0, n, lam);
    __syncthreads();
    // ---- 3. eigenvectors of T, one per thread: column k of U
    if (tnorm > 0.0) {
        for (int k = tid; k < n; k += nth)
            if (!twisted_vec(S.d, S.e, e2, n, lam[k], pivmin, U + k, lu, Dm + k, n, 0, U + k, lu)) S.flag = 1;
        __syncthreads();
        // A vector from step 3 overlaps its neighbour's by about
        // eps ||T|| / gap, which moves a sketch built from eigenpairs weighted
        // by their eigenvalues by about eps |lambda| / gap relative to ||T||.
        // Neighbours closer than 1e-6 |lambda| (and not below 1e-10 ||T|| in
        // size) therefore form clusters, where the vectors may share
        // directions.  Each cluster goes to one
        // wavefront: every member after the first is made orthogonal to the
        // earlier ones (two Gram-Schmidt passes); when too little is left, the
        // vector is recomputed with a twist index of higher |gamma| rank and
        // tried again (Jacobi fallback after 8 tries).
        int* clist = (int*)S.y;  // cluster [start, end) pairs, at most 512
        if (tid == 0) {
            int nc = 0;
            for (int k0 = 0; k0 < n;) {
                int k1 = k0 + 1;
                while (k1 < n) {
                    const double mag = fmax(fabs(lam[k1 - 1]), fabs(lam[k1]));
                    if (!(lam[k1 - 1] - lam[k1] <= 1e-6 * mag && mag >= 1e-10 * tnorm)) break;
                    ++k1;
                }
                if (k1 - k0 > 8) S.flag = 1;  // many equal eigenvalues: the Jacobi method
                if (k1 - k0 > 1) {
                    clist[2 * nc] = k0;
                    clist[2 * nc + 1] = k1;
                    ++nc;
                }
                k0 = k1;
            }
            S.ncl = nc;
        }
        __syncthreads();
        if (!S.flag)
            for (int c = wave; c < S.ncl; c += nw) {
                const int k0 = clist[2 * c], k1 = clist[2 * c + 1];
                for (int m = k0 + 1; m < k1; ++m) {
                    double* zm = U + m;
                    bool ok = false;
                    for (int rank = 0; rank < 8 && !ok; ++rank) {
                        if (rank > 0) {
                            bool fin = true;
                            if (lane == 0)
                                fin = twisted_vec(S.d, S.e, e2, n, lam[m], pivmin, zm, lu, Dm + m, n,
                                                  (m - k0) + rank - 1, zm, lu);
                            __threadfence();
                            __builtin_amdgcn_wave_barrier();
                            if (!__shfl(fin ? 1 : 0, 0, 64)) break;
                        }
                        for (int pass = 0; pass < 2; ++pass)
                            for (int q = k0; q < m; ++q) {
                                double dot = 0.0;
                                for (int i = lane; i < n; i += 64)
                                    dot = fma(U[(int64_t)i * lu + q], zm[(int64_t)i * lu], dot);
                                dot = tri_wave_sum(dot);
                                for (int i = lane; i < n; i += 64)
                                    zm[(int64_t)i * lu] = fma(-dot, U[(int64_t)i * lu + q], zm[(int64_t)i * lu]);
                            }
                        double nrm2 = 0.0;
                        for (int i = lane; i < n; i += 64) nrm2 = fma(zm[(int64_t)i * lu], zm[(int64_t)i * lu], nrm2);
                        nrm2 = tri_wave_sum(nrm2);
                        if (nrm2 > 0.25) {
                            const double inv = 1.0 / sqrt(nrm2);
                            for (int i = lane; i < n; i += 64) zm[(int64_t)i * lu] *= inv;
                            ok = true;
                        }
                        __threadfence();
                        __builtin_amdgcn_wave_barrier();
                    }
                    if (!ok) S.flag = 1;
                }
            }
    } else {  // the zero matrix
        for (int e = tid; e < n * n; e += nth) {
            const int i = e / n, j = e - i * n;
            U[(int64_t)i * lu + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    if (S.flag) {
        if (tid == 0) atomicAdd(&info[2], 1);  // fallback count (diagnostics)
        jacobi_body(Ain, ldin, n, W, Dm, U, lu, lam, info, nullptr);
    }
    __syncthreads();
    // Dm[0] tells the back-transformation whether U still needs Q applied
    if (tid == 0) Dm[0] = S.flag ? 1.0 : 0.0;
}

// U = Q U for the reflectors in W (row j: v_j beyond the super-diagonal,
// W[j][j] = tau_j), skipped when the Jacobi fallback produced U.  One
// wavefront per 4-column strip of U; the sixteen lanes of a row of the
// wavefront take one column, lane p holding rows p, p + 16, ... of it in
// registers, so the product with v_j is 16 (or 32) independent LDS loads and
// FMAs and a DPP row sum, and the update reuses the loaded v.  The reflectors
// arrive in blocks of tri_rb(n) rows of W through LDS, the next block's loads
// issued before the current block is applied.
constexpr int TRI_SC = 4;
__host__ __device__ constexpr int tri_rb(int n) { return n <= 256 ? 8 : 4; }
__host__ __device__ constexpr int tri_back_lds(int n) { return tri_rb(n) * n; }

template <int NS>
__device__ __forceinline__ void tri_back_strip(const double* W, double* U, int lu, int n, double* vb) {
    const int lane = threadIdx.x, c = lane >> 4, p = lane & 15;  // a row of 16 lanes per column
    const int c0 = blockIdx.x * TRI_SC;
    const bool act = c0 + c < n;
    const int RB = tri_rb(n);
    double z[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int r = p + 16 * u;
        z[u] = (act && r < n) ? U[(int64_t)r * lu + c0 + c] : 0.0;
    }
    double pf[32];  // RB * n <= 2048 = 32 per lane
    int jhi = n - 2;
    if (jhi >= 0) {
        const int jl = max(0, jhi - RB + 1), cnt = (jhi - jl + 1) * n;
        const double* src = W + (int64_t)jl * n;
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            const int e = lane + 64 * t;
            pf[t] = e < cnt ? src[e] : 0.0;
        }
    }
    while (jhi >= 0) {
        const int jlo = max(0, jhi - RB + 1), cnt = (jhi - jlo + 1) * n;
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            const int e = lane + 64 * t;
            if (e < cnt) vb[e] = pf[t];
        }
        __syncthreads();
        if (jlo > 0) {  // the next block, in flight while this one is applied
            const int jh = jlo - 1, jl = max(0, jh - RB + 1), cn = (jh - jl + 1) * n;
            const double* src = W + (int64_t)jl * n;
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                const int e = lane + 64 * t;
                pf[t] = e < cn ? src[e] : 0.0;
            }
        }
        for (int j = jhi; j >= jlo; --j) {
            const double* row = vb + (j - jlo) * n;
            const double tau = row[j];
            if (tau == 0.0) continue;
            // v over rows r > j: 1 at r = j + 1, W[j][r] beyond
            double v[NS];
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int r = p + 16 * u;
                v[u] = (r > j + 1 && r < n) ? row[r] : (r == j + 1 ? 1.0 : 0.0);
            }
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
            for (int u = 0; u < NS; u += 4) {
                a0 = fma(v[u], z[u], a0);
                a1 = fma(v[u + 1], z[u + 1], a1);
                a2 = fma(v[u + 2], z[u + 2], a2);
                a3 = fma(v[u + 3], z[u + 3], a3);
            }
            const double y = tau * tri_row_sum((a0 + a1) + (a2 + a3));
#pragma unroll
            for (int u = 0; u < NS; ++u) z[u] = fma(-v[u], y, z[u]);
        }
        jhi = jlo - 1;
        __syncthreads();
    }
    if (act) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int r = p + 16 * u;
            if (r < n) U[(int64_t)r * lu + c0 + c] = z[u];
        }
    }
}

__device__ __forceinline__ void tri_back_body(const double* W, const double* Dm, double* U, int lu, int n,
                                              double* lds) {
    if (Dm[0] != 0.0) return;
    if (blockIdx.x * TRI_SC >= n) return;
    if (n <= 64) tri_back_strip<4>(W, U, lu, n, lds);
    else if (n <= 128) tri_back_strip<8>(W, U, lu, n, lds);
    else if (n <= 256) tri_back_strip<16>(W, U, lu, n, lds);
    else tri_back_strip<32>(W, U, lu, n, lds);
}

// Task form: the eigen-problem of a shrink / query task (not the
// cooperative ones).
#define TRI_TASK_PROLOGUE                                                   \
    const Task& t = tasks[blockIdx.z];                                      \
    if (t.kind == T_INGEST || (t.flags & TF_COOP_EIG)) return;              \
    const SkDev* s = t.s;                                                   \
    const int n = eig_n(t);                                                 \
    if (n < 1) return;                                                      \
    const bool rnd = t.kind == T_SHRINK_RAND;                               \
    (void)rnd;

// Tasks of order xmin..512 take the multi-workgroup reduction (k_trix.hip).
__device__ __forceinline__ bool tri_by_x(int n, int xmin) { return n >= xmin && n <= TRI_NMAX; }

__global__ __launch_bounds__(1024) void k_tri_reduce(const Task* tasks, int lds_doubles, int blk_ok, int xmin) {
    extern __shared__ double lds[];
    TRI_TASK_PROLOGUE
    if (tri_blocked(n, blk_ok) || tri_by_x(n, xmin)) return;
    tri_reduce_unblk_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], s->slot[S_U],
                          s->sld[S_U], lds, lds_doubles);
}

__global__ __launch_bounds__(1024) void k_tri_reduce_blk(const Task* tasks, int xmin) {
    extern __shared__ double lds[];
    TRI_TASK_PROLOGUE
    if (!tri_blocked(n, 1) || tri_by_x(n, xmin)) return;
    tri_reduce_blk_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], s->slot[S_U],
                        s->sld[S_U], lds);
}

// Eigenvalues of the tasks' T split over the workgroups of blockIdx.x
// (n / gridDim.x each, so several compute units bisect one problem).
__global__ __launch_bounds__(1024) void k_tri_eigval(const Task* tasks) {
    __shared__ double d[TRI_NMAX], e[TRI_NMAX], e2[TRI_NMAX];
    TRI_TASK_PROLOGUE
    const int G = gridDim.x, per = (n + G - 1) / G, k0 = blockIdx.x * per, k1 = min(n, k0 + per);
    if (k0 >= k1) return;
    const double* U = s->slot[S_U];
    const int lu = s->sld[S_U];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        d[i] = U[i];
        if (i + 1 < n) {
            e[i] = U[lu + i];
            e2[i] = e[i] * e[i];
        }
    }
    // workgroup 0 leaves T (d at Dm[1..n], e at Dm[n+1..2n-1]) for the vector
    // kernel, which overwrites U, and clears the fallback flag Dm[0]
    if (blockIdx.x == 0) {
        double* Dm = s->slot[S_EV];
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            Dm[1 + i] = d[i];
            if (i + 1 < n) Dm[1 + n + i] = e[i];
        }
        if (threadIdx.x == 0) Dm[0] = 0.0;
    }
    __syncthreads();
    const TriBounds tb = tri_bounds_wave(d, e, n);
    tri_bisect(d, e2, n, tb, k0, k1, s->slot[S_LAM]);
}

__global__ __launch_bounds__(1024) void k_tri_eig(const Task* tasks, int have_lam) {
    TRI_TASK_PROLOGUE
    tri_eig_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], s->slot[S_EV], s->slot[S_U],
                 s->sld[S_U], s->slot[S_LAM], s->info, have_lam);
}

// Eigenvectors of T for the eigenvalues in lam, split over workgroups of one
// wavefront.  Neighbours closer than 1e-6 |lambda| (and not below 1e-10 ||T||)
// form clusters, as in tri_eig_body; workgroup b takes the clusters that
// start in [b TRI_VPER, (b + 1) TRI_VPER), so a cluster's re-orthogonalisation
// stays in one workgroup.  Two lanes per eigenvalue run the forward and the
// backward pivot recurrences of the twisted factorisation side by side (one
// instruction stream, the direction chosen by the lane), with the pivots in
// LDS; the twist index is the largest index of the smallest |gamma_i| (the
// one tri_eig_body picks); then the two lanes build the vector upwards and
// downwards from the twist.  A cluster of more than 8 or a vector that is not
// finite sets the flag Dm[0], and k_tri_fix solves the problem again by the
// Jacobi method.  The arithmetic of a vector does not depend on the split.
constexpr int TRI_VPER = 8;
constexpr int TRI_VMAX = TRI_VPER + 7;  // a range ends inside a cluster of at most 8
__host__ __device__ constexpr int tri_vec_lds(int n) { return 2 * TRI_VMAX * (n + 1); }

__device__ __forceinline__ bool tri_close(const double* lam, int k, double tnorm) {
    const double mag = fmax(fabs(lam[k - 1]), fabs(lam[k]));
    return lam[k - 1] - lam[k] <= 1e-6 * mag && mag >= 1e-10 * tnorm;
}

__global__ __launch_bounds__(64) void k_tri_vec(const Task* tasks) {
    extern __shared__ double lds[];
    __shared__ double d[TRI_NMAX], e[TRI_NMAX], e2[TRI_NMAX], lam[TRI_NMAX];
    __shared__ unsigned char start[TRI_NMAX + 1];
    __shared__ int rng[2], bad;
    TRI_TASK_PROLOGUE
    const int lane = threadIdx.x;
    const int b0 = blockIdx.x * TRI_VPER;
    if (b0 >= n) return;
    double* Dm = s->slot[S_EV];
    double* U = s->slot[S_U];
    const int lu = s->sld[S_U];
    const double* glam = s->slot[S_LAM];
    for (int i = lane; i < n; i += 64) {
        d[i] = Dm[1 + i];
        if (i + 1 < n) {
            e[i] = Dm[1 + n + i];
            e2[i] = e[i] * e[i];
        }
        lam[i] = glam[i];
    }
    __syncthreads();
    const TriBounds tb = tri_bounds_wave(d, e, n);
    const double tnorm = tb.tnorm, pivmin = tb.pivmin;
    for (int k = lane; k <= n; k += 64) start[k] = (k == 0 || k == n || !tri_close(lam, k, tnorm)) ? 1 : 0;
    __syncthreads();
    if (lane == 0) {
        int lo = b0, hi = min(n, b0 + TRI_VPER);
        while (!start[lo]) ++lo;
        while (!start[hi]) ++hi;
        int flag = 0;
        for (int k = lo, run = 0; k < hi; ++k) {  // cluster lengths inside the range
            run = start[k] ? 1 : run + 1;
            if (run > 8) flag = 1;
        }
        rng[0] = lo;
        rng[1] = hi;
        bad = flag || hi - lo > TRI_VMAX;
    }
    __syncthreads();
    const int lo = rng[0], hi = rng[1], V = hi - lo;
    if (bad) {
        if (lane == 0) Dm[0] = 1.0;
        return;
    }
    if (V <= 0) return;
    if (!(tnorm > 0.0)) {  // the zero matrix: unit vectors
        for (int x = lane; x < V * n; x += 64) {
            const int i = x / V, c = lo + (x - (x / V) * V);
            U[(int64_t)i * lu + c] = (i == c) ? 1.0 : 0.0;
        }
        return;
    }
    const int ns = n + 1;  // odd row stride: the lanes' rows fall in different banks
    const int v = lane >> 1, half = lane & 1;
    const bool act = v < V;
    double* Pp = lds + (int64_t)min(v, V - 1) * ns;           // forward pivots, later the vector
    double* Pm = lds + (int64_t)(TRI_VMAX + min(v, V - 1)) * ns;  // backward pivots
    const double x = lam[lo + min(v, V - 1)];
    // forward (half 0: i = 0 .. n-1) and backward (half 1: i = n-1 .. 0) pivots
    {
        double* P = half ? Pm : Pp;
        int i = half ? n - 1 : 0;
        double q = d[i] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        if (act) P[i] = q;
        for (int st = 1; st < n; ++st) {
            i = half ? n - 1 - st : st;
            q = (d[i] - x) - tri_div(e2[half ? i : i - 1], q);
            if (fabs(q) < pivmin) q = -pivmin;
            if (act) P[i] = q;
        }
    }
    __syncthreads();
    // twist: half 0 scans [0, n/2), half 1 [n/2, n), each keeping the largest
    // index of its smallest |gamma|; the upper half wins ties
    int r;
    {
        const int h = n >> 1, i0 = half ? h : 0, i1 = half ? n : h;
        double gb = 1e308;
        int rb = -1;
        for (int i = i0; i < i1; ++i) {
            const double g = fabs(Pp[i] + Pm[i] - (d[i] - x));
            if (rb < 0 || g <= gb) {
                gb = g;
                rb = i;
            }
        }
        const double go = __shfl_xor(gb, 1, 64);
        const int ro = __shfl_xor(rb, 1, 64);
        if (half) r = (rb >= 0 && (ro < 0 || gb <= go)) ? rb : ro;
        else r = (ro >= 0 && (rb < 0 || go <= gb)) ? ro : rb;
        if (r < 0) r = n - 1;  // no comparable |gamma| (not finite): flagged below
    }
    __syncthreads();
    // z_r = 1; half 0 upwards with the forward pivots, half 1 downwards with
    // the backward ones (vector stored over the forward pivots)
    double nrm = half ? 0.0 : 1.0;
    {
        const int len = half ? n - 1 - r : r;
        double z = 1.0;
        for (int st = 0; st < len; ++st) {
            const int i = half ? r + 1 + st : r - 1 - st;
            z = -tri_div(half ? e[i - 1] : e[i], half ? Pm[i] : Pp[i]) * z;
            if (act) Pp[i] = z;
            nrm = fma(z, z, nrm);
        }
        if (act && !half) Pp[r] = 1.0;
    }
    const double nrm2 = nrm + __shfl_xor(nrm, 1, 64);
    __syncthreads();
    if (act && !(nrm2 < 1e300)) bad = 1;
    {
        const double inv = 1.0 / sqrt(nrm2);
        const int a = half ? r + 1 : 0, bnd = half ? n : r + 1;
        if (act)
            for (int i = a; i < bnd; ++i) Pp[i] *= inv;
    }
    __syncthreads();
    if (bad) {
        if (lane == 0) Dm[0] = 1.0;
        return;
    }
    // clusters: every member after the first made orthogonal to the earlier
    // ones (two Gram-Schmidt passes), recomputed with a twist of higher
    // |gamma| rank when too little is left
    for (int k0 = lo; k0 < hi;) {
        int k1 = k0 + 1;
        while (k1 < hi && !start[k1]) ++k1;
        for (int m = k0 + 1; m < k1; ++m) {
            double* zm = lds + (int64_t)(m - lo) * ns;
            double* pm = lds + (int64_t)(TRI_VMAX + m - lo) * ns;
            bool ok = false;
            for (int rank = 0; rank < 8 && !ok; ++rank) {
                if (rank > 0) {
                    int fin = 1;
                    if (lane == 0)
                        fin = twisted_vec(d, e, e2, n, lam[m], pivmin, zm, 1, pm, 1, (m - k0) + rank - 1, zm, 1);
                    __syncthreads();
                    if (!__shfl(fin, 0, 64)) break;
                }
                for (int pass = 0; pass < 2; ++pass)
                    for (int q = k0; q < m; ++q) {
                        const double* zq = lds + (int64_t)(q - lo) * ns;
                        double dot = 0.0;
                        for (int i = lane; i < n; i += 64) dot = fma(zq[i], zm[i], dot);
                        dot = tri_wave_sum(dot);
                        for (int i = lane; i < n; i += 64) zm[i] = fma(-dot, zq[i], zm[i]);
                        __syncthreads();
                    }
                double nr = 0.0;
                for (int i = lane; i < n; i += 64) nr = fma(zm[i], zm[i], nr);
                nr = tri_wave_sum(nr);
                if (nr > 0.25) {
                    const double inv = 1.0 / sqrt(nr);
                    for (int i = lane; i < n; i += 64) zm[i] *= inv;
                    ok = true;
                }
                __syncthreads();
            }
            if (!ok) {
                if (lane == 0) Dm[0] = 1.0;
                return;
            }
        }
        k0 = k1;
    }
    // columns lo .. hi-1 of U, row by row
    for (int xx = lane; xx < V * n; xx += 64) {
        const int i = xx / V, c = xx - i * V;
        U[(int64_t)i * lu + lo + c] = lds[(int64_t)c * ns + i];
    }
}

// The Jacobi method for a problem whose vector kernel set the flag Dm[0]
// (info[2] counts these; Dm[0] = 1 then tells the back-transformation to
// skip).
__global__ __launch_bounds__(1024) void k_tri_fix(const Task* tasks) {
    TRI_TASK_PROLOGUE
    double* Dm = s->slot[S_EV];
    if (Dm[0] == 0.0) return;
    if (threadIdx.x == 0) atomicAdd(&s->info[2], 1);
    jacobi_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], Dm, s->slot[S_U], s->sld[S_U],
                s->slot[S_LAM], s->info, nullptr);
    __syncthreads();
    if (threadIdx.x == 0) Dm[0] = 1.0;
}

__global__ __launch_bounds__(64) void k_tri_back(const Task* tasks) {
    extern __shared__ double lds[];
    TRI_TASK_PROLOGUE
    tri_back_body(s->slot[S_EA], s->slot[S_EV], s->slot[S_U], s->sld[S_U], n, lds);
}

// Descriptor form (window sketches): A (n x n) -> X (eigenvectors), lam.
__global__ __launch_bounds__(1024) void k_tri_reduce_desc(DescArg<SmallDesc> ds, int lds_doubles, int blk_ok) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n < 1 || tri_blocked(q.n, blk_ok)) return;
    tri_reduce_unblk_body(q.A, q.lda, q.n, q.work, q.X, q.ldx, lds, lds_doubles);
}

__global__ __launch_bounds__(1024) void k_tri_reduce_blk_desc(DescArg<SmallDesc> ds) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (!tri_blocked(q.n, 1)) return;
    tri_reduce_blk_body(q.A, q.lda, q.n, q.work, q.X, q.ldx, lds);
}

__global__ __launch_bounds__(1024) void k_tri_eig_desc(DescArg<SmallDesc> ds) {
    const SmallDesc q = ds.get();
    if (q.n < 1) return;
    tri_eig_body(q.A, q.lda, q.n, q.work, q.work2, q.X, q.ldx, q.lam, q.info, 0);
}

__global__ __launch_bounds__(64) void k_tri_back_desc(DescArg<SmallDesc> ds) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n < 1) return;
    tri_back_body(q.work, q.work2, q.X, q.ldx, q.n, lds);
}

static int g_tri_lds = -1, g_back_ok = 0, g_blk_ok = 0;

static int set_dyn_lds(const void* f, int want_doubles) {
    int dev = 0, maxl = 0;
    hipFuncAttributes a{};
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&a, f) != hipSuccess)
        return 0;
    int dbl = (int)(((size_t)maxl - a.sharedSizeBytes) / sizeof(double));
    if (dbl > want_doubles) dbl = want_doubles;
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(double) * (size_t)dbl)) !=
        hipSuccess)
        dbl = 0;
    return dbl;
}

// Dynamic LDS (doubles): the unblocked reduction up to a 128 x 129 matrix;
// the blocked one its panels at n = 256 (else the unblocked reduction takes
// every size); the back-transformation up to a 256 x 64 strip.
int tri_lds_doubles() {
    if (g_tri_lds < 0) {
        const int a = set_dyn_lds((const void*)k_tri_reduce, 128 * 129);
        const int b = set_dyn_lds((const void*)k_tri_reduce_desc, 128 * 129);
        g_tri_lds = std::min(a, b);
        const int c0 = set_dyn_lds((const void*)k_tri_reduce_blk, tri_blk_lds(256));
        const int c1 = set_dyn_lds((const void*)k_tri_reduce_blk_desc, tri_blk_lds(256));
        g_blk_ok = std::min(c0, c1) >= tri_blk_lds(256) ? 1 : 0;
        const int want = std::max(tri_back_lds(256), tri_back_lds(TRI_NMAX));
        const int c = set_dyn_lds((const void*)k_tri_back, want);
        const int d = set_dyn_lds((const void*)k_tri_back_desc, want);
        g_back_ok = std::min(c, d) >= want ? 1 : 0;
        (void)hipGetLastError();
    }
    return g_tri_lds;
}

// LDS of a back-transformation launch covering sizes up to max_n
static int back_lds(int max_n) {
    int w = 0;
    for (int m : {std::min(max_n, 256), max_n}) w = std::max(w, tri_back_lds(m));
    return w;
}

hipError_t launch_tri_reduce(const Task* tasks, int count, int min_n, int max_n, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 65) return hipErrorInvalidConfiguration;
    const int xmin = trix_min_n();
    // sizes outside the multi-workgroup range
    const bool below_x = min_n < xmin, above_x = max_n > TRI_NMAX;
    const int lo_max = std::min(max_n, xmin - 1);  // largest size the one-workgroup kernels may see
    const bool any_blk = g_blk_ok && below_x && lo_max > 128 && min_n <= 256;
    const bool any_unblk = (below_x && (!g_blk_ok || min_n <= 128 || lo_max > 256)) || above_x;
    const bool any_x = max_n >= xmin && min_n <= TRI_NMAX;
    hipError_t e = hipSuccess;
    if (any_unblk) {
        hipLaunchKernelGGL(k_tri_reduce, dim3(1, 1, (unsigned)count), dim3(1024), sizeof(double) * (size_t)dbl, st,
                           tasks, dbl, g_blk_ok, xmin);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (any_blk) {
        hipLaunchKernelGGL(k_tri_reduce_blk, dim3(1, 1, (unsigned)count), dim3(1024),
                           sizeof(double) * (size_t)tri_blk_lds(std::min(lo_max, 256)), st, tasks, xmin);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (any_x) e = launch_tri_reduce_x(tasks, count, max_n, st);
    return e;
}

// Workgroups that bisect one problem's eigenvalues: n / 8 (8 eigenvalues,
// 32 lanes each, per workgroup), at most 64; SK_TRI_EIGVAL_GROUPS overrides
// (1 leaves the bisection inside the eigenpair kernel).
static int eigval_groups(int max_n) {
    static int v = -2;
    if (v == -2) {
        const char* e = getenv("SK_TRI_EIGVAL_GROUPS");
        v = e ? std::max(1, std::min(64, atoi(e))) : -1;
    }
    if (v > 0) return v;
    return std::max(1, std::min(64, max_n / 8));
}

static int g_vec_ok = -1;

hipError_t launch_tri_eig(const Task* tasks, int count, int max_n, hipStream_t st) {
    const int G = eigval_groups(max_n);
    if (g_vec_ok < 0) {  // SK_TRI_VEC=0 keeps the eigenvectors in the one-workgroup kernel
        const char* env = getenv("SK_TRI_VEC");
        g_vec_ok = (!env || atoi(env) != 0) &&
                   set_dyn_lds((const void*)k_tri_vec, tri_vec_lds(TRI_NMAX)) >= tri_vec_lds(TRI_NMAX);
        (void)hipGetLastError();
    }
    if (G > 1) {
        hipLaunchKernelGGL(k_tri_eigval, dim3((unsigned)G, 1, (unsigned)count), dim3(1024), 0, st, tasks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (g_vec_ok && max_n <= TRI_NMAX) {
            hipLaunchKernelGGL(k_tri_vec, dim3((unsigned)((max_n + TRI_VPER - 1) / TRI_VPER), 1, (unsigned)count),
                               dim3(64), sizeof(double) * (size_t)tri_vec_lds(max_n), st, tasks);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_tri_fix, dim3(1, 1, (unsigned)count), dim3(1024), 0, st, tasks);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL(k_tri_eig, dim3(1, 1, (unsigned)count), dim3(1024), 0, st, tasks, G > 1 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_tri_back(const Task* tasks, int count, int max_n, hipStream_t st) {
    tri_lds_doubles();
    if (!g_back_ok || max_n > TRI_NMAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_tri_back, dim3((unsigned)((max_n + TRI_SC - 1) / TRI_SC), 1, (unsigned)count), dim3(64),
                       sizeof(double) * (size_t)back_lds(max_n), st, tasks);
    return hipGetLastError();
}

// The same for `count` descriptors in device memory, one workgroup (group of
// workgroups for the back-transformation) per descriptor.
hipError_t launch_tri_eig_desc(const SmallDesc* ds, int count, int max_n, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 65 || !g_back_ok || max_n > TRI_NMAX) return hipErrorInvalidConfiguration;
    DescArg<SmallDesc> a{ds, {}};
    hipLaunchKernelGGL(k_tri_reduce_desc, dim3(1, 1, (unsigned)count), dim3(1024), sizeof(double) * (size_t)dbl, st,
                       a, dbl, g_blk_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g_blk_ok && max_n > 128) {
        hipLaunchKernelGGL(k_tri_reduce_blk_desc, dim3(1, 1, (unsigned)count), dim3(1024),
                           sizeof(double) * (size_t)tri_blk_lds(256), st, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_tri_eig_desc, dim3(1, 1, (unsigned)count), dim3(1024), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tri_back_desc, dim3((unsigned)((max_n + TRI_SC - 1) / TRI_SC), 1, (unsigned)count), dim3(64),
                       sizeof(double) * (size_t)back_lds(max_n), st, a);
    return hipGetLastError();
}

hipError_t launch_tri_eig1(const SmallDesc& q, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 65) return hipErrorInvalidConfiguration;
    DescArg<SmallDesc> a{nullptr, q};
    hipLaunchKernelGGL(k_tri_reduce_desc, dim3(1, 1, 1), dim3(1024), sizeof(double) * (size_t)dbl, st, a, dbl,
                       g_blk_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g_blk_ok && q.n > 128 && q.n <= 256) {
        hipLaunchKernelGGL(k_tri_reduce_blk_desc, dim3(1, 1, 1), dim3(1024), sizeof(double) * (size_t)tri_blk_lds(q.n),
                           st, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_tri_eig_desc, dim3(1, 1, 1), dim3(1024), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!g_back_ok || q.n > TRI_NMAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_tri_back_desc, dim3((unsigned)((q.n + TRI_SC - 1) / TRI_SC), 1, 1), dim3(64),
                       sizeof(double) * (size_t)tri_back_lds(q.n), st, a);
    return hipGetLastError();
}

}  // namespace sk
