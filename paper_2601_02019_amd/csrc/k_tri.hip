// k_tri.hip -- symmetric eigen-decomposition of the shrink's core (the eigen
// step of Algorithm "Simultaneous Iteration" on the k x k Rayleigh-Ritz
// matrix; the exact FD shrink's eigen-decomposition of the 2 ell x 2 ell
// buffer Gram, Sec. 2.3) by one workgroup per problem:
//
//   1. Householder tridiagonalisation A = Q T Q^T (unblocked; A in LDS when
//      it fits, else in the global work matrix, which then stays in L2);
//   2. eigenvalues of T by bisection on Sturm counts, one eigenvalue per
//      thread, to absolute accuracy eps ||T||;
//   3. eigenvectors of T by a twisted factorisation at each eigenvalue (the
//      forward and backward pivots of T - lambda I meet at the index where
//      the twist is smallest; the vector follows from one pass each way),
//      one eigenvector per thread;
//   4. U = Q Z by a second kernel: one wavefront per 64-column strip of Z
//      applies the reflectors from the last to the first (lane = column, so
//      the products with v_j need no cross-lane reduction).
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
    double red[16];
    double y[1024];
    int flag, ncl;
};

__device__ __forceinline__ double tri_block_sum(double x, double* red) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

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
    for (int i = n - 2; i >= 0; --i) {
        qb = (d[i] - x) - tri_div(e2[i], qb);
        if (fabs(qb) < pivmin) qb = -pivmin;
        Pm[(int64_t)i * sm] = qb;
        const double g = fabs(Pp[(int64_t)i * sp] + qb - (d[i] - x));
        if (g < gbest) {
            gbest = g;
            r = i;
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
    for (int i = r - 1; i >= 0; --i) {
        z = -tri_div(e[i], Pp[(int64_t)i * sp]) * z;
        Z[(int64_t)i * sz] = z;
        nrm2 = fma(z, z, nrm2);
    }
    Z[(int64_t)r * sz] = 1.0;
    z = 1.0;
    for (int i = r + 1; i < n; ++i) {
        z = -tri_div(e[i - 1], Pm[(int64_t)i * sm]) * z;
        Z[(int64_t)i * sz] = z;
        nrm2 = fma(z, z, nrm2);
    }
    if (!(nrm2 < 1e300)) return false;
    const double inv = 1.0 / sqrt(nrm2);
    for (int i = 0; i < n; ++i) Z[(int64_t)i * sz] *= inv;
    return true;
}

// Returns true when the problem was solved by the Jacobi fallback.
// W: n x n global work (ld n): A when it does not fit LDS, then the
// reflectors (row j holds v_j beyond the super-diagonal, W[j][j] = tau_j).
// Dm: n x n global scratch.  lds: dynamic LDS of lds_doubles doubles.
__device__ void tri_body(const double* Ain, int ldin, int n, double* W, double* Dm, double* U, int lu,
                         double* lam, int* info, double* lds, int lds_doubles) {
    __shared__ TriShared S;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    // A in LDS (row stride n + 1: the rows of a column map to different banks)
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
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
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
                acc += __shfl_xor(acc, 1, 64);
                acc += __shfl_xor(acc, 2, 64);
                if (i < L && sub == 0) {
                    S.w[i] = tau * acc;
                    S.y[i] = tau * acc * S.v[i];
                }
            } else {  // one wave per row
                for (int i = wave; i < L; i += nw) {
                    const double* Ai = A22 + (int64_t)i * la;
                    double acc = 0.0;
                    for (int k = lane; k < L; k += 64) acc = fma(Ai[k], S.v[k], acc);
                    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
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
                for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
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
                for (int off = 32; off > 0; off >>= 1) nx += __shfl_xor(nx, off, 64);
                if (lane == 0) S.red[1] = nx;
            }
        } else if (wave == 0) {  // no reflection: the next column as it stands
            double acc = 0.0;
            for (int k = 2 + lane; k < L; k += 64) acc = fma(A22[k], A22[k], acc);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) S.red[1] = acc;
        }
        __syncthreads();
    }
    if (tid == 0) {
        S.d[n - 1] = A[(int64_t)(n - 1) * la + n - 1];
        A[(int64_t)(n - 1) * la + n - 1] = 0.0;
        S.flag = 0;
    }
    __syncthreads();
    if (inl)  // the reflectors (ld n) for the back-transformation
        for (int e = tid; e < n * n; e += nth) {
            const int i = e / n, k = e - i * n;
            W[e] = lds[(int64_t)i * la + k];
        }

    // ---- 2. eigenvalues by bisection
    double emax2 = 0.0;
    for (int i = 0; i + 1 < n; ++i) emax2 = fmax(emax2, S.e[i] * S.e[i]);
    double* e2 = S.w;
    for (int i = tid; i + 1 < n; i += nth) e2[i] = S.e[i] * S.e[i];
    double gl = 1e308, gu = -1e308;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(S.e[i - 1]) : 0.0) + (i + 1 < n ? fabs(S.e[i]) : 0.0);
        gl = fmin(gl, S.d[i] - r);
        gu = fmax(gu, S.d[i] + r);
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    gl -= 2.0 * eps * tnorm + 2.0 * pivmin;
    gu += 2.0 * eps * tnorm + 2.0 * pivmin;
    __syncthreads();
    // multisection: tpe threads (contiguous lanes) per eigenvalue count at the
    // tpe interior points that cut the interval into tpe + 1 parts; the first
    // point with more than m eigenvalues below it bounds the next interval
    int tpe = 1;  // tpe * n <= nth: one eigenvalue per group of lanes
    while (tpe < 32 && tpe * 2 * n <= nth) tpe *= 2;
    {
        const int sub = lane % tpe, k = tid / tpe;
        const unsigned long long gmask = (1ull << tpe) - 1ull;
        const bool act = k < n;
        const int m = n - 1 - (act ? k : 0);  // k-th largest = ascending index n - 1 - k
        double lo = gl, hi = gu;
        for (int it = 0; it < 200; ++it) {
            const double tol = fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), eps * tnorm) + pivmin;
            const bool more = act && hi - lo > tol;
            if (!__any(more)) break;  // wave-uniform: every ballot sees whole groups
            const double h = (hi - lo) / (double)(tpe + 1);
            bool gt = false;
            if (more) gt = sturm_count(S.d, e2, n, lo + h * (double)(sub + 1), pivmin) > m;
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
                                for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
                                for (int i = lane; i < n; i += 64)
                                    zm[(int64_t)i * lu] = fma(-dot, U[(int64_t)i * lu + q], zm[(int64_t)i * lu]);
                            }
                        double nrm2 = 0.0;
                        for (int i = lane; i < n; i += 64) nrm2 = fma(zm[(int64_t)i * lu], zm[(int64_t)i * lu], nrm2);
                        for (int off = 32; off > 0; off >>= 1) nrm2 += __shfl_xor(nrm2, off, 64);
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
// W[j][j] = tau_j): a workgroup of four wavefronts per 64-column strip (lane
// = column), the rows of each reflector split between the wavefronts; the
// strip lives in LDS when it fits.  Skipped when the Jacobi fallback
// produced U.
__device__ void tri_back_body(const double* W, const double* Dm, double* U, int lu, int n, double* lds,
                              int lds_doubles) {
    __shared__ double vs[TRI_NMAX];
    __shared__ double part[2][4][64];
    if (Dm[0] != 0.0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c0 = blockIdx.x * 64;
    if (c0 >= n) return;
    const int nc = min(64, n - c0);
    const bool act = lane < nc;
    const bool inl = n * 64 <= lds_doubles;
    // the strip: LDS when it fits, else the columns of U in place (idle lanes
    // then work on a clamped column and do not write it)
    double* Z = inl ? lds : U + c0;
    const int lz = inl ? 64 : lu;
    const int col = inl ? lane : (act ? lane : 0);
    const bool wr = inl || act;
    if (inl)
        for (int i = wave; i < n; i += 4) Z[i * 64 + lane] = act ? U[(int64_t)i * lu + c0 + lane] : 0.0;
    int buf = 0;
    for (int j = n - 2; j >= 0; --j) {
        const double tau = W[(int64_t)j * n + j];
        if (tau == 0.0) continue;
        const int L = n - j - 1;
        __syncthreads();  // the previous reflector is done with vs
        for (int i = tid; i < L; i += 256) vs[i] = (i == 0) ? 1.0 : W[(int64_t)j * n + j + 1 + i];
        __syncthreads();
        double* z = Z + (int64_t)(j + 1) * lz + col;
        double y0 = 0.0, y1 = 0.0;
        int i = wave;
        for (; i + 4 < L; i += 8) {
            y0 = fma(vs[i], z[(int64_t)i * lz], y0);
            y1 = fma(vs[i + 4], z[(int64_t)(i + 4) * lz], y1);
        }
        for (; i < L; i += 4) y0 = fma(vs[i], z[(int64_t)i * lz], y0);
        part[buf][wave][lane] = y0 + y1;
        __syncthreads();
        const double y = tau * ((part[buf][0][lane] + part[buf][1][lane]) + (part[buf][2][lane] + part[buf][3][lane]));
        buf ^= 1;  // the next reflector writes the other buffer: no barrier before its partials
        if (wr)
            for (int r = wave; r < L; r += 4) z[(int64_t)r * lz] = fma(-vs[r], y, z[(int64_t)r * lz]);
    }
    __syncthreads();
    if (inl && act)
        for (int i = wave; i < n; i += 4) U[(int64_t)i * lu + c0 + lane] = Z[i * 64 + lane];
}

// Task form: the eigen-problem of a shrink / query task (not the
// cooperative ones).
__global__ __launch_bounds__(1024) void k_tri_eig(const Task* tasks, int lds_doubles) {
    extern __shared__ double lds[];
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST || (t.flags & TF_COOP_EIG)) return;
    const SkDev* s = t.s;
    const int n = eig_n(t);
    if (n < 1) return;
    const bool rnd = t.kind == T_SHRINK_RAND;
    tri_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], s->slot[S_EV], s->slot[S_U],
             s->sld[S_U], s->slot[S_LAM], s->info, lds, lds_doubles);
}

__global__ __launch_bounds__(256) void k_tri_back(const Task* tasks, int lds_doubles) {
    extern __shared__ double lds[];
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST || (t.flags & TF_COOP_EIG)) return;
    const SkDev* s = t.s;
    tri_back_body(s->slot[S_EA], s->slot[S_EV], s->slot[S_U], s->sld[S_U], eig_n(t), lds, lds_doubles);
}

__global__ __launch_bounds__(256) void k_tri_back_desc(DescArg<SmallDesc> ds, int lds_doubles) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n < 1) return;
    tri_back_body(q.work, q.work2, q.X, q.ldx, q.n, lds, lds_doubles);
}

// Descriptor form (window sketches): A (n x n) -> X (eigenvectors), lam.
__global__ __launch_bounds__(1024) void k_tri_eig_desc(DescArg<SmallDesc> ds, int lds_doubles) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n < 1) return;
    tri_body(q.A, q.lda, q.n, q.work, q.work2, q.X, q.ldx, q.lam, q.info, lds, lds_doubles);
}

static int g_tri_lds = -1, g_back_lds = -1;

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

// Dynamic LDS (doubles) of the tridiagonalisation kernels: up to a 128 x 129
// matrix; of the back-transformation kernels: up to a 256 x 64 strip.
int tri_lds_doubles() {
    if (g_tri_lds < 0) {
        const int a = set_dyn_lds((const void*)k_tri_eig, 128 * 129);
        const int b = set_dyn_lds((const void*)k_tri_eig_desc, 128 * 129);
        g_tri_lds = a < b ? a : b;
        const int c = set_dyn_lds((const void*)k_tri_back, 256 * 64);
        const int d = set_dyn_lds((const void*)k_tri_back_desc, 256 * 64);
        g_back_lds = c < d ? c : d;
        (void)hipGetLastError();
    }
    return g_tri_lds;
}

static int back_lds(int max_n) {
    tri_lds_doubles();
    const int want = max_n * 64;
    return want <= g_back_lds ? want : 0;
}

hipError_t launch_tri_eig(const Task* tasks, int count, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 65) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_tri_eig, dim3(1, 1, (unsigned)count), dim3(1024), sizeof(double) * (size_t)dbl, st, tasks,
                       dbl);
    return hipGetLastError();
}

hipError_t launch_tri_back(const Task* tasks, int count, int max_n, hipStream_t st) {
    const int bl = back_lds(max_n);
    hipLaunchKernelGGL(k_tri_back, dim3((unsigned)((max_n + 63) / 64), 1, (unsigned)count), dim3(256),
                       sizeof(double) * (size_t)bl, st, tasks, bl);
    return hipGetLastError();
}

hipError_t launch_tri_eig1(const SmallDesc& q, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 65) return hipErrorInvalidConfiguration;
    DescArg<SmallDesc> a{nullptr, q};
    hipLaunchKernelGGL(k_tri_eig_desc, dim3(1, 1, 1), dim3(1024), sizeof(double) * (size_t)dbl, st, a, dbl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bl = back_lds(q.n);
    hipLaunchKernelGGL(k_tri_back_desc, dim3((unsigned)((q.n + 63) / 64), 1, 1), dim3(256), sizeof(double) * (size_t)bl,
                       st, a, bl);
    return hipGetLastError();
}

}  // namespace sk
