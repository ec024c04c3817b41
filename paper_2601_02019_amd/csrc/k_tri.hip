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
//   4. U = Q Z by applying the reflectors to column tiles of Z held in LDS.
//
// Eigenvectors from step 3 are accurate to eps ||T|| / gap.  When two
// eigenvalues of non-negligible size lie closer than 1e-9 ||T|| (or a vector
// is not finite), the workgroup solves the problem again with the Jacobi
// method instead, so clusters never cost orthogonality.  Every reduction has
// a fixed order: results repeat bit for bit.
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
    int flag;
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

// Number of eigenvalues of T (d, e2) below x.
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - tri_div(e2[i - 1], q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Returns true when the problem was solved by the Jacobi fallback.
// W: n x n global work (ld n): A when it does not fit LDS, then the
// reflectors (row j holds v_j beyond the super-diagonal, W[j][j] = tau_j).
// Dm: n x n global scratch.  lds: dynamic LDS of lds_doubles doubles.
__device__ void tri_body(const double* Ain, int ldin, int n, double* W, double* Dm, double* U, int lu,
                         double* lam, int* info, double* lds, int lds_doubles) {
    __shared__ TriShared S;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    const bool inl = n * n <= lds_doubles;
    double* A = inl ? lds : W;
    const int la = n;

    double loc = 0.0;
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - i * n;
        const double v = 0.5 * (Ain[(int64_t)i * ldin + j] + Ain[(int64_t)j * ldin + i]);
        A[(int64_t)i * la + j] = v;
        loc = fma(v, v, loc);
    }
    const double fro2 = tri_block_sum(loc, S.red);

    // ---- 1. tridiagonalisation
    for (int j = 0; j + 1 < n; ++j) {
        const int L = n - j - 1;
        double* row = A + (int64_t)j * la + j + 1;
        loc = 0.0;
        for (int i = 1 + tid; i < L; i += nth) loc = fma(row[i], row[i], loc);
        const double xn2 = tri_block_sum(loc, S.red);
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
        }
        if (tau != 0.0) {
            for (int i = tid; i < L; i += nth) S.v[i] = (i == 0) ? 1.0 : row[i] * scal;
            __syncthreads();
            // p = tau A22 v, one wave per row
            for (int i = wave; i < L; i += nw) {
                const double* Ai = A + (int64_t)(j + 1 + i) * la + j + 1;
                double acc = 0.0;
                for (int k = lane; k < L; k += 64) acc = fma(Ai[k], S.v[k], acc);
                for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
                if (lane == 0) S.w[i] = tau * acc;
            }
            __syncthreads();
            loc = 0.0;
            for (int i = tid; i < L; i += nth) loc = fma(S.w[i], S.v[i], loc);
            const double K = 0.5 * tau * tri_block_sum(loc, S.red);
            for (int i = tid; i < L; i += nth) S.w[i] = fma(-K, S.v[i], S.w[i]);
            __syncthreads();
            // A22 -= v w^T + w v^T
            for (int e = tid; e < L * L; e += nth) {
                const int i = e / L, k = e - i * L;
                double* a = A + (int64_t)(j + 1 + i) * la + j + 1 + k;
                *a = *a - (S.v[i] * S.w[k] + S.w[i] * S.v[k]);
            }
            __syncthreads();
            for (int i = 1 + tid; i < L; i += nth) row[i] = S.v[i];
        }
        __syncthreads();
        if (tid == 0) A[(int64_t)j * la + j] = tau;
        __syncthreads();
    }
    if (tid == 0) {
        S.d[n - 1] = A[(int64_t)(n - 1) * la + n - 1];
        A[(int64_t)(n - 1) * la + n - 1] = 0.0;
        S.flag = 0;
    }
    __syncthreads();
    if (inl)  // the reflectors go to global memory; LDS is needed for Z tiles
        for (int e = tid; e < n * n; e += nth) W[e] = lds[e];

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
    // clusters of non-negligible eigenvalues go to the Jacobi method
    for (int k = tid; k + 1 < n; k += nth) {
        const double a = lam[k], b = lam[k + 1];
        if (a - b <= 1e-9 * tnorm && fmax(fabs(a), fabs(b)) >= 1e-6 * tnorm && tnorm > 0.0) S.flag = 1;
    }
    __syncthreads();

    // ---- 3. eigenvectors of T, one per thread: column k of U
    if (!S.flag && tnorm > 0.0) {
        for (int k = tid; k < n; k += nth) {
            const double x = lam[k];
            // forward pivots D+ into U[i][k]
            double q = S.d[0] - x;
            if (fabs(q) < pivmin) q = -pivmin;
            U[k] = q;
            for (int i = 1; i < n; ++i) {
                q = (S.d[i] - x) - tri_div(e2[i - 1], q);
                if (fabs(q) < pivmin) q = -pivmin;
                U[(int64_t)i * lu + k] = q;
            }
            // backward pivots D- into Dm[i][k]; twist index r where |gamma| is least
            double qb = S.d[n - 1] - x;
            if (fabs(qb) < pivmin) qb = -pivmin;
            Dm[(int64_t)(n - 1) * n + k] = qb;
            int r = n - 1;
            double gbest = fabs(U[(int64_t)(n - 1) * lu + k] + qb - (S.d[n - 1] - x));
            for (int i = n - 2; i >= 0; --i) {
                qb = (S.d[i] - x) - tri_div(e2[i], qb);
                if (fabs(qb) < pivmin) qb = -pivmin;
                Dm[(int64_t)i * n + k] = qb;
                const double g = fabs(U[(int64_t)i * lu + k] + qb - (S.d[i] - x));
                if (g < gbest) {
                    gbest = g;
                    r = i;
                }
            }
            // z_r = 1; upwards with the forward pivots, downwards with the backward ones
            double z = 1.0, nrm2 = 1.0;
            for (int i = r - 1; i >= 0; --i) {
                z = -tri_div(S.e[i], U[(int64_t)i * lu + k]) * z;
                U[(int64_t)i * lu + k] = z;
                nrm2 = fma(z, z, nrm2);
            }
            U[(int64_t)r * lu + k] = 1.0;
            z = 1.0;
            for (int i = r + 1; i < n; ++i) {
                z = -tri_div(S.e[i - 1], Dm[(int64_t)i * n + k]) * z;
                U[(int64_t)i * lu + k] = z;
                nrm2 = fma(z, z, nrm2);
            }
            if (!(nrm2 < 1e300)) S.flag = 1;  // overflow or NaN: fall back
            const double inv = 1.0 / sqrt(nrm2);
            for (int i = 0; i < n; ++i) U[(int64_t)i * lu + k] *= inv;
        }
    } else if (tnorm == 0.0) {  // the zero matrix
        for (int e = tid; e < n * n; e += nth) {
            const int i = e / n, j = e - i * n;
            U[(int64_t)i * lu + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    if (S.flag) {
        jacobi_body(Ain, ldin, n, W, Dm, U, lu, lam, info, nullptr);
        return;
    }

    // ---- 4. U = Q Z: H_0 ... H_{n-2} applied right-to-left to column tiles in LDS
    int cb = lds_doubles / n;
    if (cb > 64) cb = 64;
    if (cb > n) cb = n;
    const int groups = nth / cb;  // row groups per column
    for (int c0 = 0; c0 < n; c0 += cb) {
        const int nc = min(cb, n - c0);
        for (int e = tid; e < n * nc; e += nth) {
            const int i = e / nc, c = e - i * nc;
            lds[i * cb + c] = U[(int64_t)i * lu + c0 + c];
        }
        __syncthreads();
        for (int j = n - 2; j >= 0; --j) {
            const double tau = W[(int64_t)j * n + j];
            if (tau == 0.0) continue;
            const int L = n - j - 1;
            for (int i = tid; i < L; i += nth) S.v[i] = (i == 0) ? 1.0 : W[(int64_t)j * n + j + 1 + i];
            __syncthreads();
            const int c = tid % cb, g = tid / cb;
            if (g < groups && c < nc) {
                double acc = 0.0;
                for (int i = g; i < L; i += groups) acc = fma(S.v[i], lds[(j + 1 + i) * cb + c], acc);
                S.y[g * cb + c] = acc;
            }
            __syncthreads();
            if (tid < nc) {
                double acc = 0.0;
                for (int gg = 0; gg < groups; ++gg) acc += S.y[gg * cb + tid];
                S.w[tid] = tau * acc;
            }
            __syncthreads();
            for (int e = tid; e < L * nc; e += nth) {
                const int i = e / nc, cc = e - i * nc;
                lds[(j + 1 + i) * cb + cc] -= S.v[i] * S.w[cc];
            }
            __syncthreads();
        }
        for (int e = tid; e < n * nc; e += nth) {
            const int i = e / nc, c = e - i * nc;
            U[(int64_t)i * lu + c0 + c] = lds[i * cb + c];
        }
        __syncthreads();
    }
    (void)fro2;
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

// Descriptor form (window sketches): A (n x n) -> X (eigenvectors), lam.
__global__ __launch_bounds__(1024) void k_tri_eig_desc(DescArg<SmallDesc> ds, int lds_doubles) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n < 1) return;
    tri_body(q.A, q.lda, q.n, q.work, q.work2, q.X, q.ldx, q.lam, q.info, lds, lds_doubles);
}

static int g_tri_lds = -1;

// Dynamic LDS (doubles) of the tridiagonal kernels: the device limit less
// their static LDS, at most 128 x 128.
int tri_lds_doubles() {
    if (g_tri_lds < 0) {
        int dev = 0, maxl = 0;
        hipFuncAttributes a{}, b{};
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            hipFuncGetAttributes(&a, (const void*)k_tri_eig) == hipSuccess &&
            hipFuncGetAttributes(&b, (const void*)k_tri_eig_desc) == hipSuccess) {
            const size_t st = a.sharedSizeBytes > b.sharedSizeBytes ? a.sharedSizeBytes : b.sharedSizeBytes;
            int dbl = (int)(((size_t)maxl - st) / sizeof(double));
            if (dbl > 128 * 128) dbl = 128 * 128;
            const size_t bytes = sizeof(double) * (size_t)dbl;
            if (hipFuncSetAttribute((const void*)k_tri_eig, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess ||
                hipFuncSetAttribute((const void*)k_tri_eig_desc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
                dbl = 0;
            g_tri_lds = dbl;
        } else {
            g_tri_lds = 0;
        }
        (void)hipGetLastError();
    }
    return g_tri_lds;
}

hipError_t launch_tri_eig(const Task* tasks, int count, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 64) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_tri_eig, dim3(1, 1, (unsigned)count), dim3(1024), sizeof(double) * (size_t)dbl, st, tasks,
                       dbl);
    return hipGetLastError();
}

hipError_t launch_tri_eig1(const SmallDesc& q, hipStream_t st) {
    const int dbl = tri_lds_doubles();
    if (dbl < 64 * 64) return hipErrorInvalidConfiguration;
    DescArg<SmallDesc> a{nullptr, q};
    hipLaunchKernelGGL(k_tri_eig_desc, dim3(1, 1, 1), dim3(1024), sizeof(double) * (size_t)dbl, st, a, dbl);
    return hipGetLastError();
}

}  // namespace sk
