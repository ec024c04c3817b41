// k_core.hip -- the FP64 core of the shrink (gfx950).
//
//   k_core_gemm   small FP64 products between scratch slots (power steps
//                 G Q, Rayleigh-Ritz Q^T G Q, CholeskyQR products, Z = Q U)
//   k_cholinv     Cholesky of the basis Gram W = Y^T Y with rank dropping,
//                 then L^{-1} (CholeskyQR: Q = Y L^{-T})
//   k_jacobi      symmetric eigen-decomposition by parallel-ordered cyclic
//                 Jacobi: G = C C^T (exact shrink, size m) or the k x k
//                 Rayleigh-Ritz matrix (the eigen step of Algorithm
//                 "Simultaneous Iteration"); eigenvalues sorted descending with vectors
//   k_threshold   delta = ell-th eigenvalue; T = diag(f) Z^T with
//                 f_i = sqrt(max(lambda_i - delta, 0) / lambda_i)
//                 (Sec. 2.3 FD shrink; the FD reduce of Algorithm "AeroSketch: Update")
//
// All arithmetic is FP64; reductions are in a fixed order, so results do not
// depend on how many tasks share a launch.
#include "k_jacobi_body.h"
#include "sk_device.h"
#include "sk_kernels.h"

namespace sk {

// ------------------------------------------------------------ small GEMM
// C[M x N] = op(A) op(B), op(A) = A or A^T (TA), op(B) = B or B^T (TB).
// dims: bits [1:0] M, [3:2] N, [5:4] K select 0 -> task m, 1 -> k,
// 2 -> the eigen-problem size.
__device__ __forceinline__ int dim_sel(const Task& t, int code) {
    return code == 0 ? t.m : (code == 1 ? t.s->k : eig_n(t));
}

// TS x TS output tile per workgroup of 256 threads, each thread a (TS/16)^2
// register block; every output element accumulates over k in order, so the
// result does not depend on TS (small products take TS = 32 for 4x the
// workgroups).
template <bool TA, bool TB, int TS>
__global__ __launch_bounds__(256) void k_core_gemm(const Task* tasks, int sa, int sb, int sc,
                                                   int dims) {
    constexpr int RB = TS / 16;  // register block edge
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST) return;
    const SkDev* s = t.s;
    const int M = dim_sel(t, dims & 3), N = dim_sel(t, (dims >> 2) & 3), K = dim_sel(t, (dims >> 4) & 3);
    const int r0 = blockIdx.y * TS, c0 = blockIdx.x * TS;
    if (r0 >= M || c0 >= N) return;
    const double* A = s->slot[sa];
    const double* B = s->slot[sb];
    double* C = s->slot[sc];
    const int lda = s->sld[sa], ldb = s->sld[sb], ldc = s->sld[sc];
    __shared__ double As[16][TS + 2];
    __shared__ double Bs[16][TS + 2];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[RB][RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = 0.0;
    // the next 16-deep slices of A and B are loaded into registers while the
    // current ones are multiplied out of LDS
    double pa[RB], pb[RB];
    auto fetch = [&](int kk) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int e = tid + 256 * u;  // 16 * TS elements of a TS x 16 slice
            if (!TA) {  // A row-major: consecutive threads walk k
                const int r = e >> 4, k = e & 15;
                pa[u] = (r0 + r < M && kk + k < K) ? A[(int64_t)(r0 + r) * lda + kk + k] : 0.0;
            } else {    // A^T: consecutive threads walk the row index of op(A)
                const int r = e % TS, k = e / TS;
                pa[u] = (r0 + r < M && kk + k < K) ? A[(int64_t)(kk + k) * lda + r0 + r] : 0.0;
            }
            if (!TB) {
                const int c = e % TS, k = e / TS;
                pb[u] = (c0 + c < N && kk + k < K) ? B[(int64_t)(kk + k) * ldb + c0 + c] : 0.0;
            } else {
                const int c = e >> 4, k = e & 15;
                pb[u] = (c0 + c < N && kk + k < K) ? B[(int64_t)(c0 + c) * ldb + kk + k] : 0.0;
            }
        }
    };
    if (K > 0) fetch(0);
    for (int kk = 0; kk < K; kk += 16) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int e = tid + 256 * u;
            if (!TA) As[e & 15][e >> 4] = pa[u];
            else As[e / TS][e % TS] = pa[u];
            if (!TB) Bs[e / TS][e % TS] = pb[u];
            else Bs[e & 15][e >> 4] = pb[u];
        }
        __syncthreads();
        if (kk + 16 < K) fetch(kk + 16);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            double a[RB], b[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                a[i] = As[k][ty * RB + i];
                b[i] = Bs[k][tx * RB + i];
            }
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < RB; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int r = r0 + ty * RB + i;
        if (r >= M) continue;
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int c = c0 + tx * RB + j;
            if (c < N) C[(int64_t)r * ldc + c] = acc[i][j];
        }
    }
}

// Index pair (a <= b) of the e-th entry of an upper triangle of order n,
// counted row by row over (b, a) with a <= b: e = b (b + 1) / 2 + a.
__device__ __forceinline__ void tri_index(int e, int& a, int& b) {
    int bb = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((bb + 1) * (bb + 2) / 2 <= e) ++bb;
    while (bb * (bb + 1) / 2 > e) --bb;
    b = bb;
    a = e - bb * (bb + 1) / 2;
}

// ------------------------------------------------------------ Cholesky
// W (k x k, slot sw) -> X = L^{-1} (slot sx, lower), L L^T = W.  A pivot at
// or below 1e-14 of its original diagonal marks the column as numerically
// dependent: its row and column of X are zero, so the basis Q = Y X^T gets a
// zero column there and the spanned subspace keeps only the independent part.

// Cholesky-inverse of one n x n matrix by the whole workgroup; L is the
// n x n work matrix (LDS or global).
__device__ void cholinv_body(const double* W, int ldw, double* X, int ldx, int n, double* L) {
    const int ldl = n;
    __shared__ double diag0[512];
    __shared__ int drop[512];
    __shared__ double dj_sh;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e % n;
        L[(int64_t)i * ldl + j] = (j <= i) ? 0.5 * (W[(int64_t)i * ldw + j] + W[(int64_t)j * ldw + i]) : 0.0;
        if (i == j) diag0[i] = W[(int64_t)i * ldw + i];
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double piv = L[(int64_t)j * ldl + j];
            const bool ok = piv > 1e-14 * diag0[j] && piv > 1e-300;
            drop[j] = ok ? 0 : 1;
            dj_sh = ok ? sqrt(piv) : 0.0;
            L[(int64_t)j * ldl + j] = dj_sh;
        }
        __syncthreads();
        const double dj = dj_sh;
        const bool dr = drop[j] != 0;
        for (int i = j + 1 + tid; i < n; i += nth) {
            double* p = &L[(int64_t)i * ldl + j];
            *p = dr ? 0.0 : *p / dj;
        }
        __syncthreads();
        const int rem = n - j - 1;
        if (!dr && rem > 0) {
            const int cnt = rem * (rem + 1) / 2;
            for (int e = tid; e < cnt; e += nth) {
                int a, b;
                tri_index(e, a, b);          // a <= b
                const int l = j + 1 + a, i = j + 1 + b;  // l <= i
                L[(int64_t)i * ldl + l] -= L[(int64_t)i * ldl + j] * L[(int64_t)l * ldl + j];
            }
        }
        __syncthreads();
    }
    // X = L^{-1}: row i from rows < i (forward substitution, columns in parallel)
    for (int i = 0; i < n; ++i) {
        const double lii = L[(int64_t)i * ldl + i];
        for (int c = tid; c < n; c += nth) {
            double v = 0.0;
            if (c <= i && !drop[i]) {
                double acc = (c == i) ? 1.0 : 0.0;
                for (int l = c; l < i; ++l) acc -= L[(int64_t)i * ldl + l] * X[(int64_t)l * ldx + c];
                v = acc / lii;
            }
            X[(int64_t)i * ldx + c] = v;
        }
        __syncthreads();
    }
}

template <bool LDS>
__global__ __launch_bounds__(1024) void k_cholinv(const Task* tasks, int sw, int sx, int lds_max) {
    extern __shared__ double lds[];
    const Task& t = tasks[blockIdx.z];
    if (t.kind != T_SHRINK_RAND || (t.flags & (TF_COOP_CHOL | TF_X_CHOL))) return;
    const SkDev* s = t.s;
    const int n = s->k;
    if (LDS != (n <= lds_max)) return;
    cholinv_body(s->slot[sw], s->sld[sw], s->slot[sx], s->sld[sx], n, LDS ? lds : s->slot[S_EA]);
}

// Descriptor form: X = chol(W)^{-1} for each descriptor (blockIdx.z).
template <bool LDS>
__global__ __launch_bounds__(1024) void k_cholinv_desc(DescArg<SmallDesc> ds, int lds_max) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n <= 0 || LDS != (q.n <= lds_max)) return;
    cholinv_body(q.A, q.lda, q.X, q.ldx, q.n, LDS ? lds : q.work);
}

template <bool LDS>
__global__ __launch_bounds__(1024) void k_jacobi(const Task* tasks, int lds_max, int lds_doubles) {
    extern __shared__ double lds[];
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST || (t.flags & TF_COOP_EIG)) return;
    const SkDev* s = t.s;
    const int n = eig_n(t);
    if (LDS != (n <= lds_max)) return;
    const bool rnd = t.kind == T_SHRINK_RAND;
    // Vt joins A in LDS only when both fit in what this launch allocated
    double* vt = (LDS && 2 * n * n <= lds_doubles) ? lds + n * n : nullptr;
    jacobi_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, LDS ? lds : s->slot[S_EA],
                s->slot[S_EV], s->slot[S_U], s->sld[S_U], s->slot[S_LAM], s->info, vt);
}

// Descriptor form: eigen-decomposition of A (n x n) into U / lam.
template <bool LDS>
__global__ __launch_bounds__(1024) void k_jacobi_desc(DescArg<SmallDesc> ds, int lds_max, int lds_doubles) {
    extern __shared__ double lds[];
    const SmallDesc q = ds.get();
    if (q.n <= 0 || LDS != (q.n <= lds_max)) return;
    double* vt = (LDS && 2 * q.n * q.n <= lds_doubles) ? lds + q.n * q.n : nullptr;
    jacobi_body(q.A, q.lda, q.n, LDS ? lds : q.work, q.work2, q.X, q.ldx, q.lam, q.info, vt);
}

// ------------------------------------------------------------ threshold
// T (ell x m) = diag(f) Z^T with Z = U (exact) or Q U (randomized);
// delta = lambda_ell (0 when fewer than ell eigenvalues); rows i >= min(n, ell)
// and rows with f = 0 are zero.
__global__ __launch_bounds__(256) void k_threshold(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST) return;
    const SkDev* s = t.s;
    const int n = eig_n(t), m = t.m, ell = s->ell;
    const double* lam = s->slot[S_LAM];
    const bool rnd = t.kind == T_SHRINK_RAND;
    const double* Z = s->slot[rnd ? S_Z : S_U];
    const int ldz = s->sld[rnd ? S_Z : S_U];
    double* T = s->slot[S_T];
    const int ldt = s->sld[S_T];
    const double delta = (n >= ell) ? fmax(lam[ell - 1], 0.0) : 0.0;
    const int keep = n < ell ? n : ell;
    const double lmax = fmax(lam[0], 0.0);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < ell * m; e += gridDim.x * 256) {
        const int i = e / m, j = e % m;
        double f = 0.0;
        if (i < keep) {
            const double li = lam[i];
            if (li > 1e-300 && li > 1e-30 * lmax && li - delta > 0.0) f = sqrt((li - delta) / li);
        }
        T[(int64_t)i * ldt + j] = (i < keep) ? f * Z[(int64_t)j * ldz + i] : 0.0;
    }
}

// ------------------------------------------------------------ launchers
// Largest n whose n x n FP64 matrix fits the dynamic LDS a kernel may take
// (device limit minus the kernel's static LDS), capped at 128.
static int g_jac_lds = -1, g_chol_lds = -1;

static int lds_cap(const void* f) {
    int dev = 0, maxsh = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, f) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int avail = maxsh - (int)fa.sharedSizeBytes;
    int n = 0;
    while ((n + 2) <= 128 && 8 * (n + 2) * (n + 2) <= avail) n += 2;
    if (n > 0 && 8 * n * n > 65536) {
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 8 * n * n) != hipSuccess) {
            (void)hipGetLastError();
            while (n > 0 && 8 * n * n > 65536) n -= 2;
        }
    }
    return n;
}

static void init_lds_caps() {
    if (g_jac_lds < 0) {
        const int a = lds_cap((const void*)k_jacobi<true>), b = lds_cap((const void*)k_jacobi_desc<true>);
        g_jac_lds = a < b ? a : b;
    }
    if (g_chol_lds < 0) {
        const int a = lds_cap((const void*)k_cholinv<true>), b = lds_cap((const void*)k_cholinv_desc<true>);
        g_chol_lds = a < b ? a : b;
    }
}

int jacobi_lds_max() {
    init_lds_caps();
    return g_jac_lds;
}
int chol_lds_max() {
    init_lds_caps();
    return g_chol_lds;
}

template <int TS>
static void core_gemm_ts(const Task* tasks, int count, int max_M, int max_N, bool ta, bool tb, int sa, int sb,
                         int sc, int dims, hipStream_t st) {
    const dim3 grid((unsigned)((max_N + TS - 1) / TS), (unsigned)((max_M + TS - 1) / TS), (unsigned)count);
    if (!ta && !tb) hipLaunchKernelGGL((k_core_gemm<false, false, TS>), grid, dim3(256), 0, st, tasks, sa, sb, sc, dims);
    else if (ta && !tb) hipLaunchKernelGGL((k_core_gemm<true, false, TS>), grid, dim3(256), 0, st, tasks, sa, sb, sc, dims);
    else if (!ta && tb) hipLaunchKernelGGL((k_core_gemm<false, true, TS>), grid, dim3(256), 0, st, tasks, sa, sb, sc, dims);
    else hipLaunchKernelGGL((k_core_gemm<true, true, TS>), grid, dim3(256), 0, st, tasks, sa, sb, sc, dims);
}

// 64 x 64 tiles when they give the launch at least 256 workgroups, else
// 32 x 32 tiles (the same values either way).
hipError_t launch_core_gemm(const Task* tasks, int count, int max_M, int max_N, bool ta, bool tb,
                            int sa, int sb, int sc, int dims, hipStream_t st) {
    const int64_t t64 = (int64_t)((max_N + 63) / 64) * ((max_M + 63) / 64) * count;
    if (t64 >= 256) core_gemm_ts<64>(tasks, count, max_M, max_N, ta, tb, sa, sb, sc, dims, st);
    else core_gemm_ts<32>(tasks, count, max_M, max_N, ta, tb, sa, sb, sc, dims, st);
    return hipGetLastError();
}

hipError_t launch_cholinv(const Task* tasks, int count, int max_k, bool any_small, bool any_large,
                          int sw, int sx, hipStream_t st) {
    const int cap = chol_lds_max();
    const dim3 grid(1, 1, (unsigned)count);
    if (any_small && cap > 0) {
        const int kk = max_k < cap ? max_k : cap;
        hipLaunchKernelGGL((k_cholinv<true>), grid, dim3(1024), sizeof(double) * (size_t)kk * kk, st,
                           tasks, sw, sx, cap);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (any_large || cap == 0) hipLaunchKernelGGL((k_cholinv<false>), grid, dim3(1024), 0, st, tasks, sw, sx, cap);
    return hipGetLastError();
}

hipError_t launch_jacobi(const Task* tasks, int count, int max_n, bool any_small, bool any_large,
                         hipStream_t st) {
    const int cap = jacobi_lds_max();
    const dim3 grid(1, 1, (unsigned)count);
    if (any_small && cap > 0) {
        const int nn = max_n < cap ? max_n : cap;
        const int ldsd = 2 * nn * nn <= cap * cap ? 2 * nn * nn : nn * nn;
        hipLaunchKernelGGL((k_jacobi<true>), grid, dim3(1024), sizeof(double) * (size_t)ldsd, st, tasks, cap, ldsd);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (any_large || cap == 0) hipLaunchKernelGGL((k_jacobi<false>), grid, dim3(1024), 0, st, tasks, cap, 0);
    return hipGetLastError();
}

static hipError_t cholinv_desc_impl(DescArg<SmallDesc> ds, int count, int max_n, hipStream_t st) {
    const int cap = chol_lds_max();
    if (cap > 0) {
        const int nn = max_n < cap ? max_n : cap;
        hipLaunchKernelGGL((k_cholinv_desc<true>), dim3(1, 1, (unsigned)count), dim3(1024),
                           sizeof(double) * (size_t)nn * nn, st, ds, cap);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (max_n > cap) hipLaunchKernelGGL((k_cholinv_desc<false>), dim3(1, 1, (unsigned)count), dim3(1024), 0, st, ds, cap);
    return hipGetLastError();
}

static hipError_t jacobi_desc_impl(DescArg<SmallDesc> ds, int count, int max_n, hipStream_t st) {
    const int cap = jacobi_lds_max();
    if (cap > 0) {
        const int nn = max_n < cap ? max_n : cap;
        const int ldsd = 2 * nn * nn <= cap * cap ? 2 * nn * nn : nn * nn;
        hipLaunchKernelGGL((k_jacobi_desc<true>), dim3(1, 1, (unsigned)count), dim3(1024), sizeof(double) * (size_t)ldsd,
                           st, ds, cap, ldsd);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (max_n > cap) hipLaunchKernelGGL((k_jacobi_desc<false>), dim3(1, 1, (unsigned)count), dim3(1024), 0, st, ds, cap, 0);
    return hipGetLastError();
}

hipError_t launch_cholinv_desc(const SmallDesc* ds, int count, int max_n, hipStream_t st) {
    return cholinv_desc_impl(DescArg<SmallDesc>{ds, {}}, count, max_n, st);
}
hipError_t launch_jacobi_desc(const SmallDesc* ds, int count, int max_n, hipStream_t st) {
    return jacobi_desc_impl(DescArg<SmallDesc>{ds, {}}, count, max_n, st);
}
hipError_t launch_cholinv1(const SmallDesc& q, hipStream_t st) {
    return cholinv_desc_impl(DescArg<SmallDesc>{nullptr, q}, 1, q.n, st);
}
hipError_t launch_jacobi1(const SmallDesc& q, hipStream_t st) {
    return jacobi_desc_impl(DescArg<SmallDesc>{nullptr, q}, 1, q.n, st);
}

hipError_t launch_threshold(const Task* tasks, int count, int max_ell, int max_m, hipStream_t st) {
    int blocks = (max_ell * max_m + 255) / 256;
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(k_threshold, dim3((unsigned)blocks, 1, (unsigned)count), dim3(256), 0, st, tasks);
    return hipGetLastError();
}

}  // namespace sk
