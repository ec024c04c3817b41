// k_cholx.hip -- CholeskyQR of a shrink's m x k iterate Y (the
// orthonormalisation of Algorithm "Simultaneous Iteration", done as the
// Gram W = Y^T Y, its Cholesky factor L L^T = W and Q = Y L^{-T}; one or two
// passes) by P = ceil(k / 16) workgroups ("members") per task.
//
// Member b holds rows [16 b, 16 b + 16) of W in LDS.  The Cholesky factor is
// formed block row by block row: when member b's rows have received the
// updates of every earlier block, it factors its 16 x 16 diagonal block
// (one wavefront, a row per lane in registers), forms
// X_b = L_bb^{-1} W[block b, :] -- block row b of L^T -- and publishes it;
// every later member subtracts X_b[:, its rows]^T X_b from its rows.  So
// there is one exchange per 16 columns, from one member to the later ones,
// and nothing waits on a grid-wide barrier.  Q = Y L^{-T} is then solved
// by row blocks of 32 against the published L^T.
//
// Rank dropping as in the one-workgroup kernel: a pivot at or below 1e-14
// of its column's original diagonal (or below 1e-300) drops the column: its
// 1 / L_jj is taken as 0, so column j of L and of Q are zero.
//
// Every sum has a fixed order and P depends on k alone, so a task's result
// does not depend on the batch it runs in.
#include "sk_device.h"
#include "sk_kernels.h"
#include "sk_xwg.h"

namespace sk {

constexpr int CB = 16;        // rows of W per member
constexpr int CTH = 256;      // threads per member
constexpr int CKMAX = 512;    // largest k

__host__ __device__ __forceinline__ int cx_members(int k) { return (k + CB - 1) / CB; }

__device__ __forceinline__ double cx_bcast(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// rows x cols block of a row-major global matrix (leading dimension ldg,
// first column c0) into LDS (leading dimension ldl, first column lc0), by all
// threads, eight independent loads in flight per thread; entries outside
// [0, vr) x [0, vc) of the source read as zero.
__device__ __forceinline__ void cx_g2l(const double* __restrict__ g, int64_t ldg, int c0, int rows, int cols, int vr,
                                       int vc, double* l, int ldl, int lc0) {
    const int n = rows * cols;
    for (int base = threadIdx.x; base < n; base += 8 * CTH) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * CTH;
            const int r = e / cols, c = e - r * cols;
            v[u] = (e < n && r < vr && c0 + c < vc) ? g[(int64_t)r * ldg + c0 + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + u * CTH;
            if (e < n) {
                const int r = e / cols, c = e - r * cols;
                l[r * ldl + lc0 + c] = v[u];
            }
        }
    }
}

// stage of the flags in a pass (grows with the pass within a launch): block
// row p of L^T is published in flags[p], the end of a pass in flags[32 + b]
__device__ __forceinline__ unsigned cx_stage_x(int pass) { return (unsigned)(pass * 256 + 1); }
__device__ __forceinline__ unsigned cx_stage_end(int pass) { return (unsigned)(pass * 256 + 200); }

// rows of Y per block of the Q step, so that the block and one column block
// of L^T fit the LDS next to each other (chosen from the launch's largest K,
// so that every task of the launch fits the LDS sized for it)
__host__ __device__ __forceinline__ int cx_qrows(int K) { return K <= 256 ? 32 : 16; }
__host__ __device__ __forceinline__ size_t cx_lds_doubles(int K) {
    const size_t a = (size_t)2 * CB * K, b = (size_t)cx_qrows(K) * K + (size_t)K * CB;
    const size_t g = (size_t)32 * K;  // Gram staging
    size_t x = a > b ? a : b;
    return x > g ? x : g;
}

__device__ void cholqr_x_body(const Task& t, int sy, int sq, int passes, int member, uint64_t epoch, int QR) {
    extern __shared__ double lds[];
    const SkDev* s = t.s;
    const int m = t.m, k = s->k, K = cx_members(k) * CB, P = K / CB;
    const int ldk = s->sld[S_Q];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* Wb = lds;                 // [CB][K] this member's rows of W
    double* Xs = lds + CB * K;        // [CB][K] a published block row of L^T
    double* Ystage = lds;             // [32][K] rows of Y (Gram step)
    double* Qs = lds;                 // [QR][K] rows of Q (Q step)
    double* Lc = lds + QR * K;        // [K][CB] one column block of L^T (Q step)
    double* Lt = s->slot[S_EA];       // K x K: L^T, block row p from member p
    uint64_t* flags = s->xflags;      // [0, 32): block rows of L^T; [32, 64): pass ends
    __shared__ double Ld[CB][CB + 1], rd[CB], d0[CB];
    __shared__ int bad;
    if (tid == 0) bad = 0;
    const int g0 = CB * member;       // first row of W held here
    for (int pass = 0; pass < passes; ++pass) {
        const double* src = s->slot[pass == 0 ? sy : S_Q1];
        double* dst = s->slot[pass == passes - 1 ? sq : S_Q1];
        // ---- 1. rows g0 .. g0 + 15 of W = src^T src (columns c = tid, tid + 256),
        // src staged 32 rows at a time
        {
            double acc0[CB], acc1[CB];
#pragma unroll
            for (int i = 0; i < CB; ++i) acc0[i] = acc1[i] = 0.0;
            const int c0 = tid, c1 = tid + CTH;
            for (int r0 = 0; r0 < m; r0 += 32) {
                __syncthreads();
                cx_g2l(src + (int64_t)r0 * ldk, ldk, 0, 32, K, m - r0, k, Ystage, K, 0);
                __syncthreads();
                const int nr = min(32, m - r0);
                for (int rr = 0; rr < nr; ++rr) {
                    const double* yr = Ystage + rr * K;
                    const double y0 = c0 < K ? yr[c0] : 0.0;
                    const double y1 = c1 < K ? yr[c1] : 0.0;
#pragma unroll
                    for (int i = 0; i < CB; ++i) {
                        const double yi = yr[g0 + i];
                        acc0[i] = fma(yi, y0, acc0[i]);
                        acc1[i] = fma(yi, y1, acc1[i]);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                if (c0 < K) Wb[i * K + c0] = acc0[i];
                if (c1 < K) Wb[i * K + c1] = acc1[i];
            }
        }
        __syncthreads();
        if (tid < CB) d0[tid] = Wb[tid * K + g0 + tid];
        // ---- 2. updates from the earlier block rows, then this block row
        for (int p = 0; p < member; ++p) {
            if (wave == 0 && !xwg_wait(flags + p, 1, xwg_flag(epoch, cx_stage_x(pass))) && lane == 0) bad = 1;
            __syncthreads();
            if (bad) break;
            // block row p of L^T, columns g0 .. K - 1
            cx_g2l(Lt + (int64_t)CB * p * K, K, g0, CB, K - g0, CB, K, Xs, K, g0);
            __syncthreads();
            // W[block b, c] -= X_p[:, block b]^T X_p[:, c], c >= g0
            for (int c = g0 + tid; c < K; c += CTH) {
                double xc[CB];
#pragma unroll
                for (int j = 0; j < CB; ++j) xc[j] = Xs[j * K + c];
                // the 16 x 16 coefficients are read from LDS at each use (all
                // lanes read the same word), not held in registers
#pragma unroll 1
                for (int i = 0; i < CB; ++i) {
                    double a = Wb[i * K + c];
#pragma unroll
                    for (int j = 0; j < CB; ++j) a = fma(-Xs[j * K + g0 + i], xc[j], a);
                    Wb[i * K + c] = a;
                }
            }
            __syncthreads();
        }
        if (bad) break;
        // factor the diagonal block: one wavefront, lane i holding row i
        if (wave == 0) {
            const int i = lane < CB ? lane : 0;
            double a[CB];
#pragma unroll
            for (int l = 0; l < CB; ++l) a[l] = Wb[i * K + g0 + l];
            double rdi = 0.0;
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const double piv = cx_bcast(a[j], j);
                const bool ok = piv > 1e-14 * d0[j] && piv > 1e-300;
                double r = 0.0, dj = 0.0;
                if (ok) {
                    r = __builtin_amdgcn_rsq(piv);
                    r = r * fma(-0.5 * piv * r, r, 1.5);
                    r = r * fma(-0.5 * piv * r, r, 1.5);
                    dj = piv * r;
                }
                const double ci = a[j] * r;
                if (ok) {
#pragma unroll
                    for (int l = j + 1; l < CB; ++l) {
                        const double cl = cx_bcast(ci, l);
                        if (l <= i) a[l] = fma(-ci, cl, a[l]);
                    }
                }
                a[j] = (i > j) ? ci : (i == j ? dj : 0.0);
                if (i == j) rdi = r;
            }
            if (lane < CB) {
#pragma unroll
                for (int l = 0; l < CB; ++l) Ld[lane][l] = l <= lane ? a[l] : 0.0;
                rd[lane] = rdi;
            }
        }
        __syncthreads();
        // X_b = L_bb^{-1} W[block b, c] for c >= g0 + 16, by substitution per
        // column; the diagonal block of X_b is L_bb^T itself
        for (int e = tid; e < CB * CB; e += CTH) {
            const int i = e / CB, c = e - i * CB;
            Xs[i * K + g0 + c] = Ld[c][i];
        }
        for (int c = g0 + CB + tid; c < K; c += CTH) {
            double x[CB];
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                double v = Wb[i * K + c];
#pragma unroll
                for (int j = 0; j < i; ++j) v = fma(-Ld[i][j], x[j], v);
                x[i] = v * rd[i];
            }
#pragma unroll
            for (int i = 0; i < CB; ++i) Xs[i * K + c] = x[i];
        }
        __syncthreads();
        {
            // block row b of L^T to global by every wavefront, each one
            // releasing its own stores before the flag
            double* xr = Lt + (int64_t)g0 * K;
            const int w = K - g0;
            for (int e = tid; e < CB * w; e += CTH) {
                const int j = e / w, c = g0 + (e - j * w);
                xr[(int64_t)j * K + c] = Xs[j * K + c];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        __syncthreads();
        if (wave == 0) {
            if (lane == 0)
                __hip_atomic_store(flags + member, xwg_flag(epoch, cx_stage_x(pass)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            // every member's block row before the Q step
            if (!xwg_wait(flags, P, xwg_flag(epoch, cx_stage_x(pass))) && lane == 0) bad = 1;
        }
        __syncthreads();
        if (bad) break;
        // ---- 3. Q = src L^{-T} for row blocks member, member + P, ...
        for (int r0 = QR * member; r0 < m; r0 += QR * P) {
            cx_g2l(src + (int64_t)r0 * ldk, ldk, 0, QR, K, m - r0, k, Qs, K, 0);
            for (int p = 0; p < P; ++p) {
                const int cp = CB * p;
                __syncthreads();
                // column block p of L^T, rows 0 .. cp + 15
                cx_g2l(Lt, K, cp, cp + CB, CB, K, K, Lc, CB, 0);
                __syncthreads();
                // z = y[:, block p] - q[:, blocks < p] L[block p, blocks < p]^T
                for (int e = tid; e < QR * CB; e += CTH) {
                    const int rr = e / CB, c = e - rr * CB;
                    double z = Qs[rr * K + cp + c];
                    for (int j = 0; j < cp; ++j) z = fma(-Qs[rr * K + j], Lc[j * CB + c], z);
                    Qs[rr * K + cp + c] = z;
                }
                __syncthreads();
                // q[:, block p] L_pp^T = z, one row per thread (a zero pivot
                // -- a dropped column -- gives a zero column)
                if (tid < QR) {
                    double q[CB];
#pragma unroll
                    for (int i = 0; i < CB; ++i) {
                        double v = Qs[tid * K + cp + i];
#pragma unroll
                        for (int j = 0; j < i; ++j) v = fma(-Lc[(cp + j) * CB + i], q[j], v);
                        const double lii = Lc[(cp + i) * CB + i];
                        q[i] = lii != 0.0 ? v / lii : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < CB; ++i) Qs[tid * K + cp + i] = q[i];
                }
            }
            __syncthreads();
            for (int e = tid; e < QR * K; e += CTH) {
                const int rr = e / K, c = e - rr * K, row = r0 + rr;
                if (row < m && c < k) dst[(int64_t)row * ldk + c] = Qs[e];
            }
            __syncthreads();
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        // ---- 4. every member's Q rows before the next pass reads them, and
        // every member done with this pass's L^T before it is overwritten
        if (pass + 1 < passes) {
            if (wave == 0) {
                if (lane == 0)
                    __hip_atomic_store(flags + 32 + member, xwg_flag(epoch, cx_stage_end(pass)), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                if (!xwg_wait(flags + 32, P, xwg_flag(epoch, cx_stage_end(pass))) && lane == 0) bad = 1;
            }
            __syncthreads();
            if (bad) break;
        }
    }
    if (bad && tid == 0) atomicAdd(&s->info[3], 1);
}

// Members b of task i are workgroups P i + b (consecutive: spread over the
// XCDs); tasks with fewer members leave the surplus idle.
__global__ __launch_bounds__(CTH) void k_cholqr_x(const Task* tasks, int count, int Pmax, int sy, int sq,
                                                  int passes, uint64_t epoch, int qrows) {
    const int task = blockIdx.x / Pmax, member = blockIdx.x % Pmax;
    if (task >= count) return;
    const Task& t = tasks[task];
    if (t.kind != T_SHRINK_RAND || !(t.flags & TF_X_CHOL)) return;
    if (member >= cx_members(t.s->k)) return;
    cholqr_x_body(t, sy, sq, passes, member, epoch, qrows);
}

// CholeskyQR (passes 1 or 2) of every randomized task of the list, P = members
// of the largest k, as many tasks per cooperative launch as are resident.
hipError_t launch_cholqr_x(const Task* tasks, int count, int max_k, int sy, int sq, int passes, hipStream_t st) {
    if (max_k > CKMAX) return hipErrorInvalidConfiguration;
    const int Pmax = cx_members(max_k), K = Pmax * CB;
    const size_t lds = sizeof(double) * cx_lds_doubles(K);
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        if (hipFuncSetAttribute((const void*)k_cholqr_x, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(double) * cx_lds_doubles(CKMAX))) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_cholqr_x, CTH,
                                                         sizeof(double) * cx_lds_doubles(CKMAX)) != hipSuccess ||
            per_cu < 1)
            return hipErrorInvalidConfiguration;
    }
    const int chunk = std::max(1, (per_cu * cus) / Pmax);
    for (int off = 0; off < count; off += chunk) {
        const Task* tl = tasks + off;
        int cnt = std::min(chunk, count - off);
        uint64_t epoch = xwg_next_epoch();
        int pm = Pmax, a = sy, b = sq, ps = passes, qr = cx_qrows(K);
        void* args[] = {(void*)&tl, (void*)&cnt, (void*)&pm, (void*)&a, (void*)&b, (void*)&ps, (void*)&epoch,
                        (void*)&qr};
        hipError_t e = hipLaunchCooperativeKernel((const void*)k_cholqr_x, dim3((unsigned)(Pmax * cnt)), dim3(CTH),
                                                  args, (unsigned)lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sk
