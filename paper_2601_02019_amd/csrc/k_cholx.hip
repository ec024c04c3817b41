// k_cholx.hip -- CholeskyQR of a shrink's m x k iterate Y (the
// orthonormalisation of Algorithm "Simultaneous Iteration", done as the
// Gram W = Y^T Y, its Cholesky factor L L^T = W and Q = Y L^{-T}): the
// factor and Q of one pass by P = ceil(k / 16) workgroups ("members") per
// task, after the Gram (a separate product launch).
//
// Member b holds rows [16 b, 16 b + 16) of W in LDS.  The Cholesky factor is
// formed block row by block row: when member b's rows have received the
// updates of every earlier block, it factors its 16 x 16 diagonal block
// (one wavefront, a row per lane in registers), forms
// X_b = L_bb^{-1} W[block b, :] -- block row b of L^T -- and publishes it;
// every later member subtracts X_b[:, its rows]^T X_b from its rows.  So
// there is one exchange per 16 columns, from one member to the later ones,
// and nothing waits on a grid-wide barrier.  Q = Y L^{-T} is then solved
// by row blocks against the published L^T.
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

// stage of the flags (grows with the pass within a launch): block row p of
// L^T is published in flags[p]
__device__ __forceinline__ unsigned cx_stage(int pass) { return (unsigned)(pass + 1); }

// rows of Y per block of the Q step (the block and one column block of L^T
// share the LDS; chosen from the launch's largest K, so that every task of
// the launch fits the LDS sized for it)
__host__ __device__ __forceinline__ int cx_qrows(int K) { return K <= 256 ? 32 : 16; }
__host__ __device__ __forceinline__ size_t cx_lds_doubles(int K) {
    const size_t a = (size_t)CB * K, b = (size_t)cx_qrows(K) * K + (size_t)K * CB;
    return a > b ? a : b;
}

// One CholeskyQR pass: W (k x k, slot S_W, the Gram of src computed before
// the launch) -> L; dst = src L^{-T}.
__device__ void cholqr_x_body(const Task& t, int src_slot, int dst_slot, int member, uint64_t epoch, int QR,
                              int pass) {
    extern __shared__ double lds[];
    const SkDev* s = t.s;
    const int m = t.m, k = s->k, K = cx_members(k) * CB, P = K / CB;
    const int ldk = s->sld[S_Q], ldw = s->sld[S_W];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* src = s->slot[src_slot];
    double* dst = s->slot[dst_slot];
    const double* Wg = s->slot[S_W];
    double* Wb = lds;                 // [CB][K] this member's rows of W
    double* Qs = lds;                 // [QR][K] rows of Q (Q step, after the factor)
    double* Lc = lds + QR * K;        // [K][CB] one column block of L^T (Q step)
    double* Lt = s->slot[S_EA];       // K x K: L^T, block row p from member p
    uint64_t* flags = s->xflags;
    __shared__ double Ld[CB][CB + 1], rd[CB], d0[CB], coef[CB * CB];
    __shared__ int bad;
    if (tid == 0) bad = 0;
    const int g0 = CB * member;       // first row of W held here
    // ---- 1. this member's rows of W; thread columns c = tid, tid + 256
    {
        double w0[CB], w1[CB];
        const int c0 = tid, c1 = tid + CTH;
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int row = g0 + i;
            w0[i] = (row < k && c0 < k) ? Wg[(int64_t)row * ldw + c0] : 0.0;
            w1[i] = (row < k && c1 < k) ? Wg[(int64_t)row * ldw + c1] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            if (c0 < K) Wb[i * K + c0] = w0[i];
            if (c1 < K) Wb[i * K + c1] = w1[i];
        }
    }
    __syncthreads();
    if (tid < CB) d0[tid] = Wb[tid * K + g0 + tid];
    // ---- 2. updates from the earlier block rows: W[block b, c] -= X_p[:, block b]^T X_p[:, c]
    for (int p = 0; p < member; ++p) {
        if (wave == 0 && !xwg_wait(flags + p, 1, xwg_flag(epoch, cx_stage(pass))) && lane == 0) bad = 1;
        __syncthreads();
        if (bad) break;
        const double* xr = Lt + (int64_t)CB * p * K;
        coef[tid] = xr[(int64_t)(tid >> 4) * K + g0 + (tid & 15)];  // X_p[j][g0 + i], j = tid / 16
        double x0[CB], x1[CB];
        const int c0 = g0 + tid, c1 = g0 + tid + CTH;
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            x0[j] = c0 < K ? xr[(int64_t)j * K + c0] : 0.0;
            x1[j] = c1 < K ? xr[(int64_t)j * K + c1] : 0.0;
        }
        __syncthreads();
        if (c0 < K) {
#pragma unroll 1
            for (int i = 0; i < CB; ++i) {
                double a = Wb[i * K + c0];
#pragma unroll
                for (int j = 0; j < CB; ++j) a = fma(-coef[j * CB + i], x0[j], a);
                Wb[i * K + c0] = a;
            }
        }
        if (c1 < K) {
#pragma unroll 1
            for (int i = 0; i < CB; ++i) {
                double a = Wb[i * K + c1];
#pragma unroll
                for (int j = 0; j < CB; ++j) a = fma(-coef[j * CB + i], x1[j], a);
                Wb[i * K + c1] = a;
            }
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) atomicAdd(&s->info[3], 1);
        return;
    }
    // ---- 3. factor the diagonal block: one wavefront, lane i holding row i
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
    // ---- 4. block row b of L^T to global: the diagonal block is L_bb^T, the
    // rest X_b = L_bb^{-1} W[block b, c] by substitution per column; every
    // wavefront releases its stores, then the flag
    {
        double* xr = Lt + (int64_t)g0 * K;
        if (tid < CB * CB) xr[(int64_t)(tid >> 4) * K + g0 + (tid & 15)] = Ld[tid & 15][tid >> 4];
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
            for (int i = 0; i < CB; ++i) xr[(int64_t)i * K + c] = x[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (wave == 0) {
        if (lane == 0)
            __hip_atomic_store(flags + member, xwg_flag(epoch, cx_stage(pass)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        // every member's block row before the Q step
        if (!xwg_wait(flags, P, xwg_flag(epoch, cx_stage(pass))) && lane == 0) bad = 1;
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) atomicAdd(&s->info[3], 1);
        return;
    }
    // ---- 5. Q = src L^{-T} for row blocks member, member + P, ...
    for (int r0 = QR * member; r0 < m; r0 += QR * P) {
        {
            const int c0 = tid, c1 = tid + CTH;
            for (int rr0 = 0; rr0 < QR; rr0 += 16) {
                double y0[16], y1[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int row = r0 + rr0 + u;
                    y0[u] = (row < m && c0 < k) ? src[(int64_t)row * ldk + c0] : 0.0;
                    y1[u] = (row < m && c1 < k) ? src[(int64_t)row * ldk + c1] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (c0 < K) Qs[(rr0 + u) * K + c0] = y0[u];
                    if (c1 < K) Qs[(rr0 + u) * K + c1] = y1[u];
                }
            }
        }
        for (int p = 0; p < P; ++p) {
            const int cp = CB * p;
            __syncthreads();
            // column block p of L^T, rows 0 .. cp + 15
            for (int base = 0, ne = (cp + CB) * CB; base < ne; base += 16 * CTH) {
                double lv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = base + tid + CTH * u;
                    lv[u] = e < ne ? Lt[(int64_t)(e >> 4) * K + cp + (e & 15)] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = base + tid + CTH * u;
                    if (e < ne) Lc[e] = lv[u];
                }
            }
            __syncthreads();
            // z = y[:, block p] - q[:, blocks < p] L[block p, blocks < p]^T
            for (int e = tid; e < QR * CB; e += CTH) {
                const int rr = e >> 4, c = e & 15;
                double z0 = Qs[rr * K + cp + c], z1 = 0.0;
                for (int j = 0; j < cp; j += 2) {
                    z0 = fma(-Qs[rr * K + j], Lc[j * CB + c], z0);
                    z1 = fma(-Qs[rr * K + j + 1], Lc[(j + 1) * CB + c], z1);
                }
                Qs[rr * K + cp + c] = z0 + z1;
            }
            __syncthreads();
            // q[:, block p] L_pp^T = z, one row per thread (a zero pivot --
            // a dropped column -- gives a zero column)
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
        {
            const int c0 = tid, c1 = tid + CTH;
#pragma unroll 4
            for (int rr = 0; rr < QR; ++rr) {
                const int row = r0 + rr;
                if (row < m && c0 < k) dst[(int64_t)row * ldk + c0] = Qs[rr * K + c0];
                if (row < m && c1 < k) dst[(int64_t)row * ldk + c1] = Qs[rr * K + c1];
            }
        }
        __syncthreads();
    }
}

// Members b of task i are workgroups P i + b (consecutive: spread over the
// XCDs); tasks with fewer members leave the surplus idle.
__global__ __launch_bounds__(CTH) void k_cholqr_x(const Task* tasks, int count, int Pmax, int src_slot,
                                                  int dst_slot, uint64_t epoch, int qrows, int pass) {
    const int task = blockIdx.x / Pmax, member = blockIdx.x % Pmax;
    if (task >= count) return;
    const Task& t = tasks[task];
    if (t.kind != T_SHRINK_RAND || !(t.flags & TF_X_CHOL)) return;
    if (member >= cx_members(t.s->k)) return;
    cholqr_x_body(t, src_slot, dst_slot, member, epoch, qrows, pass);
}

// One CholeskyQR pass (W in slot S_W already) of every task flagged
// TF_X_CHOL, P = members of the largest k, as many tasks per cooperative
// launch as are resident.
hipError_t launch_cholqr_x(const Task* tasks, int count, int max_k, int src_slot, int dst_slot, int pass,
                           hipStream_t st) {
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
        int pm = Pmax, a = src_slot, b = dst_slot, qr = cx_qrows(K), ps = pass;
        void* args[] = {(void*)&tl, (void*)&cnt, (void*)&pm, (void*)&a, (void*)&b, (void*)&epoch, (void*)&qr,
                        (void*)&ps};
        hipError_t e = hipLaunchCooperativeKernel((const void*)k_cholqr_x, dim3((unsigned)(Pmax * cnt)), dim3(CTH),
                                                  args, (unsigned)lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sk
