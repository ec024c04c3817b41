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

// dynamic LDS: this member's rows of W
__host__ __device__ __forceinline__ size_t cx_lds_doubles(int K) { return (size_t)CB * K; }

// Barrier over LDS only: waits for this wave's LDS accesses, not for its
// global loads (a plain __syncthreads also drains the global loads in
// flight, which would serialise the prefetch of L^T below).
__device__ __forceinline__ void cx_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Q = src L^{-T} for the row blocks of QR rows from QR member, stride QR P,
// right-looking by column blocks of 16.  Thread t keeps an 8-row x 4-column
// tile of the block in registers (row group t mod RG, RG = QR / 8; column
// group t / RG).  For block p the owners of its 16 columns hand them to LDS,
// QR threads solve q L_pp^T = z row by row, and every thread with later
// columns subtracts q L[its columns, block p]^T (its 4 x 16 entries of L^T,
// loaded while the solve runs; 8 x 16 q values from LDS per 512 FMAs).  Two
// LDS buffers alternate by block, so one LDS-only barrier on each side of
// the solve suffices.
template <int QR>
__device__ __forceinline__ void cholqr_x_qstep(const double* src, double* dst, const double* Lt, int m, int k, int K,
                                               int ldk, int member, int P) {
    constexpr int RG = QR / 8;  // row groups of 8 (K = 64 * 4 * (CTH / RG / 64) columns)
    __shared__ double Zs[2][QR][CB + 1], Lp[2][CB][CB + 1], dinv[2][CB];
    const int tid = threadIdx.x;
    const int rg = tid % RG, c0 = 4 * (tid / RG);  // rows 8 rg .. 8 rg + 7, columns c0 .. c0 + 3
    for (int r0 = QR * member; r0 < m; r0 += QR * P) {
        double y[8][4];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int row = r0 + 8 * rg + i;
#pragma unroll
            for (int jc = 0; jc < 4; ++jc) {
                const int c = c0 + jc;
                y[i][jc] = (row < m && c < k) ? src[(int64_t)row * ldk + c] : 0.0;
            }
        }
        for (int p = 0; p < K / CB; ++p) {
            const int cp = CB * p, bf = p & 1;
            // block p's columns to LDS; its diagonal block of L and the
            // reciprocals of its pivots (a dropped column has pivot 0: 0)
            if (c0 >= cp && c0 < cp + CB)
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int jc = 0; jc < 4; ++jc) Zs[bf][8 * rg + i][c0 - cp + jc] = y[i][jc];
            {
                const int i = tid >> 4, j = tid & 15;  // L_pp[i][j] = L^T[cp + j][cp + i]
                const double l = Lt[(int64_t)(cp + j) * K + cp + i];
                Lp[bf][i][j] = j <= i ? l : 0.0;
                if (i == j) dinv[bf][i] = l != 0.0 ? 1.0 / l : 0.0;
            }
            // L[c, block p] for this thread's later columns, in flight during the solve
            const bool later = c0 >= cp + CB && c0 < K;
            double lc[CB][4];
#pragma unroll
            for (int i = 0; i < CB; ++i)
#pragma unroll
                for (int jc = 0; jc < 4; ++jc) lc[i][jc] = later ? Lt[(int64_t)(cp + i) * K + c0 + jc] : 0.0;
            cx_lds_barrier();
            if (tid < QR) {
                double q[CB];
#pragma unroll
                for (int i = 0; i < CB; ++i) {
                    double v = Zs[bf][tid][i];
#pragma unroll
                    for (int j = 0; j < i; ++j) v = fma(-Lp[bf][i][j], q[j], v);
                    q[i] = v * dinv[bf][i];
                }
#pragma unroll
                for (int i = 0; i < CB; ++i) Zs[bf][tid][i] = q[i];
            }
            cx_lds_barrier();
            if (c0 >= cp && c0 < cp + CB) {
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int jc = 0; jc < 4; ++jc) y[i][jc] = Zs[bf][8 * rg + i][c0 - cp + jc];
            } else if (later) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    double qv[CB];
#pragma unroll
                    for (int l = 0; l < CB; ++l) qv[l] = Zs[bf][8 * rg + i][l];
#pragma unroll
                    for (int jc = 0; jc < 4; ++jc) {
                        double acc = y[i][jc];
#pragma unroll
                        for (int l = 0; l < CB; ++l) acc = fma(-qv[l], lc[l][jc], acc);
                        y[i][jc] = acc;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int row = r0 + 8 * rg + i;
#pragma unroll
            for (int jc = 0; jc < 4; ++jc) {
                const int c = c0 + jc;
                if (row < m && c < k) dst[(int64_t)row * ldk + c] = y[i][jc];
            }
        }
        __syncthreads();
    }
}

// One CholeskyQR pass: W (k x k, slot S_W, the Gram of src computed before
// the launch) -> L; dst = src L^{-T}.
__device__ void cholqr_x_body(const Task& t, int src_slot, int dst_slot, int member, uint64_t epoch, int pass) {
    extern __shared__ double lds[];
    const SkDev* s = t.s;
    const int m = t.m, k = s->k, K = cx_members(k) * CB, P = K / CB;
    const int ldk = s->sld[S_Q], ldw = s->sld[S_W];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* src = s->slot[src_slot];
    double* dst = s->slot[dst_slot];
    const double* Wg = s->slot[S_W];
    double* Wb = lds;                 // [CB][K] this member's rows of W
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
    // 256 threads x 4 columns cover K <= 256 with 32-row blocks, K <= 512 with 16
    if (K <= 256) cholqr_x_qstep<32>(src, dst, Lt, m, k, K, ldk, member, P);
    else cholqr_x_qstep<16>(src, dst, Lt, m, k, K, ldk, member, P);
}

// The second CholeskyQR pass when the first left Q1 nearly orthonormal: with
// W = Q1^T Q1 = I + E and max |E_ij| <= CX_POLAR_TOL, Q2 = Q1 (3I - W) / 2 (one
// Newton-Schulz step towards the polar factor) has Q2^T Q2 = I - 3E^2/4 + O(E^3)
// and the span of Q1, so it serves as the orthonormal basis as well as the
// Cholesky pass does, with one product instead of a chain of block steps.
// This kernel writes X = (3I - W) / 2 into S_X (the product is the
// X-multiply launch of the one-workgroup path) and the decision into info[8];
// the multi-workgroup pass then skips the task.  Rank-deficient iterates
// (a dropped column gives W_jj = 0) always take the Cholesky pass.
constexpr double CX_POLAR_TOL = 1e-8;

__global__ __launch_bounds__(1024) void k_cholx_polar(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind != T_SHRINK_RAND || !(t.flags & TF_X_CHOL)) return;
    const SkDev* s = t.s;
    const int k = s->k, ldw = s->sld[S_W], ldx = s->sld[S_X];
    const double* W = s->slot[S_W];
    double* X = s->slot[S_X];
    double dev = 0.0;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e - i * k;
        const double w = W[(int64_t)i * ldw + j], id = i == j ? 1.0 : 0.0;
        X[(int64_t)i * ldx + j] = 1.5 * id - 0.5 * w;
        dev = fmax(dev, fabs(w - id));
    }
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dev;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        s->info[8] = m <= CX_POLAR_TOL ? 1 : 0;  // a NaN deviation keeps the Cholesky pass
    }
}

hipError_t launch_cholx_polar(const Task* tasks, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_cholx_polar, dim3(1, 1, (unsigned)count), dim3(1024), 0, st, tasks);
    return hipGetLastError();
}

// Members b of task i are workgroups P i + b (consecutive: spread over the
// XCDs); tasks with fewer members leave the surplus idle.
__global__ __launch_bounds__(CTH) void k_cholqr_x(const Task* tasks, int count, int Pmax, int src_slot,
                                                  int dst_slot, uint64_t epoch, int pass, int polar) {
    const int task = blockIdx.x / Pmax, member = blockIdx.x % Pmax;
    if (task >= count) return;
    const Task& t = tasks[task];
    if (t.kind != T_SHRINK_RAND || !(t.flags & TF_X_CHOL)) return;
    if (polar && t.s->info[8]) return;  // the polar step has written dst
    if (member >= cx_members(t.s->k)) return;
    cholqr_x_body(t, src_slot, dst_slot, member, epoch, pass);
}

// One CholeskyQR pass (W in slot S_W already) of every task flagged
// TF_X_CHOL, P = members of the largest k, as many tasks per cooperative
// launch as are resident.
hipError_t launch_cholqr_x(const Task* tasks, int count, int max_k, int src_slot, int dst_slot, int pass,
                           int polar, hipStream_t st) {
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
        int pm = Pmax, a = src_slot, b = dst_slot, ps = pass, pl = polar;
        void* args[] = {(void*)&tl, (void*)&cnt, (void*)&pm, (void*)&a, (void*)&b, (void*)&epoch, (void*)&ps,
                        (void*)&pl};
        hipError_t e = hipLaunchCooperativeKernel((const void*)k_cholqr_x, dim3((unsigned)(Pmax * cnt)), dim3(CTH),
                                                  args, (unsigned)lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sk
