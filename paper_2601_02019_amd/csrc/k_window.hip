// k_window.hip -- kernels of the sliding-window sketch (Algorithm
// "ML-AeroSketch") on gfx950.  The window engine (sk_window.cpp) drives them
// with plain pointer descriptors, one descriptor per level.
//
//   k_rownorm     |a|^2 of every arriving row (FP64), for the raw-row test
//   k_philox_mat  Gaussian d x k matrix from Philox4x64-10 (power-iteration
//                 start vector, simul_iter test matrix)
//   k_win_pi      Algorithm "Power Iteration" on C'^T C' for one level:
//                 ceil(log2 d) + 1 normalised steps x <- C'^T C' x, then the
//                 Rayleigh quotient |C' x|^2 (the power-iteration test of
//                 Algorithm "AeroSketch: Update")
//   k_gemm_desc   FP64 C = alpha op(A) op(B) + beta C for snapshot, residual
//                 and restore products
//   k_blockmask   zeroes the off-entry blocks of W Z (the restore of Algorithm
//                 "AeroSketch: Query" is per snapshot)
//   k_shrink_rows rows sqrt(max(lambda_i - lambda_ell, 0)) v_i^T (the query's
//                 final shrink)
#include "sk_device.h"
#include "sk_kernels.h"

namespace sk {

__device__ __forceinline__ void w_philox(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t y0 = hi1 ^ c[1] ^ k0;
        const uint64_t y2 = hi0 ^ c[3] ^ k1;
        c[0] = y0;
        c[1] = lo1;
        c[2] = y2;
        c[3] = lo0;
    }
}

// Normal number `which` (0..3) of the block at counter (c0, c1, c2, c3).
__device__ __forceinline__ double w_gauss(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1,
                                          uint64_t c2, uint64_t c3, int which) {
    uint64_t c[4] = {c0, c1, c2, c3};
    w_philox(c, seed, stream);
    const int h = which >> 1;
    const double u1 = (double)((c[2 * h] >> 11) + 1) * 0x1p-53;
    const double u2 = (double)(c[2 * h + 1] >> 11) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
    return (which & 1) ? rad * sn : rad * cs;
}

template <typename T> __device__ __forceinline__ double wf64(T v);
template <> __device__ __forceinline__ double wf64<double>(double v) { return v; }
template <> __device__ __forceinline__ double wf64<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double wf64<uint16_t>(uint16_t b) {
    return (double)__uint_as_float(((uint32_t)b) << 16);
}

// one wavefront per row, fixed-order reduction
template <typename T>
__global__ __launch_bounds__(256) void k_rownorm(const T* rows, int64_t ld, int64_t n, int d,
                                                 double* out) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const T* a = rows + row * ld;
    double acc = 0.0;
    for (int t = lane; t < d; t += 64) {
        const double v = wf64(a[t]);
        acc = fma(v, v, acc);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) out[row] = acc;
}


// M[t][c] = normal (c mod 4) of the block at counter (t, c / 4, c2, c3)
__global__ __launch_bounds__(256) void k_philox_mat(const MatGenDesc* ds) {
    const MatGenDesc& q = ds[blockIdx.z];
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (t >= q.rows || c >= q.cols) return;
    q.M[(int64_t)t * q.ld + c] = w_gauss(q.seed, q.stream, (uint64_t)t, (uint64_t)(c >> 2), q.c2, q.c3, c & 3);
}


__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// One workgroup per level; x (d) and y (r) live in LDS.
__global__ __launch_bounds__(256) void k_win_pi(const PiDesc* ds) {
    extern __shared__ double sm[];
    __shared__ double red[4];
    const PiDesc& q = ds[blockIdx.z];
    const int r = q.r, d = q.d, tid = threadIdx.x;
    double* x = sm;
    double* y = sm + d;
    if (r <= 0) {
        if (tid == 0) *q.out = 0.0;
        return;
    }
    double loc = 0.0;
    for (int t = tid; t < d; t += 256) {
        x[t] = w_gauss(q.seed, q.stream, (uint64_t)t, 0ull, q.c2, q.c3, 0);
        loc = fma(x[t], x[t], loc);
    }
    double nrm = sqrt(block_sum(loc, red));
    if (nrm > 0.0)
        for (int t = tid; t < d; t += 256) x[t] /= nrm;
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    bool zero = false;
    for (int it = 0; it < q.steps && !zero; ++it) {
        for (int i = wave; i < r; i += 4) {  // y = C x
            double acc = 0.0;
            for (int t = lane; t < d; t += 64) acc = fma(q.C[(int64_t)i * q.ldc + t], x[t], acc);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if (lane == 0) y[i] = acc;
        }
        __syncthreads();
        loc = 0.0;
        for (int t = tid; t < d; t += 256) {  // x = C^T y
            double acc = 0.0;
            for (int i = 0; i < r; ++i) acc = fma(q.C[(int64_t)i * q.ldc + t], y[i], acc);
            x[t] = acc;
            loc = fma(acc, acc, loc);
        }
        nrm = sqrt(block_sum(loc, red));
        if (nrm == 0.0) {
            zero = true;
        } else {
            for (int t = tid; t < d; t += 256) x[t] /= nrm;
        }
        __syncthreads();
    }
    if (zero) {
        if (tid == 0) *q.out = 0.0;
        return;
    }
    for (int i = wave; i < r; i += 4) {
        double acc = 0.0;
        for (int t = lane; t < d; t += 64) acc = fma(q.C[(int64_t)i * q.ldc + t], x[t], acc);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) y[i] = acc;
    }
    __syncthreads();
    loc = 0.0;
    for (int i = tid; i < r; i += 256) loc = fma(y[i], y[i], loc);
    const double rq = block_sum(loc, red);
    if (tid == 0) *q.out = rq;
}

// ---------------------------------------------------------------- GEMM
__global__ __launch_bounds__(256) void k_gemm_desc(const GemmDesc* ds) {
    const GemmDesc& g = ds[blockIdx.z];
    const int M = g.M, N = g.N, K = g.K;
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    if (r0 >= M || c0 >= N) return;
    __shared__ double As[16][64 + 2];
    __shared__ double Bs[16][64 + 2];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int kk = 0; kk < K; kk += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            if (!g.ta) {
                const int r = e >> 4, k = e & 15;
                As[k][r] = (r0 + r < M && kk + k < K) ? g.A[(int64_t)(r0 + r) * g.lda + kk + k] : 0.0;
            } else {
                const int r = e & 63, k = e >> 6;
                As[k][r] = (r0 + r < M && kk + k < K) ? g.A[(int64_t)(kk + k) * g.lda + r0 + r] : 0.0;
            }
            if (!g.tb) {
                const int c = e & 63, k = e >> 6;
                Bs[k][c] = (c0 + c < N && kk + k < K) ? g.B[(int64_t)(kk + k) * g.ldb + c0 + c] : 0.0;
            } else {
                const int c = e >> 4, k = e & 15;
                Bs[k][c] = (c0 + c < N && kk + k < K) ? g.B[(int64_t)(c0 + c) * g.ldb + kk + k] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[k][ty * 4 + i];
                b[i] = Bs[k][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + ty * 4 + i;
        if (r >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + tx * 4 + j;
            if (c >= N) continue;
            double* p = g.C + (int64_t)r * g.ldc + c;
            *p = (g.beta == 0.0) ? g.alpha * acc[i][j] : fma(g.alpha, acc[i][j], g.beta * *p);
        }
    }
}

// S (D x D): keep S[a][b] only when directions a and b belong to one snapshot
__global__ __launch_bounds__(256) void k_blockmask(double* S, int ld, int D, const int32_t* ent) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)D * D) return;
    const int a = (int)(e / D), b = (int)(e % D);
    if (ent[a] != ent[b]) S[(int64_t)a * ld + b] = 0.0;
}

// X (ell x d, ld ldx): row i = sqrt(max(lam_i - lam_ell, 0)) * column i of V
// (V: n x n, ld ldv, sorted descending); rows beyond n are zero.
__global__ __launch_bounds__(256) void k_shrink_rows(const double* V, int ldv, const double* lam, int n,
                                                     int ell, double* X, int64_t ldx, int d) {
    const int i = blockIdx.y;
    if (i >= ell) return;
    const double de = (n >= ell) ? lam[ell - 1] : 0.0;
    const double f = (i < n && lam[i] - de > 0.0) ? sqrt(lam[i] - de) : 0.0;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < d; t += gridDim.x * 256)
        X[(int64_t)i * ldx + t] = (i < n) ? f * V[(int64_t)t * ldv + i] : 0.0;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_rownorm(const void* rows, int64_t ld, int dtype, int64_t n, int d, double* out,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 3) / 4));
    if (dtype == DT_F64) hipLaunchKernelGGL((k_rownorm<double>), grid, dim3(256), 0, st, (const double*)rows, ld, n, d, out);
    else if (dtype == DT_F32) hipLaunchKernelGGL((k_rownorm<float>), grid, dim3(256), 0, st, (const float*)rows, ld, n, d, out);
    else hipLaunchKernelGGL((k_rownorm<uint16_t>), grid, dim3(256), 0, st, (const uint16_t*)rows, ld, n, d, out);
    return hipGetLastError();
}

hipError_t launch_philox_mat(const void* descs, int count, int max_rows, int max_cols, hipStream_t st) {
    hipLaunchKernelGGL(k_philox_mat, dim3((unsigned)((max_rows + 255) / 256), (unsigned)max_cols, (unsigned)count),
                       dim3(256), 0, st, (const MatGenDesc*)descs);
    return hipGetLastError();
}

hipError_t launch_win_pi(const void* descs, int count, int max_d, int max_r, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)(max_d + max_r);
    hipLaunchKernelGGL(k_win_pi, dim3(1, 1, (unsigned)count), dim3(256), lds, st, (const PiDesc*)descs);
    return hipGetLastError();
}

hipError_t launch_gemm_desc(const GemmDesc* ds, int count, int max_M, int max_N, hipStream_t st) {
    hipLaunchKernelGGL(k_gemm_desc, dim3((unsigned)((max_N + 63) / 64), (unsigned)((max_M + 63) / 64), (unsigned)count),
                       dim3(256), 0, st, ds);
    return hipGetLastError();
}

hipError_t launch_blockmask(double* S, int ld, int D, const int32_t* ent, hipStream_t st) {
    if (D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_blockmask, dim3((unsigned)(((int64_t)D * D + 255) / 256)), dim3(256), 0, st, S, ld, D, ent);
    return hipGetLastError();
}

hipError_t launch_shrink_rows(const double* V, int ldv, const double* lam, int n, int ell, double* X,
                              int64_t ldx, int d, hipStream_t st) {
    const int bx = (d + 255) / 256 < 16 ? (d + 255) / 256 : 16;
    hipLaunchKernelGGL(k_shrink_rows, dim3((unsigned)bx, (unsigned)ell), dim3(256), 0, st, V, ldv, lam, n, ell, X, ldx, d);
    return hipGetLastError();
}

size_t matgen_desc_size() { return sizeof(MatGenDesc); }
size_t pi_desc_size() { return sizeof(PiDesc); }

}  // namespace sk

namespace sk {

// dst (cols x rows, ld ldd) = src (rows x cols, ld lds) transposed
__global__ __launch_bounds__(256) void k_transpose(const double* src, int lds, double* dst, int64_t ldd,
                                                   int rows, int cols) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols || r >= rows) return;
    dst[(int64_t)c * ldd + r] = src[(int64_t)r * lds + c];
}

hipError_t launch_transpose(const double* src, int lds, double* dst, int64_t ldd, int rows, int cols,
                            hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0, st,
                       src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

}  // namespace sk
