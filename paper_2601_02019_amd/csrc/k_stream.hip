// k_stream.hip -- the d-sized kernels of the shrink and the row ingest
// (gfx950).  Everything here reads task lists (sk_device.h); one launch per
// stage serves every task of a batch.
//
//   k_ingest       rows -> buffer rows [row0, row0 + n) with dtype conversion
//                  (the insert of Algorithm "AeroSketch: Update")
//   k_ingest_csr   the same for CSR rows
//   k_omega        Omega^T (k x d) from Philox4x64-10 + Box-Muller
//                  (the test matrix of Algorithm "Simultaneous Iteration")
//   k_nt_partial   split-K partial products C C^T (Gram of the buffer) and
//                  C Omega (the first product of the sketch step), FP64 accumulation
//   k_reduce       fixed-order sum of the split-K partials (deterministic)
//   k_rebuild      B' = T C: the FD rebuild diag(f) Z^T C (Sec. 2.3)
//   k_convert_rows FP64 staging -> caller dtype
#include "sk_device.h"
#include "sk_kernels.h"
#include "sk_philox.h"

namespace sk {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(uint16_t b) {
    return (double)__uint_as_float(((uint32_t)b) << 16);
}
template <typename T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
// bfloat16 with round-to-nearest-even from float (the float itself RNE from double)
template <> __device__ __forceinline__ uint16_t from_f64<uint16_t>(double v) {
    float f = (float)v;
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- ingest
template <typename Tin, typename Tst>
__global__ __launch_bounds__(256) void k_ingest(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    const int row = blockIdx.y;
    if (t.kind != T_INGEST || row >= t.nrows) return;
    const SkDev* s = t.s;
    Tst* dst = (Tst*)s->buf[t.par] + (int64_t)(t.row0 + row) * s->ld;
    const Tin* src = (const Tin*)t.src + (int64_t)row * t.src_ld;
    const int d = s->d;
    for (int c = (blockIdx.x * 256 + threadIdx.x) * 4; c < d; c += gridDim.x * 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c + u < d) dst[c + u] = from_f64<Tst>(to_f64(src[c + u]));
    }
}

// One workgroup per sparse row, written out densely.  Duplicate column
// indices within a row are summed in the order they appear in the row: the
// first position of every column is found with an integer atomicMin in LDS
// (exact, order-free), duplicates set bit 31 of that entry, and the thread of
// a column with duplicates adds them up sequentially from its first
// position.  No floating-point atomics: the result does not depend on thread
// timing.  Columns without duplicates cost one store.
template <typename Tst>
__global__ __launch_bounds__(256) void k_ingest_csr(const Task* tasks) {
    extern __shared__ int first[];
    const Task& t = tasks[blockIdx.z];
    const int row = blockIdx.y;
    if (t.kind != T_INGEST || row >= t.nrows) return;
    const SkDev* s = t.s;
    const int d = s->d;
    constexpr int NONE = 0x7fffffff;
    for (int c = threadIdx.x; c < d; c += 256) first[c] = NONE;
    __syncthreads();
    const int64_t b = t.indptr[row], e = t.indptr[row + 1];
    for (int64_t p = b + threadIdx.x; p < e; p += 256) {
        const int j = t.indices[p];
        if (j >= 0 && j < d) atomicMin(&first[j], (int)(p - b));
    }
    __syncthreads();
    for (int64_t p = b + threadIdx.x; p < e; p += 256) {
        const int j = t.indices[p];
        if (j >= 0 && j < d && (first[j] & NONE) != (int)(p - b)) atomicOr(&first[j], (int)0x80000000);
    }
    __syncthreads();
    Tst* dst = (Tst*)s->buf[t.par] + (int64_t)(t.row0 + row) * s->ld;
    for (int c = threadIdx.x; c < d; c += 256) {
        const int f = first[c];
        double v = 0.0;
        if (f != NONE) {
            const int64_t p0 = b + (f & NONE);
            v = (double)t.values[p0];
            if (f < 0)  // duplicates: the later positions in row order
                for (int64_t p = p0 + 1; p < e; ++p)
                    if (t.indices[p] == c) v += (double)t.values[p];
        }
        dst[c] = from_f64<Tst>(v);
    }
}

// ---------------------------------------------------------------- Omega^T
template <typename Tp>
__global__ __launch_bounds__(256) void k_omega(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind != T_SHRINK_RAND) return;
    const SkDev* s = t.s;
    const int i = blockIdx.x * 256 + threadIdx.x;  // coordinate in R^d
    const int jg = blockIdx.y;                       // column group of 4
    if (i >= s->d || 4 * jg >= s->k) return;
    double g[4];
    gauss4(s->seed, s->stream, (uint64_t)i, (uint64_t)jg, (uint64_t)t.shrink_idx, 0ull, g);
    Tp* om = (Tp*)s->omegaT;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (4 * jg + u < s->k) om[(int64_t)(4 * jg + u) * s->ld + i] = from_f64<Tp>(g[u]);
}

// ---------------------------------------------------------------- A B^T
// MODE 0: Gram C C^T over the m buffer rows (upper tiles only);
// MODE 1: C Omega with Omega^T stored k x ld.
// 64 x 64 output tile, 16-deep k slices through LDS, 4 x 4 per thread.
template <typename TA, typename TB, int MODE>
__global__ __launch_bounds__(256) void k_nt_partial(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST) return;
    if (MODE == 1 && t.kind != T_SHRINK_RAND) return;
    const SkDev* s = t.s;
    const int M = t.m;
    const int N = MODE == 0 ? t.m : s->k;
    const int splits = MODE == 0 ? s->sg : s->sp;
    const int kc = MODE == 0 ? s->kcg : s->kcp;
    const int ntm = (M + 63) >> 6, ntn = (N + 63) >> 6;
    const int tiles = MODE == 0 ? ntm * (ntm + 1) / 2 : ntm * ntn;
    const int L = blockIdx.x + blockIdx.y * gridDim.x;
    if (L >= tiles * splits) return;
    int tile, split;
    xcd_tile_split(L, tiles, splits, &tile, &split);
    int ti, tj;
    if (MODE == 0) {
        int idx = tile;
        ti = 0;
        while (idx >= ntm - ti) {
            idx -= ntm - ti;
            ++ti;
        }
        tj = ti + idx;
    } else {
        ti = tile / ntn;
        tj = tile % ntn;
    }
    const TA* A = (const TA*)s->buf[t.par];
    const TB* B = MODE == 0 ? (const TB*)s->buf[t.par] : (const TB*)s->omegaT;
    const int64_t ld = s->ld;
    const int kend = (s->d + 15) & ~15;
    const int k0 = split * kc;
    const int k1 = min(k0 + kc, kend);

    __shared__ double As[16][64 + 2];
    __shared__ double Bs[16][64 + 2];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int lr = tid >> 2, lk = (tid & 3) * 4;
    const int ga = ti * 64 + lr, gb = tj * 64 + lr;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    // the next 16-deep slices are loaded into registers while the current
    // ones are multiplied out of LDS
    double pa[4], pb[4];
    auto fetch = [&](int kk) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pa[u] = (ga < M) ? to_f64(A[(int64_t)ga * ld + kk + lk + u]) : 0.0;
            pb[u] = (gb < N) ? to_f64(B[(int64_t)gb * ld + kk + lk + u]) : 0.0;
        }
    };
    if (k0 < k1) fetch(k0);
    for (int kk = k0; kk < k1; kk += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[lk + u][lr] = pa[u];
            Bs[lk + u][lr] = pb[u];
        }
        __syncthreads();
        if (kk + 16 < k1) fetch(kk + 16);
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
    const int ldp = s->sld[MODE == 0 ? S_GPART : S_PPART];
    const int64_t pstride = (int64_t)s->n2 * ldp;
    double* part = s->slot[MODE == 0 ? S_GPART : S_PPART] + (int64_t)split * pstride;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = ti * 64 + ty * 4 + i;
        if (r >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = tj * 64 + tx * 4 + j;
            if (c < N) part[(int64_t)r * ldp + c] = acc[i][j];
        }
    }
}

// P = sum of the split-K partials of C Omega in split order (MODE 1: FP64
// partials; MODE 2: the FP32 partials of the bfloat16 matrix-core product,
// summed in FP64).
template <int MODE>
__global__ __launch_bounds__(256) void k_reduce(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind != T_SHRINK_RAND) return;
    const SkDev* s = t.s;
    const int M = t.m;
    const int N = s->k;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= M * N) return;
    const int i = idx / N, j = idx % N;
    const int splits = s->sp;
    const int ldp = s->sld[S_PPART];
    const int64_t pstride = (int64_t)s->n2 * ldp;
    double acc = 0.0;
    if (MODE == 2) {
        const float* part = (const float*)s->slot[S_PPART];
        for (int q = 0; q < splits; ++q) acc += (double)part[q * pstride + (int64_t)i * ldp + j];
    } else {
        const double* part = s->slot[S_PPART];
        for (int q = 0; q < splits; ++q) acc += part[q * pstride + (int64_t)i * ldp + j];
    }
    s->slot[S_P][(int64_t)i * s->sld[S_P] + j] = acc;
}

// G = sum of the split-K partials of C C^T in split order, for the upper
// 64 x 64 tiles the partial kernel computed; one workgroup per 16-row band
// of an upper tile writes the band and, through LDS, its mirror below the
// diagonal, both row-contiguous.
__global__ __launch_bounds__(256) void k_reduce_gram(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST) return;
    const SkDev* s = t.s;
    const int M = t.m;
    const int ntm = (M + 63) >> 6;
    const int band = blockIdx.x & 3;
    int idx = blockIdx.x >> 2;
    if (idx >= ntm * (ntm + 1) / 2) return;
    int ti = 0;
    while (idx >= ntm - ti) {
        idx -= ntm - ti;
        ++ti;
    }
    const int tj = ti + idx;
    const int splits = s->sg;
    const int ldp = s->sld[S_GPART];
    const int64_t pstride = (int64_t)s->n2 * ldp;
    const double* part = s->slot[S_GPART];
    double* G = s->slot[S_G];
    const int ldg = s->sld[S_G];
    __shared__ double tile[16][64 + 1];
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u, r = e >> 6, c = e & 63;
        const int gi = ti * 64 + band * 16 + r, gj = tj * 64 + c;
        double acc = 0.0;
        if (gi < M && gj < M) {
            for (int q = 0; q < splits; ++q) acc += part[q * pstride + (int64_t)gi * ldp + gj];
            G[(int64_t)gi * ldg + gj] = acc;
        }
        tile[r][c] = acc;
    }
    if (ti == tj) return;  // the diagonal tile holds both triangles
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u, r = e >> 4, c = e & 15;  // 64 rows x 16 columns of the mirror
        const int gi = tj * 64 + r, gj = ti * 64 + band * 16 + c;
        if (gi < M && gj < M) G[(int64_t)gi * ldg + gj] = tile[c][r];
    }
}

// ---------------------------------------------------------------- rebuild
// rows_out x d = T (rows_out x m, FP64) . C (m x d).  QUERY writes ell rows
// to the FP64 query staging; otherwise ell-1 rows to the other buffer.
template <typename Tst, bool QUERY>
__global__ __launch_bounds__(256) void k_rebuild(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind == T_INGEST) return;
    if (QUERY != (t.kind == T_QUERY)) return;
    const SkDev* s = t.s;
    const int rows_out = QUERY ? s->ell : s->ell - 1;
    const int K = t.m;
    const int N = s->d;
    // the row tiles of one column slab of C run on one XCD (xcd_tile_split
    // with the column tiles in the role of the splits): the slab is fetched once
    const int R = (rows_out + 63) >> 6, Cn = (N + 63) >> 6;
    const int L = blockIdx.x + blockIdx.y * gridDim.x;
    if (L >= R * Cn) return;
    int rt, ct;
    xcd_tile_split(L, R, Cn, &rt, &ct);
    const int r0 = rt * 64, c0 = ct * 64;
    const double* T = s->slot[S_T];
    const int ldt = s->sld[S_T];
    const Tst* X = (const Tst*)s->buf[t.par];
    const int64_t ld = s->ld;

    __shared__ double As[16][64 + 2];
    __shared__ double Bs[16][64 + 2];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    // T tile (64 rows x 16 k) and C tile (16 k rows x 64 columns; columns < ld
    // are always allocated), the next pair loaded into registers while the
    // current one is multiplied out of LDS
    const int lr = tid >> 2, lk = (tid & 3) * 4, kr = tid >> 4, lc = (tid & 15) * 4;
    double pa[4], pb[4];
    auto fetch = [&](int kk) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + lr, k = kk + lk + u;
            pa[u] = (r < rows_out && k < K) ? T[(int64_t)r * ldt + k] : 0.0;
            pb[u] = (kk + kr < K) ? to_f64(X[(int64_t)(kk + kr) * ld + c0 + lc + u]) : 0.0;
        }
    };
    if (K > 0) fetch(0);
    for (int kk = 0; kk < K; kk += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[lk + u][lr] = pa[u];
            Bs[kr][lc + u] = pb[u];
        }
        __syncthreads();
        if (kk + 16 < K) fetch(kk + 16);
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
        if (r >= rows_out) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + tx * 4 + j;
            if (c >= N) continue;
            if (QUERY)
                s->slot[S_QOUT][(int64_t)r * ld + c] = acc[i][j];
            else
                ((Tst*)s->buf[1 - t.par])[(int64_t)r * ld + c] = from_f64<Tst>(acc[i][j]);
        }
    }
}

template <typename To>
__global__ __launch_bounds__(256) void k_convert_rows(const double* src, int64_t lds, To* dst,
                                                      int64_t ldd, int rows, int cols) {
    const int r = blockIdx.y;
    if (r >= rows) return;
    for (int c = blockIdx.x * 256 + threadIdx.x; c < cols; c += gridDim.x * 256)
        dst[(int64_t)r * ldd + c] = from_f64<To>(src[(int64_t)r * lds + c]);
}

template <typename Tst>
__global__ __launch_bounds__(256) void k_rows_to_f64(const Tst* src, int64_t lds, double* dst,
                                                     int64_t ldd, int rows, int cols) {
    const int r = blockIdx.y;
    if (r >= rows) return;
    for (int c = blockIdx.x * 256 + threadIdx.x; c < cols; c += gridDim.x * 256)
        dst[(int64_t)r * ldd + c] = to_f64(src[(int64_t)r * lds + c]);
}

// ---------------------------------------------------------------- launchers
static inline dim3 g3(int x, int y, int z) { return dim3((unsigned)x, (unsigned)y, (unsigned)z); }

hipError_t launch_ingest(const Task* tasks, int count, int max_rows, int max_d, int in_dtype,
                         int st_dtype, hipStream_t st) {
    const dim3 grid = g3((max_d + 1023) / 1024, max_rows, count);
    if (st_dtype == DT_F64) {
        if (in_dtype == DT_F64) hipLaunchKernelGGL((k_ingest<double, double>), grid, dim3(256), 0, st, tasks);
        else if (in_dtype == DT_F32) hipLaunchKernelGGL((k_ingest<float, double>), grid, dim3(256), 0, st, tasks);
        else hipLaunchKernelGGL((k_ingest<uint16_t, double>), grid, dim3(256), 0, st, tasks);
    } else {
        if (in_dtype == DT_F64) hipLaunchKernelGGL((k_ingest<double, float>), grid, dim3(256), 0, st, tasks);
        else if (in_dtype == DT_F32) hipLaunchKernelGGL((k_ingest<float, float>), grid, dim3(256), 0, st, tasks);
        else hipLaunchKernelGGL((k_ingest<uint16_t, float>), grid, dim3(256), 0, st, tasks);
    }
    return hipGetLastError();
}

hipError_t launch_ingest_csr(const Task* tasks, int count, int max_rows, int max_d, int st_dtype,
                             hipStream_t st) {
    const dim3 grid = g3(1, max_rows, count);
    const size_t lds = sizeof(int) * (size_t)max_d;
    if (st_dtype == DT_F64) hipLaunchKernelGGL((k_ingest_csr<double>), grid, dim3(256), lds, st, tasks);
    else hipLaunchKernelGGL((k_ingest_csr<float>), grid, dim3(256), lds, st, tasks);
    return hipGetLastError();
}

hipError_t launch_omega(const Task* tasks, int count, int max_d, int max_k, int pj_dtype,
                        hipStream_t st) {
    const dim3 grid = g3((max_d + 255) / 256, (max_k + 3) / 4, count);
    if (pj_dtype == DT_F64) hipLaunchKernelGGL((k_omega<double>), grid, dim3(256), 0, st, tasks);
    else if (pj_dtype == DT_F32) hipLaunchKernelGGL((k_omega<float>), grid, dim3(256), 0, st, tasks);
    else hipLaunchKernelGGL((k_omega<uint16_t>), grid, dim3(256), 0, st, tasks);
    return hipGetLastError();
}

hipError_t launch_gram(const Task* tasks, int count, int max_m, int max_splits, int st_dtype,
                       hipStream_t st) {
    const int nt = (max_m + 63) / 64;
    const dim3 grid = g3(nt * (nt + 1) / 2, max_splits, count);
    if (st_dtype == DT_F64) hipLaunchKernelGGL((k_nt_partial<double, double, 0>), grid, dim3(256), 0, st, tasks);
    else hipLaunchKernelGGL((k_nt_partial<float, float, 0>), grid, dim3(256), 0, st, tasks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2 = g3(4 * (nt * (nt + 1) / 2), 1, count);
    hipLaunchKernelGGL(k_reduce_gram, g2, dim3(256), 0, st, tasks);
    return hipGetLastError();
}

hipError_t launch_project(const Task* tasks, int count, int max_m, int max_k, int max_splits,
                          int st_dtype, int pj_dtype, hipStream_t st) {
    const int ntm = (max_m + 63) / 64, ntn = (max_k + 63) / 64;
    const dim3 grid = g3(ntm * ntn, max_splits, count);
    if (st_dtype == DT_F64) {
        if (pj_dtype == DT_F64) hipLaunchKernelGGL((k_nt_partial<double, double, 1>), grid, dim3(256), 0, st, tasks);
        else if (pj_dtype == DT_F32) hipLaunchKernelGGL((k_nt_partial<double, float, 1>), grid, dim3(256), 0, st, tasks);
        else hipLaunchKernelGGL((k_nt_partial<double, uint16_t, 1>), grid, dim3(256), 0, st, tasks);
    } else {
        if (pj_dtype == DT_F64) hipLaunchKernelGGL((k_nt_partial<float, double, 1>), grid, dim3(256), 0, st, tasks);
        else if (pj_dtype == DT_F32) hipLaunchKernelGGL((k_nt_partial<float, float, 1>), grid, dim3(256), 0, st, tasks);
        else return launch_project_bf16(tasks, count, max_m, max_k, max_splits, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2 = g3((max_m * max_k + 255) / 256, 1, count);
    hipLaunchKernelGGL((k_reduce<1>), g2, dim3(256), 0, st, tasks);
    return hipGetLastError();
}

hipError_t launch_reduce_proj_f32(const Task* tasks, int count, int max_m, int max_k, hipStream_t st) {
    const dim3 g2 = g3((max_m * max_k + 255) / 256, 1, count);
    hipLaunchKernelGGL((k_reduce<2>), g2, dim3(256), 0, st, tasks);
    return hipGetLastError();
}

hipError_t launch_rebuild(const Task* tasks, int count, int max_ell, int max_d, int st_dtype,
                          bool query, hipStream_t st) {
    const dim3 grid = g3((max_d + 63) / 64, (max_ell + 63) / 64, count);
    if (st_dtype == DT_F64) {
        if (query) hipLaunchKernelGGL((k_rebuild<double, true>), grid, dim3(256), 0, st, tasks);
        else hipLaunchKernelGGL((k_rebuild<double, false>), grid, dim3(256), 0, st, tasks);
    } else {
        if (query) hipLaunchKernelGGL((k_rebuild<float, true>), grid, dim3(256), 0, st, tasks);
        else hipLaunchKernelGGL((k_rebuild<float, false>), grid, dim3(256), 0, st, tasks);
    }
    return hipGetLastError();
}

hipError_t launch_convert_rows(const double* src, int64_t lds, void* dst, int64_t ldd, int rows,
                               int cols, int out_dtype, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid = g3((cols + 255) / 256 < 64 ? (cols + 255) / 256 : 64, rows, 1);
    if (out_dtype == DT_F64)
        hipLaunchKernelGGL((k_convert_rows<double>), grid, dim3(256), 0, st, src, lds, (double*)dst, ldd, rows, cols);
    else
        hipLaunchKernelGGL((k_convert_rows<float>), grid, dim3(256), 0, st, src, lds, (float*)dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_rows_to_f64(const void* src, int64_t lds, int st_dtype, double* dst, int64_t ldd,
                              int rows, int cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid = g3((cols + 255) / 256 < 64 ? (cols + 255) / 256 : 64, rows, 1);
    if (st_dtype == DT_F64)
        hipLaunchKernelGGL((k_rows_to_f64<double>), grid, dim3(256), 0, st, (const double*)src, lds, dst, ldd, rows, cols);
    else
        hipLaunchKernelGGL((k_rows_to_f64<float>), grid, dim3(256), 0, st, (const float*)src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

}  // namespace sk
