// k_window.hip -- kernels of the sliding-window sketch (Algorithm
// "ML-AeroSketch") on gfx950.  The window engine (sk_window.cpp) drives them
// with plain pointer descriptors, one descriptor per level.
//
//   k_rownorm     |a|^2 of every arriving row (FP64), for the raw-row test
//   k_philox_mat  Gaussian d x k matrix from Philox4x64-10 (power-iteration
//                 start vector, simul_iter test matrix)
//   k_win_pi_reg  Algorithm "Power Iteration" on C'^T C' for many buffers:
//                 ceil(log2 d) + 1 normalised steps x <- C'^T C' x, then the
//                 Rayleigh quotient |C' x|^2 (the power-iteration test of
//                 Algorithm "AeroSketch: Update"), each buffer's column slabs
//                 held in the registers of its workgroups
//   k_win_gemv,   the same power iteration in the row space of C' through
//   k_win_pig     the level's Gram C' C'^T, kept between rows: one pass over
//                 C' (start vector, new Gram row), then r x r steps on one
//                 workgroup per level
//   k_gemm_desc   FP64 C = alpha op(A) op(B) + beta C for snapshot, residual
//                 and restore products and the batched simul_iter stages
//                 (split-K partials summed by k_gemm_reduce in fixed order)
//   k_blockmask   zeroes the off-entry blocks of W Z (the restore of Algorithm
//                 "AeroSketch: Query" is per snapshot)
//   k_shrink_rows rows sqrt(max(lambda_i - lambda_ell, 0)) v_i^T (the query's
//                 final shrink)
#include "sk_device.h"
#include "sk_kernels.h"
#include "sk_philox.h"

namespace sk {

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
__global__ __launch_bounds__(256) void k_philox_mat(DescArg<MatGenDesc> ds) {
    const MatGenDesc q = ds.get();
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (t >= q.rows || c >= q.cols) return;
    q.M[(int64_t)t * q.ld + c] = gauss_pick(q.seed, q.stream, (uint64_t)t, (uint64_t)(c >> 2), q.c2, q.c3, c & 3);
}


__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Power iteration of many buffers in one cooperative launch: blockIdx.y is
// the buffer, its G = ceil(d / 64) workgroups of 512 threads own 64-column
// slabs of C (r x d) and of x.  A workgroup reads its slab once into
// registers (lane = column, wave v = rows v, v + 8, ...; RPT rows per thread)
// and keeps it for every step.  One barrier per step: each workgroup writes
// the partial y = C x of its slab (x not yet normalised) and its slab's
// |x|^2; after the barrier every workgroup sums the G partials in a fixed
// order, scales y by 1 / |x| and forms its slab of the next x = C^T y.  The
// partial buffers alternate, so a buffer is rewritten only two barriers
// after it was read.
template <int RPT>
__global__ __launch_bounds__(512, (RPT > 32 ? 2 : 4)) void k_win_pi_reg(const PiDesc* ds, int G, int rmax, double* part,
                                                   unsigned* bars) {
    __shared__ double ys[8 * RPT];  // y (rows beyond r stay zero)
    __shared__ double xp[8][64];    // C^T y partials of the eight waves
    __shared__ double red[8];
    __shared__ double tb[8][8][65]; // per wave: 8 rows x 64 column products
    const int lv = blockIdx.y, wg = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const PiDesc& q = ds[lv];
    const int r = q.r, d = q.d;
    if (r <= 0) {
        if (wg == 0 && tid == 0) *q.out = 0.0;
        return;
    }
    GridBar bar{bars + 2 * lv, (unsigned)G, 0u};
    const int c = wg * 64 + lane;
    const bool cin = c < d;
    double* py = part + (int64_t)lv * 2 * G * (rmax + 1);
    double* pn = py + (int64_t)2 * G * rmax;
    double cr[RPT];
#pragma unroll
    for (int ii = 0; ii < RPT; ++ii) {
        const int i = wv + 8 * ii;
        cr[ii] = (cin && i < r) ? q.C[(int64_t)i * q.ldc + c] : 0.0;
    }
    for (int i = tid; i < 8 * RPT; i += 512) ys[i] = 0.0;
    double x = cin ? gauss_pick(q.seed, q.stream, (uint64_t)c, 0ull, q.c2, q.c3, 0) : 0.0;

    // y = C x / |x| in LDS; returns |x|^2 (the same value in every workgroup)
    // rows of y summed per step: `per` threads share a row's G partials
    const int per = r <= 64 ? 8 : r <= 128 ? 4 : r <= 256 ? 2 : 1;
    auto apply_C = [&](int b) {
        double* pyb = py + ((int64_t)b * G + wg) * rmax;
        // the slab's y partial, 8 rows of each wave at a time: the 64 column
        // products go through LDS, lane l sums row l & 7 over columns
        // 8 (l >> 3) .. 8 (l >> 3) + 7, and three exchanges add the segments
        const int jj = lane & 7, seg = lane >> 3;
#pragma unroll
        for (int h = 0; h < RPT; h += 8) {
#pragma unroll
            for (int q8 = 0; q8 < 8; ++q8) tb[wv][q8][lane] = cr[h + q8] * x;
            __syncthreads();
            double sacc = 0.0;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) sacc += tb[wv][jj][seg * 8 + cc];
            sacc += __shfl_xor(sacc, 8, 64);
            sacc += __shfl_xor(sacc, 16, 64);
            sacc += __shfl_xor(sacc, 32, 64);
            const int i = wv + 8 * (h + jj);
            if (seg == 0 && i < r) pyb[i] = sacc;
            __syncthreads();
        }
        if (wv == 0) {
            double s2 = x * x;
            for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
            if (lane == 0) pn[b * G + wg] = s2;
        }
        bar.sync();
        double tot = 0.0;
        for (int ww = 0; ww < G; ++ww) tot += pn[b * G + ww];
        const double inv = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
        {
            const int i = tid / per, p = tid % per;
            double acc = 0.0;
            if (i < r) {
#pragma unroll 4
                for (int ww = p; ww < G; ww += per) acc += py[((int64_t)b * G + ww) * rmax + i];
            }
            for (int off = 1; off < per; off <<= 1) acc += __shfl_xor(acc, off, 64);
            if (p == 0 && i < r) ys[i] = acc * inv;
        }
        __syncthreads();
        return tot;
    };

    bool zero = false;
    for (int it = 0; it < q.steps; ++it) {
        if (apply_C(it & 1) == 0.0) {  // uniform across the buffer's workgroups
            zero = true;
            break;
        }
        double a = 0.0;
#pragma unroll
        for (int ii = 0; ii < RPT; ++ii) a = fma(cr[ii], ys[wv + 8 * ii], a);
        xp[wv][lane] = a;
        __syncthreads();
        x = ((xp[0][lane] + xp[1][lane]) + (xp[2][lane] + xp[3][lane])) +
            ((xp[4][lane] + xp[5][lane]) + (xp[6][lane] + xp[7][lane]));
        __syncthreads();
    }
    double rq = 0.0;
    if (!zero && apply_C(q.steps & 1) > 0.0 && wg == 0) {
        double loc = 0.0;
        for (int i = tid; i < r; i += 512) loc = fma(ys[i], ys[i], loc);
        for (int off = 32; off > 0; off >>= 1) loc += __shfl_xor(loc, off, 64);
        if (lane == 0) red[wv] = loc;
        __syncthreads();
        rq = ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7]));
    }
    if (wg == 0 && tid == 0) {
        const bool timed_out = __hip_atomic_load(bars + 2 * lv + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        *q.out = timed_out ? __builtin_nan("") : rq;
    }
}

// ------------------------------------------------- row-space power iteration
// Pass over C: blockIdx.y = level, 4 rpw rows of C per workgroup (rpw per
// wave).  x0 (the draws of the column-slab kernel: normal 0 of the Philox
// block at counter (c, 0, c2, c3) for column c) is generated into LDS; a
// wave forms u_i = C_i . x0 and, for i <= grow, G_{grow,i} = C_i . C_grow,
// each with a fixed-order lane reduction.  Workgroup 0 also writes |x0|^2.
__global__ __launch_bounds__(256) void k_win_gemv(const GramPiDesc* ds, int rpw) {
    extern __shared__ double x0[];  // d doubles
    __shared__ double red[4];
    const GramPiDesc& q = ds[blockIdx.y];
    const int r = q.r, d = q.d;
    const int i0 = blockIdx.x * 4 * rpw;
    if (r <= 0 || i0 >= r) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int c = tid; c < d; c += 256) x0[c] = gauss_pick(q.seed, q.stream, (uint64_t)c, 0ull, q.c2, q.c3, 0);
    __syncthreads();
    if (blockIdx.x == 0) {
        double s = 0.0;
        for (int c = tid; c < d; c += 256) s = fma(x0[c], x0[c], s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[wv] = s;
        __syncthreads();
        if (tid == 0) q.u[q.ldg] = (red[0] + red[1]) + (red[2] + red[3]);
    }
    const double* a = q.grow >= 0 ? q.C + (int64_t)q.grow * q.ldc : nullptr;
    for (int t = 0; t < rpw; ++t) {
        const int i = i0 + wv * rpw + t;
        if (i >= r) break;
        const double* ci = q.C + (int64_t)i * q.ldc;
        const bool g = a != nullptr && i <= q.grow;
        double sx = 0.0, sa = 0.0;
        if (g) {
            for (int c = lane; c < d; c += 64) {
                const double v = ci[c];
                sx = fma(v, x0[c], sx);
                sa = fma(v, a[c], sa);
            }
        } else {
            for (int c = lane; c < d; c += 64) sx = fma(ci[c], x0[c], sx);
        }
        for (int off = 32; off > 0; off >>= 1) {
            sx += __shfl_xor(sx, off, 64);
            sa += __shfl_xor(sa, off, 64);
        }
        if (lane == 0) {
            q.u[i] = sx;
            if (g) {
                q.G[(int64_t)q.grow * q.ldg + i] = sa;
                q.G[(int64_t)i * q.ldg + q.grow] = sa;
            }
        }
    }
}

// Steps, one workgroup of 1024 threads per level.  With y = u / |x0|:
// `steps` times { v = G y; n = y . v; y = v / sqrt(n) }, then out = |y|^2.
// In exact arithmetic this is the column-slab kernel's sequence (its
// y = C x / |x|, x <- C^T y, and |x|^2 = y^T G y for the next x).  Column j
// of G goes to the threads j mod R (R = r rounded up to a power of two
// >= 64); the rows are cut into P = 1024 / R chunks, one per thread group,
// and the chunk partials are added in chunk order.  G is read once from
// memory: the first cpc rows of every chunk are kept in LDS (lds_doubles of
// dynamic LDS) and the next kPigRegs in each thread's registers; only the
// rest of a chunk is re-read at every step.
static constexpr int kPigRegs = 16;
__global__ __launch_bounds__(1024) void k_win_pig(const GramPiDesc* ds, int lds_doubles) {
    extern __shared__ double gl[];
    __shared__ double y[1024];
    __shared__ double part[1024];
    __shared__ double red[16];
    const GramPiDesc& q = ds[blockIdx.x];
    const int r = q.r, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (r <= 0) {
        if (tid == 0) *q.out = 0.0;
        return;
    }
    int R = 64;
    while (R < r) R <<= 1;
    const int P = 1024 / R, j = tid % R, p = tid / R;
    const int per = (r + P - 1) / P;
    const int ib = p * per, ie = min(r, ib + per);
    const int cpc = min(per, lds_doubles / (P * r));
    const double* G = q.G;
    const int64_t ldg = q.ldg;
    for (int e = tid; e < P * cpc * r; e += 1024) {
        const int row = e / r, c = e - row * r;
        const int i = (row / cpc) * per + row % cpc;
        gl[e] = i < r ? G[(int64_t)i * ldg + c] : 0.0;
    }
    double rg[kPigRegs];
#pragma unroll
    for (int t = 0; t < kPigRegs; ++t) {
        const int i = ib + cpc + t;
        rg[t] = (j < r && i < ie) ? G[(int64_t)i * ldg + j] : 0.0;
    }
    const int i_mem = min(ie, ib + cpc + kPigRegs);
    const double* gll = gl + (int64_t)p * cpc * r;
    // block sum in a fixed order (the same value in every thread)
    auto block_total = [&](double v) -> double {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        __syncthreads();
        if (lane == 0) red[wv] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) s += red[w];
        return s;
    };
    const double n0 = q.u[q.ldg];
    const double inv0 = n0 > 0.0 ? 1.0 / sqrt(n0) : 0.0;
    if (tid < r) y[tid] = q.u[tid] * inv0;
    __syncthreads();
    bool zero = !(n0 > 0.0);
    for (int it = 0; it < q.steps && !zero; ++it) {
        double acc = 0.0;
        if (j < r) {
            const int il = min(ie, ib + cpc);
#pragma unroll 8
            for (int i = ib; i < il; ++i) acc = fma(gll[(i - ib) * r + j], y[i], acc);
#pragma unroll
            for (int t = 0; t < kPigRegs; ++t) {
                const int i = ib + cpc + t;
                if (i < ie) acc = fma(rg[t], y[i], acc);
            }
#pragma unroll 8
            for (int i = i_mem; i < ie; ++i) acc = fma(G[(int64_t)i * ldg + j], y[i], acc);
        }
        part[tid] = acc;
        __syncthreads();
        double v = 0.0;
        if (tid < r)
            for (int pp = 0; pp < P; ++pp) v += part[pp * R + tid];
        const double n = block_total(tid < r ? v * y[tid] : 0.0);
        if (!(n > 0.0)) {
            zero = true;
            break;
        }
        if (tid < r) y[tid] = v * (1.0 / sqrt(n));
        __syncthreads();
    }
    const double rq = zero ? 0.0 : block_total(tid < r ? y[tid] * y[tid] : 0.0);
    if (tid == 0) *q.out = rq;
}

hipError_t launch_win_pi_gram(const void* descs, int count, int max_r, int max_d, hipStream_t st) {
    if (count <= 0 || max_r <= 0) return hipSuccess;
    if (max_r > 1024 || max_d < 1 || max_d > 4096) return hipErrorInvalidValue;
    // dynamic LDS of the step kernel: what the device grants beyond the
    // static arrays, at most 160 KiB in all (none if the request fails)
    static int pig_lds = -1;
    if (pig_lds < 0) {
        int dev = 0, cap = 0;
        pig_lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cap, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess) {
            const int stat = (int)(sizeof(double) * (1024 + 1024 + 16));
            int want = (cap < 160 * 1024 ? cap : 160 * 1024) - stat;
            want = want / 8 * 8;
            if (want > 0 && hipFuncSetAttribute((const void*)k_win_pig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                want) == hipSuccess)
                pig_lds = want;
        }
        (void)hipGetLastError();
    }
    hipError_t e = launch_win_gemv(descs, count, max_r, max_d, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_win_pig, dim3((unsigned)count), dim3(1024), (size_t)pig_lds, st, (const GramPiDesc*)descs,
                       pig_lds / 8);
    return hipGetLastError();
}

hipError_t launch_win_gemv(const void* descs, int count, int max_r, int max_d, hipStream_t st) {
    if (count <= 0 || max_r <= 0) return hipSuccess;
    if (max_d < 1 || max_d > 4096) return hipErrorInvalidValue;
    // rows of C per wave: enough workgroups to cover the chip (about 1024)
    const int wg4 = count * ((max_r + 15) / 16);
    const int rpw = wg4 >= 1024 ? 4 : wg4 >= 512 ? 2 : 1;
    const int rows_wg = 4 * rpw;
    hipLaunchKernelGGL(k_win_gemv, dim3((unsigned)((max_r + rows_wg - 1) / rows_wg), (unsigned)count), dim3(256),
                       sizeof(double) * (size_t)max_d, st, (const GramPiDesc*)descs, rpw);
    return hipGetLastError();
}

// ---------------------------------------------------------------- GEMM
// One 64 x 64 tile (r0, c0) of C = alpha op(A) op(B) + beta C, 256 threads.
__device__ void gemm_tile(const GemmDesc& g, int r0, int c0) {
    const int M = g.M, N = g.N, K = g.K;
    if (r0 >= M || c0 >= N) return;
    __shared__ double As[16][64 + 2];
    __shared__ double Bs[16][64 + 2];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    // the next K slice is fetched into registers while the current one is
    // multiplied (the sum over K keeps its order)
    double pa[4], pb[4];
    auto fetch = [&](int kk) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            if (!g.ta) {
                const int r = e >> 4, k = e & 15;
                pa[u] = (r0 + r < M && kk + k < K) ? g.A[(int64_t)(r0 + r) * g.lda + kk + k] : 0.0;
            } else {
                const int r = e & 63, k = e >> 6;
                pa[u] = (r0 + r < M && kk + k < K) ? g.A[(int64_t)(kk + k) * g.lda + r0 + r] : 0.0;
            }
            if (!g.tb) {
                const int c = e & 63, k = e >> 6;
                pb[u] = (c0 + c < N && kk + k < K) ? g.B[(int64_t)(kk + k) * g.ldb + c0 + c] : 0.0;
            } else {
                const int c = e >> 4, k = e & 15;
                pb[u] = (c0 + c < N && kk + k < K) ? g.B[(int64_t)(c0 + c) * g.ldb + kk + k] : 0.0;
            }
        }
    };
    fetch(0);
    for (int kk = 0; kk < K; kk += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            if (!g.ta) As[e & 15][e >> 4] = pa[u];
            else As[e >> 6][e & 63] = pa[u];
            if (!g.tb) Bs[e >> 6][e & 63] = pb[u];
            else Bs[e & 15][e >> 4] = pb[u];
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

__global__ __launch_bounds__(256) void k_gemm_desc(DescArg<GemmDesc> ds) {
    gemm_tile(ds.get(), blockIdx.y * 64, blockIdx.x * 64);
}

// Split-K partial of one GEMM descriptor: blockIdx.z = split, blockIdx.y/x
// = 64 x 64 tile; part[split] = op(A)[:, chunk] op(B)[chunk, :].
__global__ __launch_bounds__(256) void k_gemm_part(DescArg<GemmDesc> dp) {
    GemmDesc g = dp.one;
    const int s = blockIdx.z;
    const int kb = s * g.kchunk, ke = min(g.K, kb + g.kchunk);
    if (kb >= ke) return;
    // shift A and B to the chunk and compute an ordinary product into part[s]
    g.A = g.ta ? g.A + (int64_t)kb * g.lda : g.A + kb;
    g.B = g.tb ? g.B + kb : g.B + (int64_t)kb * g.ldb;
    g.K = ke - kb;
    g.C = g.part + (int64_t)s * g.M * g.N;
    g.ldc = g.N;
    g.alpha = 1.0;
    g.beta = 0.0;
    gemm_tile(g, blockIdx.y * 64, blockIdx.x * 64);
}

// C = alpha * (sum of the splits in order) + beta C.
__global__ __launch_bounds__(256) void k_gemm_reduce(DescArg<GemmDesc> dp) {
    const GemmDesc g = dp.get();
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)g.M * g.N) return;
    double acc = 0.0;
    for (int s = 0; s < g.nsplit; ++s) acc += g.part[(int64_t)s * g.M * g.N + e];
    const int r = (int)(e / g.N), c = (int)(e % g.N);
    double* p = g.C + (int64_t)r * g.ldc + c;
    *p = (g.beta == 0.0) ? g.alpha * acc : fma(g.alpha, acc, g.beta * *p);
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
    DescArg<MatGenDesc> a{(const MatGenDesc*)descs, {}};
    hipLaunchKernelGGL(k_philox_mat, dim3((unsigned)((max_rows + 255) / 256), (unsigned)max_cols, (unsigned)count),
                       dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_philox_mat1(const MatGenDesc& m, hipStream_t st) {
    DescArg<MatGenDesc> a{nullptr, m};
    hipLaunchKernelGGL(k_philox_mat, dim3((unsigned)((m.rows + 255) / 256), (unsigned)m.cols, 1u), dim3(256), 0, st, a);
    return hipGetLastError();
}

int win_pi_groups(int d) {
    const int g = (d + 63) / 64;
    return g < 1 ? 1 : g;
}

template <int RPT>
static hipError_t launch_pi_rpt(const PiDesc* dp, int count, int G, int max_r, double* part, unsigned* bars,
                                hipStream_t st) {
    // buffers per cooperative launch: as many as are resident at once
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0, nb = 0;
        hipDeviceProp_t prop{};
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_win_pi_reg<RPT>, 512, 0) != hipSuccess)
            return hipErrorInvalidConfiguration;
        per_cu = nb;
        cus = prop.multiProcessorCount;
    }
    const int fit = per_cu * cus / G;
    if (fit < 1) return hipErrorCooperativeLaunchTooLarge;
    for (int b = 0; b < count; b += fit) {
        const int n = count - b < fit ? count - b : fit;
        hipError_t e = hipMemsetAsync(bars, 0, sizeof(unsigned) * 2 * (size_t)n, st);
        if (e != hipSuccess) return e;
        const PiDesc* d0 = dp + b;
        int gg = G, rm = max_r;
        void* kargs[] = {(void*)&d0, (void*)&gg, (void*)&rm, (void*)&part, (void*)&bars};
        e = hipLaunchCooperativeKernel((const void*)k_win_pi_reg<RPT>, dim3((unsigned)G, (unsigned)n), dim3(512), kargs,
                                       0, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_win_pi(const void* descs, int count, int d, int max_r, double* part, unsigned* bars,
                         hipStream_t st) {
    const int G = win_pi_groups(d);
    const PiDesc* dp = (const PiDesc*)descs;
    if (max_r <= 64) return launch_pi_rpt<8>(dp, count, G, max_r, part, bars, st);
    if (max_r <= 128) return launch_pi_rpt<16>(dp, count, G, max_r, part, bars, st);
    if (max_r <= 256) return launch_pi_rpt<32>(dp, count, G, max_r, part, bars, st);
    if (max_r <= 512) return launch_pi_rpt<64>(dp, count, G, max_r, part, bars, st);
    return hipErrorInvalidValue;
}

hipError_t launch_gemm_split(const GemmDesc& g, hipStream_t st) {
    DescArg<GemmDesc> a{nullptr, g};
    hipLaunchKernelGGL(k_gemm_part, dim3((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)g.nsplit),
                       dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gemm_reduce_desc(const GemmDesc* ds, int count, int64_t max_MN, hipStream_t st) {
    DescArg<GemmDesc> a{ds, {}};
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((max_MN + 255) / 256), 1u, (unsigned)count), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

hipError_t launch_gemm_desc(const GemmDesc* ds, int count, int max_M, int max_N, hipStream_t st) {
    DescArg<GemmDesc> a{ds, {}};
    hipLaunchKernelGGL(k_gemm_desc, dim3((unsigned)((max_N + 63) / 64), (unsigned)((max_M + 63) / 64), (unsigned)count),
                       dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gemm1(const GemmDesc& g, hipStream_t st) {
    DescArg<GemmDesc> a{nullptr, g};
    hipLaunchKernelGGL(k_gemm_desc, dim3((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), 1u), dim3(256), 0,
                       st, a);
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
