// k_cod.hip -- kernels of the approximate-matrix-multiplication window
// (Algorithm "AeroSketchCOD Framework") on gfx950:
//
//   k_cod_scale  columns of a matrix scaled by functions of eigenvalues: the
//                factors of the co-occurring-directions reduce (square roots
//                and inverse square roots of a Gram's eigenvalues, the shrink
//                gains sqrt(max(s - s_ell, 0)) / s) and the query's shrink
//   k_cod_pi     Algorithm "Power Iteration" on M = A^T B (x <- M^T M x in
//                R^{d_y}) carried out in the row space of the buffers: with
//                u = B x, G_x = A A^T and G_y = B B^T one step is
//                u <- G_y G_x u / |B^T G_x u| and |M x|^2 = u^T G_x u, the
//                same iteration in exact arithmetic
#include "sk_device.h"
#include "sk_kernels.h"

namespace sk {

// f(c) of column c from the eigenvalues lam (n of them, descending).
__device__ __forceinline__ double cod_factor(const double* lam, int n, int c, int mode, double tol, int ell) {
    const double l0 = n > 0 ? lam[0] : 0.0;
    const double lc = c < n ? lam[c] : 0.0;
    const bool kept = l0 > 0.0 && lc > tol * l0;
    switch (mode) {
        case COD_SQRT: return kept ? sqrt(lc) : 0.0;
        case COD_INVSQRT: return kept ? 1.0 / sqrt(lc) : 0.0;
        case COD_KEPT: return kept ? 1.0 : 0.0;
        default: break;
    }
    // shrink of the singular values s_c = sqrt(lam_c) by s_ell; eigenvalues
    // at or below tol lam_0 are taken as zero (below that the rounding of
    // the Gram, about n eps lam_0, decides them)
    const double sc = kept ? sqrt(lc) : 0.0;
    const double le = n >= ell ? lam[ell - 1] : 0.0;
    const double de = (l0 > 0.0 && le > tol * l0) ? sqrt(le) : 0.0;
    const double sh = fmax(sc - de, 0.0);
    if (mode == COD_SHRINK_SQRT) return sqrt(sh);
    return (sc > 0.0 && sh > 0.0) ? sqrt(sh) / sc : 0.0;  // COD_SHRINK_GAIN
}

// dst[i][c] = src[i][c] * f(c), i < rows, c < cols; blockIdx.y = column.
__global__ __launch_bounds__(256) void k_cod_scale(const double* src, int lds, double* dst, int ldd, int rows, int cols,
                                                  const double* lam, int n, int mode, double tol, int ell) {
    const int c = blockIdx.y;
    if (c >= cols) return;
    const double f = cod_factor(lam, n, c, mode, tol, ell);
    for (int i = blockIdx.x * 256 + threadIdx.x; i < rows; i += gridDim.x * 256)
        dst[(int64_t)i * ldd + c] = src[(int64_t)i * lds + c] * f;
}

hipError_t launch_cod_scale(const double* src, int lds, double* dst, int ldd, int rows, int cols, const double* lam,
                            int n, int mode, double tol, int ell, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    int bx = (rows + 255) / 256;
    if (bx > 64) bx = 64;
    hipLaunchKernelGGL(k_cod_scale, dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, st, src, lds, dst, ldd, rows, cols,
                       lam, n, mode, tol, ell);
    return hipGetLastError();
}

__device__ double cod_block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += red[w];
    __syncthreads();
    return s;
}

// One workgroup; r <= 512.  u0 = B x0, n0 = |x0|^2; out = |M x|^2 after
// `steps` normalised steps (0 when an iterate vanishes).  With IN_LDS the two
// Grams are first copied to LDS (dynamic, 2 r^2 doubles).  The Grams are
// exactly symmetric (both triangles come from the same products), so row i
// of a product is read as column i: consecutive threads then read
// consecutive words (no LDS bank conflicts, coalesced from memory).
template <bool IN_LDS>
__global__ __launch_bounds__(256) void k_cod_pi(const double* Gx0, const double* Gy0, int ld0, const double* u0,
                                               const double* n0, int r, int steps, double* out) {
    __shared__ double u[512], v[512], w[512];
    __shared__ double red[4];
    extern __shared__ double gl[];
    const int tid = threadIdx.x;
    // (a compile-time choice, so that LDS reads compile to LDS instructions)
    if (IN_LDS)
        for (int e = tid; e < r * r; e += 256) {
            gl[e] = Gx0[(int64_t)(e / r) * ld0 + e % r];
            gl[r * r + e] = Gy0[(int64_t)(e / r) * ld0 + e % r];
        }
    const double* Gx = IN_LDS ? gl : Gx0;
    const double* Gy = IN_LDS ? gl + r * r : Gy0;
    const int ld = IN_LDS ? r : ld0;
    const double nn = *n0;
    const double inv0 = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int i = tid; i < r; i += 256) u[i] = u0[i] * inv0;
    __syncthreads();
    bool zero = !(nn > 0.0);
    for (int it = 0; it < steps && !zero; ++it) {
        for (int i = tid; i < r; i += 256) {
            double a = 0.0;
#pragma unroll 8
            for (int j = 0; j < r; ++j) a = fma(Gx[(int64_t)j * ld + i], u[j], a);
            v[i] = a;
        }
        __syncthreads();
        double loc = 0.0;
        for (int i = tid; i < r; i += 256) {
            double a = 0.0;
#pragma unroll 8
            for (int j = 0; j < r; ++j) a = fma(Gy[(int64_t)j * ld + i], v[j], a);
            w[i] = a;
            loc = fma(v[i], a, loc);
        }
        const double nz2 = cod_block_sum(loc, red);
        if (!(nz2 > 0.0)) {
            zero = true;
            break;
        }
        const double inv = 1.0 / sqrt(nz2);
        for (int i = tid; i < r; i += 256) u[i] = w[i] * inv;
        __syncthreads();
    }
    double loc = 0.0;
    if (!zero)
        for (int i = tid; i < r; i += 256) {
            double a = 0.0;
#pragma unroll 8
            for (int j = 0; j < r; ++j) a = fma(Gx[(int64_t)j * ld + i], u[j], a);
            loc = fma(u[i], a, loc);
        }
    const double rq = cod_block_sum(loc, red);
    if (tid == 0) *out = zero ? 0.0 : rq;
}

hipError_t launch_cod_pi(const double* Gx, const double* Gy, int ld, const double* u0, const double* n0, int r,
                         int steps, double* out, hipStream_t st) {
    if (r < 1 || r > 512) return hipErrorInvalidValue;
    // LDS for the Grams of r <= 64 (64 KiB beside the 12 KiB of vectors)
    static int lds_cap = -1;
    if (lds_cap < 0) {
        const int want = (int)(sizeof(double) * 2 * 64 * 64);
        lds_cap = hipFuncSetAttribute((const void*)k_cod_pi<true>, hipFuncAttributeMaxDynamicSharedMemorySize, want) ==
                          hipSuccess
                      ? want
                      : 0;
        (void)hipGetLastError();
    }
    const size_t need = sizeof(double) * 2 * (size_t)r * r;
    const int in_lds = need <= (size_t)lds_cap ? 1 : 0;
    if (in_lds)
        hipLaunchKernelGGL(k_cod_pi<true>, dim3(1), dim3(256), need, st, Gx, Gy, ld, u0, n0, r, steps, out);
    else
        hipLaunchKernelGGL(k_cod_pi<false>, dim3(1), dim3(256), 0, st, Gx, Gy, ld, u0, n0, r, steps, out);
    return hipGetLastError();
}

}  // namespace sk
