// k_mfma.hip -- the random projection C Omega on the bfloat16 matrix cores of
// gfx950 (v_mfma_f32_32x32x16_bf16), FP32 accumulation within a K chunk,
// FP64 across chunks (the FP32 split-K partials go through k_reduce<2>).
//
// Operands come straight from global memory into registers: for the
// 32x32x16 instruction lane l holds row (l mod 32) of the A tile and column
// (l mod 32) of the B tile, each with the 8 consecutive k-values starting at
// 8 * (l / 32).  Both C (m x d) and Omega^T (k x d) are k-contiguous, so each
// lane reads 8 consecutive elements of one row.  The buffer is FP32 and is
// rounded to bfloat16 (nearest-even) in registers; Omega^T is stored in
// bfloat16.  Each wave owns a 32 x 32 output tile; a workgroup of 4 waves
// covers 64 x 64.
#include "sk_device.h"
#include "sk_kernels.h"

namespace sk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

union Bf8 {
    bf16x8 v;
    uint16_t h[8];
    uint4 q;
};

__global__ __launch_bounds__(256) void k_proj_bf16(const Task* tasks) {
    const Task& t = tasks[blockIdx.z];
    if (t.kind != T_SHRINK_RAND) return;
    const SkDev* s = t.s;
    const int M = t.m, N = s->k;
    const int splits = s->sp, kc = s->kcp;
    const int ntn = (N + 63) >> 6, ntm = (M + 63) >> 6;
    const int L = blockIdx.x + blockIdx.y * gridDim.x;
    if (L >= ntm * ntn * splits) return;
    int tile, split;
    xcd_tile_split(L, ntm * ntn, splits, &tile, &split);
    const int ti = tile / ntn, tj = tile % ntn;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = ti * 64 + (wave >> 1) * 32;   // first row of this wave's tile
    const int wc = tj * 64 + (wave & 1) * 32;    // first column
    const int64_t ld = s->ld;
    const float* A = (const float*)s->buf[t.par];
    const uint16_t* B = (const uint16_t*)s->omegaT;
    const int kend = (s->d + 15) & ~15;
    const int k0 = split * kc;
    const int k1 = min(k0 + kc, kend);
    const int ar = wr + (lane & 31), bc = wc + (lane & 31);
    const int koff = (lane >> 5) * 8;
    const bool a_ok = ar < M, b_ok = bc < N;
    const float* ap = A + (int64_t)(a_ok ? ar : 0) * ld + koff;
    const uint16_t* bp = B + (int64_t)(b_ok ? bc : 0) * ld + koff;
    floatx16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int kk = k0; kk < k1; kk += 16) {
        Bf8 a, b;
        if (a_ok) {
            const float4 x0 = *(const float4*)(ap + kk);
            const float4 x1 = *(const float4*)(ap + kk + 4);
            a.h[0] = f32_to_bf16_rne(x0.x); a.h[1] = f32_to_bf16_rne(x0.y);
            a.h[2] = f32_to_bf16_rne(x0.z); a.h[3] = f32_to_bf16_rne(x0.w);
            a.h[4] = f32_to_bf16_rne(x1.x); a.h[5] = f32_to_bf16_rne(x1.y);
            a.h[6] = f32_to_bf16_rne(x1.z); a.h[7] = f32_to_bf16_rne(x1.w);
        } else {
            a.q = make_uint4(0u, 0u, 0u, 0u);
        }
        if (b_ok) b.q = *(const uint4*)(bp + kk);
        else b.q = make_uint4(0u, 0u, 0u, 0u);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b.v, acc, 0, 0, 0);
    }
    // FP32 partials (what the matrix cores accumulated; summed in FP64 by
    // k_reduce<2>)
    const int ldp = s->sld[S_PPART];
    float* part = (float*)s->slot[S_PPART] + (int64_t)split * (int64_t)s->n2 * ldp;
    const int col = wc + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = wr + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
        if (row < M && col < N) part[(int64_t)row * ldp + col] = acc[i];
    }
}

hipError_t launch_project_bf16(const Task* tasks, int count, int max_m, int max_k, int max_splits,
                               hipStream_t st) {
    const int ntm = (max_m + 63) / 64, ntn = (max_k + 63) / 64;
    hipLaunchKernelGGL(k_proj_bf16, dim3((unsigned)(ntm * ntn), (unsigned)max_splits, (unsigned)count),
                       dim3(256), 0, st, tasks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_proj_f32(tasks, count, max_m, max_k, st);
}

}  // namespace sk
