// sk_device.h -- structures shared by the host engine and the gfx950 kernels.
//
// Every pipeline kernel reads a list of Task records from device memory; the
// task index is blockIdx.z.  A single sketch is a batch of one; the batched
// update and the merge tree launch the same kernels with longer lists, so
// sketches of different d and ell share one launch per stage.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

enum DType : int32_t { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// FP64 scratch matrices of a sketch, addressed by slot so that one generic
// small-GEMM kernel serves every product of the shrink's core.
enum Slot : int32_t {
    S_G = 0,   // m x m   Gram of the buffer rows, C C^T
    S_P,       // m x k   C Omega
    S_Y,       // m x k   power-step iterate
    S_Q,       // m x k   orthonormal basis
    S_Q1,      // m x k   first CholeskyQR pass
    S_W,       // k x k   Gram of the basis being orthonormalised
    S_X,       // k x k   inverse Cholesky factor (lower)
    S_T1,      // m x k   G Q
    S_M,       // k x k   Rayleigh-Ritz matrix Q^T G Q
    S_U,       // n x n   eigenvectors (sorted, descending eigenvalues)
    S_Z,       // m x k   Q U
    S_T,       // ell x m rebuild matrix diag(f) Z^T
    S_LAM,     // n       eigenvalues, descending
    S_EA,      // n x n   eigen-solver work matrix (matrices too big for LDS)
    S_EV,      // n x n   eigen-solver rotations
    S_GPART,   // splits x m x m   split-K partials of the Gram
    S_PPART,   // splits x m x k   split-K partials of C Omega
    S_QOUT,    // ell x d query staging (FP64)
    NSLOT
};

struct SkDev {
    int32_t d, ell, n2, k;     // n2 = 2 ell buffer rows; k = target rank (rand)
    int32_t st, pj;            // state dtype, projection dtype
    int32_t sg, kcg;           // Gram split-K: number of splits, chunk (columns)
    int32_t sp, kcp;           // projection split-K
    int64_t ld;                // buffer leading dimension (elements), multiple of 64
    void* buf[2];              // the two state buffers, n2 x ld each
    void* omegaT;              // k x ld, projection dtype
    double* slot[NSLOT];
    int32_t sld[NSLOT];        // leading dimension of each slot
    int32_t* info;             // [0]: non-converged eigen-solves, [1]: max sweeps, [2]: eigen fall-backs,
                               // [3]: exchange timeouts, [8]: second CholeskyQR pass taken by the polar step
    uint64_t seed, stream;
    double* coop;              // cooperative-solver scratch (COOP_* layout)
    int32_t* coop_ctrl;        // [0..1] rotation counters, [8..9] grid barrier
    uint64_t* xflags;          // 64 exchange flags of the multi-workgroup CholeskyQR
};

// Cooperative scratch layout (doubles): 16 pair-block rotations of 32 x 32,
// 256 partial sums, 16 inverse diagonal blocks of 32 x 32, 512 pivots, stats.
constexpr int64_t COOP_UBUF = 0, COOP_PART = 16 * 1024, COOP_LINV = COOP_PART + 256,
                  COOP_D0 = COOP_LINV + 16 * 1024, COOP_STATS = COOP_D0 + 512,
                  COOP_DOUBLES = COOP_STATS + 16;


enum TaskFlags : int32_t { TF_COOP_EIG = 1, TF_COOP_CHOL = 2, TF_X_CHOL = 4 };

enum TaskKind : int32_t { T_INGEST = 0, T_SHRINK_EXACT = 1, T_SHRINK_RAND = 2, T_QUERY = 3 };

struct Task {
    const SkDev* s;
    int32_t kind;
    int32_t par;               // index of the current buffer
    int32_t m;                 // buffer rows taking part (2 ell for a shrink)
    int32_t row0;              // ingest: first destination row
    int32_t nrows;             // ingest: rows to copy
    int32_t src_dtype;         // ingest: dtype of src
    int32_t flags;             // TF_*: stages solved by the cooperative / multi-workgroup kernels
    int32_t pad0;
    int64_t shrink_idx;        // Philox counter word of this shrink
    int64_t src_ld;            // ingest: leading dimension of src
    const void* src;           // ingest: source rows (device)
    const int64_t* indptr;     // CSR ingest (src == nullptr)
    const int32_t* indices;
    const float* values;
};

// Task list of one multi-task cooperative launch: task idx[i] of `tasks`
// owns workgroups [i * gper, (i + 1) * gper).
constexpr int COOP_MAX_TASKS = 64;
struct CoopList {
    const Task* tasks;
    int32_t count, gper;
    int32_t sy, sq, passes, pad;   // CholeskyQR: input / output slots, passes
    int32_t idx[COOP_MAX_TASKS];
};

// Descriptor of one small dense FP64 problem for the pointer-driven kernels
// (window sketches): Cholesky-inverse (A -> X) or eigen-decomposition
// (A -> X = eigenvectors, lam).  work / work2: n x n scratch.
struct SmallDesc {
    const double* A;
    double* X;
    double* lam;
    double* work;
    double* work2;
    int32_t* info;
    int32_t n, lda, ldx, pad;
};

// Descriptor of one FP64 product C = alpha op(A) op(B) + beta C.
// With nsplit > 1 the K range is cut into nsplit chunks of kchunk: the
// partial products go to part (nsplit x M x N) and a fixed-order reduction
// writes C, so the result does not depend on the launch shape.
struct GemmDesc {
    const double* A;
    const double* B;
    double* C;
    int32_t M, N, K;
    int32_t lda, ldb, ldc;
    int32_t ta, tb;
    double alpha, beta;
    double* part;
    int32_t nsplit, kchunk;
};

// Gaussian matrix from Philox: M[t][c] = normal (c mod 4) of the block at
// counter (t, c / 4, c2, c3), key (seed, stream).
struct MatGenDesc {
    double* M;
    int32_t rows, cols, ld, pad;
    uint64_t seed, stream, c2, c3;
};

// Column factors of the approximate-matrix-multiplication kernels (k_cod.hip).
enum CodScale { COD_SQRT = 0, COD_INVSQRT = 1, COD_KEPT = 2, COD_SHRINK_GAIN = 3, COD_SHRINK_SQRT = 4 };

// Power iteration of one window level on C (r x d).  out receives the
// Rayleigh quotient, or NaN when a grid barrier of the cooperative kernel
// timed out.
struct PiDesc {
    const double* C;
    double* out;
    int64_t ldc;
    int32_t r, d, steps, pad;
    uint64_t seed, stream, c2, c3;
};

// The same power iteration carried out in the row space of C through the
// level's Gram G = C C^T (r x r, ld ldg, kept between rows): u = C x0 and
// |x0|^2 come from one pass over C, which also fills row and column grow of
// G (the row appended since G was last complete; grow < 0: G is complete),
// and the steps are r x r products.  u holds ldg + 1 doubles (u, then
// |x0|^2).
struct GramPiDesc {
    const double* C;
    double* out;
    double* G;
    double* u;
    int64_t ldc;
    int32_t r, d, steps, grow, ldg, pad;
    uint64_t seed, stream, c2, c3;
};

// Arguments of the cooperative block-Jacobi eigen-solver.
struct CoopEig {
    const double* Ain;   // n x n symmetric input (ld ldin)
    double* A;           // N x N work (N = n rounded up to 32)
    double* V;           // N x N rotations
    double* U;           // n x n sorted eigenvectors (ld lu)
    double* lam;         // n eigenvalues, descending
    int32_t* info;       // [0] non-converged solves, [1] max sweeps
    double* ubuf;        // (N / 32) x 32 x 32 pair-block rotations
    double* part;        // >= gridDim doubles
    int32_t* ctrl;       // 2 rotation counters
    double* stats;       // 8 diagnostic accumulators
    uint32_t* bar;       // grid barrier (2 words, zeroed before launch)
    int32_t n, ldin, lu, pad;
};

// Grid barrier for a cooperative launch: an arrival counter (zeroed by the
// host before the launch) with agent-scope release on arrival and acquire
// while waiting.  Every workgroup is resident (cooperative launch), so every
// wait ends; the spin is bounded all the same and records a timeout in
// bar[1] instead of hanging.
struct GridBar {
    unsigned* bar;
    unsigned nblk;
    unsigned epoch;
    __device__ void sync() {
        __syncthreads();
        if (threadIdx.x == 0) {
            ++epoch;
            const unsigned target = epoch * nblk;
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            // relaxed polls, then one acquire fence: the fence pairs with the
            // release increments whose count the last poll read, without a
            // cache invalidation per poll
            unsigned spins = 0;
            while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1u << 26)) {
                    __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
    }
};

// Descriptor argument of the pointer-driven kernels: a device list indexed by
// blockIdx.z, or (list == nullptr) one descriptor passed by value, which
// saves the host-to-device copy of a single descriptor.
template <typename D>
struct DescArg {
    const D* list;
    D one;
    __device__ D get() const { return list ? list[blockIdx.z] : one; }
};

// Eigen-problem size of a task: the buffer rows (exact shrink / query) or k.
__host__ __device__ inline int eig_n(const Task& t) {
    return t.kind == T_SHRINK_RAND ? t.s->k : t.m;
}

// Workgroups are handed to the eight XCDs (each with its own L2) round-robin
// in linear launch order.  xcd_tile_split maps a workgroup's linear index L
// in [0, tiles * splits) of one task to (tile, split) so that, when splits is
// a multiple of 8, every tile of one split (one K chunk of the operands) runs
// on the same XCD: the chunk is fetched from HBM once and re-read from that
// L2.  Any other split count gets the plain row-major map.  Results do not
// depend on the map (each (tile, split) product is the same arithmetic).
__device__ __forceinline__ void xcd_tile_split(int L, int tiles, int splits, int* tile, int* split) {
    if ((splits & 7) == 0) {
        const int j = L >> 3;
        *split = (L & 7) + 8 * (j / tiles);
        *tile = j % tiles;
    } else {
        *tile = L % tiles;
        *split = L / tiles;
    }
}

}  // namespace sk
