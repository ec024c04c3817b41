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
    int32_t* info;             // [0]: non-converged eigen-solves, [1]: max sweeps
    uint64_t seed, stream;
};

enum TaskKind : int32_t { T_INGEST = 0, T_SHRINK_EXACT = 1, T_SHRINK_RAND = 2, T_QUERY = 3 };

struct Task {
    const SkDev* s;
    int32_t kind;
    int32_t par;               // index of the current buffer
    int32_t m;                 // buffer rows taking part (2 ell for a shrink)
    int32_t row0;              // ingest: first destination row
    int32_t nrows;             // ingest: rows to copy
    int32_t src_dtype;         // ingest: dtype of src
    int64_t shrink_idx;        // Philox counter word of this shrink
    int64_t src_ld;            // ingest: leading dimension of src
    const void* src;           // ingest: source rows (device)
    const int64_t* indptr;     // CSR ingest (src == nullptr)
    const int32_t* indices;
    const float* values;
};

// Eigen-problem size of a task: the buffer rows (exact shrink / query) or k.
__host__ __device__ inline int eig_n(const Task& t) {
    return t.kind == T_SHRINK_RAND ? t.s->k : t.m;
}

}  // namespace sk
