// sk_kernels.h -- host-side launchers of the gfx950 kernels.  Every launcher
// takes a device array of `count` Task records; the max_* arguments size the
// grid to the largest task, smaller tasks exit their surplus workgroups.
#pragma once
#include <hip/hip_runtime.h>
#include "sk_device.h"

namespace sk {

hipError_t launch_ingest(const Task* tasks, int count, int max_rows, int max_d, int in_dtype,
                         int st_dtype, hipStream_t st);
hipError_t launch_ingest_csr(const Task* tasks, int count, int max_rows, int max_d, int st_dtype,
                             hipStream_t st);
hipError_t launch_omega(const Task* tasks, int count, int max_d, int max_k, int pj_dtype,
                        hipStream_t st);
hipError_t launch_gram(const Task* tasks, int count, int max_m, int max_splits, int st_dtype,
                       hipStream_t st);
hipError_t launch_project(const Task* tasks, int count, int max_m, int max_k, int max_splits,
                          int st_dtype, int pj_dtype, hipStream_t st);
hipError_t launch_project_bf16(const Task* tasks, int count, int max_m, int max_k, int max_splits,
                               hipStream_t st);
hipError_t launch_reduce_proj_f32(const Task* tasks, int count, int max_m, int max_k, hipStream_t st);
hipError_t launch_rebuild(const Task* tasks, int count, int max_ell, int max_d, int st_dtype,
                          bool query, hipStream_t st);
hipError_t launch_convert_rows(const double* src, int64_t lds, void* dst, int64_t ldd, int rows,
                               int cols, int out_dtype, hipStream_t st);
hipError_t launch_rows_to_f64(const void* src, int64_t lds, int st_dtype, double* dst, int64_t ldd,
                              int rows, int cols, hipStream_t st);

hipError_t launch_core_gemm(const Task* tasks, int count, int max_M, int max_N, bool ta, bool tb,
                            int sa, int sb, int sc, int dims, hipStream_t st);
hipError_t launch_cholinv(const Task* tasks, int count, int max_k, bool any_small, bool any_large,
                          int sw, int sx, hipStream_t st);
hipError_t launch_jacobi(const Task* tasks, int count, int max_n, bool any_small, bool any_large,
                         hipStream_t st);
hipError_t launch_threshold(const Task* tasks, int count, int max_ell, int max_m, hipStream_t st);
hipError_t launch_jacobi_coop(const CoopEig& args, hipStream_t st);
hipError_t launch_rownorm(const void* rows, int64_t ld, int dtype, int64_t n, int d, double* out,
                          hipStream_t st);
hipError_t launch_philox_mat(const void* descs, int count, int max_rows, int max_cols, hipStream_t st);
// Workgroups per level of the cooperative power iteration for dimension d.
int win_pi_groups(int d);
// part: count * 2 * win_pi_groups(d) * (max_r + 1) doubles; bars: 2 * count words
// (max_r <= 512).  Launched cooperatively, in as many launches as residency
// requires; the buffers are reused by the launches in stream order.
hipError_t launch_win_pi(const void* descs, int count, int d, int max_r, double* part, unsigned* bars,
                         hipStream_t st);
// Row-space power iteration (GramPiDesc list on the device, r <= 1024): one
// pass over every C (u = C x0, |x0|^2, the new row and column of G), then
// one workgroup per level for the steps.
hipError_t launch_win_pi_gram(const void* descs, int count, int max_r, int max_d, hipStream_t st);
// The pass over C alone (u = C x0, |x0|^2 in u[ldg], the new Gram row and
// column); descriptors with r = 0 are skipped.  max_d <= 4096.
hipError_t launch_win_gemv(const void* descs, int count, int max_r, int max_d, hipStream_t st);
// One split-K product (descriptor by value, with part, nsplit, kchunk set).
hipError_t launch_gemm_split(const GemmDesc& g, hipStream_t st);
// Single-descriptor launches with the descriptor passed by value.
hipError_t launch_gemm1(const GemmDesc& g, hipStream_t st);
hipError_t launch_philox_mat1(const MatGenDesc& m, hipStream_t st);
hipError_t launch_cholinv1(const SmallDesc& q, hipStream_t st);
hipError_t launch_jacobi1(const SmallDesc& q, hipStream_t st);
hipError_t launch_blockmask(double* S, int ld, int D, const int32_t* ent, hipStream_t st);
hipError_t launch_shrink_rows(const double* V, int ldv, const double* lam, int n, int ell, double* X,
                              int64_t ldx, int d, hipStream_t st);
// Tridiagonal eigen-solver, one workgroup per problem (n <= 512): the
// non-cooperative tasks of a list, or one descriptor by value.
// The tridiagonal solver in three launches: the reduction (tasks' sizes in
// [min_n, max_n]), the eigenpairs of T, the back-transformation.
hipError_t launch_tri_reduce(const Task* tasks, int count, int min_n, int max_n, hipStream_t st);
hipError_t launch_tri_eig(const Task* tasks, int count, int max_n, hipStream_t st);
hipError_t launch_tri_back(const Task* tasks, int count, int max_n, hipStream_t st);
hipError_t launch_tri_eig1(const SmallDesc& q, hipStream_t st);
hipError_t launch_tri_eig_desc(const SmallDesc* ds, int count, int max_n, hipStream_t st);
int tri_lds_doubles();
// Multi-workgroup reduction (one group of workgroups on one XCD per problem)
// of the tasks of order trix_min_n() .. 512.
hipError_t launch_tri_reduce_x(const Task* tasks, int count, int max_n, hipStream_t st);
int trix_min_n();
// One pass of the multi-workgroup CholeskyQR (the Gram of src already in
// slot S_W) of the tasks flagged TF_X_CHOL: src -> dst.
hipError_t launch_cholqr_x(const Task* tasks, int count, int max_k, int src_slot, int dst_slot, int pass,
                           int polar, hipStream_t st);
// X = (3I - W) / 2 and the polar decision (info[8]) for the second CholeskyQR
// pass of the multi-workgroup tasks.
hipError_t launch_cholx_polar(const Task* tasks, int count, hipStream_t st);
// Multi-task cooperative solvers: tasks[idx[i]] for i < count, each by its
// own group of workgroups (several launches when residency requires).
hipError_t launch_jacobi_coop_tasks(const Task* tasks, const int* idx, int count, int max_n, hipStream_t st);
hipError_t launch_cholqr_coop_tasks(const Task* tasks, const int* idx, int count, int m, int k, int sy, int sq,
                                    int passes, hipStream_t st);
hipError_t launch_cholinv_desc(const SmallDesc* ds, int count, int max_n, hipStream_t st);
hipError_t launch_jacobi_desc(const SmallDesc* ds, int count, int max_n, hipStream_t st);
hipError_t launch_gemm_desc(const GemmDesc* ds, int count, int max_M, int max_N, hipStream_t st);
// Fixed-order sum of the split-K partials of `count` descriptors (part,
// nsplit set): C = alpha * sum + beta C.
hipError_t launch_gemm_reduce_desc(const GemmDesc* ds, int count, int64_t max_MN, hipStream_t st);
hipError_t launch_transpose(const double* src, int lds, double* dst, int64_t ldd, int rows, int cols,
                            hipStream_t st);
// dst = src with column c scaled by f(c) from the n eigenvalues lam (descending):
// COD_SQRT sqrt(lam_c), COD_INVSQRT 1/sqrt(lam_c), COD_KEPT 1 (0 for columns with
// lam_c <= tol lam_0), COD_SHRINK_GAIN sqrt(max(s_c - s_ell, 0)) / s_c and
// COD_SHRINK_SQRT sqrt(max(s_c - s_ell, 0)) with s = sqrt(lam).
hipError_t launch_cod_scale(const double* src, int lds, double* dst, int ldd, int rows, int cols, const double* lam,
                            int n, int mode, double tol, int ell, hipStream_t st);
// Power iteration on A^T B in the row space (Gx = A A^T, Gy = B B^T, ld; r <= 512).
hipError_t launch_cod_pi(const double* Gx, const double* Gy, int ld, const double* u0, const double* n0, int r,
                         int steps, double* out, hipStream_t st);
int jacobi_lds_max();
int chol_lds_max();

}  // namespace sk
