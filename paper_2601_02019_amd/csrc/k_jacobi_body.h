// k_jacobi_body.h -- the single-workgroup parallel Jacobi eigen-solver as a
// device function, shared by the kernels of k_core.hip and k_tri.hip (each
// translation unit gets its own copy: the library is built without
// relocatable device code).
#pragma once
#include "sk_device.h"

namespace sk {

// ------------------------------------------------------------ Jacobi
// Parallel cyclic Jacobi, round-robin ("chess tournament") ordering: in each
// of the ne-1 steps of a sweep the ne/2 index pairs are disjoint, so all
// rotations of a step commute and are applied together as A <- J^T A J on
// 2 x 2 blocks, V <- V J.  Rotation of pair (p, q): Golub & Van Loan's
// symmetric Schur step (tau = (a_qq - a_pp) / (2 a_pq)).  A pair is skipped
// when |a_pq| <= 1e-15 sqrt(|a_pp a_qq|) or below 1e-17 ||A||_F; the solve
// ends after a sweep without rotations.
constexpr int JAC_MAX_SWEEPS = 40;

__device__ __forceinline__ int rr_player(int slot, int step, int ne) {
    return slot == 0 ? 0 : 1 + (slot - 1 + step) % (ne - 1);
}

// Jacobi eigen-decomposition of one n x n symmetric matrix by the whole
// workgroup.  A: n x n work matrix (LDS or global).  The rotations are
// accumulated in Vt = V^T (n x n, rows = eigenvectors), so that a pair's
// update rotates two contiguous rows; Vt lives in LDS after A when both fit
// (vt_lds), else in the global scratch Vg.  U (ld lu) / lam: sorted output;
// info[0] counts non-converged solves, info[1] keeps the largest sweep count.
static __device__ void jacobi_body(const double* Ain, int ldin, int n, double* A, double* Vg, double* U,
                            int lu, double* lam, int* info, double* vt_lds) {
    const int la = n;
    double* Vt = vt_lds ? vt_lds : Vg;
    __shared__ double cs_c[256], cs_s[256];
    __shared__ int pp[256], qq[256];
    __shared__ int rot_count[2];
    __shared__ double red[32];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int ne = (n + 1) & ~1;
    const int np = ne / 2;
    // threads per row-pair of A (a power of two <= np) and per pair of Vt rows
    int tpr = 1;
    while (tpr * 2 <= np && tpr * 2 * np <= nth * 2 && tpr < 64) tpr *= 2;
    if (tpr > nth) tpr = nth;
    int tpv = 1;
    while (tpv * 2 <= n && tpv < 64) tpv *= 2;

    double loc = 0.0;
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - (e / n) * n;
        const double v = 0.5 * (Ain[(int64_t)i * ldin + j] + Ain[(int64_t)j * ldin + i]);
        A[(int64_t)i * la + j] = v;
        Vt[(int64_t)i * n + j] = (i == j) ? 1.0 : 0.0;
        loc += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) loc += __shfl_down(loc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = loc;
    if (tid < 2) rot_count[tid] = 0;
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < (nth + 63) / 64; ++w) fro2 += red[w];
    const double floor_abs = 1e-300 + 1e-17 * sqrt(fro2);

    int sweep = 0;
    bool done = (n <= 1);
    while (!done && sweep < JAC_MAX_SWEEPS) {
        const int sb = sweep & 1;
        if (tid == 0) rot_count[sb] = 0;
        __syncthreads();
        for (int step = 0; step < ne - 1; ++step) {
            for (int m = tid; m < np; m += nth) {
                int p = rr_player(m, step, ne), q = rr_player(ne - 1 - m, step, ne);
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double c = 1.0, sn = 0.0;
                if (q < n) {
                    const double apq = A[(int64_t)p * la + q];
                    const double app = A[(int64_t)p * la + p];
                    const double aqq = A[(int64_t)q * la + q];
                    if (fabs(apq) > floor_abs && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
                        // symmetric Schur rotation (Golub & Van Loan 8.5.2), tan from the hypot
                        const double dd = aqq - app, bb = 2.0 * apq;
                        const double hyp = sqrt(dd * dd + bb * bb);
                        const double tt = (dd >= 0.0 ? bb : -bb) / (fabs(dd) + hyp);
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        sn = tt * c;
                        rot_count[sb] = 1;  // any rotation: another sweep follows
                    }
                }
                cs_c[m] = c;
                cs_s[m] = sn;
                pp[m] = p;
                qq[m] = q;
            }
            __syncthreads();
            // A <- J^T A J: every 2 x 2 block (m1, m2) by one thread, no mirrors;
            // a thread walks one m1 and strided m2, keeping m1's rotation in registers
            for (int m1 = tid / tpr; m1 < np; m1 += nth / tpr) {
                const int p1 = pp[m1], q1 = qq[m1];
                const double c1 = cs_c[m1], s1 = cs_s[m1];
                const bool hq1 = q1 < n;
                for (int m2 = tid % tpr; m2 < np; m2 += tpr) {
                    const int p2 = pp[m2], q2 = qq[m2];
                    const double c2 = cs_c[m2], s2 = cs_s[m2];
                    const bool hq2 = q2 < n;
                    const double a00 = A[(int64_t)p1 * la + p2];
                    const double a01 = hq2 ? A[(int64_t)p1 * la + q2] : 0.0;
                    const double a10 = hq1 ? A[(int64_t)q1 * la + p2] : 0.0;
                    const double a11 = (hq1 && hq2) ? A[(int64_t)q1 * la + q2] : 0.0;
                    const double r00 = c1 * a00 - s1 * a10, r01 = c1 * a01 - s1 * a11;
                    const double r10 = s1 * a00 + c1 * a10, r11 = s1 * a01 + c1 * a11;
                    double n00 = r00 * c2 - r01 * s2, n01 = r00 * s2 + r01 * c2;
                    double n10 = r10 * c2 - r11 * s2, n11 = r10 * s2 + r11 * c2;
                    if (m1 == m2) {
                        n01 = 0.0;
                        n10 = 0.0;
                    }
                    A[(int64_t)p1 * la + p2] = n00;
                    if (hq2) A[(int64_t)p1 * la + q2] = n01;
                    if (hq1) A[(int64_t)q1 * la + p2] = n10;
                    if (hq1 && hq2) A[(int64_t)q1 * la + q2] = n11;
                }
            }
            // Vt <- J^T Vt: rows p and q of every pair, contiguous along the row
            for (int mm = tid / tpv; mm < np; mm += nth / tpv) {
                const int p = pp[mm], q = qq[mm];
                if (q >= n) continue;
                const double cc = cs_c[mm], sn = cs_s[mm];
                if (cc == 1.0 && sn == 0.0) continue;
                for (int c = tid % tpv; c < n; c += tpv) {
                    const double vp = Vt[(int64_t)p * n + c], vq = Vt[(int64_t)q * n + c];
                    Vt[(int64_t)p * n + c] = cc * vp - sn * vq;
                    Vt[(int64_t)q * n + c] = sn * vp + cc * vq;
                }
            }
            __syncthreads();
        }
        done = rot_count[sb] == 0;
        ++sweep;
    }
    // eigenvalues sorted descending (ties by index), vectors permuted along
    for (int i = tid; i < n; i += nth) {
        const double li = A[(int64_t)i * la + i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[(int64_t)j * la + j];
            rank += (lj > li) || (lj == li && j < i);
        }
        lam[rank] = li;
        for (int r = 0; r < n; ++r) U[(int64_t)r * lu + rank] = Vt[(int64_t)i * n + r];
    }
    if (tid == 0) {
        if (!done) atomicAdd(&info[0], 1);
        atomicMax(&info[1], sweep);
    }
}


}  // namespace sk
