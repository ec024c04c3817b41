// k_coop.hip -- multi-workgroup (cooperative) versions of the FP64 core for
// one large problem at a time (gfx950): the single-stream case, where one
// shrink's eigen-solve and CholeskyQR would otherwise sit on one CU.
//
//   k_jacobi_coop  two-sided block Jacobi: indices in blocks of 16, block
//                  pairs in round-robin order; in each step every pair's
//                  32 x 32 diagonal sub-problem is diagonalised in LDS by one
//                  workgroup (phase A), then all workgroups apply the block
//                  rotations U_P^T A_PQ U_Q and V_P U_P as 32 x 32 tiles
//                  (phase B).  Ends after a sweep in which no sub-problem
//                  needed a rotation.
//   k_cholqr_coop  CholeskyQR: W = Y^T Y (tiles over all workgroups),
//                  right-looking blocked Cholesky with rank dropping, then
//                  Q = Y L^{-T} by row blocks; optionally a second pass.
//
// Launched with hipLaunchCooperativeKernel so that every workgroup is
// resident; the grid barriers are agent-scope arrival counters (GridBar).
// Every floating-point reduction runs in a fixed order, so results repeat
// bit for bit.
#include "sk_device.h"
#include "sk_kernels.h"

namespace sk {

constexpr int BW = 16;    // block width
constexpr int PB = 32;    // pair-block size (two blocks)
constexpr int PBL = 33;   // padded LDS leading dimension
constexpr int COOP_MAX_SWEEPS = 40;

__device__ __forceinline__ int rrp(int slot, int step, int ne) {
    return slot == 0 ? 0 : 1 + (slot - 1 + step) % (ne - 1);
}

// Global index of entry e (0..31) of pair-block P at block step `step`.
__device__ __forceinline__ int pb_index(int P, int e, int step, int nb) {
    const int blk = (e < BW) ? rrp(P, step, nb) : rrp(nb - 1 - P, step, nb);
    return blk * BW + (e & (BW - 1));
}

// Parallel cyclic Jacobi sweeps (at most max_sweeps) of a 32 x 32 symmetric
// matrix in LDS (ld PBL) with the rotations accumulated in V (LDS).  Returns
// the rotations performed.
__device__ int lds_jacobi32(double* A, double* V, double floor_abs, int* sh_rot, double* cs,
                            int* pq, int max_sweeps) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int n = PB, np = PB / 2;
    int total = 0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) *sh_rot = 0;
        __syncthreads();
        for (int step = 0; step < n - 1; ++step) {
            if (tid < np) {
                int p = rrp(tid, step, n), q = rrp(n - 1 - tid, step, n);
                if (p > q) { const int x = p; p = q; q = x; }
                double c = 1.0, s = 0.0;
                const double apq = A[p * PBL + q], app = A[p * PBL + p], aqq = A[q * PBL + q];
                if (fabs(apq) > floor_abs && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                    atomicAdd(sh_rot, 1);
                }
                cs[2 * tid] = c;
                cs[2 * tid + 1] = s;
                pq[2 * tid] = p;
                pq[2 * tid + 1] = q;
            }
            __syncthreads();
            for (int e = tid; e < np * np; e += nth) {  // all 2 x 2 blocks (m1, m2)
                const int m1 = e / np, m2 = e % np;
                const int p1 = pq[2 * m1], q1 = pq[2 * m1 + 1], p2 = pq[2 * m2], q2 = pq[2 * m2 + 1];
                const double c1 = cs[2 * m1], s1 = cs[2 * m1 + 1], c2 = cs[2 * m2], s2 = cs[2 * m2 + 1];
                const double a00 = A[p1 * PBL + p2], a01 = A[p1 * PBL + q2];
                const double a10 = A[q1 * PBL + p2], a11 = A[q1 * PBL + q2];
                const double r00 = c1 * a00 - s1 * a10, r01 = c1 * a01 - s1 * a11;
                const double r10 = s1 * a00 + c1 * a10, r11 = s1 * a01 + c1 * a11;
                double n00 = r00 * c2 - r01 * s2, n01 = r00 * s2 + r01 * c2;
                double n10 = r10 * c2 - r11 * s2, n11 = r10 * s2 + r11 * c2;
                if (m1 == m2) { n01 = 0.0; n10 = 0.0; }
                A[p1 * PBL + p2] = n00;
                A[p1 * PBL + q2] = n01;
                A[q1 * PBL + p2] = n10;
                A[q1 * PBL + q2] = n11;
            }
            for (int e = tid; e < n * np; e += nth) {
                const int i = e / np, mm = e % np;
                const int p = pq[2 * mm], q = pq[2 * mm + 1];
                const double c = cs[2 * mm], s = cs[2 * mm + 1];
                const double vp = V[i * PBL + p], vq = V[i * PBL + q];
                V[i * PBL + p] = c * vp - s * vq;
                V[i * PBL + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
        const int r = *sh_rot;
        total += r;
        __syncthreads();
        if (r == 0) break;
    }
    return total;
}

// C (32 x 32, LDS) = op(X) Y with X, Y in LDS (ld PBL); 256 threads, 2 x 2 each.
template <bool TX>
__device__ __forceinline__ void lds_mm32(const double* X, const double* Y, double* C) {
    const int tid = threadIdx.x;
    const int r = (tid >> 4) * 2, c = (tid & 15) * 2;
    double a00 = 0, a01 = 0, a10 = 0, a11 = 0;
#pragma unroll 8
    for (int k = 0; k < PB; ++k) {
        const double x0 = TX ? X[k * PBL + r] : X[r * PBL + k];
        const double x1 = TX ? X[k * PBL + r + 1] : X[(r + 1) * PBL + k];
        const double y0 = Y[k * PBL + c], y1 = Y[k * PBL + c + 1];
        a00 = fma(x0, y0, a00);
        a01 = fma(x0, y1, a01);
        a10 = fma(x1, y0, a10);
        a11 = fma(x1, y1, a11);
    }
    C[r * PBL + c] = a00;
    C[r * PBL + c + 1] = a01;
    C[(r + 1) * PBL + c] = a10;
    C[(r + 1) * PBL + c + 1] = a11;
}

// The solve of one problem by G workgroups (wg = 0 .. G-1).  Every value
// computed depends on the problem alone, not on G: tiles and pair problems
// are independent of which workgroup takes them, and the norm used for the
// rotation floor is summed over a fixed set of 64 chunks.
__device__ void jacobi_coop_body(const CoopEig& args, int wg, int G) {
    GridBar grid{args.bar, (unsigned)G, 0u};
    const int n = args.n;
    const double* Ain = args.Ain;
    const int ldin = args.ldin;
    double* ubuf = args.ubuf;
    double* part = args.part;
    int* ctrl = args.ctrl;
    double* stats = args.stats;
    const int N = (n + PB - 1) / PB * PB;
    const int nb = N / BW, np = nb / 2;
    double* A = args.A;
    double* V = args.V;
    const int tid = threadIdx.x;

    __shared__ double sA[PB * PBL], sV[PB * PBL], sT[PB * PBL];
    __shared__ double cs[PB];
    __shared__ int pq[PB];
    __shared__ int sh_rot;
    __shared__ double red[4];

    // A = sym(Ain) zero-padded to N x N, V = I; ||A||_F^2 by 64 fixed chunks
    const int64_t NN = (int64_t)N * N;
    for (int ch = wg; ch < 64; ch += G) {
        const int64_t e0 = NN * ch / 64, e1 = NN * (ch + 1) / 64;
        double loc = 0.0;
        for (int64_t e = e0 + tid; e < e1; e += 256) {
            const int i = (int)(e / N), j = (int)(e % N);
            double v = 0.0;
            if (i < n && j < n) v = 0.5 * (Ain[(int64_t)i * ldin + j] + Ain[(int64_t)j * ldin + i]);
            A[e] = v;
            V[e] = (i == j) ? 1.0 : 0.0;
            loc += v * v;
        }
        for (int off = 32; off > 0; off >>= 1) loc += __shfl_down(loc, off, 64);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = loc;
        __syncthreads();
        if (tid == 0) part[ch] = red[0] + red[1] + red[2] + red[3];
    }
    if (wg == 0 && tid == 0) {
        ctrl[0] = 0;
        ctrl[1] = 0;
    }
    grid.sync();
    double fro2 = 0.0;
    for (int ch = 0; ch < 64; ++ch) fro2 += part[ch];
    // off-diagonal entries below eps ||A||_F are rounding noise: not rotated
    const double floor_abs = 1e-300 + 1.1e-16 * sqrt(fro2);

    // workgroup 0 keeps a wall-clock account of its phases (diagnostics)
    const bool timer = (wg == 0 && tid == 0);
    uint64_t tA = 0, tSA = 0, tB = 0, tSB = 0, t0 = timer ? wall_clock64() : 0, t1;
    int steps_done = 0;
    int sweep = 0;
    for (; sweep < COOP_MAX_SWEEPS; ++sweep) {
        const int par = sweep & 1;
        for (int step = 0; step < nb - 1; ++step) {
            ++steps_done;
            // ---- phase A: diagonalise each pair's 32 x 32 sub-problem
            for (int P = wg; P < np; P += G) {
                for (int e = tid; e < PB * PB; e += 256) {
                    const int i = e / PB, j = e % PB;
                    sA[i * PBL + j] = A[(int64_t)pb_index(P, i, step, nb) * N + pb_index(P, j, step, nb)];
                    sV[i * PBL + j] = (i == j) ? 1.0 : 0.0;
                }
                __syncthreads();
                // one sweep per block step: the outer cycle revisits every pair
                const int rot = lds_jacobi32(sA, sV, floor_abs, &sh_rot, cs, pq, 1);
                if (tid == 0 && rot > 0) atomicAdd(&ctrl[par], rot);
                double* U = ubuf + (int64_t)P * PB * PB;
                for (int e = tid; e < PB * PB; e += 256) U[e] = sV[(e / PB) * PBL + (e % PB)];
                __syncthreads();
            }
            if (timer) { t1 = wall_clock64(); tA += t1 - t0; t0 = t1; }
            grid.sync();
            if (timer) { t1 = wall_clock64(); tSA += t1 - t0; t0 = t1; }
            // ---- phase B: block rotations, sandwich tiles then V tiles
            const int nsand = np * (np + 1) / 2;
            const int nvt = (N / PB) * np;
            for (int tile = wg; tile < nsand + nvt; tile += G) {
                if (tile < nsand) {
                    int Q = 0, rem = tile;
                    while (rem >= Q + 1) {
                        rem -= Q + 1;
                        ++Q;
                    }
                    const int P = rem;  // P <= Q
                    const double* UP = ubuf + (int64_t)P * PB * PB;
                    const double* UQ = ubuf + (int64_t)Q * PB * PB;
                    for (int e = tid; e < PB * PB; e += 256) {
                        const int i = e / PB, j = e % PB;
                        sA[i * PBL + j] = A[(int64_t)pb_index(P, i, step, nb) * N + pb_index(Q, j, step, nb)];
                        sV[i * PBL + j] = UQ[e];
                    }
                    __syncthreads();
                    lds_mm32<false>(sA, sV, sT);   // sT = A_PQ U_Q
                    __syncthreads();
                    for (int e = tid; e < PB * PB; e += 256) sV[(e / PB) * PBL + (e % PB)] = UP[e];
                    __syncthreads();
                    lds_mm32<true>(sV, sT, sA);    // sA = U_P^T sT
                    __syncthreads();
                    for (int e = tid; e < PB * PB; e += 256) {
                        const int i = e / PB, j = e % PB;
                        const double v = sA[i * PBL + j];
                        const int gi = pb_index(P, i, step, nb), gj = pb_index(Q, j, step, nb);
                        A[(int64_t)gi * N + gj] = v;
                        if (P != Q) A[(int64_t)gj * N + gi] = v;
                    }
                    __syncthreads();
                } else {
                    const int vt = tile - nsand;
                    const int rb = vt / np, P = vt % np;
                    const double* UP = ubuf + (int64_t)P * PB * PB;
                    for (int e = tid; e < PB * PB; e += 256) {
                        const int i = e / PB, j = e % PB;
                        sA[i * PBL + j] = V[(int64_t)(rb * PB + i) * N + pb_index(P, j, step, nb)];
                        sV[i * PBL + j] = UP[e];
                    }
                    __syncthreads();
                    lds_mm32<false>(sA, sV, sT);
                    __syncthreads();
                    for (int e = tid; e < PB * PB; e += 256) {
                        const int i = e / PB, j = e % PB;
                        V[(int64_t)(rb * PB + i) * N + pb_index(P, j, step, nb)] = sT[i * PBL + j];
                    }
                    __syncthreads();
                }
            }
            if (timer) { t1 = wall_clock64(); tB += t1 - t0; t0 = t1; }
            grid.sync();
            if (timer) { t1 = wall_clock64(); tSB += t1 - t0; t0 = t1; }
        }
        const bool done = ctrl[par] == 0;
        grid.sync();  // everyone has read ctrl[par] before it is reset
        if (wg == 0 && tid == 0) ctrl[par ^ 1] = 0;
        grid.sync();
        if (done) break;
    }
    // eigenvalues (real indices only) sorted descending, vectors permuted along
    double* U = args.U;
    const int lu = args.lu;
    double* lam = args.lam;
    for (int i = wg * 256 + tid; i < n; i += G * 256) {
        const double li = A[(int64_t)i * N + i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[(int64_t)j * N + j];
            rank += (lj > li) || (lj == li && j < i);
        }
        lam[rank] = li;
        for (int r = 0; r < n; ++r) U[(int64_t)r * lu + rank] = V[(int64_t)r * N + i];
    }
    if (wg == 0 && tid == 0) {
        if (sweep >= COOP_MAX_SWEEPS) atomicAdd(&args.info[0], 1);
        atomicMax(&args.info[1], sweep + 1);
        stats[0] += (double)(sweep + 1);
        stats[1] += (double)steps_done;
        stats[2] += (double)tA;
        stats[3] += (double)tSA;
        stats[4] += (double)tB;
        stats[5] += (double)tSB;
        stats[6] += 1.0;
        stats[7] = (double)G;
    }
}

__global__ __launch_bounds__(256) void k_jacobi_coop(CoopEig args) {
    jacobi_coop_body(args, blockIdx.x, gridDim.x);
}

// Problem of a shrink / query task: the Rayleigh-Ritz matrix (randomized) or
// the buffer Gram (exact), into the sketch's slots and cooperative scratch.
__device__ CoopEig coop_eig_of(const Task& t) {
    const SkDev* s = t.s;
    const bool rnd = t.kind == T_SHRINK_RAND;
    CoopEig a{};
    a.Ain = s->slot[rnd ? S_M : S_G];
    a.ldin = s->sld[rnd ? S_M : S_G];
    a.n = eig_n(t);
    a.A = s->slot[S_EA];
    a.V = s->slot[S_EV];
    a.U = s->slot[S_U];
    a.lu = s->sld[S_U];
    a.lam = s->slot[S_LAM];
    a.info = s->info;
    a.ubuf = s->coop + COOP_UBUF;
    a.part = s->coop + COOP_PART;
    a.ctrl = s->coop_ctrl;
    a.stats = s->coop + COOP_STATS;
    a.bar = (uint32_t*)(s->coop_ctrl + 8);
    return a;
}

__global__ __launch_bounds__(256) void k_jacobi_coop_tasks(CoopList L) {
    const int i = blockIdx.x / L.gper;
    const CoopEig a = coop_eig_of(L.tasks[L.idx[i]]);
    jacobi_coop_body(a, blockIdx.x % L.gper, L.gper);
}

// Zeroes the grid-barrier words of every task of a multi-task launch.
__global__ void k_coop_zero_bars(CoopList L) {
    const int i = threadIdx.x;
    if (i < L.count) {
        int32_t* c = L.tasks[L.idx[i]].s->coop_ctrl;
        c[8] = 0;
        c[9] = 0;
    }
}

// ------------------------------------------------------------ CholeskyQR
__device__ __forceinline__ double lane_bcast(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Factor the 32 x 32 diagonal block in LDS (lower, with rank dropping against
// the original diagonal d0), then its lower inverse.  drop[] per column.
// One wavefront, lane i holding row i in registers: per column the pivot and
// the scaled column come by lane reads, 1/sqrt by the hardware estimate and
// two Newton steps; no LDS traffic and no barrier.  The
// inverse: lane c holds column c and substitutes row by row.
__device__ void lds_chol32(double* L, double* Li, const double* d0, int* drop, double* piv) {
    __shared__ double rd[PB];
    const int tid = threadIdx.x;
    (void)piv;
    if (tid < PB) {
        const int i = tid;
        double a[PB];
#pragma unroll
        for (int t = 0; t < PB; ++t) a[t] = L[i * PBL + t];
        double rdi = 0.0;
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const double p = lane_bcast(a[j], j);
            const bool ok = p > 1e-14 * d0[j] && p > 1e-300;
            double r = 0.0, dj = 0.0;
            if (ok) {
                r = __builtin_amdgcn_rsq(p);
                r = r * fma(-0.5 * p * r, r, 1.5);
                r = r * fma(-0.5 * p * r, r, 1.5);
                dj = p * r;
            }
            const double ci = a[j] * r;
            if (ok) {
#pragma unroll
                for (int l = j + 1; l < PB; ++l) {
                    const double cl = lane_bcast(ci, l);
                    if (l <= i) a[l] -= ci * cl;
                }
            }
            a[j] = (i > j) ? ci : (i == j ? dj : 0.0);
            if (i == j) rdi = r;
            if (i == 0) drop[j] = ok ? 0 : 1;
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int t = 0; t < PB; ++t) L[i * PBL + t] = t <= i ? a[t] : 0.0;
        rd[i] = rdi;
    }
    __syncthreads();
    if (tid < PB) {
        const int c = tid;
        double x[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            double s0 = (i == c) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int l = 0; l < i; l += 2) {
                s0 = fma(-L[i * PBL + l], x[l], s0);
                if (l + 1 < i) s1 = fma(-L[i * PBL + l + 1], x[l + 1], s1);
            }
            x[i] = (i >= c) ? (s0 + s1) * rd[i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) Li[i * PBL + c] = x[i];
    }
    __syncthreads();
}

// CholeskyQR of one task by G workgroups; every value is independent of G.
__device__ void cholqr_coop_body(const Task& t, int sy, int sq, int passes, int wg, int G) {
    const SkDev* s = t.s;
    double* linv = s->coop + COOP_LINV;
    double* d0g = s->coop + COOP_D0;
    GridBar grid{(unsigned*)(s->coop_ctrl + 8), (unsigned)G, 0u};
    const int m = t.m, k = s->k;
    const int K = (k + PB - 1) / PB * PB;   // padded rank
    const int kb = K / PB;
    const int mb = (m + PB - 1) / PB;
    const int tid = threadIdx.x;
    double* W = s->slot[S_EA];              // K x K (ld K)
    const int ldk = s->sld[S_Q];

    __shared__ double sX[PB * PBL], sY[PB * PBL], sZ[PB * PBL];
    __shared__ double sd0[PB];
    __shared__ int sdrop[PB];
    __shared__ double spiv;

    for (int pass = 0; pass < passes; ++pass) {
        const double* src = s->slot[pass == 0 ? sy : S_Q1];
        double* dst = s->slot[pass == passes - 1 ? sq : S_Q1];
        // ---- W = src^T src, upper tiles (ti <= tj) over all workgroups, K padded with zeros
        const int ntile = kb * (kb + 1) / 2;
        for (int tile = wg; tile < ntile; tile += G) {
            int tj = 0, rem = tile;
            while (rem >= tj + 1) {
                rem -= tj + 1;
                ++tj;
            }
            const int ti = rem;
            const int r = (tid >> 4) * 2, c = (tid & 15) * 2;
            double a00 = 0, a01 = 0, a10 = 0, a11 = 0;
            for (int r0 = 0; r0 < m; r0 += PB) {
                for (int e = tid; e < PB * PB; e += 256) {
                    const int rr = e / PB, cc = e % PB;
                    const int row = r0 + rr;
                    const int ci = ti * PB + cc, cj = tj * PB + cc;
                    sX[rr * PBL + cc] = (row < m && ci < k) ? src[(int64_t)row * ldk + ci] : 0.0;
                    sY[rr * PBL + cc] = (row < m && cj < k) ? src[(int64_t)row * ldk + cj] : 0.0;
                }
                __syncthreads();
#pragma unroll 8
                for (int q = 0; q < PB; ++q) {
                    const double x0 = sX[q * PBL + r], x1 = sX[q * PBL + r + 1];
                    const double y0 = sY[q * PBL + c], y1 = sY[q * PBL + c + 1];
                    a00 = fma(x0, y0, a00);
                    a01 = fma(x0, y1, a01);
                    a10 = fma(x1, y0, a10);
                    a11 = fma(x1, y1, a11);
                }
                __syncthreads();
            }
            const double vals[4] = {a00, a01, a10, a11};
            for (int u = 0; u < 4; ++u) {
                const int gi = ti * PB + r + (u >> 1), gj = tj * PB + c + (u & 1);
                W[(int64_t)gi * K + gj] = vals[u];
                W[(int64_t)gj * K + gi] = vals[u];
            }
        }
        grid.sync();
        for (int i = wg * 256 + tid; i < K; i += G * 256) d0g[i] = W[(int64_t)i * K + i];
        grid.sync();
        // ---- blocked right-looking Cholesky, lower factor overwrites W
        for (int j = 0; j < kb; ++j) {
            if (wg == 0) {
                for (int e = tid; e < PB * PB; e += 256) {
                    const int i = e / PB, l = e % PB;
                    sX[i * PBL + l] = W[(int64_t)(j * PB + i) * K + j * PB + l];
                }
                if (tid < PB) sd0[tid] = d0g[j * PB + tid];
                __syncthreads();
                lds_chol32(sX, sY, sd0, sdrop, &spiv);
                for (int e = tid; e < PB * PB; e += 256) {
                    const int i = e / PB, l = e % PB;
                    W[(int64_t)(j * PB + i) * K + j * PB + l] = sX[i * PBL + l];
                    linv[(int64_t)j * PB * PB + e] = sY[i * PBL + l];
                }
                __syncthreads();
            }
            grid.sync();
            // panel: L_ij = W_ij Linv_jj^T for i > j
            for (int i = j + 1 + wg; i < kb; i += G) {
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    sX[a * PBL + b] = W[(int64_t)(i * PB + a) * K + j * PB + b];
                    sY[b * PBL + a] = linv[(int64_t)j * PB * PB + e];  // transpose
                }
                __syncthreads();
                lds_mm32<false>(sX, sY, sZ);
                __syncthreads();
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    W[(int64_t)(i * PB + a) * K + j * PB + b] = sZ[a * PBL + b];
                }
                __syncthreads();
            }
            grid.sync();
            // trailing update: W_il -= L_ij L_lj^T for j < l <= i
            const int rem = kb - j - 1;
            const int ntr = rem * (rem + 1) / 2;
            for (int tt = wg; tt < ntr; tt += G) {
                int ii = 0, rr = tt;
                while (rr >= ii + 1) {
                    rr -= ii + 1;
                    ++ii;
                }
                const int i = j + 1 + ii, l = j + 1 + rr;  // l <= i
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    sX[a * PBL + b] = W[(int64_t)(i * PB + a) * K + j * PB + b];
                    sY[b * PBL + a] = W[(int64_t)(l * PB + a) * K + j * PB + b];  // L_lj^T
                }
                __syncthreads();
                lds_mm32<false>(sX, sY, sZ);
                __syncthreads();
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    W[(int64_t)(i * PB + a) * K + l * PB + b] -= sZ[a * PBL + b];
                }
                __syncthreads();
            }
            grid.sync();
        }
        // ---- dst = src L^{-T}, one workgroup per 32-row block, column blocks in order
        for (int rb = wg; rb < mb; rb += G) {
            for (int j = 0; j < kb; ++j) {
                // sZ = src[rb, j] - sum_{l<j} dst[rb, l] L_jl^T
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    const int row = rb * PB + a, col = j * PB + b;
                    sZ[a * PBL + b] = (row < m && col < k) ? src[(int64_t)row * ldk + col] : 0.0;
                }
                __syncthreads();
                for (int l = 0; l < j; ++l) {
                    for (int e = tid; e < PB * PB; e += 256) {
                        const int a = e / PB, b = e % PB;
                        const int row = rb * PB + a, col = l * PB + b;
                        sX[a * PBL + b] = (row < m && col < k) ? dst[(int64_t)row * ldk + col] : 0.0;
                        sY[b * PBL + a] = W[(int64_t)(j * PB + a) * K + l * PB + b];  // L_jl^T
                    }
                    __syncthreads();
                    const int r = (tid >> 4) * 2, c = (tid & 15) * 2;
                    double a00 = 0, a01 = 0, a10 = 0, a11 = 0;
                    for (int q = 0; q < PB; ++q) {
                        const double x0 = sX[r * PBL + q], x1 = sX[(r + 1) * PBL + q];
                        const double y0 = sY[q * PBL + c], y1 = sY[q * PBL + c + 1];
                        a00 = fma(x0, y0, a00);
                        a01 = fma(x0, y1, a01);
                        a10 = fma(x1, y0, a10);
                        a11 = fma(x1, y1, a11);
                    }
                    __syncthreads();
                    sZ[r * PBL + c] -= a00;
                    sZ[r * PBL + c + 1] -= a01;
                    sZ[(r + 1) * PBL + c] -= a10;
                    sZ[(r + 1) * PBL + c + 1] -= a11;
                    __syncthreads();
                }
                // dst[rb, j] = sZ Linv_jj^T
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    sY[b * PBL + a] = linv[(int64_t)j * PB * PB + e];
                }
                __syncthreads();
                lds_mm32<false>(sZ, sY, sX);
                __syncthreads();
                for (int e = tid; e < PB * PB; e += 256) {
                    const int a = e / PB, b = e % PB;
                    const int row = rb * PB + a, col = j * PB + b;
                    if (row < m && col < k) dst[(int64_t)row * ldk + col] = sX[a * PBL + b];
                }
                __syncthreads();
            }
        }
        grid.sync();
    }
}

__global__ __launch_bounds__(256) void k_cholqr_coop_tasks(CoopList L) {
    const int i = blockIdx.x / L.gper;
    cholqr_coop_body(L.tasks[L.idx[i]], L.sy, L.sq, L.passes, blockIdx.x % L.gper, L.gper);
}

// ------------------------------------------------------------ launchers
static int coop_grid(const void* f, int want) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 256, 0) != hipSuccess) return 0;
    const int cap = cus * per;
    return want < cap ? want : cap;
}

hipError_t launch_jacobi_coop(const CoopEig& a, hipStream_t st) {
    const int N = (a.n + PB - 1) / PB * PB;
    const int nb = N / BW, np = nb / 2;
    const int tiles = np * (np + 1) / 2 + (N / PB) * np;
    int G = coop_grid((const void*)k_jacobi_coop, tiles < 128 ? tiles : 128);
    if (G < 1) return hipErrorInvalidConfiguration;
    hipError_t e = hipMemsetAsync(a.bar, 0, 2 * sizeof(unsigned), st);
    if (e != hipSuccess) return e;
    CoopEig args = a;
    void* kargs[] = {(void*)&args};
    return hipLaunchCooperativeKernel((const void*)k_jacobi_coop, dim3((unsigned)G), dim3(256), kargs, 0, st);
}

// Runs the listed tasks in as few cooperative launches as residency allows;
// want = workgroups per task that keep every tile busy.
static hipError_t launch_multi(const void* kern, const Task* tasks, const int* idx, int count, int want,
                               int sy, int sq, int passes, hipStream_t st) {
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 256, 0);
    if (e != hipSuccess) return e;
    const int cap = cus * per;
    if (cap < 1) return hipErrorInvalidConfiguration;
    int done = 0;
    while (done < count) {
        // tasks of this launch: at least 16 workgroups each while they fit
        int batch = count - done;
        if (batch > COOP_MAX_TASKS) batch = COOP_MAX_TASKS;
        while (batch > 1 && cap / batch < 16) --batch;
        int gper = cap / batch;
        if (gper > want) gper = want;
        if (gper < 1) return hipErrorInvalidConfiguration;
        CoopList L{};
        L.tasks = tasks;
        L.count = batch;
        L.gper = gper;
        L.sy = sy;
        L.sq = sq;
        L.passes = passes;
        for (int i = 0; i < batch; ++i) L.idx[i] = idx[done + i];
        hipLaunchKernelGGL(k_coop_zero_bars, dim3(1), dim3(COOP_MAX_TASKS), 0, st, L);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        void* kargs[] = {(void*)&L};
        e = hipLaunchCooperativeKernel(kern, dim3((unsigned)(batch * gper)), dim3(256), kargs, 0, st);
        if (e != hipSuccess) return e;
        done += batch;
    }
    return hipSuccess;
}

hipError_t launch_jacobi_coop_tasks(const Task* tasks, const int* idx, int count, int max_n, hipStream_t st) {
    const int N = (max_n + PB - 1) / PB * PB;
    const int nb = N / BW, np = nb / 2;
    int want = np * (np + 1) / 2 + (N / PB) * np;
    if (want > 128) want = 128;
    return launch_multi((const void*)k_jacobi_coop_tasks, tasks, idx, count, want, 0, 0, 0, st);
}

hipError_t launch_cholqr_coop_tasks(const Task* tasks, const int* idx, int count, int m, int k, int sy, int sq,
                                    int passes, hipStream_t st) {
    const int kb = (k + PB - 1) / PB, mb = (m + PB - 1) / PB;
    int want = kb * (kb + 1) / 2;
    if (mb > want) want = mb;
    if (want > 64) want = 64;
    return launch_multi((const void*)k_cholqr_coop_tasks, tasks, idx, count, want, sy, sq, passes, st);
}

}  // namespace sk
