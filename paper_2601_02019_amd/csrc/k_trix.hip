// k_trix.hip -- Householder tridiagonalisation of one symmetric eigen-problem
// (the k x k Rayleigh-Ritz matrix of Algorithm "Simultaneous Iteration", or
// the 2 ell x 2 ell buffer Gram of the exact FD shrink, Sec. 2.3) by a group
// of P workgroups on one XCD.
//
// The rows of A are dealt out cyclically (row i to member i mod P, at most
// XR rows each) and stay in LDS for the whole reduction.  Column j's
// reflector needs row j of the current matrix, A22 v over every row, and the
// scalar p.v; each member computes its rows' part of A22 v, and one exchange
// per column (through L2) gives every member all of p, the partial dots and
// the not-yet-updated row j + 1.  Every member then derives w, applies the
// rank-2 update to its own rows and forms row j + 1 of the updated matrix
// itself, so the next reflector starts without another exchange.  All
// members run the same arithmetic on the same inputs, so they agree bit for
// bit; every sum has a fixed order (results repeat exactly).
//
// Output as the one-workgroup reductions: W row j holds v_j beyond the
// super-diagonal and W[j][j] = tau_j (H_j = I - tau_j v_j v_j^T, v_j[j+1] = 1),
// U row 0 the diagonal of T and U row 1 its off-diagonal.
//
// Exchange words: each member publishes (epoch << 32 | step) in its flag
// after its step data; the epoch grows with every launch, so flags left by
// earlier launches never satisfy a wait.  A wait gives up after a bounded
// number of polls and counts the failure in info[3] (the solve then reports
// SK_EDEVICE); no wait can hang.
#include <atomic>

#include "sk_device.h"
#include "sk_kernels.h"
#include "sk_xwg.h"

namespace sk {

constexpr int XR = 16;          // rows per member
constexpr int XTHREADS = 256;   // 16 rows x 16 lanes
constexpr int XNMAX = 512;
constexpr int XSLOT = 2 * XNMAX + 32;  // p, row, partial dots

// Sums within each 16-lane row of a wavefront by DPP exchanges (every lane
// of the row gets the row's sum): lane ^ 1, lane ^ 2 by quad permutes, then
// the half-row and row mirrors pair the (by then uniform) quads.
template <int CTRL>
__device__ __forceinline__ double x_dpp(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double x_sum16(double x) {
    x += x_dpp<0xB1>(x);
    x += x_dpp<0x4E>(x);
    x += x_dpp<0x141>(x);
    x += x_dpp<0x140>(x);
    return x;
}
__device__ __forceinline__ double x_lane(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
// wave sum (every lane gets it), rows summed in order
__device__ __forceinline__ double x_wave_sum(double x) {
    x = x_sum16(x);
    return (x_lane(x, 0) + x_lane(x, 16)) + (x_lane(x, 32) + x_lane(x, 48));
}

// The member group of workgroup b.  Workgroups are dealt to the 8 XCDs round
// robin, so with `local` the P members of a problem share one XCD (b = xcd +
// 8 (P g + m), m < P); otherwise they are consecutive (b = P problem + m) and
// spread over the XCDs.
struct XMap {
    int problem, member;
};
__device__ __forceinline__ XMap x_map(int P, int local) {
    const int b = blockIdx.x;
    if (!local) return {b / P, b % P};
    const int xcd = b & 7, slot = b >> 3;
    return {(slot / P) * 8 + xcd, slot % P};
}

__host__ __device__ __forceinline__ int x_members(int n) { return (n + XR - 1) / XR; }

// LDS row stride of the member's rows: 16 doubles past a multiple of 32, so
// the four rows a wavefront touches at once fall in two bank halves.
__host__ __device__ __forceinline__ int x_ald(int n) { return (n + 31) / 32 * 32 + 16; }
// LDS (doubles) of a problem of order n: the rows, four waves' private
// reflector pairs, and the arrivals p and row j + 1.
__host__ __device__ __forceinline__ int x_lds_doubles(int n) { return XR * x_ald(n) + 10 * n; }

// Row jj + 1 of the reflector pair, in every wavefront of every member (no
// barrier): lane l holds xr[t] = x[c] for c = jj + lane + 64 t of the row x
// that column jj reduces (x[jj + 1] = alpha).  Writes v[jj + 1 ..] into this
// wave's v (v[jj + 1] = 1) and returns tau; member 0's wave 0 also writes
// the reflector (W row jj), the diagonal entry and beta.  Identical
// arithmetic in every wavefront and member.
template <int LPL>
__device__ __forceinline__ double trix_reflector_w(int jj, int n, const double (&xr)[LPL], double xn2, double* v,
                                                   double* Wr, double* U, int lu, bool writer) {
    const int lane = threadIdx.x & 63;
    const double alpha = x_lane(xr[0], 1);  // x[jj + 1]
    double beta = alpha, tau = 0.0, scal = 0.0;
    if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
    }
#pragma unroll
    for (int t = 0; t < LPL; ++t) {
        const int c = jj + lane + 64 * t;
        if (c > jj && c < n) v[c] = (c == jj + 1) ? 1.0 : xr[t] * scal;
    }
    if (writer) {
        if (lane == 0) {
            U[jj] = xr[0];
            U[lu + jj] = beta;
            Wr[(int64_t)jj * n + jj] = tau;
        }
#pragma unroll
        for (int t = 0; t < LPL; ++t) {
            const int c = jj + lane + 64 * t;
            if (c > jj + 1 && c < n) Wr[(int64_t)jj * n + c] = xr[t] * scal;
        }
    }
    return tau;
}

// Exchange of step j, wave 0 only: this member's p (pl) and partial dot (the
// sum of pvw), row j + 1 as it stands if this member owns it; then every
// member's data into pb, rb and *pvs.  Returns false on a timed-out wait.
__device__ __forceinline__ bool trix_exchange(int j, int n, int P, int member, const double* Al, int ald,
                                              const double* pl, const double* pvw, double* xch, uint64_t* flags,
                                              uint64_t epoch, double* pb, double* rb, double* pvs) {
    const int lane = threadIdx.x & 63;
    double* slot = xch + (j & 1) * XSLOT;
    if (lane < XR) {
        const int i = member + P * lane;
        if (i > j && i < n) slot[i] = pl[lane];
    }
    if (lane == 0) slot[2 * XNMAX + member] = (pvw[0] + pvw[1]) + (pvw[2] + pvw[3]);
    if (member == (j + 1) % P) {
        const double* ar = Al + ((j + 1) / P) * ald;
        for (int c = j + 1 + lane; c < n; c += 64) slot[XNMAX + c] = ar[c];
    }
    const uint64_t target = xwg_flag(epoch, (unsigned)(j + 1));
    xwg_publish(flags + member, target);
    const bool ok = xwg_wait(flags, P, target);
    double pvv = lane < P ? slot[2 * XNMAX + lane] : 0.0;
    constexpr int LPL = XNMAX / 64;
    double pr[LPL], rr_[LPL];
#pragma unroll
    for (int u = 0; u < LPL; ++u) {
        const int c = j + 1 + lane + 64 * u;
        pr[u] = c < n ? slot[c] : 0.0;
        rr_[u] = c < n ? slot[XNMAX + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LPL; ++u) {
        const int c = j + 1 + lane + 64 * u;
        if (c < n) {
            pb[c] = pr[u];
            rb[c] = rr_[u];
        }
    }
    double sum = 0.0;  // partial dots in member order (the same sum in every member)
    for (int m = 0; m < P; ++m) sum += x_lane(pvv, m);
    if (lane == 0) *pvs = sum;
    return ok;
}

// One pass over this thread's part of its row: the rank-2 update of column
// j (skipped for j < 0, the first column) and the dot with the reflector vb
// over columns from jv; the loads of four columns are issued together.
__device__ __forceinline__ double trix_row_pass(double* ar, int c0, int n, int jv, const double* va, const double* pb,
                                                const double* vb, double K, double vi, double wi, bool update) {
    double acc = 0.0;
    for (int cb = c0; cb < n; cb += 64) {
        double av[4], vv[4], pv[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = min(cb + 16 * u, n - 1);
            av[u] = ar[c];
            bv[u] = vb[c];
            if (update) {
                vv[u] = va[c];
                pv[u] = pb[c];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = cb + 16 * u;
            if (c < n) {
                double a = av[u];
                if (update) {
                    const double wc = fma(-K, vv[u], pv[u]);
                    a = fma(-vi, wc, fma(-wi, vv[u], a));
                    ar[c] = a;
                }
                if (c >= jv) acc = fma(a, bv[u], acc);
            }
        }
    }
    return acc;
}

__device__ void trix_body(const double* __restrict__ Ain, int ldin, int n, double* __restrict__ Wr,
                          double* __restrict__ U, int lu, double* xch, uint64_t* flags, int* info, uint64_t epoch,
                          int member) {
    extern __shared__ double lds[];
    constexpr int LPL = XNMAX / 64;
    const int P = x_members(n);
    const int ald = x_ald(n);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = tid >> 4, part = tid & 15;  // row slot and lane within it
    double* Al = lds;                          // [XR][ald] this member's rows
    double* va = lds + XR * ald + wave * 2 * n;  // this wave's reflector of the current column
    double* vb = va + n;                       // ... and of the next column
    double* pb = lds + XR * ald + 8 * n;       // p of every row, on arrival
    double* rb = pb + n;                       // shipped row j + 1, on arrival
    __shared__ double pl[XR], pvw[4], pvs_s;
    __shared__ int bad;
    const int my_i = member + P * r;           // this thread's row
    const bool has_row = my_i < n;
    const bool writer = member == 0 && wave == 0;
    for (int e = tid; e < XR * n; e += XTHREADS) {
        const int rr = e / n, c = e - rr * n, i = member + P * rr;
        Al[rr * ald + c] = i < n ? 0.5 * (Ain[(int64_t)i * ldin + c] + Ain[(int64_t)c * ldin + i]) : 0.0;
    }
    if (tid == 0) bad = 0;
    // (n >= 3 here: the launcher takes orders from trix_min_n() >= 8)
    // column 0 in every wave: row 0 of A, its reflector into va
    double tau;
    {
        double xr[LPL], s2 = 0.0;
#pragma unroll
        for (int t = 0; t < LPL; ++t) {
            const int c = lane + 64 * t;
            xr[t] = c < n ? 0.5 * (Ain[c] + Ain[(int64_t)c * ldin]) : 0.0;
            if (c >= 2 && c < n) s2 = fma(xr[t], xr[t], s2);
        }
        s2 = x_wave_sum(s2);
        tau = trix_reflector_w<LPL>(0, n, xr, s2, va, Wr, U, lu, writer);
    }
    __syncthreads();  // rows in LDS; every wave's va
    {
        const bool live = has_row && my_i > 0;
        double acc = 0.0;
        if (live) acc = trix_row_pass(Al + r * ald, 1 + part, n, 1, va, pb, va, 0.0, 0.0, 0.0, false);
        acc = x_sum16(acc);
        const double pi = tau * acc;
        if (part == 0) pl[r] = live ? pi : 0.0;
        const double pv = (live && part == 0) ? pi * va[my_i] : 0.0;
        const double wsum = (x_lane(pv, 0) + x_lane(pv, 16)) + (x_lane(pv, 32) + x_lane(pv, 48));
        if (lane == 0) pvw[wave] = wsum;
    }
    __syncthreads();
    if (wave == 0 && !trix_exchange(0, n, P, member, Al, ald, pl, pvw, xch, flags, epoch, pb, rb, &pvs_s) &&
        lane == 0)
        bad = 1;
    __syncthreads();
    for (int j = 0; j + 2 < n && !bad; ++j) {
        // (1) in every wave: w = p - K v (on the fly) and row j + 1 after this
        // column's update (lane l: columns j + 1 + l + 64 t), with the squared
        // norm of its part beyond j + 2
        const double K = 0.5 * tau * pvs_s;
        const double w1 = fma(-K, va[j + 1], pb[j + 1]);
        const bool next = j + 3 < n;
        double xr[LPL], s2 = 0.0;
#pragma unroll
        for (int t = 0; t < LPL; ++t) {
            const int c = j + 1 + lane + 64 * t;
            double x = 0.0;
            if (c < n) {
                const double wc = fma(-K, va[c], pb[c]);
                x = fma(-1.0, wc, fma(-w1, va[c], rb[c]));
                if (c >= j + 3) s2 = fma(x, x, s2);
            }
            xr[t] = x;
        }
        // (2) the next column's reflector, in every wave (its v into vb)
        double tau2 = 0.0;
        if (next) {
            s2 = x_wave_sum(s2);
            tau2 = trix_reflector_w<LPL>(j + 1, n, xr, s2, vb, Wr, U, lu, writer);
        } else {  // j = n - 3: the last 2 x 2 block of T
            const double last = x_lane(xr[0], 1);  // row n - 2, column n - 1
            if (writer && lane == 0) {
                U[n - 2] = xr[0];
                U[lu + n - 2] = last;
                Wr[(int64_t)(n - 2) * n + n - 2] = 0.0;
                Wr[(int64_t)(n - 1) * n + n - 1] = 0.0;
            }
        }
        __builtin_amdgcn_wave_barrier();  // the wave's vb before its reads
        // (3) one pass over this member's rows: the update of column j and
        // the products with the next reflector
        {
            const bool live = has_row && my_i > j, live2 = has_row && my_i > j + 1;
            double acc = 0.0;
            if (live) {
                const double vi = va[my_i], wi = fma(-K, vi, pb[my_i]);
                acc = trix_row_pass(Al + r * ald, j + 1 + part, n, j + 2, va, pb, vb, K, vi, wi, true);
            }
            if (next) {
                acc = x_sum16(acc);
                const double pi = tau2 * acc;
                if (part == 0) pl[r] = live2 ? pi : 0.0;
                const double pv = (live2 && part == 0) ? pi * vb[my_i] : 0.0;
                const double wsum = (x_lane(pv, 0) + x_lane(pv, 16)) + (x_lane(pv, 32) + x_lane(pv, 48));
                if (lane == 0) pvw[wave] = wsum;
            }
        }
        __syncthreads();
        if (!next) break;
        // (4) exchange of column j + 1
        if (wave == 0 &&
            !trix_exchange(j + 1, n, P, member, Al, ald, pl, pvw, xch, flags, epoch, pb, rb, &pvs_s) && lane == 0)
            bad = 1;
        __syncthreads();
        double* t = va;
        va = vb;
        vb = t;
        tau = tau2;
    }
    if (bad) {
        if (tid == 0 && member == 0) atomicAdd(&info[3], 1);
        return;
    }
    // A[n-1][n-1] after every update: its owner holds it
    if (member == (n - 1) % P && tid == 0) U[n - 1] = Al[((n - 1) / P) * ald + n - 1];
}

// Task form: eigen-problems of shrink / query tasks that the tridiagonal
// solver takes and whose size is in [xmin, XNMAX].
__global__ __launch_bounds__(XTHREADS) void k_tri_reduce_x(const Task* tasks, int count, int P, int xmin,
                                                            uint64_t epoch, int local) {
    const XMap mp = x_map(P, local);
    if (mp.problem >= count) return;
    const Task& t = tasks[mp.problem];
    if (t.kind == T_INGEST || (t.flags & TF_COOP_EIG)) return;
    const int n = eig_n(t);
    if (n < xmin || n > XNMAX || mp.member >= x_members(n)) return;
    const SkDev* s = t.s;
    const bool rnd = t.kind == T_SHRINK_RAND;
    trix_body(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], s->slot[S_U], s->sld[S_U],
              s->slot[S_EV], s->xflags, s->info, epoch, mp.member);
}

static std::atomic<uint64_t> g_xwg_epoch{0};
uint64_t xwg_next_epoch() { return ++g_xwg_epoch; }

// Members of a problem on one XCD (SK_TRIX_LOCAL=1) or spread (0).
static int trix_local() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_TRIX_LOCAL");
        v = e ? atoi(e) : 0;
    }
    return v;
}

int trix_min_n() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_TRIX_MIN_N");
        v = e ? atoi(e) : 160;
        if (v < 8) v = 8;
    }
    return v;
}

// Every task with xmin <= n <= XNMAX (that the tridiagonal solver takes) by
// cooperative launches of 8 P ceil(count / 8) workgroups, P = members of the
// largest problem (smaller problems leave their surplus members idle); as
// many tasks per launch as can be resident at once.
hipError_t launch_tri_reduce_x(const Task* tasks, int count, int max_n, hipStream_t st) {
    const int nmax = std::min(max_n, XNMAX);
    int P = x_members(nmax);
    const size_t lds = sizeof(double) * (size_t)x_lds_doubles(nmax);
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        if (hipFuncSetAttribute((const void*)k_tri_reduce_x, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(double) * x_lds_doubles(XNMAX))) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_tri_reduce_x, XTHREADS,
                                                         sizeof(double) * x_lds_doubles(XNMAX)) != hipSuccess ||
            per_cu < 1)
            return hipErrorInvalidConfiguration;
    }
    // resident workgroups at the largest LDS size; 8 P per group of 8 tasks
    const int chunk = std::max(8, ((per_cu * cus) / (8 * P)) * 8);
    int xmin = trix_min_n(), local = trix_local();
    for (int off = 0; off < count; off += chunk) {
        const Task* tl = tasks + off;
        int cnt = std::min(chunk, count - off);
        const int groups = (cnt + 7) / 8;
        uint64_t epoch = xwg_next_epoch();
        void* args[] = {(void*)&tl, (void*)&cnt, (void*)&P, (void*)&xmin, (void*)&epoch, (void*)&local};
        const unsigned grid = local ? (unsigned)(8 * P * groups) : (unsigned)(P * cnt);
        hipError_t e = hipLaunchCooperativeKernel((const void*)k_tri_reduce_x, dim3(grid), dim3(XTHREADS), args,
                                                  (unsigned)lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sk
