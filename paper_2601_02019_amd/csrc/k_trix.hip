// k_trix.hip -- Householder tridiagonalisation of one symmetric eigen-problem
// (the k x k Rayleigh-Ritz matrix of Algorithm "Simultaneous Iteration", or
// the 2 ell x 2 ell buffer Gram of the exact FD shrink, Sec. 2.3) by P
// one-wavefront workgroups ("members").
//
// Member m holds rows i = m + P q (q < XR) of A in registers, lane l the
// columns c = l + 64 t; every vector of the reduction (the current and the
// next reflector, p = tau A v, the shipped row) is kept the same way, so a
// lane only ever touches its own columns and no LDS or barrier is needed.
// Column j's reflector needs row j of the current matrix, A v over every row
// and the scalar p.v; each member computes its rows' part of A v, and one
// exchange per column gives every member all of p, the members' partial dots
// and the not-yet-updated row j + 1.  Every member then derives w, applies
// the rank-2 update to its own rows and forms row j + 1 of the updated
// matrix itself, so the next reflector starts without another exchange.
// All members run the same arithmetic on the same inputs, so they agree bit
// for bit; every sum has a fixed order (results repeat exactly).
//
// The exchange goes through self-tagged 64-bit words: a double travels as two
// words, each carrying 32 bits of it and the 32-bit tag of the step
// ((launch epoch << 10) | step, the epoch growing with every launch).  Words
// are written and read with relaxed agent-scope atomics, which are
// single-copy atomic, so a reader that sees the step's tag in a word has that
// word's payload, whatever the order in which the words arrive: no flag, no
// fence.  Two buffers alternate by step parity; a member writes step s + 2
// only after it has read every member's step s + 1, which every member
// publishes only after reading step s, so no word is overwritten before it
// is read.  Polls are bounded: a wait that gives up counts the failure in
// info[3] (the solve then reports SK_EDEVICE); no wait can hang.
//
// Output as the one-workgroup reductions: W row j holds v_j beyond the
// super-diagonal and W[j][j] = tau_j (H_j = I - tau_j v_j v_j^T, v_j[j+1] = 1),
// U row 0 the diagonal of T and U row 1 its off-diagonal.
#include <atomic>

#include "sk_device.h"
#include "sk_kernels.h"
#include "sk_xwg.h"

namespace sk {

constexpr int XR = 4;             // rows per member
constexpr int XNMAX = 512;
// columns per lane: NT = 4 for orders up to 256, 8 up to 512 (templates)
// A step buffer of a problem of order n holds p (2 words per row, from word
// 0), the shipped row (2 per column, from 2 n) and the members' partial dots
// (2 per member, from 4 n): 4 n + 2 P words; the two buffers take at most
// 9 n + 4 words, inside the n x n scratch slot for every n >= 10.
__host__ __device__ __forceinline__ int x_slot_words(int n) { return 4 * n + 2 * ((n + 3) / 4); }

__host__ __device__ __forceinline__ int x_members(int n) { return (n + XR - 1) / XR; }

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
// Element k of a register array (k uniform).  The entries arrive as values,
// not as a reference to the array: a select among loads of the array could
// be folded into one load at a computed address, which would move the array
// out of registers.
__device__ __forceinline__ double x_pick4(int k, double v0, double v1, double v2, double v3) {
    return k == 0 ? v0 : k == 1 ? v1 : k == 2 ? v2 : v3;
}
__device__ __forceinline__ double x_pick8(int k, double v0, double v1, double v2, double v3, double v4, double v5,
                                          double v6, double v7) {
    return k < 4 ? x_pick4(k, v0, v1, v2, v3) : x_pick4(k - 4, v4, v5, v6, v7);
}
template <int NT> __device__ __forceinline__ double x_pickv(int k, const double (&v)[NT]);
template <> __device__ __forceinline__ double x_pickv<8>(int k, const double (&v)[8]) {
    return x_pick8(k, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
}
template <> __device__ __forceinline__ double x_pickv<4>(int k, const double (&v)[4]) {
    return x_pick4(k, v[0], v[1], v[2], v[3]);
}
static_assert(XR == 4, "x_row picks from 4 rows per member");
// entry c of a lane-distributed vector (c uniform)
#define x_at(v, c) x_lane(x_pickv<NT>((c) >> 6, v), (c) & 63)
// column slot t of row slot q (q uniform) of the member's rows
#define x_row(a, q, t) x_pick4(q, a[0][t], a[1][t], a[2][t], a[3][t])

__device__ __forceinline__ uint32_t x_tag(uint64_t epoch, int step) {
    return (uint32_t)((epoch << 10) | (uint64_t)step);
}
// global (not flat) accesses: the compiler then waits for just the loads a
// check needs, not for every load in flight
typedef __attribute__((address_space(1))) uint64_t xg_u64;
__device__ __forceinline__ void x_put(uint64_t* w, int half, uint32_t tag, double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint64_t p = half ? (b >> 32) : (b & 0xffffffffull);
    __hip_atomic_store((xg_u64*)(w + half), ((uint64_t)tag << 32) | p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t x_get(const uint64_t* w) {
    return __hip_atomic_load((const xg_u64*)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double x_join(uint64_t lo, uint64_t hi) {
    return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
}

// Reflector of column jj from the row x that it reduces (x[jj + 1] = alpha),
// in every member (no exchange): v[jj + 1 ..] into v (v[jj + 1] = 1, zero
// before), returns tau; member 0 also writes the reflector (W row jj), the
// diagonal entry and beta.  xn2 = |x beyond jj + 1|^2.
template <int NT>
__device__ __forceinline__ double x_reflector(int jj, int n, const double (&x)[NT], double xn2, double (&v)[NT],
                                              double* Wr, double* U, int lu, bool writer) {
    const int lane = threadIdx.x & 63;
    const double alpha = x_at(x, jj + 1);
    double beta = alpha, tau = 0.0, scal = 0.0;
    if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = lane + 64 * t;
        v[t] = (c <= jj || c >= n) ? 0.0 : (c == jj + 1) ? 1.0 : x[t] * scal;
    }
    if (writer) {
        const double xjj = x_at(x, jj);
        if (lane == 0) {
            U[jj] = xjj;
            U[lu + jj] = beta;
            Wr[(int64_t)jj * n + jj] = tau;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            if (c > jj + 1 && c < n) Wr[(int64_t)jj * n + c] = v[t];
        }
    }
    return tau;
}

// The words of one step a lane reads: p and the shipped row at its columns
// beyond jj, the partial dots of members lane and lane + 64.
template <int NT>
struct XWords {
    uint64_t p[NT][2], r[NT][2], d[2][2];
    __device__ __forceinline__ void load(const uint64_t* buf, int op, int orow, int odot, int lane, int jj, int n,
                                         int P) {
        // straight-line loads from clamped (always valid) addresses; the
        // words a lane does not need are ignored by tagged()
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = min(lane + 64 * t, n - 1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                p[t][h] = x_get(buf + op + 2 * c + h);
                r[t][h] = x_get(buf + orow + 2 * c + h);
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int m = min(lane + 64 * k, P - 1);
#pragma unroll
            for (int h = 0; h < 2; ++h) d[k][h] = x_get(buf + odot + 2 * m + h);
        }
    }
    __device__ __forceinline__ bool tagged(uint32_t tag, int lane, int jj, int n, int P) const {
        bool ok = true;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            const bool need = c > jj && c < n;
#pragma unroll
            for (int h = 0; h < 2; ++h)
                ok &= !need || ((uint32_t)(p[t][h] >> 32) == tag && (uint32_t)(r[t][h] >> 32) == tag);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bool need = lane + 64 * k < P;
#pragma unroll
            for (int h = 0; h < 2; ++h) ok &= !need || (uint32_t)(d[k][h] >> 32) == tag;
        }
        return ok;
    }
};

// Publishes step s (column jj = s - 1): p of this member's rows beyond jj,
// its partial dot, and row jj + 1 (columns from jj + 1) if this member holds
// it; then reads every member's step s into p, row and the dot sum.
// Returns false on a timed-out wait.
template <int NT>
__device__ __forceinline__ bool x_exchange(int s, int n, int P, int member, const double (&a)[XR][NT],
                                           const double (&pl)[XR], double dot, uint64_t* xw, uint64_t epoch,
                                           double (&p)[NT], double (&row)[NT], double* dsum) {
    const int lane = threadIdx.x & 63;
    const int jj = s - 1;
    const uint32_t tag = x_tag(epoch, s);
    uint64_t* buf = xw + (s & 1) * x_slot_words(n);
    const int XW_P = 0, XW_ROW = 2 * n, XW_DOT = 4 * n;
    if (lane < 2 * XR) {
        const int q = lane >> 1, i = member + P * q;
        const double v = x_pick4(q, pl[0], pl[1], pl[2], pl[3]);
        if (i > jj && i < n) x_put(buf + XW_P + 2 * i, lane & 1, tag, v);
    } else if (lane < 2 * XR + 2) {
        x_put(buf + XW_DOT + 2 * member, lane & 1, tag, dot);
    }
    if (member == (jj + 1) % P) {
        const int q = (jj + 1) / P;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            if (c > jj && c < n) {
                const double v = x_row(a, q, t);
                x_put(buf + XW_ROW + 2 * c, 0, tag, v);
                x_put(buf + XW_ROW + 2 * c, 1, tag, v);
            }
        }
    }
    // every word of the step this lane needs, until all carry the tag
    XWords<NT> A;
    bool ok = false;
    for (unsigned polls = 0; polls <= XWG_POLLS; ++polls) {
        A.load(buf, XW_P, XW_ROW, XW_DOT, lane, jj, n, P);
        if (__all(A.tagged(tag, lane, jj, n, P))) {
            ok = true;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    uint64_t wp[NT][2], wr[NT][2], wd[2][2];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            wp[t][h] = A.p[t][h];
            wr[t][h] = A.r[t][h];
        }
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2)
#pragma unroll
        for (int h = 0; h < 2; ++h) wd[k2][h] = A.d[k2][h];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = lane + 64 * t;
        const bool live = c > jj && c < n;
        p[t] = live ? x_join(wp[t][0], wp[t][1]) : 0.0;
        row[t] = live ? x_join(wr[t][0], wr[t][1]) : 0.0;
    }
    // partial dots in member order through a fixed tree (the same sum in every member)
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (lane + 64 * k < P) d += x_join(wd[k][0], wd[k][1]);
    *dsum = x_wave_sum(d);
    return ok;
}

template <int NT>
__device__ void trix_body(const double* __restrict__ Ain, int ldin, int n, double* __restrict__ Wr,
                          double* __restrict__ U, int lu, uint64_t* xw, int* info, uint64_t epoch, int member) {
    const int P = x_members(n);
    const int lane = threadIdx.x & 63;
    const bool writer = member == 0;
    double a[XR][NT];  // rows member + P q, columns lane + 64 t
#pragma unroll
    for (int q = 0; q < XR; ++q) {
        const int i = member + P * q;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            a[q][t] = (i < n && c < n) ? 0.5 * (Ain[(int64_t)i * ldin + c] + Ain[(int64_t)c * ldin + i]) : 0.0;
        }
    }
    // (n >= 16 here: the launcher takes orders from trix_min_n() >= 16)
    // column 0: row 0 of A, its reflector, p of this member's rows
    double va[NT], vb[NT], p[NT], row[NT], x[NT];
    double tau, dsum;
    {
        double s2 = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            x[t] = c < n ? 0.5 * (Ain[c] + Ain[(int64_t)c * ldin]) : 0.0;
            if (c >= 2 && c < n) s2 = fma(x[t], x[t], s2);
        }
        s2 = x_wave_sum(s2);
        tau = x_reflector(0, n, x, s2, va, Wr, U, lu, writer);
    }
    double pl[XR], dot = 0.0;
#pragma unroll
    for (int q = 0; q < XR; ++q) {
        const int i = member + P * q;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc = fma(a[q][t], va[t], acc);  // va is zero up to column 0
        acc = x_wave_sum(acc);
        pl[q] = (i > 0 && i < n) ? tau * acc : 0.0;
        if (i > 0 && i < n) dot = fma(pl[q], x_at(va, i), dot);
    }
    bool bad = !x_exchange(1, n, P, member, a, pl, dot, xw, epoch, p, row, &dsum);
    for (int j = 0; j + 2 < n && !bad; ++j) {
        // row j + 1 after this column's update, w = p - K v on the fly, with
        // the squared norm of its part beyond j + 2
        const double K = 0.5 * tau * dsum;
        const double w1 = fma(-K, x_at(va, j + 1), x_at(p, j + 1));
        const bool next = j + 3 < n;
        double wv[NT], s2 = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = lane + 64 * t;
            wv[t] = fma(-K, va[t], p[t]);
            x[t] = (c > j && c < n) ? fma(-1.0, wv[t], fma(-w1, va[t], row[t])) : 0.0;
            if (c >= j + 3 && c < n) s2 = fma(x[t], x[t], s2);
        }
        double tau2 = 0.0;
        if (next) {
            s2 = x_wave_sum(s2);
            tau2 = x_reflector(j + 1, n, x, s2, vb, Wr, U, lu, writer);
        } else {  // j = n - 3: the last 2 x 2 block of T
            const double d0 = x_at(x, n - 2), e0 = x_at(x, n - 1);
            if (writer && lane == 0) {
                U[n - 2] = d0;
                U[lu + n - 2] = e0;
                Wr[(int64_t)(n - 2) * n + n - 2] = 0.0;
                Wr[(int64_t)(n - 1) * n + n - 1] = 0.0;
            }
        }
        // the update of column j on this member's rows and their products
        // with the next reflector
        dot = 0.0;
#pragma unroll
        for (int q = 0; q < XR; ++q) {
            const int i = member + P * q;
            if (i > j && i < n) {  // uniform
                const double vi = x_at(va, i), wi = fma(-K, vi, x_at(p, i));
                double acc = 0.0;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int c = lane + 64 * t;
                    if (c > j && c < n) a[q][t] = fma(-vi, wv[t], fma(-wi, va[t], a[q][t]));
                    acc = fma(a[q][t], vb[t], acc);  // vb is zero up to column j + 1
                }
                if (next && i > j + 1) {
                    acc = x_wave_sum(acc);
                    pl[q] = tau2 * acc;
                    dot = fma(pl[q], x_at(vb, i), dot);
                }
            }
        }
        if (!next) break;
        bad = !x_exchange(j + 2, n, P, member, a, pl, dot, xw, epoch, p, row, &dsum);
#pragma unroll
        for (int t = 0; t < NT; ++t) va[t] = vb[t];
        tau = tau2;
    }
    if (bad) {
        if (lane == 0) atomicAdd(&info[3], 1);
        return;
    }
    // A[n-1][n-1] after every update: its holder writes it
    if (member == (n - 1) % P) {
        const int q = (n - 1) / P, t = (n - 1) >> 6;
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < NT; ++u)
            if (u == t) v = x_row(a, q, u);
        v = x_lane(v, (n - 1) & 63);
        if (lane == 0) U[n - 1] = v;
    }
}

// Task form: eigen-problems of shrink / query tasks that the tridiagonal
// solver takes and whose size is in [xmin, XNMAX]; workgroup b is member
// b mod P of problem b / P.
template <int NT>
__global__ __launch_bounds__(64) void k_tri_reduce_x(const Task* tasks, int count, int P, int xmin, uint64_t epoch) {
    const int problem = blockIdx.x / P, member = blockIdx.x % P;
    if (problem >= count) return;
    const Task& t = tasks[problem];
    if (t.kind == T_INGEST || (t.flags & TF_COOP_EIG)) return;
    const int n = eig_n(t);
    if (n < xmin || n > 64 * NT || member >= x_members(n)) return;
    const SkDev* s = t.s;
    const bool rnd = t.kind == T_SHRINK_RAND;
    trix_body<NT>(s->slot[rnd ? S_M : S_G], s->sld[rnd ? S_M : S_G], n, s->slot[S_EA], s->slot[S_U], s->sld[S_U],
              (uint64_t*)s->slot[S_EV], s->info, epoch, member);
}

static std::atomic<uint64_t> g_xwg_epoch{0};
uint64_t xwg_next_epoch() { return ++g_xwg_epoch; }

int trix_min_n() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_TRIX_MIN_N");
        v = e ? atoi(e) : 160;
        if (v < 16) v = 16;  // the step buffers fit the n x n scratch slot
    }
    return v;
}

// Every task with xmin <= n <= XNMAX (that the tridiagonal solver takes) by
// cooperative launches of P workgroups per task, P = members of the largest
// problem (smaller problems leave their surplus members idle); as many tasks
// per launch as can be resident at once.  The step buffers live in the
// eigen-solver's scratch slot (at least n x n doubles).
hipError_t launch_tri_reduce_x(const Task* tasks, int count, int max_n, hipStream_t st) {
    const int nmax = std::min(max_n, XNMAX);
    const bool small = nmax <= 256;
    const void* kern = small ? (const void*)k_tri_reduce_x<4> : (const void*)k_tri_reduce_x<8>;
    int P = x_members(nmax);
    static int per_cu[2] = {-1, -1}, cus = 0;
    int& pc = per_cu[small ? 0 : 1];
    if (pc < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, 64, 0) != hipSuccess || pc < 1) {
            pc = -1;
            return hipErrorInvalidConfiguration;
        }
    }
    const int chunk = std::max(1, (pc * cus) / P);
    int xmin = trix_min_n();
    for (int off = 0; off < count; off += chunk) {
        const Task* tl = tasks + off;
        int cnt = std::min(chunk, count - off);
        uint64_t epoch = xwg_next_epoch();
        void* args[] = {(void*)&tl, (void*)&cnt, (void*)&P, (void*)&xmin, (void*)&epoch};
        hipError_t e = hipLaunchCooperativeKernel(kern, dim3((unsigned)(P * cnt)), dim3(64), args, 0, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sk
