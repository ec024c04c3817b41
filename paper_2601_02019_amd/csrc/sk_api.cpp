// sk_api.cpp -- host engine and C ABI (include/sketch.h).
//
// The host owns each sketch's state machine: it knows from row counts alone
// when the buffer fills (Algorithm "AeroSketch: Update"), so a whole
// update call is planned on the host as a list of Task records (ingest
// segments and shrinks), uploaded once, and executed as a stream-ordered
// sequence of task-list launches without any device-to-host round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sk_internal.h"
#include "sk_window.h"

thread_local std::string g_err;
thread_local const char* g_stage = "";
std::atomic<int64_t> g_in_use{0};
std::atomic<int64_t> g_budget{0};

// Problem sizes from which one task alone runs the cooperative solvers:
// CholeskyQR from k = 64 (SK_COOP_MIN_N; 4 % more rows/s than the
// one-workgroup kernel on the 64 CSR sites at k = 128), the eigen-solve from n = 513
// (SK_COOP_EIG_MIN_N; up to 512 the tridiagonal solver, whose reduction
// runs on several workgroups from n = 160, is faster than the block Jacobi
// method: the exact shrink with a 512 x 512 core took 6.9 ms against 25 ms
// at d = 4096; with SK_EIG_SOLVER=jacobi the one-workgroup Jacobi solver
// stops at 128).
static int coop_min_n() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_COOP_MIN_N");
        v = e ? atoi(e) : 64;
    }
    return v;
}

bool eig_solver_jacobi();

// CholeskyQR of 64 <= k <= 512 (SK_CHOLX_MIN_K moves the lower end) runs on
// ceil(k / 16) workgroups with one exchange per 16 columns (k_cholx.hip).
static int cholx_min_k() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_CHOLX_MIN_K");
        v = e ? atoi(e) : 64;
    }
    return v;
}

static int coop_eig_min_n() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_COOP_EIG_MIN_N");
        v = e ? atoi(e) : (eig_solver_jacobi() ? 129 : 513);
    }
    return v;
}

// The one-workgroup eigen-solver: the tridiagonal solver, or the Jacobi
// method with SK_EIG_SOLVER=jacobi (both exact to rounding; the choice is
// fixed for the process, so results do not depend on batch composition).
bool eig_solver_jacobi() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_EIG_SOLVER");
        v = (e && std::string(e) == "jacobi") ? 1 : 0;
    }
    return v == 1;
}

// Marks the stages of a shrink / query task that the cooperative solvers
// take: a property of the task alone, so a sketch computes the same thing
// whatever else shares its launches.
static void mark_coop(Task& t, const sketch_s* h) {
    const int n = (t.kind == T_SHRINK_RAND) ? h->k : t.m;
    t.flags = 0;
    if (n >= coop_eig_min_n()) t.flags |= TF_COOP_EIG;
    if (t.kind == T_SHRINK_RAND && h->k >= cholx_min_k() && h->k <= 512) t.flags |= TF_X_CHOL;
    else if (t.kind == T_SHRINK_RAND && h->k >= coop_min_n()) t.flags |= TF_COOP_CHOL;
}

// Split-K plan: about 512 workgroups in total for a launch, the split count
// rounded up to a multiple of 8 so that each K chunk stays on one XCD
// (xcd_tile_split), and chunks of at least 128 columns.
static void splitk_plan(int tiles, int d, int* splits, int* chunk, int target = 512) {
    int s = std::max(1, (target + tiles - 1) / tiles);
    if (s > 1) s = (s + 7) / 8 * 8;
    s = std::min(s, std::max(1, (d + 127) / 128));
    int kc = (int)round_up((d + s - 1) / s, 16);
    s = (d + kc - 1) / kc;
    *splits = std::max(1, s);
    *chunk = kc;
}

// Workgroups the Gram's split-K plan aims at (SK_GRAM_SPLITK_TARGET).
static int gram_splitk_target() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("SK_GRAM_SPLITK_TARGET");
        v = e ? std::max(1, atoi(e)) : 512;
    }
    return v;
}

static sk_status build_device_state(sketch_t h) {
    const int d = h->d, ell = h->ell, n2 = h->n2, k = h->k;
    const int neig = std::max(n2, k);
    const int neig32 = (int)round_up(neig, 32);  // cooperative solvers pad to 32
    const int kk = std::max(k, 1);
    SkDev& s = h->host;
    std::memset(&s, 0, sizeof(s));
    s.d = d;
    s.ell = ell;
    s.n2 = n2;
    s.k = k;
    s.st = h->st;
    s.pj = h->pj;
    s.ld = h->ld;
    s.seed = h->cfg.seed;
    s.stream = h->cfg.stream_id;
    const int ntg = (n2 + 63) / 64;
    splitk_plan(ntg * (ntg + 1) / 2, d, &s.sg, &s.kcg, gram_splitk_target());
    splitk_plan(ntg * ((kk + 63) / 64), d, &s.sp, &s.kcp);
    const size_t es = (size_t)dtype_size(h->st);
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(h, h->dalloc(&s.buf[b], es * (size_t)n2 * (size_t)h->ld));
        HIP_TRY(h, h->dzero(s.buf[b], es * (size_t)n2 * (size_t)h->ld));
    }
    if (h->rnd) {
        const size_t ps = (size_t)dtype_size(h->pj);
        HIP_TRY(h, h->dalloc(&s.omegaT, ps * (size_t)k * (size_t)h->ld));
        HIP_TRY(h, h->dzero(s.omegaT, ps * (size_t)k * (size_t)h->ld));
    }
    struct Sz { int slot; int64_t rows, cols; };
    const int64_t mk = h->rnd ? kk : 1;
    const Sz sizes[] = {
        {S_G, n2, n2},       {S_P, n2, mk},        {S_Y, n2, mk},      {S_Q, n2, mk},
        {S_Q1, n2, mk},      {S_W, mk, mk},        {S_X, mk, mk},      {S_T1, n2, mk},
        {S_M, mk, mk},       {S_U, neig, neig},    {S_Z, n2, mk},      {S_T, ell, n2},
        {S_LAM, 1, neig},    {S_EA, neig32, neig32}, {S_EV, neig32, neig32},
        {S_GPART, (int64_t)s.sg * n2, n2},
        {S_PPART, (int64_t)(h->rnd ? s.sp : 1) * n2, mk},
        {S_QOUT, ell, h->ld},
    };
    for (const Sz& z : sizes) {
        void* p = nullptr;
        HIP_TRY(h, h->dalloc(&p, sizeof(double) * (size_t)z.rows * (size_t)z.cols));
        s.slot[z.slot] = (double*)p;
        s.sld[z.slot] = (int32_t)z.cols;
    }
    s.sld[S_LAM] = 1;
    {
        void* p = nullptr;
        HIP_TRY(h, h->dalloc(&p, sizeof(double) * COOP_DOUBLES));
        h->coop = (double*)p;
        HIP_TRY(h, h->dalloc(&p, 64 * sizeof(int)));
        HIP_TRY(h, h->dzero(p, 64 * sizeof(int)));
        h->coop_ctrl = (int*)p;
        s.coop = h->coop;
        s.coop_ctrl = h->coop_ctrl;
    }
    void* info = nullptr;
    HIP_TRY(h, h->dalloc(&info, 64));
    HIP_TRY(h, h->dzero(info, 64));
    s.info = (int32_t*)info;
    {
        void* p = nullptr;
        HIP_TRY(h, h->dalloc(&p, 64 * sizeof(uint64_t)));
        HIP_TRY(h, h->dzero(p, 64 * sizeof(uint64_t)));
        s.xflags = (uint64_t*)p;
    }
    HIP_TRY(h, h->dalloc((void**)&h->dev, sizeof(SkDev)));
    if (!h->dry) HIP_TRY(h, hipMemcpy(h->dev, &s, sizeof(SkDev), hipMemcpyHostToDevice));
    return SK_OK;
}

// ---------------------------------------------------------- stage sequences
namespace {

struct Group {
    int count = 0;
    int max_m = 0, max_k = 0, max_d = 0, max_ell = 0, max_sg = 1, max_sp = 1, max_n = 0, min_n = 1 << 30;
    bool small = false, large = false, small_k = false, large_k = false;
    int q = 0, st = DT_F64, pj = DT_F64;
    double* coop = nullptr;
    int* coop_ctrl = nullptr;
    Prof* prof = nullptr;
    const SkDev* hs = nullptr;   // host mirror of the (single) task's sketch
    int kind = 0;
    // tasks (offsets in the group) whose eigen-solve / CholeskyQR is cooperative
    std::vector<int> coop_eig, coop_chol;
    int x_chol_k = 0;             // largest k of the tasks on the multi-workgroup CholeskyQR
    std::vector<sketch_t> own;
    std::vector<int> ns;          // eigen-problem size of each task
    bool any_plain_eig = false, any_plain_chol = false;
};

Group describe(const std::vector<sketch_t>& owners, const std::vector<Task>& tasks, size_t first,
               size_t count) {
    Group g;
    g.count = (int)count;
    for (size_t i = first; i < first + count; ++i) {
        const sketch_t h = owners[i];
        const Task& t = tasks[i];
        g.max_m = std::max(g.max_m, t.m);
        g.max_k = std::max(g.max_k, h->k);
        g.max_d = std::max(g.max_d, h->d);
        g.max_ell = std::max(g.max_ell, h->ell);
        g.max_sg = std::max(g.max_sg, h->host.sg);
        g.max_sp = std::max(g.max_sp, h->host.sp);
        const int n = (t.kind == T_SHRINK_RAND) ? h->k : t.m;
        g.max_n = std::max(g.max_n, n);
        g.min_n = std::min(g.min_n, n);
        if (n <= jacobi_lds_max()) g.small = true;
        else g.large = true;
        if (h->k <= chol_lds_max()) g.small_k = true;
        else g.large_k = true;
        g.q = h->q;
        g.st = h->st;
        g.pj = h->pj;
        g.coop = h->coop;
        g.coop_ctrl = h->coop_ctrl;
        g.hs = &h->host;
        g.kind = t.kind;
        g.own.push_back(h);
        g.ns.push_back(n);
        if (t.flags & TF_COOP_EIG) g.coop_eig.push_back((int)(i - first));
        else g.any_plain_eig = true;
        if (t.flags & TF_X_CHOL) g.x_chol_k = std::max(g.x_chol_k, h->k);
        else if (t.flags & TF_COOP_CHOL) g.coop_chol.push_back((int)(i - first));
        else if (t.kind == T_SHRINK_RAND) g.any_plain_chol = true;
    }
    return g;
}

inline int dims(int M, int N, int K) { return M | (N << 2) | (K << 4); }  // 0 m, 1 k, 2 n

hipError_t cholqr(const Task* t, const Group& g, int sy, int sq, int passes, hipStream_t st) {
    hipError_t e;
    StageScope sc(g.prof, ST_CHOLQR, st);
    if (g.any_plain_chol || g.x_chol_k > 0) {
        // batched CholeskyQR passes: the Gram of every task, then the
        // one-workgroup Cholesky-inverse and Q = Y X^T (which skip or are
        // overwritten for the other tasks), then the multi-workgroup pass of
        // the tasks flagged for it; cooperative tasks are rewritten below from
        // the unchanged input sy
        // The second pass of the multi-workgroup tasks may be the polar step
        // (k_cholx.hip): X = (3I - W) / 2 goes to S_X, the same X-multiply
        // launch as the one-workgroup tasks' applies it, and the Cholesky pass
        // skips the tasks it served.
        int src = sy;
        for (int pass = 0; pass < passes; ++pass) {
            const int dst = (pass == passes - 1) ? sq : S_Q1;
            const bool polar = g.x_chol_k > 0 && pass == 1;
            if ((g_stage = "core_gemm", e = launch_core_gemm(t, g.count, g.max_k, g.max_k, true, false, src, src, S_W, dims(1, 1, 0), st))) return e;
            if (g.any_plain_chol && (g_stage = "cholinv", e = launch_cholinv(t, g.count, g.max_k, g.small_k, g.large_k, S_W, S_X, st)))
                return e;
            if (polar && (g_stage = "cholx_polar", e = launch_cholx_polar(t, g.count, st))) return e;
            if ((g.any_plain_chol || polar) &&
                (g_stage = "core_gemm", e = launch_core_gemm(t, g.count, g.max_m, g.max_k, false, true, src, S_X, dst, dims(0, 1, 1), st)))
                return e;
            if (g.x_chol_k > 0 &&
                (g_stage = "cholqr_x", e = launch_cholqr_x(t, g.count, g.x_chol_k, src, dst, pass, polar ? 1 : 0, st)))
                return e;
            src = dst;
        }
    }
    if (!g.coop_chol.empty()) {
        // every cooperative CholeskyQR of the group in one launch (same m and k
        // within a task; the launch is sized by the largest)
        int m = 0, k = 0;
        for (int off : g.coop_chol) {
            m = std::max(m, g.own[(size_t)off]->n2);
            k = std::max(k, g.own[(size_t)off]->k);
        }
        g_stage = "cholqr_coop";
        if ((e = launch_cholqr_coop_tasks(t, g.coop_chol.data(), (int)g.coop_chol.size(), m, k, sy, sq, passes, st)))
            return e;
    }
    return hipSuccess;
}

hipError_t eig(const Task* t, const Group& g, hipStream_t st) {
    if (g.any_plain_eig) {
        hipError_t e;
        if (eig_solver_jacobi()) {
            StageScope sc(g.prof, ST_EIG, st);
            g_stage = "jacobi";
            e = launch_jacobi(t, g.count, g.max_n, g.small, g.large, st);
        } else {
            {
                StageScope sc(g.prof, ST_EIG_REDUCE, st);
                g_stage = "tridiagonal reduction";
                e = launch_tri_reduce(t, g.count, g.min_n, g.max_n, st);
            }
            if (e == hipSuccess) {
                StageScope sc(g.prof, ST_EIG, st);
                g_stage = "tridiagonal eig";
                e = launch_tri_eig(t, g.count, g.max_n, st);
            }
            if (e == hipSuccess) {
                StageScope sc(g.prof, ST_EIG_BACK, st);
                g_stage = "eig back-transformation";
                e = launch_tri_back(t, g.count, g.max_n, st);
            }
        }
        if (e != hipSuccess) return e;
    }
    if (!g.coop_eig.empty()) {
        StageScope sc(g.prof, ST_EIG, st);
        // every cooperative eigen-solve of the group in one launch
        int max_n = 0;
        for (int off : g.coop_eig) max_n = std::max(max_n, g.ns[(size_t)off]);
        g_stage = "jacobi_coop";
        hipError_t e = launch_jacobi_coop_tasks(t, g.coop_eig.data(), (int)g.coop_eig.size(), max_n, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Runs the shrink stages for `count` tasks of one kind starting at t.
hipError_t run_shrinks(const Task* t, const Group& g, int kind, hipStream_t st) {
    hipError_t e;
    if (kind == T_SHRINK_RAND) {
        { StageScope sc(g.prof, ST_OMEGA, st); if ((g_stage = "omega", e = launch_omega(t, g.count, g.max_d, g.max_k, g.pj, st))) return e; }
        { StageScope sc(g.prof, ST_GRAM, st); if ((g_stage = "gram", e = launch_gram(t, g.count, g.max_m, g.max_sg, g.st, st))) return e; }
        { StageScope sc(g.prof, ST_PROJECT, st); if ((g_stage = "project", e = launch_project(t, g.count, g.max_m, g.max_k, g.max_sp, g.st, g.pj, st))) return e; }
        int cur = S_P;
        for (int it = 0; it < g.q; ++it) {
            // a well-conditioned basis of the iterate's span is enough between steps
            if ((e = cholqr(t, g, cur, S_Q, 1, st))) return e;
            { StageScope sc(g.prof, ST_CORE, st); if ((g_stage = "core_gemm", e = launch_core_gemm(t, g.count, g.max_m, g.max_k, false, false, S_G, S_Q, S_Y, dims(0, 1, 0), st))) return e; }
            cur = S_Y;
        }
        if ((e = cholqr(t, g, cur, S_Q, 2, st))) return e;
        { StageScope sc(g.prof, ST_CORE, st); if ((g_stage = "core_gemm", e = launch_core_gemm(t, g.count, g.max_m, g.max_k, false, false, S_G, S_Q, S_T1, dims(0, 1, 0), st))) return e; }
        { StageScope sc(g.prof, ST_CORE, st); if ((g_stage = "core_gemm", e = launch_core_gemm(t, g.count, g.max_k, g.max_k, true, false, S_Q, S_T1, S_M, dims(1, 1, 0), st))) return e; }
        if ((e = eig(t, g, st))) return e;
        { StageScope sc(g.prof, ST_CORE, st); if ((g_stage = "core_gemm", e = launch_core_gemm(t, g.count, g.max_m, g.max_k, false, false, S_Q, S_U, S_Z, dims(0, 1, 1), st))) return e; }
    } else {
        { StageScope sc(g.prof, ST_GRAM, st); if ((g_stage = "gram", e = launch_gram(t, g.count, g.max_m, g.max_sg, g.st, st))) return e; }
        if ((e = eig(t, g, st))) return e;
    }
    { StageScope sc(g.prof, ST_THRESH, st); if ((g_stage = "threshold", e = launch_threshold(t, g.count, g.max_ell, g.max_m, st))) return e; }
    g_stage = "rebuild";
    StageScope sc(g.prof, ST_REBUILD, st);
    return launch_rebuild(t, g.count, g.max_ell, g.max_d, g.st, kind == T_QUERY, st);
}

}  // namespace

// Executes a planned list: consecutive tasks of one kind form a launch group.
static sk_status execute(sketch_t h, std::vector<sketch_t>& owners, std::vector<Task>& tasks,
                         int in_dtype, bool csr) {
    if (tasks.empty()) return SK_OK;
    Task* dt = nullptr;
    HIP_TRY(h, h->arena.upload(tasks, h->stream, &dt));
    size_t i = 0;
    while (i < tasks.size()) {
        size_t j = i + 1;
        while (j < tasks.size() && tasks[j].kind == tasks[i].kind && tasks[j].kind != T_QUERY) {
            // a sketch may appear once per group only (its stages are not reentrant)
            bool dup = false;
            for (size_t u = i; u < j; ++u)
                if (owners[u] == owners[j]) dup = true;
            if (dup) break;
            ++j;
        }
        Group g = describe(owners, tasks, i, j - i);
        g.prof = &h->prof;
        if (tasks[i].kind == T_INGEST) {
            int max_rows = 0;
            for (size_t u = i; u < j; ++u) max_rows = std::max(max_rows, tasks[u].nrows);
            StageScope sc(g.prof, ST_INGEST, h->stream);
            if (csr) HIP_TRY(h, launch_ingest_csr(dt + i, g.count, max_rows, g.max_d, g.st, h->stream));
            else HIP_TRY(h, launch_ingest(dt + i, g.count, max_rows, g.max_d, in_dtype, g.st, h->stream));
        } else {
            HIP_TRY(h, run_shrinks(dt + i, g, tasks[i].kind, h->stream));
        }
        i = j;
    }
    HIP_TRY(h, h->arena.done(h->stream));
    return SK_OK;
}

// Plans ingest segments and shrinks for n rows appended to h.
void plan_rows(sketch_t h, int64_t n, const char* src, int64_t src_ld, int in_dtype,
                      const int64_t* indptr, const int32_t* idx, const float* val,
                      std::vector<sketch_t>& owners, std::vector<Task>& tasks) {
    const int64_t esz = src ? dtype_size(in_dtype) : 0;
    int64_t pos = 0;
    while (pos < n) {
        const int64_t take = std::min<int64_t>(n - pos, h->n2 - h->fill);
        Task t{};
        t.s = h->dev;
        t.kind = T_INGEST;
        t.par = h->par;
        t.row0 = (int32_t)h->fill;
        t.nrows = (int32_t)take;
        t.src_dtype = in_dtype;
        t.src_ld = src_ld;
        t.src = src ? src + pos * src_ld * esz : nullptr;
        t.indptr = indptr ? indptr + pos : nullptr;
        t.indices = idx;
        t.values = val;
        owners.push_back(h);
        tasks.push_back(t);
        h->fill += take;
        h->rows_seen += take;
        pos += take;
        if (h->fill == h->n2) {
            Task s{};
            s.s = h->dev;
            s.kind = h->rnd ? T_SHRINK_RAND : T_SHRINK_EXACT;
            s.par = h->par;
            s.m = h->n2;
            s.shrink_idx = h->shrinks;
            mark_coop(s, h);
            owners.push_back(h);
            tasks.push_back(s);
            h->par ^= 1;
            h->fill = h->ell - 1;
            h->shrinks += 1;
        }
    }
}

sk_status check_handle(sketch_t h, const char* what) {
    if (!h) return fail(SK_EINVAL, std::string(what) + ": NULL handle");
    if (h->sticky) return fail(SK_EDEVICE, std::string(what) + ": sketch is in a failed state: " + h->sticky_msg);
    return SK_OK;
}

// ---------------------------------------------------------------- C ABI
static sk_status validate_config(const sketch_config* cfg) {
    if (cfg->d < 1 || cfg->ell < 2) return fail(SK_EINVAL, "sketch_create: need d >= 1 and ell >= 2");
    if (cfg->ell > 256) return fail(SK_EINVAL, "sketch_create: ell > 256 is not supported");
    if (cfg->state_dtype != SK_F64 && cfg->state_dtype != SK_F32)
        return fail(SK_EINVAL, "sketch_create: state_dtype must be SK_F64 or SK_F32");
    if (cfg->proj_dtype < SK_F64 || cfg->proj_dtype > SK_BF16)
        return fail(SK_EINVAL, "sketch_create: bad proj_dtype");
    if (cfg->shrink != SK_SHRINK_EXACT && cfg->shrink != SK_SHRINK_RAND)
        return fail(SK_EINVAL, "sketch_create: bad shrink");
    if (cfg->kind != SK_PERSISTENT && cfg->kind != SK_WINDOW && cfg->kind != SK_ATTP && cfg->kind != SK_P5 &&
        cfg->kind != SK_COD)
        return fail(SK_EINVAL, "sketch_create: bad kind");
    if (cfg->kind == SK_COD) {
        if (cfg->d_y < 1 || cfg->d > 4096 || cfg->d_y > 4096 || std::min(cfg->d, cfg->d_y) > 512)
            return fail(SK_EINVAL, "sketch_create: COD needs 1 <= d, d_y <= 4096 and min(d, d_y) <= 512");
        if (cfg->window_N < 1 || !(cfg->theta > 0.0))
            return fail(SK_EINVAL, "sketch_create: COD needs window_N >= 1 and theta > 0");
        if (cfg->amplify_r != 1 || cfg->amplify_s != 0)
            return fail(SK_EINVAL, "sketch_create: amplification is not available for COD sketches");
    }
    if (cfg->kind == SK_P5 && (cfg->sites < 1 || cfg->sites > 4096))
        return fail(SK_EINVAL, "sketch_create: P5 needs 1 <= sites <= 4096");
    if (cfg->q < 0 || cfg->q > 64 || cfg->oversample < 0)
        return fail(SK_EINVAL, "sketch_create: bad q or oversample");
    if (cfg->kind == SK_WINDOW && (cfg->window_N < 1 || !(cfg->R >= 1.0)))
        return fail(SK_EINVAL, "sketch_create: window needs window_N >= 1 and R >= 1");
    if (cfg->d > (1 << 20)) return fail(SK_EINVAL, "sketch_create: d too large");
    if (cfg->amplify_r < 1 || cfg->amplify_r > 16 || cfg->amplify_s < 0 || cfg->amplify_s > 16)
        return fail(SK_EINVAL, "sketch_create: need 1 <= amplify_r <= 16 and 0 <= amplify_s <= 16");
    if (cfg->kind == SK_PERSISTENT && (cfg->amplify_r != 1 || cfg->amplify_s != 0))
        return fail(SK_EINVAL, "sketch_create: amplification applies to window and ATTP sketches only");
    return SK_OK;
}

static void init_fields(sketch_t h, const sketch_config* cfg) {
    h->cfg = *cfg;
    h->d = cfg->d;
    h->ell = cfg->ell;
    h->n2 = 2 * cfg->ell;
    h->rnd = cfg->kind == SK_PERSISTENT && cfg->shrink == SK_SHRINK_RAND;
    h->k = h->rnd ? std::min(std::min(cfg->ell + cfg->oversample, 2 * cfg->ell), cfg->d) : 0;
    h->q = cfg->q;
    h->st = cfg->state_dtype;
    h->pj = cfg->proj_dtype;
    h->ld = round_up(cfg->d, 64);
}

int64_t sketch_state_bytes(const sketch_config* cfg) {
    if (!cfg || validate_config(cfg) != SK_OK || cfg->kind != SK_PERSISTENT) return -1;
    sketch_s tmp;
    tmp.dry = true;
    init_fields(&tmp, cfg);
    if (build_device_state(&tmp) != SK_OK) return -1;
    return tmp.bytes;
}

sk_status sketch_reset(sketch_t h, uint64_t seed, uint64_t stream_id) {
    if (h->win || h->cod) return fail(SK_EUNSUPPORTED, "sketch_reset: window sketch");
    h->cfg.seed = seed;
    h->cfg.stream_id = stream_id;
    h->host.seed = seed;
    h->host.stream = stream_id;
    h->fill = 0;
    h->shrinks = 0;
    h->rows_seen = 0;
    h->par = 0;
    h->sticky = false;
    h->sticky_msg.clear();
    h->prof.drain();
    for (int i = 0; i < NSTAGE; ++i) {
        h->prof.calls[i] = 0;
        h->prof.ms[i] = 0.0;
    }
    h->prof.mask = 0;
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    // stream-ordered: kernels queued later read the new seed; the zeroed
    // buffer rows keep a query of the empty sketch exact
    HIP_TRY(h, hipMemsetAsync(h->host.buf[0], 0, (size_t)dtype_size(h->st) * (size_t)h->n2 * (size_t)h->ld,
                              h->stream));
    // the solver status words (non-convergence counts) belong to the previous
    // stream: a reused sketch starts with a clean record
    HIP_TRY(h, hipMemsetAsync(h->host.info, 0, 64, h->stream));
    // h->host is not written again before the sketch is next idle, so the
    // asynchronous copy may read it late
    HIP_TRY(h, hipMemcpyAsync(h->dev, &h->host, sizeof(SkDev), hipMemcpyHostToDevice, h->stream));
    return SK_OK;
}

extern "C" {

sk_status sketch_config_init(sketch_config* cfg) {
    if (!cfg) return fail(SK_EINVAL, "sketch_config_init: cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->kind = SK_PERSISTENT;
    cfg->shrink = SK_SHRINK_EXACT;
    cfg->state_dtype = SK_F64;
    cfg->proj_dtype = SK_F64;
    cfg->q = 1;
    cfg->R = 1.0;
    cfg->amplify_r = 1;
    cfg->amplify_s = 0;
    return SK_OK;
}

sk_status sketch_create(const sketch_config* cfg, sketch_t* out) {
    if (!cfg || !out) return fail(SK_EINVAL, "sketch_create: NULL argument");
    *out = nullptr;
    sk_status vr = validate_config(cfg);
    if (vr) return vr;
    sketch_t h = new sketch_s();
    init_fields(h, cfg);
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) {
        delete h;
        return fail(SK_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    if (cfg->hip_stream || cfg->use_given_stream) {
        h->stream = (hipStream_t)cfg->hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return fail(SK_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    sk_status rc;
    if (cfg->kind == SK_WINDOW || cfg->kind == SK_ATTP || cfg->kind == SK_P5) rc = window_create(h);
    else if (cfg->kind == SK_COD) rc = cod_create(h);
    else rc = build_device_state(h);
    const int64_t budget = g_budget.load();
    if (rc == SK_OK && budget > 0 && g_in_use.load() + h->bytes > budget) {
        rc = fail(SK_ENOMEM, "sketch_create: memory budget exceeded");
    }
    if (rc != SK_OK) {
        std::string msg = g_err;
        sketch_destroy(h);
        g_err = msg;
        return rc == SK_EDEVICE ? SK_ENOMEM : rc;
    }
    g_in_use += h->bytes;
    h->counted = true;
    *out = h;
    return SK_OK;
}


sk_status sketch_update(sketch_t h, const void* rows, int64_t n_rows, int64_t ld, int32_t dtype,
                        int32_t on_device) {
    sk_status rc = check_handle(h, "sketch_update");
    if (rc) return rc;
    if (n_rows < 0) return fail(SK_EINVAL, "sketch_update: n_rows < 0");
    if (n_rows == 0) return SK_OK;
    if (!rows) return fail(SK_EINVAL, "sketch_update: rows is NULL");
    if (ld < h->d) return fail(SK_EINVAL, "sketch_update: ld < d");
    if (dtype < SK_F64 || dtype > SK_BF16) return fail(SK_EINVAL, "sketch_update: bad dtype");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const char* src = (const char*)rows;
    const size_t es = (size_t)dtype_size(dtype);
    if (!on_device) {
        const size_t nb = es * (size_t)((n_rows - 1) * ld + h->d);
        HIP_TRY(h, h->ensure_stage(nb));
        HIP_TRY(h, hipMemcpyAsync(h->stage, rows, nb, hipMemcpyHostToDevice, h->stream));
        src = (const char*)h->stage;
    }
    if (h->cod) {
        rc = fail(SK_EUNSUPPORTED, "sketch_update: COD sketches take pairs by cod_update");
    } else if (h->win) {
        rc = h->cfg.kind == SK_P5 ? fail(SK_EUNSUPPORTED, "sketch_update: P5 sketches take rows by p5_update")
                                  : window_update(h, src, n_rows, ld, dtype);
    } else {
        std::vector<sketch_t> owners;
        std::vector<Task> tasks;
        plan_rows(h, n_rows, src, ld, dtype, nullptr, nullptr, nullptr, owners, tasks);
        rc = execute(h, owners, tasks, dtype, false);
    }
    if (rc) return rc;
    if (!on_device) HIP_TRY(h, hipStreamSynchronize(h->stream));
    return SK_OK;
}

sk_status sketch_update_csr(sketch_t h, const int64_t* indptr, const int32_t* indices,
                            const float* values, int64_t n_rows, int32_t on_device) {
    sk_status rc = check_handle(h, "sketch_update_csr");
    if (rc) return rc;
    if (n_rows < 0) return fail(SK_EINVAL, "sketch_update_csr: n_rows < 0");
    if (n_rows == 0) return SK_OK;
    if (!indptr || !indices || !values) return fail(SK_EINVAL, "sketch_update_csr: NULL array");
    if (h->win || h->cod) return fail(SK_EUNSUPPORTED, "sketch_update_csr: window sketches take dense rows");
    if (h->d > 16384) return fail(SK_EUNSUPPORTED, "sketch_update_csr: d > 16384");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const int64_t* ip = indptr;
    const int32_t* ix = indices;
    const float* vv = values;
    if (!on_device) {
        const int64_t nnz0 = indptr[0], nnz = indptr[n_rows] - indptr[0];
        if (nnz < 0) return fail(SK_EINVAL, "sketch_update_csr: indptr not non-decreasing");
        const size_t b1 = sizeof(int64_t) * (size_t)(n_rows + 1);
        const size_t b2 = sizeof(int32_t) * (size_t)nnz, b3 = sizeof(float) * (size_t)nnz;
        HIP_TRY(h, h->ensure_stage(b1 + round_up((int64_t)b2, 256) + b3 + 512));
        char* base = (char*)h->stage;
        std::vector<int64_t> shifted(indptr, indptr + n_rows + 1);
        for (auto& v : shifted) v -= nnz0;
        HIP_TRY(h, hipMemcpyAsync(base, shifted.data(), b1, hipMemcpyHostToDevice, h->stream));
        char* pix = base + round_up((int64_t)b1, 256);
        char* pv = pix + round_up((int64_t)b2, 256);
        HIP_TRY(h, hipMemcpyAsync(pix, indices + nnz0, b2, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync(pv, values + nnz0, b3, hipMemcpyHostToDevice, h->stream));
        ip = (const int64_t*)base;
        ix = (const int32_t*)pix;
        vv = (const float*)pv;
    }
    std::vector<sketch_t> owners;
    std::vector<Task> tasks;
    plan_rows(h, n_rows, nullptr, 0, DT_F32, ip, ix, vv, owners, tasks);
    rc = execute(h, owners, tasks, DT_F32, true);
    if (rc) return rc;
    if (!on_device) HIP_TRY(h, hipStreamSynchronize(h->stream));
    return SK_OK;
}

// Query into the sketch's FP64 staging (QOUT, ell x ld), on its stream.
static sk_status query_to_qout(sketch_t h) {
    const int64_t r = h->fill;
    double* qout = h->host.slot[S_QOUT];
    if (r >= h->ell) {
        std::vector<sketch_t> owners{h};
        Task t{};
        t.s = h->dev;
        t.kind = T_QUERY;
        t.par = h->par;
        t.m = (int32_t)r;
        mark_coop(t, h);
        std::vector<Task> tasks{t};
        return execute(h, owners, tasks, DT_F64, false);
    }
    HIP_TRY(h, hipMemsetAsync(qout, 0, sizeof(double) * (size_t)h->ell * (size_t)h->ld, h->stream));
    HIP_TRY(h, launch_rows_to_f64(h->host.buf[h->par], h->ld, h->st, qout, h->ld, (int)r, h->d, h->stream));
    return SK_OK;
}

static sk_status check_info(sketch_t h) {
    int32_t info[4] = {0, 0, 0, 0};
    const int32_t* dinfo = h->win ? window_info_ptr(h) : h->cod ? cod_info_ptr(h) : h->host.info;
    HIP_TRY(h, hipMemcpy(info, dinfo, sizeof(info), hipMemcpyDeviceToHost));
    if (info[0] != 0) return h->device_fail("eigen-solver did not converge");
    if (info[3] != 0) return h->device_fail("multi-workgroup reduction: exchange wait timed out");
    if (h->coop_ctrl) {
        unsigned bar[2] = {0, 0};
        HIP_TRY(h, hipMemcpy(bar, h->coop_ctrl + 8, sizeof(bar), hipMemcpyDeviceToHost));
        if (bar[1] != 0) return h->device_fail("cooperative grid barrier timed out");
    }
    return SK_OK;
}

// Copies the FP64 ell x ld result src to B_out (dtype, host or device) and
// waits for it.
static sk_status query_out(sketch_t h, const double* src, void* B_out, int32_t dtype, int32_t on_device);

sk_status sketch_query(sketch_t h, void* B_out, int32_t dtype, int32_t on_device) {
    sk_status rc = check_handle(h, "sketch_query");
    if (rc) return rc;
    if (!B_out) return fail(SK_EINVAL, "sketch_query: B_out is NULL");
    if (dtype != SK_F64 && dtype != SK_F32) return fail(SK_EINVAL, "sketch_query: dtype must be F64 or F32");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    if (h->cod) return fail(SK_EUNSUPPORTED, "sketch_query: COD sketches answer cod_query");
    const double* src = nullptr;
    if (h->win) {
        rc = window_query(h, &src);
    } else {
        rc = query_to_qout(h);
        src = h->host.slot[S_QOUT];
    }
    if (rc) return rc;
    return query_out(h, src, B_out, dtype, on_device);
}

sk_status sketch_query_at(sketch_t h, int64_t t, void* B_out, int32_t dtype, int32_t on_device) {
    sk_status rc = check_handle(h, "sketch_query_at");
    if (rc) return rc;
    if (!B_out) return fail(SK_EINVAL, "sketch_query_at: B_out is NULL");
    if (dtype != SK_F64 && dtype != SK_F32) return fail(SK_EINVAL, "sketch_query_at: dtype must be F64 or F32");
    if (!h->win || h->cfg.kind != SK_ATTP) return fail(SK_EUNSUPPORTED, "sketch_query_at: not an ATTP sketch");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const double* src = nullptr;
    if ((rc = window_query_at(h, t, &src))) return rc;
    return query_out(h, src, B_out, dtype, on_device);
}

static sk_status query_out(sketch_t h, const double* src, void* B_out, int32_t dtype, int32_t on_device) {
    const size_t es = (size_t)dtype_size(dtype);
    const size_t nb = es * (size_t)h->ell * (size_t)h->d;
    if (on_device) {
        HIP_TRY(h, launch_convert_rows(src, h->ld, B_out, h->d, h->ell, h->d, dtype, h->stream));
    } else {
        HIP_TRY(h, h->ensure_stage(nb));
        HIP_TRY(h, launch_convert_rows(src, h->ld, h->stage, h->d, h->ell, h->d, dtype, h->stream));
        HIP_TRY(h, hipMemcpyAsync(B_out, h->stage, nb, hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_info(h);
}

sk_status window_advance(sketch_t h, int64_t t_now) {
    sk_status rc = check_handle(h, "window_advance");
    if (rc) return rc;
    if (!h->win || h->cfg.kind != SK_WINDOW) return fail(SK_EUNSUPPORTED, "window_advance: not a window sketch");
    return window_advance_impl(h, t_now);
}

sk_status sketch_merge(sketch_t dst, const sketch_t* srcs, int32_t n_src) {
    sk_status rc = check_handle(dst, "sketch_merge");
    if (rc) return rc;
    if (n_src < 0 || (n_src > 0 && !srcs)) return fail(SK_EINVAL, "sketch_merge: bad source list");
    if (dst->win || dst->cod) return fail(SK_EUNSUPPORTED, "sketch_merge: window sketches cannot be merged");
    for (int i = 0; i < n_src; ++i) {
        if ((rc = check_handle(srcs[i], "sketch_merge"))) return rc;
        if (srcs[i]->d != dst->d) return fail(SK_ESHAPE, "sketch_merge: d differs");
        if (srcs[i]->win || srcs[i]->cod) return fail(SK_EUNSUPPORTED, "sketch_merge: window source");
        if (srcs[i] == dst) return fail(SK_EINVAL, "sketch_merge: dst listed as a source");
    }
    HIP_TRY(dst, hipSetDevice(dst->cfg.device));
    for (int i = 0; i < n_src; ++i) {
        sketch_t s = srcs[i];
        if (s->fill == 0) continue;
        if ((rc = query_to_qout(s))) return rc;
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        if ((rc = check_info(s))) return rc;
        const int64_t nz = s->fill >= s->ell ? s->ell - 1 : s->fill;
        // the rows are read on dst's stream: copy them to dst's staging first
        const size_t nb = sizeof(double) * (size_t)nz * (size_t)s->ld;
        HIP_TRY(dst, dst->ensure_stage(nb));
        HIP_TRY(dst, hipMemcpyAsync(dst->stage, s->host.slot[S_QOUT], nb, hipMemcpyDeviceToDevice, dst->stream));
        std::vector<sketch_t> owners;
        std::vector<Task> tasks;
        plan_rows(dst, nz, (const char*)dst->stage, s->ld, DT_F64, nullptr, nullptr, nullptr, owners, tasks);
        if ((rc = execute(dst, owners, tasks, DT_F64, false))) return rc;
        HIP_TRY(dst, hipStreamSynchronize(dst->stream));
    }
    return SK_OK;
}

sk_status sketch_debug_fail_solver(sketch_t h) {
    sk_status rc = check_handle(h, "sketch_debug_fail_solver");
    if (rc) return rc;
    if (h->win || h->cod) return fail(SK_EUNSUPPORTED, "sketch_debug_fail_solver: window sketch");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    // one failed solve, stream-ordered after the work queued so far (a
    // host-to-device copy: the library's kernels are not involved)
    static const int32_t one = 1;
    HIP_TRY(h, hipMemcpyAsync(h->host.info, &one, sizeof(one), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return SK_OK;
}

sk_status sketch_sync(sketch_t h) {
    sk_status rc = check_handle(h, "sketch_sync");
    if (rc) return rc;
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_info(h);
}

static void destroy_impl(sketch_t h, bool sync) {
    (void)hipSetDevice(h->cfg.device);
    if (sync && h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->win) window_destroy(h);
    if (h->cod) cod_destroy(h);
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->stage) (void)hipFree(h->stage);
    h->arena.release();
    h->prof.release();
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    if (h->counted) g_in_use -= h->bytes;
    delete h;
}

sk_status sketch_destroy(sketch_t h) {
    if (h) destroy_impl(h, true);
    return SK_OK;
}

const char* sketch_last_error(void) { return g_err.c_str(); }

sk_status sketch_info(sketch_t h, sketch_info_t* info) {
    if (!h || !info) return fail(SK_EINVAL, "sketch_info: NULL argument");
    info->rows_seen = h->win ? window_time(h) : h->cod ? cod_time(h) : h->rows_seen;
    info->fill = h->fill;
    info->shrinks = h->shrinks;
    info->device_bytes = h->bytes;
    info->k = h->k;
    info->levels = h->win ? window_levels(h) : 1;
    return SK_OK;
}

sk_status p5_update(sketch_t h, const int32_t* sites, const void* rows, int64_t n_rows, int64_t ld, int32_t dtype,
                    int32_t on_device) {
    sk_status rc = check_handle(h, "p5_update");
    if (rc) return rc;
    if (!h->win || h->cfg.kind != SK_P5) return fail(SK_EUNSUPPORTED, "p5_update: not a P5 sketch");
    if (n_rows < 0) return fail(SK_EINVAL, "p5_update: n_rows < 0");
    if (n_rows == 0) return SK_OK;
    if (!rows || !sites) return fail(SK_EINVAL, "p5_update: NULL rows or sites");
    if (ld < h->d) return fail(SK_EINVAL, "p5_update: ld < d");
    if (dtype < SK_F64 || dtype > SK_BF16) return fail(SK_EINVAL, "p5_update: bad dtype");
    for (int64_t e = 0; e < n_rows; ++e)
        if (sites[e] < 0 || sites[e] >= h->cfg.sites) return fail(SK_EINVAL, "p5_update: site outside [0, m)");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const char* src = (const char*)rows;
    if (!on_device) {
        const size_t nb = (size_t)dtype_size(dtype) * (size_t)((n_rows - 1) * ld + h->d);
        HIP_TRY(h, h->ensure_stage(nb));
        HIP_TRY(h, hipMemcpyAsync(h->stage, rows, nb, hipMemcpyHostToDevice, h->stream));
        src = (const char*)h->stage;
    }
    return p5_update_impl(h, sites, src, n_rows, ld, dtype);
}

sk_status p5_stats(sketch_t h, int64_t* stats8) {
    sk_status rc = check_handle(h, "p5_stats");
    if (rc) return rc;
    if (!h->win || h->cfg.kind != SK_P5) return fail(SK_EUNSUPPORTED, "p5_stats: not a P5 sketch");
    if (!stats8) return fail(SK_EINVAL, "p5_stats: NULL output");
    p5_counters(h, stats8);
    return SK_OK;
}

sk_status p5_coordinator(sketch_t h, double* fhat, void* gram, int32_t on_device) {
    sk_status rc = check_handle(h, "p5_coordinator");
    if (rc) return rc;
    if (!h->win || h->cfg.kind != SK_P5) return fail(SK_EUNSUPPORTED, "p5_coordinator: not a P5 sketch");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    return p5_coordinator_impl(h, fhat, gram, on_device);
}

sk_status cod_update(sketch_t h, const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t n, int32_t dtype,
                     int32_t on_device) {
    sk_status rc = check_handle(h, "cod_update");
    if (rc) return rc;
    if (!h->cod) return fail(SK_EUNSUPPORTED, "cod_update: not a COD sketch");
    if (n < 0) return fail(SK_EINVAL, "cod_update: n < 0");
    if (n == 0) return SK_OK;
    if (!X || !Y) return fail(SK_EINVAL, "cod_update: NULL X or Y");
    if (ldx < h->cfg.d || ldy < h->cfg.d_y) return fail(SK_EINVAL, "cod_update: ldx < d or ldy < d_y");
    if (dtype < SK_F64 || dtype > SK_BF16) return fail(SK_EINVAL, "cod_update: bad dtype");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const char* xs = (const char*)X;
    const char* ys = (const char*)Y;
    if (!on_device) {
        const size_t es = (size_t)dtype_size(dtype);
        const size_t nx = es * (size_t)((n - 1) * ldx + h->cfg.d), ny = es * (size_t)((n - 1) * ldy + h->cfg.d_y);
        const size_t ox = (nx + 255) / 256 * 256;
        HIP_TRY(h, h->ensure_stage(ox + ny));
        HIP_TRY(h, hipMemcpyAsync(h->stage, X, nx, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync((char*)h->stage + ox, Y, ny, hipMemcpyHostToDevice, h->stream));
        xs = (const char*)h->stage;
        ys = (const char*)h->stage + ox;
    }
    return cod_update_impl(h, xs, ldx, ys, ldy, n, dtype);
}

sk_status cod_query(sketch_t h, void* A_out, void* B_out, int32_t dtype, int32_t on_device) {
    sk_status rc = check_handle(h, "cod_query");
    if (rc) return rc;
    if (!h->cod) return fail(SK_EUNSUPPORTED, "cod_query: not a COD sketch");
    if (!A_out || !B_out) return fail(SK_EINVAL, "cod_query: NULL output");
    if (dtype != SK_F64 && dtype != SK_F32) return fail(SK_EINVAL, "cod_query: dtype must be F64 or F32");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const double *A = nullptr, *B = nullptr;
    if ((rc = cod_query_impl(h, &A, &B))) return rc;
    const int ell = h->cfg.ell, dx = h->cfg.d, dy = h->cfg.d_y;
    const size_t es = (size_t)dtype_size(dtype);
    const size_t na = es * (size_t)dx * ell, nb = es * (size_t)dy * ell;
    if (on_device) {
        HIP_TRY(h, launch_convert_rows(A, ell, A_out, ell, dx, ell, dtype, h->stream));
        HIP_TRY(h, launch_convert_rows(B, ell, B_out, ell, dy, ell, dtype, h->stream));
    } else {
        const size_t oa = (na + 255) / 256 * 256;
        HIP_TRY(h, h->ensure_stage(oa + nb));
        HIP_TRY(h, launch_convert_rows(A, ell, h->stage, ell, dx, ell, dtype, h->stream));
        HIP_TRY(h, launch_convert_rows(B, ell, (char*)h->stage + oa, ell, dy, ell, dtype, h->stream));
        HIP_TRY(h, hipMemcpyAsync(A_out, h->stage, na, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipMemcpyAsync(B_out, (char*)h->stage + oa, nb, hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_info(h);
}

sk_status cod_product(sketch_t h, void* M_out, int32_t on_device) {
    sk_status rc = check_handle(h, "cod_product");
    if (rc) return rc;
    if (!h->cod) return fail(SK_EUNSUPPORTED, "cod_product: not a COD sketch");
    if (!M_out) return fail(SK_EINVAL, "cod_product: NULL output");
    HIP_TRY(h, hipSetDevice(h->cfg.device));
    const size_t nb = sizeof(double) * (size_t)h->cfg.d * h->cfg.d_y;
    double* dst = (double*)M_out;
    if (!on_device) {
        HIP_TRY(h, h->ensure_stage(nb));
        dst = (double*)h->stage;
    }
    if ((rc = cod_product_impl(h, dst))) return rc;
    if (!on_device) HIP_TRY(h, hipMemcpyAsync(M_out, h->stage, nb, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_info(h);
}

sk_status window_stats(sketch_t h, int32_t level, int64_t* stats6) {
    sk_status rc = check_handle(h, "window_stats");
    if (rc) return rc;
    if (!h->win && !h->cod) return fail(SK_EUNSUPPORTED, "window_stats: not a window sketch");
    if (!stats6) return fail(SK_EINVAL, "window_stats: NULL output");
    if (h->cod) {
        if (level != 0) return fail(SK_EINVAL, "window_stats: COD sketches have one level");
        cod_stats(h, stats6);
        return SK_OK;
    }
    return window_level_stats(h, level, stats6);
}

sk_status sketch_set_memory_budget(int64_t bytes) {
    if (bytes < 0) return fail(SK_EINVAL, "sketch_set_memory_budget: negative");
    g_budget = bytes;
    return SK_OK;
}

int64_t sketch_memory_in_use(void) { return g_in_use.load(); }

// Lock-step rounds: round r holds every sketch's r-th ingest segment, then the
// shrinks those segments triggered, grouped by shrink flavour.  Dense rows
// (rows[i], dtype) or CSR rows (indptr[i], indices[i], values[i]).
static sk_status noalloc_tasks(sketch_t h, const std::vector<Task>& tasks, Task** out);

static sk_status update_batch_impl(const char* what, sketch_t* hs, const void* const* rows,
                                   const int64_t* const* indptr, const int32_t* const* indices,
                                   const float* const* values, const int64_t* n, int32_t count,
                                   int32_t dtype, bool noalloc = false) {
    const bool csr = indptr != nullptr;
    if (count < 0 || (count > 0 && (!hs || !n || (!csr && !rows) || (csr && (!indices || !values)))))
        return fail(SK_EINVAL, std::string(what) + ": bad arguments");
    if (count == 0) return SK_OK;
    if (dtype < SK_F64 || dtype > SK_BF16) return fail(SK_EINVAL, std::string(what) + ": bad dtype");
    sk_status rc;
    for (int i = 0; i < count; ++i) {
        if ((rc = check_handle(hs[i], what))) return rc;
        if (hs[i]->win || hs[i]->cod) return fail(SK_EUNSUPPORTED, std::string(what) + ": window sketch");
        if (hs[i]->stream != hs[0]->stream || hs[i]->cfg.device != hs[0]->cfg.device)
            return fail(SK_EINVAL, std::string(what) + ": sketches must share stream and device");
        if (n[i] < 0) return fail(SK_EINVAL, std::string(what) + ": negative row count");
        if (n[i] > 0 && !csr && !rows[i]) return fail(SK_EINVAL, std::string(what) + ": NULL rows");
        if (n[i] > 0 && csr && (!indptr[i] || !indices[i] || !values[i]))
            return fail(SK_EINVAL, std::string(what) + ": NULL CSR array");
        if (csr && hs[i]->d > 16384) return fail(SK_EUNSUPPORTED, std::string(what) + ": d > 16384");
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return fail(SK_EINVAL, std::string(what) + ": a sketch is listed twice");
    }
    sketch_t h0 = hs[0];
    HIP_TRY(h0, hipSetDevice(h0->cfg.device));
    if (noalloc) {
        // the task list must fit the static scratch: count it before any
        // sketch's state moves (one ingest segment per buffer fill, one
        // shrink per fill that completes the buffer)
        int64_t ntask = 0;
        for (int i = 0; i < count; ++i) {
            const sketch_t h = hs[i];
            const int64_t free0 = h->n2 - h->fill;
            if (n[i] == 0) continue;
            const int64_t per = h->n2 - (h->ell - 1);  // rows per later fill
            const int64_t fills = n[i] <= free0 ? 1 : 1 + (n[i] - free0 + per - 1) / per;
            const int64_t shr = n[i] < free0 ? 0 : 1 + (n[i] - free0) / per;
            ntask += fills + shr;
        }
        if (ntask > SK_NOALLOC_MAX_TASKS)
            return fail(SK_EINVAL, std::string(what) + ": " + std::to_string(ntask) +
                                       " tasks exceed the static scratch (" +
                                       std::to_string(SK_NOALLOC_MAX_TASKS) + ")");
    }
    std::vector<int64_t> cur((size_t)count, 0);
    std::vector<sketch_t> owners;
    std::vector<Task> tasks;
    const int64_t es = dtype_size(dtype);
    bool more = true;
    while (more) {
        more = false;
        std::vector<std::pair<sketch_t, Task>> ing, shr;
        for (int i = 0; i < count; ++i) {
            sketch_t h = hs[i];
            if (cur[i] >= n[i]) continue;
            const int64_t take = std::min<int64_t>(n[i] - cur[i], h->n2 - h->fill);
            Task t{};
            t.s = h->dev;
            t.kind = T_INGEST;
            t.par = h->par;
            t.row0 = (int32_t)h->fill;
            t.nrows = (int32_t)take;
            t.src_dtype = dtype;
            t.src_ld = h->d;
            if (csr) {
                t.indptr = indptr[i] + cur[i];
                t.indices = indices[i];
                t.values = values[i];
            } else {
                t.src = (const char*)rows[i] + cur[i] * h->d * es;
            }
            ing.push_back({h, t});
            h->fill += take;
            h->rows_seen += take;
            cur[i] += take;
            if (h->fill == h->n2) {
                Task s{};
                s.s = h->dev;
                s.kind = h->rnd ? T_SHRINK_RAND : T_SHRINK_EXACT;
                s.par = h->par;
                s.m = h->n2;
                s.shrink_idx = h->shrinks;
                mark_coop(s, h);
                shr.push_back({h, s});
                h->par ^= 1;
                h->fill = h->ell - 1;
                h->shrinks += 1;
            }
            if (cur[i] < n[i]) more = true;
        }
        for (auto& p : ing) {
            owners.push_back(p.first);
            tasks.push_back(p.second);
        }
        // group shrinks so that one launch sequence serves one flavour
        std::stable_sort(shr.begin(), shr.end(), [](const std::pair<sketch_t, Task>& a,
                                                     const std::pair<sketch_t, Task>& b) {
            auto key = [](const std::pair<sketch_t, Task>& p) {
                return ((int64_t)p.second.kind << 32) | ((int64_t)p.first->q << 16) |
                       ((int64_t)p.first->st << 8) | (int64_t)p.first->pj;
            };
            return key(a) < key(b);
        });
        for (auto& p : shr) {
            owners.push_back(p.first);
            tasks.push_back(p.second);
        }
    }
    if (!noalloc) return execute_batched(h0, owners, tasks, csr ? DT_F32 : dtype, csr);
    Task* dt = nullptr;
    if ((rc = noalloc_tasks(h0, tasks, &dt))) return rc;
    return execute_batched(h0, owners, tasks, dtype, false, dt);
}

sk_status sketch_update_batch(sketch_t* hs, const void* const* rows, const int64_t* n, int32_t count,
                              int32_t dtype) {
    return update_batch_impl("sketch_update_batch", hs, rows, nullptr, nullptr, nullptr, n, count, dtype);
}

sk_status sketch_update_batch_noalloc(sketch_t* hs, const void* const* rows, const int64_t* n, int32_t count,
                                      int32_t dtype) {
    return update_batch_impl("sketch_update_batch_noalloc", hs, rows, nullptr, nullptr, nullptr, n, count, dtype,
                             true);
}

sk_status sketch_update_csr_batch(sketch_t* hs, const int64_t* const* indptr, const int32_t* const* indices,
                                  const float* const* values, const int64_t* n, int32_t count) {
    if (!indptr) return fail(SK_EINVAL, "sketch_update_csr_batch: NULL indptr list");
    return update_batch_impl("sketch_update_csr_batch", hs, nullptr, indptr, indices, values, n, count,
                             SK_F32);
}

}  // extern "C"

sk_status sketch_destroy_idle(sketch_t h) {
    if (h) destroy_impl(h, false);
    return SK_OK;
}

// Batched execution: like execute(), but a group also breaks where the shrink
// flavour (q, dtypes) changes.
sk_status execute_batched(sketch_t h, std::vector<sketch_t>& owners, std::vector<Task>& tasks,
                          int in_dtype, bool csr, Task* uploaded) {
    if (tasks.empty()) return SK_OK;
    Task* dt = uploaded;
    if (!dt) HIP_TRY(h, h->arena.upload(tasks, h->stream, &dt));
    size_t i = 0;
    while (i < tasks.size()) {
        size_t j = i + 1;
        while (j < tasks.size() && tasks[j].kind == tasks[i].kind && owners[j]->q == owners[i]->q &&
               owners[j]->st == owners[i]->st && owners[j]->pj == owners[i]->pj &&
               tasks[j].kind != T_QUERY)
            ++j;
        Group g = describe(owners, tasks, i, j - i);
        g.prof = &h->prof;
        if (tasks[i].kind == T_INGEST) {
            int max_rows = 0;
            for (size_t u = i; u < j; ++u) max_rows = std::max(max_rows, tasks[u].nrows);
            StageScope sc(g.prof, ST_INGEST, h->stream);
            if (csr) HIP_TRY(h, launch_ingest_csr(dt + i, g.count, max_rows, g.max_d, g.st, h->stream));
            else HIP_TRY(h, launch_ingest(dt + i, g.count, max_rows, g.max_d, in_dtype, g.st, h->stream));
        } else {
            HIP_TRY(h, run_shrinks(dt + i, g, tasks[i].kind, h->stream));
        }
        i = j;
    }
    if (!uploaded) HIP_TRY(h, h->arena.done(h->stream));
    return SK_OK;
}

// ------------------------------------------------- allocation-free variant
// Task list of sketch_update_batch_noalloc: a static device array (each GPU
// holds its own copy for the life of the process).  In host code `scratch`
// names a host-side stand-in, never the device memory: its device address is
// taken once per device with hipGetSymbolAddress and only that address is
// used.  Calls that overlap on one GPU share the array and race.
static __device__ __align__(256) Task scratch[SK_NOALLOC_MAX_TASKS];

static std::mutex g_scratch_mu;
static Task* g_scratch_ptr[64] = {};

static sk_status noalloc_tasks(sketch_t h, const std::vector<Task>& tasks, Task** out) {
    const int dev = h->cfg.device;
    if (dev < 0 || dev >= 64) return fail(SK_EINVAL, "sketch_update_batch_noalloc: device ordinal >= 64");
    Task* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // the device is current (set by the caller of this function)
            hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(SK_EDEVICE, std::string("sketch_update_batch_noalloc: hipGetSymbolAddress: ") +
                                            hipGetErrorString(e));
            g_scratch_ptr[dev] = ptr;
        }
        ptr = g_scratch_ptr[dev];
    }
    if (tasks.empty()) {
        *out = ptr;
        return SK_OK;
    }
    // stream-ordered behind earlier work that read the array; the host copy
    // is pageable memory, which HIP stages before the call returns
    HIP_TRY(h, hipMemcpyAsync(ptr, tasks.data(), sizeof(Task) * tasks.size(), hipMemcpyHostToDevice, h->stream));
    *out = ptr;
    return SK_OK;
}

// ------------------------------------------------------------ merge tree
// Level by level, children (2i, 2i+1) are stacked into a node buffer and
// shrunk; all node shrinks of one level are one task group.
extern "C" sk_status sketch_merge_tree(sketch_t dst, const sketch_t* srcs, int32_t n_src) {
    sk_status rc = check_handle(dst, "sketch_merge_tree");
    if (rc) return rc;
    if (n_src < 1 || !srcs) return fail(SK_EINVAL, "sketch_merge_tree: need at least one source");
    if (dst->win || dst->cod) return fail(SK_EUNSUPPORTED, "sketch_merge_tree: window sketch");
    if (dst->fill != 0 || dst->rows_seen != 0) return fail(SK_ESTATE, "sketch_merge_tree: dst must be empty");
    for (int i = 0; i < n_src; ++i) {
        if ((rc = check_handle(srcs[i], "sketch_merge_tree"))) return rc;
        if (srcs[i]->d != dst->d || srcs[i]->ell != dst->ell)
            return fail(SK_ESHAPE, "sketch_merge_tree: d and ell must match");
        if (srcs[i]->win || srcs[i]->cod) return fail(SK_EUNSUPPORTED, "sketch_merge_tree: window source");
    }
    HIP_TRY(dst, hipSetDevice(dst->cfg.device));
    // leaves: each source's queried sketch
    std::vector<sketch_t> level;
    std::vector<int64_t> rows_of;
    for (int i = 0; i < n_src; ++i) {
        if ((rc = query_to_qout(srcs[i]))) return rc;
        HIP_TRY(srcs[i], hipStreamSynchronize(srcs[i]->stream));
        if ((rc = check_info(srcs[i]))) return rc;
    }
    // node sketches: same configuration as dst on dst's stream
    sketch_config ncfg = dst->cfg;
    ncfg.hip_stream = dst->stream;
    std::vector<sketch_t> temps;
    auto cleanup = [&]() {
        for (sketch_t t : temps) sketch_destroy(t);
    };
    // current level: pointers to FP64 row blocks (ld = dst->ld) and counts
    std::vector<const double*> cur_rows;
    std::vector<int64_t> cur_n;
    for (int i = 0; i < n_src; ++i) {
        cur_rows.push_back(srcs[i]->host.slot[S_QOUT]);
        cur_n.push_back(srcs[i]->fill >= srcs[i]->ell ? srcs[i]->ell - 1 : srcs[i]->fill);
    }
    int depth = 0;
    while (cur_rows.size() > 1) {
        std::vector<sketch_t> owners;
        std::vector<Task> tasks;
        std::vector<const double*> nxt_rows;
        std::vector<int64_t> nxt_n;
        std::vector<sketch_t> nodes;
        for (size_t i = 0; i + 1 < cur_rows.size(); i += 2) {
            sketch_t node = nullptr;
            ncfg.stream_id = dst->cfg.stream_id * 1315423911ull + (uint64_t)(depth * 65536 + (int)i / 2 + 1);
            if ((rc = sketch_create(&ncfg, &node))) {
                cleanup();
                return rc;
            }
            temps.push_back(node);
            nodes.push_back(node);
            // stack both children into the node buffer, then shrink the stack
            for (int c = 0; c < 2; ++c) {
                const int64_t nr = cur_n[i + c];
                if (nr == 0) continue;
                Task t{};
                t.s = node->dev;
                t.kind = T_INGEST;
                t.par = node->par;
                t.row0 = (int32_t)node->fill;
                t.nrows = (int32_t)nr;
                t.src_dtype = DT_F64;
                t.src_ld = dst->ld;
                t.src = cur_rows[i + c];
                owners.push_back(node);
                tasks.push_back(t);
                node->fill += nr;
                node->rows_seen += nr;
            }
        }
        // ingest tasks first (one group), then one shrink group for all nodes
        std::vector<sketch_t> o2;
        std::vector<Task> t2;
        for (size_t u = 0; u < tasks.size(); ++u) {
            o2.push_back(owners[u]);
            t2.push_back(tasks[u]);
        }
        // split the ingest list so that a node appears once per group
        std::vector<sketch_t> oi;
        std::vector<Task> ti;
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<sketch_t> seen;
            for (size_t u = 0; u < t2.size(); ++u) {
                bool first = std::find(seen.begin(), seen.end(), o2[u]) == seen.end();
                if ((pass == 0) == first) {
                    oi.push_back(o2[u]);
                    ti.push_back(t2[u]);
                }
                seen.push_back(o2[u]);
            }
        }
        for (sketch_t node : nodes) {
            if (node->fill >= node->ell) {
                Task s{};
                s.s = node->dev;
                s.kind = node->rnd ? T_SHRINK_RAND : T_SHRINK_EXACT;
                s.par = node->par;
                s.m = (int32_t)node->fill;
                s.shrink_idx = 0;
                mark_coop(s, node);
                oi.push_back(node);
                ti.push_back(s);
                node->par ^= 1;
                node->fill = node->ell - 1;
                node->shrinks += 1;
            }
        }
        if ((rc = execute_batched(dst, oi, ti, DT_F64))) {
            cleanup();
            return rc;
        }
        // children of the next level: the nodes' buffers (converted to FP64)
        for (sketch_t node : nodes) {
            double* q = node->host.slot[S_QOUT];
            HIP_TRY(dst, launch_rows_to_f64(node->host.buf[node->par], node->ld, node->st, q, node->ld,
                                            (int)node->fill, node->d, dst->stream));
            nxt_rows.push_back(q);
            nxt_n.push_back(node->fill);
        }
        if (cur_rows.size() % 2 == 1) {
            nxt_rows.push_back(cur_rows.back());
            nxt_n.push_back(cur_n.back());
        }
        cur_rows.swap(nxt_rows);
        cur_n.swap(nxt_n);
        ++depth;
    }
    // dst takes the root's rows
    std::vector<sketch_t> owners;
    std::vector<Task> tasks;
    plan_rows(dst, cur_n[0], (const char*)cur_rows[0], dst->ld, DT_F64, nullptr, nullptr, nullptr,
              owners, tasks);
    rc = execute(dst, owners, tasks, DT_F64, false);
    if (rc == SK_OK) {
        hipError_t e = hipStreamSynchronize(dst->stream);
        if (e != hipSuccess) rc = dst->device_fail(std::string("merge_tree sync: ") + hipGetErrorString(e));
    }
    if (rc == SK_OK) {
        for (sketch_t t : temps)
            if ((rc = check_info(t))) break;
    }
    cleanup();
    return rc;
}

// ---------------------------------------------------------------- profiling
extern "C" sk_status sketch_profile_enable(sketch_t h, uint32_t stage_mask) {
    sk_status rc = check_handle(h, "sketch_profile_enable");
    if (rc) return rc;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->prof.drain();
    h->prof.mask = stage_mask & SK_STAGE_ALL;
    for (int i = 0; i < NSTAGE; ++i) {
        h->prof.calls[i] = 0;
        h->prof.ms[i] = 0.0;
    }
    if (h->coop) HIP_TRY(h, hipMemset(h->coop + COOP_STATS, 0, 16 * sizeof(double)));
    return SK_OK;
}

extern "C" sk_status sketch_profile_read(sketch_t h, sketch_stage_time* out, int32_t max_entries,
                                         int32_t* n_out) {
    sk_status rc = check_handle(h, "sketch_profile_read");
    if (rc) return rc;
    if (!n_out || (max_entries > 0 && !out)) return fail(SK_EINVAL, "sketch_profile_read: NULL argument");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->prof.drain();
    int n = 0;
    auto put = [&](const char* name, int64_t calls, double v) {
        if (n < max_entries) {
            std::memset(out[n].name, 0, sizeof(out[n].name));
            std::strncpy(out[n].name, name, sizeof(out[n].name) - 1);
            out[n].calls = calls;
            out[n].total_ms = v;
        }
        ++n;
    };
    for (int i = 0; i < NSTAGE; ++i)
        if (h->prof.calls[i] > 0) put(STAGE_NAMES[i], h->prof.calls[i], h->prof.ms[i]);
    if (h->coop) {
        double st[16];
        HIP_TRY(h, hipMemcpy(st, h->coop + COOP_STATS, sizeof(st), hipMemcpyDeviceToHost));
        if (st[6] > 0) {
            int dev = 0, khz = 0;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
            const double tick_ms = khz > 0 ? 1.0 / khz : 0.0;
            put("eig_solves", 0, st[6]);
            put("eig_sweeps", 0, st[0]);
            put("eig_steps", 0, st[1]);
            put("eig_phaseA_ms", 0, st[2] * tick_ms);
            put("eig_syncA_ms", 0, st[3] * tick_ms);
            put("eig_phaseB_ms", 0, st[4] * tick_ms);
            put("eig_syncB_ms", 0, st[5] * tick_ms);
            put("eig_workgroups", 0, st[7]);
        }
    }
    if (!h->win) {  // eigen-solves that went from the tridiagonal solver to the Jacobi method
        int32_t inf[4] = {0, 0, 0, 0};
        HIP_TRY(h, hipMemcpy(inf, h->host.info, sizeof(inf), hipMemcpyDeviceToHost));
        put("eig_fallbacks", 0, (double)inf[2]);
    }
    *n_out = n;
    return SK_OK;
}
