// sk_internal.h -- engine internals shared by the persistent-sketch engine
// (sk_api.cpp) and the sliding-window engine (sk_window.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sketch.h"
#include "sk_device.h"
#include "sk_kernels.h"

struct WindowState;
struct CodState;

using namespace sk;

// ------------------------------------------------------------------ errors
extern thread_local std::string g_err;
extern thread_local const char* g_stage;  // last pipeline stage launched
extern std::atomic<int64_t> g_in_use;
extern std::atomic<int64_t> g_budget;

inline sk_status fail(sk_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(h, expr)                                                                    \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) return (h)->device_fail(std::string(#expr) + " [" + g_stage + \
                                                      "]: " + hipGetErrorString(_e));       \
    } while (0)

inline int dtype_size(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2); }
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// --------------------------------------------------------------- task arena
// Pinned host mirror + device array of Task records, used as a ring of NSLOT
// slots; a slot is rewritten only after the event recorded behind the last
// launch that read it has completed, so NSLOT - 1 batched calls can be queued
// on the device while the host plans the next.
struct TaskArena {
    static const int NSLOT = 4;
    Task* host = nullptr;
    Task* dev = nullptr;
    int cap = 0;  // per slot
    int slot = 0;
    hipEvent_t ev[NSLOT] = {};
    bool used[NSLOT] = {};

    hipError_t reserve(int n, hipStream_t st) {
        if (n <= cap) return hipSuccess;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        release();
        int c = std::max(n, 256);
        e = hipHostMalloc((void**)&host, sizeof(Task) * NSLOT * (size_t)c, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        e = hipMalloc((void**)&dev, sizeof(Task) * NSLOT * (size_t)c);
        if (e != hipSuccess) return e;
        for (int i = 0; i < NSLOT; ++i) {
            e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
            if (e != hipSuccess) return e;
            used[i] = false;
        }
        cap = c;
        return hipSuccess;
    }
    // Copies tasks to the next slot; returns its device pointer.
    hipError_t upload(const std::vector<Task>& tasks, hipStream_t st, Task** out) {
        hipError_t e = reserve((int)tasks.size(), st);
        if (e != hipSuccess) return e;
        slot = (slot + 1) % NSLOT;
        if (used[slot]) {
            e = hipEventSynchronize(ev[slot]);
            if (e != hipSuccess) return e;
        }
        Task* h = host + (size_t)slot * cap;
        Task* d = dev + (size_t)slot * cap;
        std::memcpy(h, tasks.data(), sizeof(Task) * tasks.size());
        e = hipMemcpyAsync(d, h, sizeof(Task) * tasks.size(), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        *out = d;
        return hipSuccess;
    }
    hipError_t done(hipStream_t st) {
        used[slot] = true;
        return hipEventRecord(ev[slot], st);
    }
    void release() {
        if (host) (void)hipHostFree(host);
        if (dev) (void)hipFree(dev);
        for (int i = 0; i < NSLOT; ++i) {
            if (ev[i]) (void)hipEventDestroy(ev[i]);
            ev[i] = nullptr;
        }
        host = nullptr;
        dev = nullptr;
        cap = 0;
    }
};

// ---------------------------------------------------------------- profiling
static const int NSTAGE = 11;
static const char* const STAGE_NAMES[NSTAGE] = {"ingest", "omega", "gram", "project", "cholqr",
                                                "core_gemm", "eig", "threshold", "rebuild", "eig_back",
                                                "eig_reduce"};
enum { ST_INGEST, ST_OMEGA, ST_GRAM, ST_PROJECT, ST_CHOLQR, ST_CORE, ST_EIG, ST_THRESH, ST_REBUILD, ST_EIG_BACK,
       ST_EIG_REDUCE };

struct Prof {
    uint32_t mask = 0;
    struct Ev { int stage; hipEvent_t a, b; };
    std::vector<Ev> pending;
    std::vector<hipEvent_t> pool;
    int64_t calls[NSTAGE] = {};
    double ms[NSTAGE] = {};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    void drain() {
        for (Ev& e : pending) {
            float t = 0.f;
            if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
                calls[e.stage] += 1;
                ms[e.stage] += t;
            }
            pool.push_back(e.a);
            pool.push_back(e.b);
        }
        pending.clear();
    }
    void release() {
        drain();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

// Records an event pair around the launches in its scope when the stage is
// enabled.
struct StageScope {
    Prof* p;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr;
    StageScope(Prof* p_, int stage_, hipStream_t st_) : p(p_), stage(stage_), st(st_) {
        if (p && (p->mask & (1u << stage))) {
            a = p->get();
            (void)hipEventRecord(a, st);
        }
    }
    ~StageScope() {
        if (a) {
            hipEvent_t b = p->get();
            (void)hipEventRecord(b, st);
            p->pending.push_back({stage, a, b});
            if (p->pending.size() > 4096) p->drain();
        }
    }
};

// ------------------------------------------------------------------ sketch
struct sketch_s {
    sketch_config cfg{};
    int d = 0, ell = 0, n2 = 0, k = 0, q = 0;
    bool rnd = false;
    int st = DT_F64, pj = DT_F64;
    int64_t ld = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    SkDev host{};
    SkDev* dev = nullptr;
    std::vector<void*> allocs;
    int64_t bytes = 0;
    int par = 0;
    int64_t fill = 0, shrinks = 0, rows_seen = 0;
    bool sticky = false;
    std::string sticky_msg;
    void* stage = nullptr;  // device staging of host inputs / outputs
    size_t stage_bytes = 0;
    int64_t* csr_stage_ptr = nullptr;
    TaskArena arena;
    WindowState* win = nullptr;
    CodState* cod = nullptr;  // SK_COD sketches (sk_cod.cpp)
    bool counted = false;
    bool dry = false;         // size computation only: dalloc counts, allocates nothing
    double* coop = nullptr;   // cooperative-kernel scratch (see coop_* offsets)
    int* coop_ctrl = nullptr;
    Prof prof;

    sk_status device_fail(const std::string& msg) {
        sticky = true;
        sticky_msg = msg;
        return fail(SK_EDEVICE, msg);
    }
    hipError_t dalloc(void** p, size_t n) {
        if (n == 0) n = 8;
        if (dry) {
            *p = nullptr;
            bytes += (int64_t)n;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(p, n);
        if (e == hipSuccess) {
            allocs.push_back(*p);
            bytes += (int64_t)n;
        }
        return e;
    }
    hipError_t dzero(void* p, size_t n) { return dry ? hipSuccess : hipMemset(p, 0, n); }
    // A grown allocation takes the place of `old` (which is freed); the
    // sketch's byte count grows by `extra`.
    void replace_alloc(void* old, void* now, size_t extra) {
        for (void*& p : allocs)
            if (p == old) {
                (void)hipFree(old);
                p = now;
            }
        bytes += (int64_t)extra;
        if (counted) g_in_use += (int64_t)extra;
    }
    hipError_t ensure_stage(size_t n) {
        if (n <= stage_bytes) return hipSuccess;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (stage) (void)hipFree(stage);
        stage = nullptr;
        stage_bytes = 0;
        e = hipMalloc(&stage, n);
        if (e == hipSuccess) stage_bytes = n;
        return e;
    }
};


// Planning and execution helpers of sk_api.cpp.
void plan_rows(sketch_t h, int64_t n, const char* src, int64_t src_ld, int in_dtype,
               const int64_t* indptr, const int32_t* idx, const float* val,
               std::vector<sketch_t>& owners, std::vector<Task>& tasks);
// uploaded != nullptr: the task list is already on the device there (the
// allocation-free entry point); otherwise it goes through the task arena
sk_status execute_batched(sketch_t h, std::vector<sketch_t>& owners, std::vector<Task>& tasks,
                          int in_dtype, bool csr = false, Task* uploaded = nullptr);
sk_status check_handle(sketch_t h, const char* what);
bool eig_solver_jacobi();
// Device bytes sketch_create would allocate for cfg (persistent sketches);
// negative on a configuration sketch_create rejects.
int64_t sketch_state_bytes(const sketch_config* cfg);
// Returns an idle persistent sketch (no work in flight on its stream) to its
// empty state with a new seed and stream id, without reallocating.
sk_status sketch_reset(sketch_t h, uint64_t seed, uint64_t stream_id);
// sketch_destroy without the stream synchronisation, for a sketch whose work
// the caller knows to have completed.
sk_status sketch_destroy_idle(sketch_t h);
