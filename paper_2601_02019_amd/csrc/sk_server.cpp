// sk_server.cpp -- request loop over many resident stream sketches.
//
// Each stream is an ordinary persistent sketch (the AeroSketch update of the
// paper, one per stream); the server adds admission by device memory and
// continuous batching: every tick launches, in one batched update, the next
// rows of every admitted stream with queued bursts, on one HIP stream.  Up to
// max_inflight ticks are on the device while the host plans the next one, so
// bursts that arrive while the GPU works join the next tick.  Ticks complete
// in launch order (one HIP stream), which the completion bookkeeping uses.
#include <chrono>
#include <deque>
#include <map>
#include <tuple>

#include "sk_internal.h"

namespace {

enum { ST_WAITING = 0, ST_ADMITTED = 1, ST_CLOSED = 2 };

struct Burst {
    int64_t ticket = 0;
    const char* rows = nullptr;
    int64_t n = 0, pos = 0;
    int dtype = SK_F32;
    double arrival = 0.0, launched = -1.0;
};

struct SStream {
    sketch_config cfg{};
    sketch_t h = nullptr;
    int state = ST_WAITING;
    bool closing = false;
    int64_t bytes = 0;
    int64_t last_seq = -1;  // last tick that launched rows of this stream
    std::deque<Burst> q;
};

struct Finished {
    int64_t ticket, stream, rows;
    double arrival, launched;
};

struct Tick {
    int64_t seq = 0;
    hipEvent_t ev = nullptr;
    std::vector<Finished> fin;
};

// the shape that decides a sketch's device layout (reuse key)
using ShapeKey = std::tuple<int, int, int, int, int, int, int, int>;
ShapeKey shape_of(const sketch_config& c) {
    return ShapeKey(c.d, c.ell, c.kind, c.shrink, c.state_dtype, c.proj_dtype, c.q, c.oversample);
}

double steady_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct sk_server_s {
    sk_server_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ref = nullptr;  // device time origin, recorded at host time t0
    double t0 = 0.0;
    std::vector<SStream> streams;
    std::deque<int64_t> waiting;
    std::multimap<ShapeKey, sketch_t> idle;  // released sketches kept for reuse
    int64_t idle_bytes = 0;
    std::deque<Tick> inflight;
    std::vector<hipEvent_t> ev_pool;
    std::deque<sk_completion> done;
    int64_t next_ticket = 0, next_seq = 0, completed_seq = -1;
    int64_t bytes = 0;  // admitted + idle sketches
    int64_t n_admitted = 0, n_closed = 0, ticks = 0, batches = 0, rows_done = 0;
    int64_t pending = 0;  // bursts not yet complete, of admitted or waiting streams
    bool failed = false;

    double now() const { return cfg.clock ? cfg.clock(cfg.clock_ctx) : steady_seconds(); }

    sk_status dev_fail(const std::string& m) {
        failed = true;
        return fail(SK_EDEVICE, m);
    }
};

#define SRV_HIP(s, expr)                                                                       \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) return (s)->dev_fail(std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

namespace {

sk_status check_server(sk_server_t s, const char* what) {
    if (!s) return fail(SK_EINVAL, std::string(what) + ": NULL server");
    if (s->failed) return fail(SK_EDEVICE, std::string(what) + ": server is in a failed state");
    return SK_OK;
}

// Completion of tick t: stamps its finished bursts.
sk_status complete(sk_server_t s, Tick& t) {
    double when;
    if (s->cfg.clock) {
        when = s->now();
    } else {
        float ms = 0.f;
        SRV_HIP(s, hipEventElapsedTime(&ms, s->ref, t.ev));
        when = s->t0 + 1e-3 * (double)ms;
    }
    for (const Finished& f : t.fin) {
        s->done.push_back({f.ticket, f.stream, f.rows, f.arrival, f.launched, when});
        s->rows_done += f.rows;
        s->pending -= 1;
    }
    s->completed_seq = t.seq;
    s->ev_pool.push_back(t.ev);
    return SK_OK;
}

// Completes finished ticks; with block, waits until at most keep are left.
sk_status reap(sk_server_t s, bool block, size_t keep) {
    while (!s->inflight.empty()) {
        Tick& t = s->inflight.front();
        if (block && s->inflight.size() > keep) {
            SRV_HIP(s, hipEventSynchronize(t.ev));
        } else {
            hipError_t e = hipEventQuery(t.ev);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return s->dev_fail(std::string("hipEventQuery: ") + hipGetErrorString(e));
        }
        sk_status rc = complete(s, t);
        if (rc) return rc;
        s->inflight.pop_front();
    }
    return SK_OK;
}

// Releases closing streams whose work has completed.
void release_closed(sk_server_t s) {
    for (size_t i = 0; i < s->streams.size(); ++i) {
        SStream& st = s->streams[i];
        if (st.state != ST_ADMITTED || !st.closing || !st.q.empty() || st.last_seq > s->completed_seq)
            continue;
        if (st.h->sticky) {  // a failed sketch is not handed to another stream
            sketch_destroy_idle(st.h);
            s->bytes -= st.bytes;
        } else {
            s->idle.emplace(shape_of(st.cfg), st.h);
            s->idle_bytes += st.bytes;
        }
        st.h = nullptr;
        st.state = ST_CLOSED;
        s->n_admitted -= 1;
        s->n_closed += 1;
    }
}

sk_status admit_one(sk_server_t s, int64_t id, bool* ok) {
    *ok = false;
    SStream& st = s->streams[(size_t)id];
    sketch_config c = st.cfg;
    auto it = s->idle.find(shape_of(c));
    if (it != s->idle.end()) {
        sketch_t h = it->second;
        s->idle.erase(it);
        s->idle_bytes -= st.bytes;
        sk_status rc = sketch_reset(h, c.seed, c.stream_id);
        if (rc) {
            sketch_destroy(h);
            s->bytes -= st.bytes;
            return rc;
        }
        st.h = h;
    } else {
        const int64_t budget = s->cfg.memory_budget;
        // free idle sketches of other shapes while that makes room
        while (budget > 0 && s->bytes + st.bytes > budget && !s->idle.empty()) {
            auto v = s->idle.begin();
            s->bytes -= v->second->bytes;
            s->idle_bytes -= v->second->bytes;
            sketch_destroy_idle(v->second);
            s->idle.erase(v);
        }
        if (budget > 0 && s->bytes + st.bytes > budget) return SK_OK;
        sk_status rc = sketch_create(&c, &st.h);
        if (rc == SK_ENOMEM) return SK_OK;  // the library-wide budget: keep waiting
        if (rc) return rc;
        s->bytes += st.bytes;
    }
    st.state = ST_ADMITTED;
    s->n_admitted += 1;
    *ok = true;
    return SK_OK;
}

// First come, first served: stops at the first stream that does not fit.
sk_status admit_waiting(sk_server_t s) {
    while (!s->waiting.empty()) {
        bool ok = false;
        sk_status rc = admit_one(s, s->waiting.front(), &ok);
        if (rc) return rc;
        if (!ok) break;
        s->waiting.pop_front();
    }
    return SK_OK;
}

}  // namespace

extern "C" {

sk_status server_config_init(sk_server_config* cfg) {
    if (!cfg) return fail(SK_EINVAL, "server_config_init: NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->max_inflight = 2;
    return SK_OK;
}

sk_status server_create(const sk_server_config* cfg, sk_server_t* out) {
    if (!cfg || !out) return fail(SK_EINVAL, "server_create: NULL argument");
    *out = nullptr;
    if (cfg->max_inflight < 1 || cfg->max_inflight > 64)
        return fail(SK_EINVAL, "server_create: max_inflight must be in [1, 64]");
    if (cfg->memory_budget < 0 || cfg->max_rows_per_tick < 0 || cfg->max_shrinks_per_tick < 0)
        return fail(SK_EINVAL, "server_create: negative budget or cap");
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return fail(SK_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    sk_server_t s = new sk_server_s();
    s->cfg = *cfg;
    if (cfg->hip_stream || cfg->use_given_stream) {
        s->stream = (hipStream_t)cfg->hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e == hipSuccess) s->own_stream = true;
    }
    if (e == hipSuccess) e = hipEventCreate(&s->ref);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ref, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->ref);
    if (e != hipSuccess) {
        std::string m = std::string("server_create: ") + hipGetErrorString(e);
        server_destroy(s);
        return fail(SK_EDEVICE, m);
    }
    s->t0 = steady_seconds();
    *out = s;
    return SK_OK;
}

double server_now(sk_server_t s) { return s ? s->now() : 0.0; }

sk_status server_open(sk_server_t s, const sketch_config* cfg, int64_t* id) {
    sk_status rc = check_server(s, "server_open");
    if (rc) return rc;
    if (!cfg || !id) return fail(SK_EINVAL, "server_open: NULL argument");
    if (cfg->kind != SK_PERSISTENT) return fail(SK_EUNSUPPORTED, "server_open: only persistent sketches");
    SStream st;
    st.cfg = *cfg;
    st.cfg.device = s->cfg.device;
    st.cfg.hip_stream = s->stream;
    st.cfg.use_given_stream = 1;
    st.bytes = sketch_state_bytes(&st.cfg);
    if (st.bytes < 0) return fail(SK_EINVAL, "server_open: invalid sketch configuration");
    if (s->cfg.memory_budget > 0 && st.bytes > s->cfg.memory_budget)
        return fail(SK_ENOMEM, "server_open: the stream alone exceeds the memory budget");
    const int64_t sid = (int64_t)s->streams.size();
    s->streams.push_back(st);
    s->waiting.push_back(sid);
    if ((rc = admit_waiting(s))) return rc;
    *id = sid;
    return SK_OK;
}

sk_status server_submit(sk_server_t s, int64_t id, const void* rows, int64_t n, int32_t dtype,
                        double arrival, int64_t* ticket) {
    sk_status rc = check_server(s, "server_submit");
    if (rc) return rc;
    if (id < 0 || id >= (int64_t)s->streams.size()) return fail(SK_EINVAL, "server_submit: bad stream id");
    SStream& st = s->streams[(size_t)id];
    if (st.closing || st.state == ST_CLOSED) return fail(SK_ESTATE, "server_submit: stream is closed");
    if (n < 1 || !rows) return fail(SK_EINVAL, "server_submit: need n >= 1 rows");
    if (dtype < SK_F64 || dtype > SK_BF16) return fail(SK_EINVAL, "server_submit: bad dtype");
    Burst b;
    b.ticket = s->next_ticket++;
    b.rows = (const char*)rows;
    b.n = n;
    b.dtype = dtype;
    b.arrival = arrival;
    st.q.push_back(b);
    s->pending += 1;
    if (ticket) *ticket = b.ticket;
    return SK_OK;
}

sk_status server_tick(sk_server_t s, int32_t* launched) {
    sk_status rc = check_server(s, "server_tick");
    if (rc) return rc;
    if (launched) *launched = 0;
    SRV_HIP(s, hipSetDevice(s->cfg.device));
    if ((rc = reap(s, false, 0))) return rc;
    release_closed(s);
    if ((rc = admit_waiting(s))) return rc;
    // segments: for each admitted stream, up to the row cap from its queue
    struct Seg { int64_t sid; size_t burst; int64_t off, n; };
    std::vector<std::vector<Seg>> rounds;
    const int64_t cap = s->cfg.max_rows_per_tick;
    for (size_t i = 0; i < s->streams.size(); ++i) {
        SStream& st = s->streams[i];
        if (st.state != ST_ADMITTED || st.q.empty()) continue;
        int64_t budget = cap > 0 ? cap : INT64_MAX;
        if (s->cfg.max_shrinks_per_tick > 0) {
            // rows up to the buffer's next shrink plus (cap - 1) more shrinks;
            // sketches with ell < 64 take 64 / ell times as many (cheaper) shrinks
            const int64_t cap_s = (int64_t)s->cfg.max_shrinks_per_tick * std::max(1, 64 / st.cfg.ell);
            const int64_t to_first = 2 * (int64_t)st.cfg.ell - st.h->fill;
            budget = std::min(budget, to_first + (cap_s - 1) * (st.cfg.ell + 1));
        }
        size_t r = 0;
        for (size_t b = 0; b < st.q.size() && budget > 0; ++b, ++r) {
            Burst& bu = st.q[b];
            const int64_t take = std::min(bu.n - bu.pos, budget);
            if (rounds.size() <= r) rounds.emplace_back();
            rounds[r].push_back({(int64_t)i, b, bu.pos, take});
            budget -= take;
        }
    }
    if (rounds.empty()) return SK_OK;
    // bound the work on the device: at most max_inflight ticks after this launch
    if ((rc = reap(s, true, (size_t)s->cfg.max_inflight - 1))) return rc;
    const double tnow = s->now();
    Tick tick;
    tick.seq = s->next_seq++;
    // one batched update per (round, dtype)
    for (auto& segs : rounds) {
        for (int dt = SK_F64; dt <= SK_BF16; ++dt) {
            std::vector<sketch_t> hs;
            std::vector<const void*> ptrs;
            std::vector<int64_t> ns;
            for (const Seg& g : segs) {
                SStream& st = s->streams[(size_t)g.sid];
                Burst& bu = st.q[g.burst];
                if (bu.dtype != dt) continue;
                hs.push_back(st.h);
                ptrs.push_back(bu.rows + (size_t)g.off * (size_t)st.cfg.d * (size_t)dtype_size(dt));
                ns.push_back(g.n);
            }
            if (hs.empty()) continue;
            rc = sketch_update_batch(hs.data(), ptrs.data(), ns.data(), (int32_t)hs.size(), dt);
            if (rc) {
                s->failed = true;
                return rc;
            }
            s->batches += 1;
        }
    }
    // bookkeeping: advance positions; bursts whose last rows went out finish with this tick
    int32_t nl = 0;
    for (auto& segs : rounds) {
        for (const Seg& g : segs) {
            SStream& st = s->streams[(size_t)g.sid];
            Burst& bu = st.q[g.burst];
            if (bu.pos == 0) bu.launched = tnow;
            bu.pos += g.n;
            st.last_seq = tick.seq;
            ++nl;
        }
    }
    for (size_t i = 0; i < s->streams.size(); ++i) {
        SStream& st = s->streams[i];
        while (!st.q.empty() && st.q.front().pos == st.q.front().n) {
            const Burst& bu = st.q.front();
            tick.fin.push_back({bu.ticket, (int64_t)i, bu.n, bu.arrival, bu.launched});
            st.q.pop_front();
        }
    }
    if (s->ev_pool.empty()) {
        hipEvent_t e = nullptr;
        SRV_HIP(s, hipEventCreate(&e));
        s->ev_pool.push_back(e);
    }
    tick.ev = s->ev_pool.back();
    s->ev_pool.pop_back();
    SRV_HIP(s, hipEventRecord(tick.ev, s->stream));
    s->inflight.push_back(std::move(tick));
    s->ticks += 1;
    if (launched) *launched = nl;
    return SK_OK;
}

sk_status server_poll(sk_server_t s, sk_completion* out, int32_t max, int32_t* n) {
    sk_status rc = check_server(s, "server_poll");
    if (rc) return rc;
    if (!n || max < 0 || (max > 0 && !out)) return fail(SK_EINVAL, "server_poll: bad arguments");
    if ((rc = reap(s, false, 0))) return rc;
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return SK_OK;
}

sk_status server_drain(sk_server_t s) {
    sk_status rc = check_server(s, "server_drain");
    if (rc) return rc;
    for (;;) {
        int32_t nl = 0;
        if ((rc = server_tick(s, &nl))) return rc;
        if (nl == 0) {
            if ((rc = reap(s, true, 0))) return rc;
            release_closed(s);
            // closes may have made room for waiting streams
            const size_t w = s->waiting.size();
            if ((rc = admit_waiting(s))) return rc;
            if (s->waiting.size() == w) break;
        }
    }
    return SK_OK;
}

sk_status server_query(sk_server_t s, int64_t id, void* B_out, int32_t dtype, int32_t on_device) {
    sk_status rc = check_server(s, "server_query");
    if (rc) return rc;
    if (id < 0 || id >= (int64_t)s->streams.size()) return fail(SK_EINVAL, "server_query: bad stream id");
    SStream& st = s->streams[(size_t)id];
    if (st.state != ST_ADMITTED) return fail(SK_ESTATE, "server_query: stream is not admitted");
    return sketch_query(st.h, B_out, dtype, on_device);
}

sk_status server_debug_fail_solver(sk_server_t s, int64_t id) {
    sk_status rc = check_server(s, "server_debug_fail_solver");
    if (rc) return rc;
    if (id < 0 || id >= (int64_t)s->streams.size()) return fail(SK_EINVAL, "server_debug_fail_solver: bad stream id");
    SStream& st = s->streams[(size_t)id];
    if (st.state != ST_ADMITTED) return fail(SK_ESTATE, "server_debug_fail_solver: stream is not admitted");
    return sketch_debug_fail_solver(st.h);
}

sk_status server_close(sk_server_t s, int64_t id) {
    sk_status rc = check_server(s, "server_close");
    if (rc) return rc;
    if (id < 0 || id >= (int64_t)s->streams.size()) return fail(SK_EINVAL, "server_close: bad stream id");
    SStream& st = s->streams[(size_t)id];
    if (st.closing || st.state == ST_CLOSED) return fail(SK_ESTATE, "server_close: already closed");
    st.closing = true;
    if (st.state == ST_WAITING) {
        for (auto it = s->waiting.begin(); it != s->waiting.end(); ++it)
            if (*it == id) {
                s->waiting.erase(it);
                break;
            }
        for (const Burst& b : st.q) {
            s->done.push_back({b.ticket, id, b.n, b.arrival, -1.0, -1.0});
            s->pending -= 1;
        }
        st.q.clear();
        st.state = ST_CLOSED;
        s->n_closed += 1;
        return SK_OK;
    }
    release_closed(s);
    return SK_OK;
}

sk_status server_stats(sk_server_t s, sk_server_stats* out) {
    if (!s || !out) return fail(SK_EINVAL, "server_stats: NULL argument");
    out->admitted = s->n_admitted;
    out->waiting = (int64_t)s->waiting.size();
    out->closed = s->n_closed;
    out->bytes_in_use = s->bytes;
    out->ticks = s->ticks;
    out->batches = s->batches;
    out->pending_bursts = s->pending;
    out->inflight = (int64_t)s->inflight.size();
    out->rows_done = s->rows_done;
    return SK_OK;
}

sk_status server_destroy(sk_server_t s) {
    if (!s) return SK_OK;
    (void)hipSetDevice(s->cfg.device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (SStream& st : s->streams)
        if (st.h) sketch_destroy_idle(st.h);
    for (auto& v : s->idle) sketch_destroy_idle(v.second);
    for (Tick& t : s->inflight) s->ev_pool.push_back(t.ev);
    for (hipEvent_t e : s->ev_pool)
        if (e) (void)hipEventDestroy(e);
    if (s->ref) (void)hipEventDestroy(s->ref);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return SK_OK;
}

}  // extern "C"
