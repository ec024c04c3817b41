// sk_window.cpp -- sliding-window sketches: Algorithm "ML-AeroSketch" on the
// GPU, behind the same C ABI.
//
// Levels j = 0 .. L-1 (L = max(1, ceil(log2 R))), threshold theta_j =
// 2^j eps N with eps = 2 / ell.  Each level keeps
//   - an FD buffer C (2 ell x d, FP64): a persistent sketch whose shrink is the
//     window's shrink (exact SVD or simul_iter), so FD reduces of all levels
//     run through the batched shrink pipeline;
//   - a queue of snapshots (Z, Z^T C'^T C') and raw rows, metadata on the
//     host, vectors in device rings.
//
// The host can plan everything that depends on row norms alone: for an
// update call it reads |a|^2 of all rows once (one transfer), then knows for
// each level which rows are stored raw and when the FD buffer fills (a dump
// never changes the number of buffer rows).  What depends on the data is
// decided per row from one small transfer: the power-iteration estimate of
// every level (one launch for all levels), and, rarely, the doubling
// simul_iter and the dump of a level.
//
// Readings shared with the FP64 oracle: simul_iter's test matrix is on the d
// side; the dump at k = min(ell, d, rows) happens even if every estimate
// reaches theta; s of an entry is the previous entry's t + 1; a level is
// valid for a query when no in-window entry was dropped by the length cap;
// random counters: power-iteration start (t, 0, i, 0x100 + j), simul_iter
// (t, c / 4, i, 0x200 + 32 j + s), FD reduce of level j keyed (seed,
// 64 stream + j + 1).
#include <algorithm>
#include <cmath>
#include <deque>
#include <functional>

#include "sk_internal.h"
#include "sk_window.h"

namespace {

struct WinEntry {
    int kind;        // 0 snapshot, 1 raw row
    int xi;          // directions of a snapshot
    int64_t s, t;
    int64_t slot;    // first ring slot
};

struct WinLevel {
    sketch_t sub = nullptr;
    double theta = 0.0;
    std::deque<WinEntry> q;
    int64_t last_t = 0, dropped_t = 0;
    double* Zp = nullptr;  // direction ring: z vectors (pcap x ld)
    double* Wp = nullptr;  // rows of Z^T C'^T C' (pcap x ld)
    int64_t pcap = 0, ptail = 0;
    double* Rp = nullptr;  // raw-row ring (rcap x ld)
    int64_t rcap = 0, rtail = 0;
    int64_t ndumps = 0, nraw = 0, ndirs = 0, nsi = 0;
    // Philox stream word and level index of the level's power iteration,
    // simul_iter and amplification draws (a P5 site: its own stream, level 0)
    uint64_t rstream = 0;
    int rlevel = 0;
    // P5 site: row clock and unsent counter F_j
    int64_t clock = 0;
    double F = 0.0;
    // the level's Gram C' C'^T (row-space power iteration): complete for the
    // first g_rows rows of buffer g_C after g_shr shrinks; g_rows < 0 after
    // any other change of the buffer
    int64_t g_rows = -1, g_shr = -1;
    const double* g_C = nullptr;
};

// one row of a P5 update call: its index in the block, the site's timestamp,
// the site's threshold when it arrives, and whether it goes out as it is
struct P5Row {
    int64_t e, i;
    double theta;
    bool raw;
};

}  // namespace

struct WindowState {
    // ATTP (Algorithm "ATTP Sketch using AeroSketch"): one level whose
    // threshold follows the stream (theta_i = eps ||A_i||_F^2), no expiry, no
    // raw rows, snapshots kept for ever in a growing store
    bool attp = false;
    double fro2 = 0.0;
    int L = 0, d = 0, ell = 0, q = 1, kmax = 0, steps = 0;
    int64_t N = 0, T = 0, ld = 0;
    uint64_t seed = 0, stream = 0;
    std::vector<WinLevel> lv;
    // per-row and simul_iter scratch
    double* norms = nullptr;
    int64_t norms_cap = 0;
    double* h_norms = nullptr;   // pinned
    double* pi_out = nullptr;
    double* h_pi = nullptr;      // pinned
    double* pg = nullptr;        // L x (2 ell)^2 level Grams
    double* pu = nullptr;        // L x (2 ell + 1): C' x0 and |x0|^2
    int32_t* info = nullptr;     // eigen-solver counters (all simul_iter slots, the query)
    // simul_iter job slots: every stage of a batch of simul_iter calls is one
    // launch over the slots it uses
    int nslots = 0;
    double *sK = nullptr, *sQ = nullptr, *sZ = nullptr;   // nslots x (d x kmax)
    double *sY = nullptr, *sCQ = nullptr, *sCZ = nullptr;  // nslots x (2 ell x kmax)
    double *sW = nullptr, *sX = nullptr, *sM = nullptr, *sU = nullptr, *sw1 = nullptr, *sw2 = nullptr;  // kmax^2
    double* slam = nullptr;      // nslots x kmax estimates
    double* h_slam = nullptr;    // pinned mirror
    double* sR = nullptr;        // nslots x (2 ell x ld): residuals of amplification candidates
    // descriptor arena (device + pinned mirror), reset after every sync.
    // While `defer` is set descriptors are only staged (from dlo on) and the
    // launches that read them wait in `queued` for one upload of the range.
    char* darena = nullptr;
    char* harena = nullptr;
    size_t acap = 0, aoff = 0;
    hipEvent_t done = nullptr;  // recorded at every wait of the engine
    bool defer = false;
    size_t dlo = 0;
    std::vector<std::function<hipError_t()>> queued;
    // query scratch
    double *Bq = nullptr, *Eq = nullptr, *Vq = nullptr, *Uq = nullptr, *lamq = nullptr;
    double *Zs = nullptr, *Ws = nullptr, *S = nullptr, *T2 = nullptr, *Rs = nullptr;
    double *Xq = nullptr, *Xq2 = nullptr;
    int32_t* ent = nullptr;
    int chunk = 0;
    double *ubuf = nullptr, *part = nullptr, *stats = nullptr;
    int32_t* ctrl = nullptr;
    // cooperative power iteration: slab partials and per-level barriers
    double* pi_part = nullptr;
    unsigned* pi_bars = nullptr;
    // split-K partials of the skinny products (long K, few output tiles)
    double* gpart = nullptr;
    int64_t gpart_cap = 0;
    // probability amplification of the dump step (amp_r candidates, amp_s
    // power iterations on each residual; 1, 0: the plain step)
    int amp_r = 1, amp_s = 0;
    double* amp_out = nullptr;   // nslots x amp_s power-iteration estimates
    double* h_amp = nullptr;     // pinned mirror
    // P5 (Algorithm "P5"): the levels are the m sites; the coordinator's
    // Fhat, the value of the last broadcast (every site holds it), the
    // messages since that broadcast and the coordinator's d x d B.  Snapshot
    // messages wait in Zs / Ws (directions as rows, ent = message index) and
    // rows sent as they are in Rs until they are added to B.
    bool p5 = false;
    int m = 0;
    double Fhat = 0.0, Fb = 0.0;
    int64_t nmsg = 0;
    int64_t fmsgs = 0, bcasts = 0, smsgs = 0, sdirs = 0, raws = 0, words = 0;
    double* Bc = nullptr;
    int qD = 0, qmsgs = 0, rawn = 0;
    std::vector<int32_t> qent;
    std::vector<std::vector<P5Row>> p5rows;
};

// power-iteration descriptors per cooperative launch (pi_part holds the slab
// partials of one launch)
static const int kPiBatch = 32;


static const int kWinDmax = 4096;  // largest d of a window sketch

#define W_TRY(expr)                                                                         \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) return h->device_fail(std::string("window: ") + #expr + ": " + \
                                                    hipGetErrorString(_e));                 \
    } while (0)

// Copies descriptors to the device arena (ordered on the stream); returns
// the device address.  While deferring, the copy waits for DeferDesc::flush.
template <typename D>
static hipError_t put_desc(sketch_t h, const std::vector<D>& ds, const D** out) {
    WindowState* w = h->win;
    const size_t nb = sizeof(D) * ds.size();
    const size_t off = (w->aoff + 255) / 256 * 256;
    if (off + nb > w->acap) return hipErrorOutOfMemory;
    std::memcpy(w->harena + off, ds.data(), nb);
    hipError_t e = hipSuccess;
    if (!w->defer) e = hipMemcpyAsync(w->darena + off, w->harena + off, nb, hipMemcpyHostToDevice, h->stream);
    w->aoff = off + nb;
    *out = (const D*)(w->darena + off);
    return e;
}

// A stream operation: issued now, or queued behind the staged descriptors.
static hipError_t w_issue(sketch_t h, std::function<hipError_t()> f) {
    WindowState* w = h->win;
    if (!w->defer) return f();
    w->queued.push_back(std::move(f));
    return hipSuccess;
}

// Scope in which every descriptor is staged in the host arena and every
// stream operation of the window engine's batches goes through w_issue;
// flush() uploads the staged range with one copy and then issues the queued
// operations in their order.  Leaving the scope without flush() drops them.
struct DeferDesc {
    sketch_t h;
    explicit DeferDesc(sketch_t hh) : h(hh) {
        WindowState* w = h->win;
        w->defer = true;
        w->dlo = (w->aoff + 255) / 256 * 256;
        w->queued.clear();
    }
    hipError_t flush() {
        WindowState* w = h->win;
        w->defer = false;
        std::vector<std::function<hipError_t()>> q;
        q.swap(w->queued);
        if (w->aoff > w->dlo) {
            hipError_t e = hipMemcpyAsync(w->darena + w->dlo, w->harena + w->dlo, w->aoff - w->dlo,
                                          hipMemcpyHostToDevice, h->stream);
            if (e != hipSuccess) return e;
        }
        for (auto& f : q) {
            hipError_t e = f();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    ~DeferDesc() {
        h->win->defer = false;
        h->win->queued.clear();
    }
};

// Waits for the stream by polling an event recorded on it (the engine's
// per-row decisions wait on short GPU stages, where a polled wait returns
// sooner than a blocking one), then resets the descriptor arena.
static hipError_t sync_reset(sketch_t h) {
    WindowState* w = h->win;
    hipError_t e = hipEventRecord(w->done, h->stream);
    while (e == hipSuccess) {
        e = hipEventQuery(w->done);
        if (e == hipErrorNotReady) e = hipSuccess;
        else break;
    }
    w->aoff = 0;
    return e;
}

static GemmDesc gd(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
                   int ldc, int M, int N, int K, double alpha = 1.0, double beta = 0.0) {
    GemmDesc g{};
    g.A = A;
    g.B = B;
    g.C = C;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = lda;
    g.ldb = ldb;
    g.ldc = ldc;
    g.ta = ta;
    g.tb = tb;
    g.alpha = alpha;
    g.beta = beta;
    return g;
}

// Algorithm "Power Iteration" for every descriptor, kPiBatch per cooperative
// launch (the launches share one partial buffer, in stream order).
static sk_status launch_pis(sketch_t h, const std::vector<PiDesc>& pis) {
    WindowState* w = h->win;
    for (size_t b = 0; b < pis.size(); b += kPiBatch) {
        const size_t cnt = std::min(pis.size() - b, (size_t)kPiBatch);
        std::vector<PiDesc> part(pis.begin() + (ptrdiff_t)b, pis.begin() + (ptrdiff_t)(b + cnt));
        const PiDesc* dp = nullptr;
        W_TRY(put_desc(h, part, &dp));
        const int d = w->d, mr = 2 * w->ell;
        double* pp = w->pi_part;
        unsigned* bars = w->pi_bars;
        hipStream_t st = h->stream;
        W_TRY(w_issue(h, [=] { return launch_win_pi(dp, (int)cnt, d, mr, pp, bars, st); }));
    }
    return SK_OK;
}

static sk_status gemm1(sketch_t h, const GemmDesc& g0) {
    if (g0.M <= 0 || g0.N <= 0) return SK_OK;
    WindowState* w = h->win;
    GemmDesc g = g0;
    // products with few output tiles and a long K (C' Omega, K^T K, C' Z ...)
    // are cut along K so that enough workgroups take part; the cut depends
    // on the shape alone and the partials are summed in a fixed order
    const int64_t tiles = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64);
    hipError_t e;
    if (tiles < 64 && g.K >= 128) {
        int ns = (int)std::min<int64_t>((g.K + 31) / 32, std::max<int64_t>(2, 256 / tiles));
        const int kc = (int)round_up((g.K + ns - 1) / ns, 16);
        ns = (g.K + kc - 1) / kc;
        if (ns > 1 && (int64_t)ns * g.M * g.N <= w->gpart_cap) {
            g.part = w->gpart;
            g.nsplit = ns;
            g.kchunk = kc;
            e = launch_gemm_split(g, h->stream);
            if (e != hipSuccess) return h->device_fail(std::string("window split gemm: ") + hipGetErrorString(e));
            return SK_OK;
        }
    }
    e = launch_gemm1(g, h->stream);
    if (e != hipSuccess) return h->device_fail(std::string("window gemm: ") + hipGetErrorString(e));
    return SK_OK;
}

// One symmetric eigen-solve (the query's d x d restore when d is small).
static sk_status small_eig(sketch_t h, const SmallDesc& q) {
    hipError_t e = eig_solver_jacobi() ? launch_jacobi1(q, h->stream) : launch_tri_eig1(q, h->stream);
    if (e != hipSuccess) return h->device_fail(std::string("window small solve: ") + hipGetErrorString(e));
    return SK_OK;
}

static const double* level_C(const WinLevel& l) { return (const double*)l.sub->host.buf[l.sub->par]; }

// Split-K factor of a batched product, from its shape alone: products with
// few 64 x 64 output tiles and a long K are cut into chunks of >= 64 so that
// about 128 workgroups work on each (at most 128 x 64 x 64 partials): a batch
// of one or two levels then spreads over half the chip instead of an eighth.
static int batch_splits(const GemmDesc& g) {
    const int tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
    return std::max(1, std::min(g.K / 64, 128 / tiles));
}

// Products of a batch (descriptors with an empty output are dropped; the
// grid covers the largest product, smaller ones exit their surplus
// workgroups): one launch of the unsplit products and of the split-K
// partials together, then one launch of the fixed-order partial sums.
static sk_status gemm_batch(sketch_t h, const std::vector<GemmDesc>& gs0) {
    WindowState* w = h->win;
    std::vector<GemmDesc> gs, fin;
    int mM = 0, mN = 0;
    int64_t used = 0, mMN = 0;
    for (const GemmDesc& g : gs0) {
        if (g.M <= 0 || g.N <= 0) continue;
        int ns = batch_splits(g);
        const int64_t need = (int64_t)ns * g.M * g.N;
        if (ns > 1 && used + need > w->gpart_cap) ns = 1;
        if (ns == 1) {
            gs.push_back(g);
            mM = std::max(mM, g.M);
            mN = std::max(mN, g.N);
            continue;
        }
        const int kc = (int)round_up((g.K + ns - 1) / ns, 16);
        ns = (g.K + kc - 1) / kc;
        GemmDesc f = g;
        f.part = w->gpart + used;
        f.nsplit = ns;
        f.kchunk = kc;
        for (int sp = 0; sp < ns; ++sp) {
            const int kb = sp * kc, ke = std::min(g.K, kb + kc);
            GemmDesc p = g;
            p.A = g.ta ? g.A + (int64_t)kb * g.lda : g.A + kb;
            p.B = g.tb ? g.B + kb : g.B + (int64_t)kb * g.ldb;
            p.K = ke - kb;
            p.C = f.part + (int64_t)sp * g.M * g.N;
            p.ldc = g.N;
            p.alpha = 1.0;
            p.beta = 0.0;
            gs.push_back(p);
        }
        mM = std::max(mM, g.M);
        mN = std::max(mN, g.N);
        used += (int64_t)ns * g.M * g.N;
        mMN = std::max(mMN, (int64_t)g.M * g.N);
        fin.push_back(f);
    }
    if (gs.empty()) return SK_OK;
    const GemmDesc* dp = nullptr;
    hipStream_t st = h->stream;
    W_TRY(put_desc(h, gs, &dp));
    const int ng = (int)gs.size();
    W_TRY(w_issue(h, [=] { return launch_gemm_desc(dp, ng, mM, mN, st); }));
    if (!fin.empty()) {
        W_TRY(put_desc(h, fin, &dp));
        const int nf = (int)fin.size();
        W_TRY(w_issue(h, [=] { return launch_gemm_reduce_desc(dp, nf, mMN, st); }));
    }
    return SK_OK;
}

// Algorithm "Power Iteration" of the levels js (descriptors pis, in the
// same order) in the row space of their buffers (GramPiDesc): a level whose
// buffer only gained its last row since its Gram was complete has that row
// and column filled by the pass over C'; after any other change (a reduce,
// a dump, the other buffer of the pair) G = C' C'^T is recomputed first.
// The estimates land in each descriptor's out, as with launch_pis.
static sk_status launch_pis_gram(sketch_t h, const std::vector<int>& js, const std::vector<PiDesc>& pis) {
    WindowState* w = h->win;
    if (js.empty()) return SK_OK;
    const int n2 = 2 * w->ell;
    hipStream_t st = h->stream;
    DeferDesc defer(h);
    std::vector<GemmDesc> full;
    std::vector<GramPiDesc> gs;
    int max_r = 0;
    for (size_t u = 0; u < js.size(); ++u) {
        WinLevel& l = w->lv[(size_t)js[u]];
        const PiDesc& p = pis[u];
        GramPiDesc g{};
        g.C = p.C;
        g.out = p.out;
        g.G = w->pg + (size_t)js[u] * n2 * n2;
        g.u = w->pu + (size_t)js[u] * (n2 + 1);
        g.ldc = p.ldc;
        g.r = p.r;
        g.d = p.d;
        g.steps = p.steps;
        g.ldg = n2;
        g.grow = -1;
        g.seed = p.seed;
        g.stream = p.stream;
        g.c2 = p.c2;
        g.c3 = p.c3;
        const bool same = l.g_rows >= 0 && l.g_C == p.C && l.g_shr == l.sub->shrinks;
        if (p.r > 0 && same && l.g_rows == p.r - 1) {
            g.grow = p.r - 1;
        } else if (p.r > 0 && !(same && l.g_rows == p.r)) {
            full.push_back(gd(p.C, (int)p.ldc, false, p.C, (int)p.ldc, true, g.G, n2, p.r, p.r, p.d));
        }
        l.g_rows = p.r;
        l.g_C = p.C;
        l.g_shr = l.sub->shrinks;
        max_r = std::max(max_r, p.r);
        gs.push_back(g);
    }
    sk_status rc = gemm_batch(h, full);
    if (rc) return rc;
    const GramPiDesc* dp = nullptr;
    W_TRY(put_desc(h, gs, &dp));
    const int cnt = (int)gs.size(), dd = w->d;
    W_TRY(w_issue(h, [=] { return launch_win_pi_gram(dp, cnt, max_r, dd, st); }));
    W_TRY(defer.flush());
    return SK_OK;
}

// One simul_iter call: level j, k columns, Philox counter word 3 = tag, row
// timestamp ts, results in job slot `slot`.
struct SiJob {
    int j, k, slot;
    uint64_t tag;
    int64_t ts;
};

// Slot views: d x kmax (K, Q, Z), 2 ell x kmax (Y, CQ, CZ; the row-space iterates), kmax x kmax
// (W, X, M, U, w1, w2), kmax (estimates).
struct SlotSz {
    size_t z, y, k;
};
static SlotSz slot_sz(const WindowState* w) {
    return SlotSz{(size_t)w->d * w->kmax, (size_t)2 * w->ell * w->kmax, (size_t)w->kmax * w->kmax};
}

// Algorithm "Simultaneous Iteration" on A = C'^T (test matrix on the d side)
// for every job at once, every product on the d side: each stage is one
// batched launch over the jobs.  Leaves Z' = Q U in the slot's Z (d x k), U
// in its U and the k estimates of every slot in h_slam.  The buffer sQ
// (d x kmax per slot) is the second iterate of the CholeskyQR passes.
static sk_status simul_iter_cols(sketch_t h, const std::vector<SiJob>& jobs) {
    WindowState* w = h->win;
    const int n = (int)jobs.size();
    if (n == 0) return SK_OK;
    const int d = w->d, lk = w->kmax;
    const SlotSz z = slot_sz(w);
    hipStream_t st = h->stream;
    DeferDesc defer(h);  // every stage's descriptors go up in one copy
    int maxk = 0, maxslot = 0;
    std::vector<double*> K((size_t)n), Q((size_t)n);
    std::vector<const double*> C((size_t)n);
    std::vector<int> ldc((size_t)n), r((size_t)n);
    std::vector<MatGenDesc> mg((size_t)n);
    for (int b = 0; b < n; ++b) {
        const SiJob& J = jobs[(size_t)b];
        const WinLevel& l = w->lv[(size_t)J.j];
        maxk = std::max(maxk, J.k);
        maxslot = std::max(maxslot, J.slot);
        K[(size_t)b] = w->sK + J.slot * z.z;
        Q[(size_t)b] = w->sQ + J.slot * z.z;
        C[(size_t)b] = level_C(l);
        ldc[(size_t)b] = (int)l.sub->ld;
        r[(size_t)b] = (int)l.sub->fill;
        MatGenDesc& m = mg[(size_t)b];
        m = MatGenDesc{};
        m.M = K[(size_t)b];
        m.rows = d;
        m.cols = J.k;
        m.ld = lk;
        m.seed = w->seed;
        m.stream = l.rstream;
        m.c2 = (uint64_t)J.ts;
        m.c3 = J.tag;
    }
    {
        const MatGenDesc* dp = nullptr;
        W_TRY(put_desc(h, mg, &dp));
        W_TRY(w_issue(h, [=] { return launch_philox_mat(dp, n, d, maxk, st); }));
    }
    auto at = [&](double* base, int b, size_t per) { return base + (size_t)jobs[(size_t)b].slot * per; };
    std::vector<GemmDesc> g;
    std::vector<SmallDesc> sd((size_t)n);
    sk_status rc;
    // CholeskyQR passes on every K (d x k): W = K^T K, X = chol(W)^-1,
    // Q1 = K X^T, then Q1 becomes K
    auto cholqr = [&](int passes) -> sk_status {
        for (int p = 0; p < passes; ++p) {
            g.clear();
            for (int b = 0; b < n; ++b) {
                const int k = jobs[(size_t)b].k;
                g.push_back(gd(K[(size_t)b], lk, true, K[(size_t)b], lk, false, at(w->sW, b, z.k), lk, k, k, d));
            }
            sk_status e = gemm_batch(h, g);
            if (e) return e;
            for (int b = 0; b < n; ++b) {
                SmallDesc& q = sd[(size_t)b];
                q = SmallDesc{};
                q.A = at(w->sW, b, z.k);
                q.lda = lk;
                q.X = at(w->sX, b, z.k);
                q.ldx = lk;
                q.n = jobs[(size_t)b].k;
                q.work = at(w->sw1, b, z.k);
            }
            const SmallDesc* dp = nullptr;
            W_TRY(put_desc(h, sd, &dp));
            W_TRY(w_issue(h, [=] { return launch_cholinv_desc(dp, n, maxk, st); }));
            g.clear();
            for (int b = 0; b < n; ++b) {
                const int k = jobs[(size_t)b].k;
                g.push_back(gd(K[(size_t)b], lk, false, at(w->sX, b, z.k), lk, true, Q[(size_t)b], lk, d, k, k));
            }
            if ((e = gemm_batch(h, g))) return e;
            std::swap(K, Q);
        }
        return SK_OK;
    };
    for (int it = 0; it <= w->q; ++it) {
        if (it > 0 && (rc = cholqr(1))) return rc;
        g.clear();
        for (int b = 0; b < n; ++b)
            g.push_back(gd(C[(size_t)b], ldc[(size_t)b], false, K[(size_t)b], lk, false, at(w->sY, b, z.y), lk,
                           r[(size_t)b], jobs[(size_t)b].k, d));
        if ((rc = gemm_batch(h, g))) return rc;
        g.clear();
        for (int b = 0; b < n; ++b)
            g.push_back(gd(C[(size_t)b], ldc[(size_t)b], true, at(w->sY, b, z.y), lk, false, K[(size_t)b], lk, d,
                           jobs[(size_t)b].k, r[(size_t)b]));
        if ((rc = gemm_batch(h, g))) return rc;
    }
    if ((rc = cholqr(2))) return rc;  // K now holds Q
    g.clear();
    for (int b = 0; b < n; ++b)
        g.push_back(gd(C[(size_t)b], ldc[(size_t)b], false, K[(size_t)b], lk, false, at(w->sCQ, b, z.y), lk,
                       r[(size_t)b], jobs[(size_t)b].k, d));
    if ((rc = gemm_batch(h, g))) return rc;
    g.clear();
    for (int b = 0; b < n; ++b) {
        const int k = jobs[(size_t)b].k;
        g.push_back(gd(at(w->sCQ, b, z.y), lk, true, at(w->sCQ, b, z.y), lk, false, at(w->sM, b, z.k), lk, k, k,
                       r[(size_t)b]));
    }
    if ((rc = gemm_batch(h, g))) return rc;
    for (int b = 0; b < n; ++b) {
        SmallDesc& q = sd[(size_t)b];
        q = SmallDesc{};
        q.A = at(w->sM, b, z.k);
        q.lda = lk;
        q.X = at(w->sU, b, z.k);
        q.ldx = lk;
        q.lam = w->slam + (size_t)jobs[(size_t)b].slot * lk;
        q.n = jobs[(size_t)b].k;
        q.work = at(w->sw1, b, z.k);
        q.work2 = at(w->sw2, b, z.k);
        q.info = w->info;
    }
    {
        const SmallDesc* dp = nullptr;
        W_TRY(put_desc(h, sd, &dp));
        const bool jac = eig_solver_jacobi();
        W_TRY(w_issue(h, [=] {
            return jac ? launch_jacobi_desc(dp, n, maxk, st) : launch_tri_eig_desc(dp, n, maxk, st);
        }));
    }
    g.clear();
    for (int b = 0; b < n; ++b) {
        const int k = jobs[(size_t)b].k;
        g.push_back(gd(K[(size_t)b], lk, false, at(w->sU, b, z.k), lk, false, at(w->sZ, b, z.z), lk, d, k, k));
    }
    if ((rc = gemm_batch(h, g))) return rc;
    W_TRY(defer.flush());
    W_TRY(hipMemcpyAsync(w->h_slam, w->slam, sizeof(double) * (size_t)(maxslot + 1) * lk, hipMemcpyDeviceToHost,
                         h->stream));
    W_TRY(sync_reset(h));
    for (const SiJob& J : jobs) w->lv[(size_t)J.j].nsi += 1;
    return SK_OK;
}

// The same batch of simul_iter calls with the iterate carried in the row
// space of each buffer.  After the first product Y = C' K0 the iterate K (d x k) is carried as
// K = C'^T T with T (r x k) in the row space of the buffer, and every later
// step goes through the level's Gram G = C' C'^T (kept by the power
// iteration of the same row): C' K = G T, K^T K = T^T G T, K X^T = C'^T (T
// X^T).  In exact arithmetic these are the d-side steps; only the first
// product and the final Z = K U = C'^T (T U) read C'.  Leaves Z in the slot's
// Z (d x k), U in its U and the k estimates of every slot in h_slam.
static sk_status simul_iter_rows(sketch_t h, const std::vector<SiJob>& jobs) {
    WindowState* w = h->win;
    const int n = (int)jobs.size();
    if (n == 0) return SK_OK;
    const int d = w->d, lk = w->kmax, n2 = 2 * w->ell;
    const SlotSz z = slot_sz(w);
    hipStream_t st = h->stream;
    DeferDesc defer(h);  // every stage's descriptors go up in one copy
    int maxk = 0, maxslot = 0;
    std::vector<const double*> C((size_t)n);
    std::vector<const double*> G((size_t)n);
    std::vector<double*> T((size_t)n), T2((size_t)n), GT((size_t)n);
    std::vector<int> ldc((size_t)n), r((size_t)n);
    std::vector<MatGenDesc> mg((size_t)n);
    std::vector<GemmDesc> g;
    auto at = [&](double* base, int b, size_t per) { return base + (size_t)jobs[(size_t)b].slot * per; };
    for (int b = 0; b < n; ++b) {
        const SiJob& J = jobs[(size_t)b];
        WinLevel& l = w->lv[(size_t)J.j];
        maxk = std::max(maxk, J.k);
        maxslot = std::max(maxslot, J.slot);
        C[(size_t)b] = level_C(l);
        ldc[(size_t)b] = (int)l.sub->ld;
        r[(size_t)b] = (int)l.sub->fill;
        double* Gl = w->pg + (size_t)J.j * n2 * n2;
        G[(size_t)b] = Gl;
        T[(size_t)b] = at(w->sY, b, z.y);
        T2[(size_t)b] = at(w->sCQ, b, z.y);
        GT[(size_t)b] = at(w->sCZ, b, z.y);
        // the Gram is complete after the power iteration of this row; any
        // level whose buffer changed since (none in the engine's order) gets
        // it recomputed here, once per level
        if (!(l.g_rows == l.sub->fill && l.g_C == level_C(l) && l.g_shr == l.sub->shrinks)) {
            g.push_back(gd(C[(size_t)b], ldc[(size_t)b], false, C[(size_t)b], ldc[(size_t)b], true, Gl, n2,
                           r[(size_t)b], r[(size_t)b], d));
            l.g_rows = l.sub->fill;
            l.g_C = level_C(l);
            l.g_shr = l.sub->shrinks;
        }
        MatGenDesc& m = mg[(size_t)b];
        m = MatGenDesc{};
        m.M = w->sK + J.slot * z.z;
        m.rows = d;
        m.cols = J.k;
        m.ld = lk;
        m.seed = w->seed;
        m.stream = l.rstream;
        m.c2 = (uint64_t)J.ts;
        m.c3 = J.tag;
    }
    sk_status rc;
    if ((rc = gemm_batch(h, g))) return rc;
    {
        const MatGenDesc* dp = nullptr;
        W_TRY(put_desc(h, mg, &dp));
        W_TRY(w_issue(h, [=] { return launch_philox_mat(dp, n, d, maxk, st); }));
    }
    std::vector<SmallDesc> sd((size_t)n);
    auto kk = [&](int b) { return jobs[(size_t)b].k; };
    // T = C' K0 (r x k): K = C'^T T is the first power step
    g.clear();
    for (int b = 0; b < n; ++b)
        g.push_back(gd(C[(size_t)b], ldc[(size_t)b], false, w->sK + jobs[(size_t)b].slot * z.z, lk, false,
                       T[(size_t)b], lk, r[(size_t)b], kk(b), d));
    if ((rc = gemm_batch(h, g))) return rc;
    // GT = G T for every job
    auto gram_times_T = [&]() -> sk_status {
        g.clear();
        for (int b = 0; b < n; ++b)
            g.push_back(gd(G[(size_t)b], n2, false, T[(size_t)b], lk, false, GT[(size_t)b], lk, r[(size_t)b], kk(b),
                           r[(size_t)b]));
        return gemm_batch(h, g);
    };
    // CholeskyQR passes on K = C'^T T: W = T^T G T, X = chol(W)^-1, T <- T X^T
    auto cholqr = [&](int passes) -> sk_status {
        for (int p = 0; p < passes; ++p) {
            sk_status e = gram_times_T();
            if (e) return e;
            g.clear();
            for (int b = 0; b < n; ++b)
                g.push_back(gd(T[(size_t)b], lk, true, GT[(size_t)b], lk, false, at(w->sW, b, z.k), lk, kk(b), kk(b),
                               r[(size_t)b]));
            if ((e = gemm_batch(h, g))) return e;
            for (int b = 0; b < n; ++b) {
                SmallDesc& q = sd[(size_t)b];
                q = SmallDesc{};
                q.A = at(w->sW, b, z.k);
                q.lda = lk;
                q.X = at(w->sX, b, z.k);
                q.ldx = lk;
                q.n = kk(b);
                q.work = at(w->sw1, b, z.k);
            }
            const SmallDesc* dp = nullptr;
            W_TRY(put_desc(h, sd, &dp));
            W_TRY(w_issue(h, [=] { return launch_cholinv_desc(dp, n, maxk, st); }));
            g.clear();
            for (int b = 0; b < n; ++b)
                g.push_back(gd(T[(size_t)b], lk, false, at(w->sX, b, z.k), lk, true, T2[(size_t)b], lk, r[(size_t)b],
                               kk(b), kk(b)));
            if ((e = gemm_batch(h, g))) return e;
            std::swap(T, T2);
        }
        return SK_OK;
    };
    for (int it = 1; it <= w->q; ++it) {
        if ((rc = cholqr(1))) return rc;
        // C' K = G T, and K <- C'^T (G T)
        if ((rc = gram_times_T())) return rc;
        std::swap(T, GT);
    }
    if ((rc = cholqr(2))) return rc;  // K = C'^T T now has orthonormal columns
    // C' Q = G T; M = (C' Q)^T (C' Q)
    if ((rc = gram_times_T())) return rc;
    g.clear();
    for (int b = 0; b < n; ++b)
        g.push_back(gd(GT[(size_t)b], lk, true, GT[(size_t)b], lk, false, at(w->sM, b, z.k), lk, kk(b), kk(b),
                       r[(size_t)b]));
    if ((rc = gemm_batch(h, g))) return rc;
    for (int b = 0; b < n; ++b) {
        SmallDesc& q = sd[(size_t)b];
        q = SmallDesc{};
        q.A = at(w->sM, b, z.k);
        q.lda = lk;
        q.X = at(w->sU, b, z.k);
        q.ldx = lk;
        q.lam = w->slam + (size_t)jobs[(size_t)b].slot * lk;
        q.n = kk(b);
        q.work = at(w->sw1, b, z.k);
        q.work2 = at(w->sw2, b, z.k);
        q.info = w->info;
    }
    {
        const SmallDesc* dp = nullptr;
        W_TRY(put_desc(h, sd, &dp));
        const bool jac = eig_solver_jacobi();
        W_TRY(w_issue(h, [=] {
            return jac ? launch_jacobi_desc(dp, n, maxk, st) : launch_tri_eig_desc(dp, n, maxk, st);
        }));
    }
    // Z = K U = C'^T (T U)
    g.clear();
    for (int b = 0; b < n; ++b)
        g.push_back(gd(T[(size_t)b], lk, false, at(w->sU, b, z.k), lk, false, T2[(size_t)b], lk, r[(size_t)b], kk(b),
                       kk(b)));
    if ((rc = gemm_batch(h, g))) return rc;
    g.clear();
    for (int b = 0; b < n; ++b)
        g.push_back(gd(C[(size_t)b], ldc[(size_t)b], true, T2[(size_t)b], lk, false, at(w->sZ, b, z.z), lk, d, kk(b),
                       r[(size_t)b]));
    if ((rc = gemm_batch(h, g))) return rc;
    W_TRY(defer.flush());
    W_TRY(hipMemcpyAsync(w->h_slam, w->slam, sizeof(double) * (size_t)(maxslot + 1) * lk, hipMemcpyDeviceToHost,
                         h->stream));
    W_TRY(sync_reset(h));
    for (const SiJob& J : jobs) w->lv[(size_t)J.j].nsi += 1;
    return SK_OK;
}

// One batch of simul_iter calls.  The row-space form trades the d-side
// products for r x r ones and one more product per CholeskyQR pass; it is
// taken when d exceeds 8 ell (four times the largest buffer), where it was
// the faster of the two on the P5 shape (d = 2048, ell = 128) and the slower
// on the window shape (d = 1024, ell = 128).
static sk_status simul_iter_batch(sketch_t h, const std::vector<SiJob>& jobs) {
    return h->win->d > 8 * h->win->ell ? simul_iter_rows(h, jobs) : simul_iter_cols(h, jobs);
}

// P5 coordinator (Receive_Update of Algorithm "P5"): adds the waiting
// messages to B -- B += R^T R for the rows sent as they are, and for the
// snapshots (directions as rows of Zs, Ws; ent = message of each direction)
// B += Z^T W + W^T Z - Z^T M Z with M = W Z^T masked to the blocks of one
// message, i.e. Z W + W^T Z^T - Z (W Z) Z^T per message.
static sk_status p5_flush(sketch_t h) {
    WindowState* w = h->win;
    const int d = w->d, li = (int)w->ld;
    sk_status rc;
    if (w->rawn > 0) {
        if ((rc = gemm1(h, gd(w->Rs, li, true, w->Rs, li, false, w->Bc, d, d, d, w->rawn, 1.0, 1.0)))) return rc;
        w->rawn = 0;
    }
    if (w->qD > 0) {
        const int D = w->qD;
        W_TRY(hipMemcpyAsync(w->ent, w->qent.data(), sizeof(int32_t) * (size_t)D, hipMemcpyHostToDevice, h->stream));
        if ((rc = gemm1(h, gd(w->Zs, li, true, w->Ws, li, false, w->Bc, d, d, d, D, 1.0, 1.0)))) return rc;
        if ((rc = gemm1(h, gd(w->Ws, li, true, w->Zs, li, false, w->Bc, d, d, d, D, 1.0, 1.0)))) return rc;
        if ((rc = gemm1(h, gd(w->Ws, li, false, w->Zs, li, true, w->S, w->chunk, D, D, d)))) return rc;
        W_TRY(launch_blockmask(w->S, w->chunk, D, w->ent, h->stream));
        if ((rc = gemm1(h, gd(w->Zs, li, true, w->S, w->chunk, false, w->T2, w->chunk, d, D, D)))) return rc;
        if ((rc = gemm1(h, gd(w->T2, w->chunk, false, w->Zs, li, false, w->Bc, d, d, d, D, -1.0, 1.0)))) return rc;
        W_TRY(sync_reset(h));  // the host entry list is reused
        w->qD = 0;
        w->qmsgs = 0;
        w->qent.clear();
    }
    return SK_OK;
}

// One dump: level j takes the first xi columns of the Z of job slot `slot`.
struct DumpJob {
    int j, slot, xi;
    int64_t ts;
    double *Zdst, *Wdst;  // xi rows each (ld = the sketch's ld)
};

// The products of a list of dumps (one batched launch per product): the
// snapshot W = (C' Z)^T C' and Z^T into their rows, then the residual
// C <- C' - (C' Z) Z^T (the dump of Algorithm "AeroSketch: Update").
static sk_status dump_exec(sketch_t h, const std::vector<DumpJob>& ds) {
    if (ds.empty()) return SK_OK;
    WindowState* w = h->win;
    const int d = w->d, lk = w->kmax, li = (int)w->ld;
    const SlotSz z = slot_sz(w);
    std::vector<GemmDesc> g;
    sk_status rc;
    hipStream_t st = h->stream;
    DeferDesc defer(h);
    for (const DumpJob& x : ds) {
        const WinLevel& l = w->lv[(size_t)x.j];
        g.push_back(gd(level_C(l), (int)l.sub->ld, false, w->sZ + x.slot * z.z, lk, false, w->sCZ + x.slot * z.y, lk,
                       (int)l.sub->fill, x.xi, d));
    }
    if ((rc = gemm_batch(h, g))) return rc;
    g.clear();
    for (const DumpJob& x : ds) {
        const WinLevel& l = w->lv[(size_t)x.j];
        g.push_back(gd(w->sCZ + x.slot * z.y, lk, true, level_C(l), (int)l.sub->ld, false, x.Wdst, li, x.xi, d,
                       (int)l.sub->fill));
    }
    if ((rc = gemm_batch(h, g))) return rc;
    for (const DumpJob& x : ds) {
        const double* src = w->sZ + x.slot * z.z;
        const int64_t ld = w->ld;
        W_TRY(w_issue(h, [=] { return launch_transpose(src, lk, x.Zdst, ld, d, x.xi, st); }));
    }
    g.clear();
    for (const DumpJob& x : ds) {
        WinLevel& l = w->lv[(size_t)x.j];
        l.g_rows = -1;  // the residual rewrites the buffer
        g.push_back(gd(w->sCZ + x.slot * z.y, lk, false, w->sZ + x.slot * z.z, lk, true, (double*)level_C(l),
                       (int)l.sub->ld, (int)l.sub->fill, d, x.xi, -1.0, 1.0));
    }
    if ((rc = gemm_batch(h, g))) return rc;
    W_TRY(defer.flush());
    return SK_OK;
}

// Places the snapshots of a list of dumps (level rings, the ATTP store, or
// the P5 coordinator's message queue) and runs their products.
static sk_status dump_batch(sketch_t h, std::vector<DumpJob>& ds) {
    WindowState* w = h->win;
    const int d = w->d;
    std::vector<DumpJob> pend;
    sk_status rc;
    for (DumpJob& x : ds) {
        WinLevel& l = w->lv[(size_t)x.j];
        const int xi = x.xi;
        if (w->p5) {
            if (w->qD + xi > w->chunk) {
                if ((rc = dump_exec(h, pend))) return rc;
                pend.clear();
                if ((rc = p5_flush(h))) return rc;
            }
            const int64_t off = w->qD;
            x.Zdst = w->Zs + off * w->ld;
            x.Wdst = w->Ws + off * w->ld;
            for (int c = 0; c < xi; ++c) w->qent.push_back(w->qmsgs);
            w->qD += xi;
            w->qmsgs += 1;
            w->smsgs += 1;
            w->sdirs += xi;
            w->words += 2 * (int64_t)d * xi;
        } else {
            if (w->attp && l.ptail + xi > l.pcap) {
                // append-only store: double it (the old vectors are copied over)
                if ((rc = dump_exec(h, pend))) return rc;
                pend.clear();
                int64_t ncap = std::max<int64_t>(2 * l.pcap, l.ptail + xi);
                double *nZ = nullptr, *nW = nullptr;
                W_TRY(hipStreamSynchronize(h->stream));
                W_TRY(hipMalloc((void**)&nZ, sizeof(double) * (size_t)ncap * w->ld));
                W_TRY(hipMalloc((void**)&nW, sizeof(double) * (size_t)ncap * w->ld));
                W_TRY(hipMemcpyAsync(nZ, l.Zp, sizeof(double) * (size_t)l.ptail * w->ld, hipMemcpyDeviceToDevice,
                                     h->stream));
                W_TRY(hipMemcpyAsync(nW, l.Wp, sizeof(double) * (size_t)l.ptail * w->ld, hipMemcpyDeviceToDevice,
                                     h->stream));
                W_TRY(hipStreamSynchronize(h->stream));
                h->replace_alloc(l.Zp, nZ, sizeof(double) * (size_t)(ncap - l.pcap) * w->ld);
                h->replace_alloc(l.Wp, nW, sizeof(double) * (size_t)(ncap - l.pcap) * w->ld);
                l.Zp = nZ;
                l.Wp = nW;
                l.pcap = ncap;
            }
            if (l.ptail + xi > l.pcap) l.ptail = 0;
            const int64_t slot = l.ptail;
            for (const WinEntry& e : l.q)
                if (e.kind == 0 && e.slot < slot + xi && slot < e.slot + e.xi)
                    return h->device_fail("window: snapshot ring overflow");
            l.ptail += xi;
            x.Zdst = l.Zp + slot * w->ld;
            x.Wdst = l.Wp + slot * w->ld;
            WinEntry e{};
            e.kind = 0;
            e.xi = xi;
            e.s = l.last_t + 1;
            e.t = x.ts;
            e.slot = slot;
            l.q.push_back(e);
            l.last_t = x.ts;
        }
        l.ndumps += 1;
        l.ndirs += xi;
        pend.push_back(x);
    }
    return dump_exec(h, pend);
}

// A level whose power-iteration estimate reached theta / 2 at row ts.
struct DJob {
    int j;
    int64_t ts;
};

// Per-level state of the doubling loop.
struct DState {
    int j, s, kmax, k, best;
    int64_t ts;
    bool done;
};

// Algorithm "Probability Amplification" in place of the simul_iter calls of
// one doubling step: level u of the batch ran amp_r candidates in slots
// u amp_r + h (candidate h's test matrix from counter word 3 = 0x200 + 32 j
// + s + 0x1000 h; h = 0 is the plain call).  Each candidate keeps xi_h
// directions (the leading estimates that reach theta) and leaves the
// residual R_h = C' - C' Z_h Z_h^T; amp_s power iterations on every R_h
// (start vectors from counter word 3 = 0x100000 + 0x10000 g + 0x1000 h +
// 32 j + s) give c_h = the largest of its estimates, and the candidate with
// the smallest c_h (the first on ties) is kept.  The squared estimates are
// compared; their order is that of c_h.
static sk_status amplify_pick(sketch_t h, std::vector<DState>& st, const std::vector<int>& act) {
    WindowState* w = h->win;
    const int R = w->amp_r, S = w->amp_s, d = w->d, lk = w->kmax;
    const SlotSz z = slot_sz(w);
    const size_t rsz = (size_t)(2 * w->ell) * w->ld;
    if (S == 0) {
        for (int u : act) st[(size_t)u].best = u * R;
        return SK_OK;
    }
    std::vector<GemmDesc> g1, g2;
    std::vector<PiDesc> pis;
    hipStream_t stm = h->stream;
    DeferDesc defer(h);
    for (int u : act) {
        const DState& x = st[(size_t)u];
        const WinLevel& l = w->lv[(size_t)x.j];
        const double* C = level_C(l);
        const int r = (int)l.sub->fill, ldc = (int)l.sub->ld;
        for (int hc = 0; hc < R; ++hc) {
            const int sl = u * R + hc;
            const double* est = w->h_slam + (size_t)sl * lk;
            int xi = 0;
            while (xi < x.k && est[xi] >= l.theta) ++xi;
            double* Rh = w->sR + sl * rsz;
            const size_t pitch = sizeof(double) * (size_t)w->ld;
            W_TRY(w_issue(h, [=] {
                return hipMemcpy2DAsync(Rh, pitch, C, sizeof(double) * (size_t)ldc, sizeof(double) * (size_t)d,
                                        (size_t)r, hipMemcpyDeviceToDevice, stm);
            }));
            if (xi > 0) {
                g1.push_back(gd(C, ldc, false, w->sZ + sl * z.z, lk, false, w->sCZ + sl * z.y, lk, r, xi, d));
                g2.push_back(gd(w->sCZ + sl * z.y, lk, false, w->sZ + sl * z.z, lk, true, Rh, (int)w->ld, r, d, xi,
                                -1.0, 1.0));
            }
            for (int gi = 0; gi < S; ++gi) {
                PiDesc p{};
                p.C = Rh;
                p.out = w->amp_out + (size_t)sl * S + gi;
                p.ldc = w->ld;
                p.r = r;
                p.d = d;
                p.steps = w->steps;
                p.seed = w->seed;
                p.stream = l.rstream;
                p.c2 = (uint64_t)x.ts;
                p.c3 = 0x100000u + 0x10000u * (uint64_t)gi + 0x1000u * (uint64_t)hc + 32u * (uint64_t)l.rlevel +
                       (uint64_t)x.s;
                pis.push_back(p);
            }
        }
    }
    sk_status rc;
    if ((rc = gemm_batch(h, g1))) return rc;
    if ((rc = gemm_batch(h, g2))) return rc;
    if ((rc = launch_pis(h, pis))) return rc;
    W_TRY(defer.flush());
    const int nsl = (act.back() + 1) * R;
    W_TRY(hipMemcpyAsync(w->h_amp, w->amp_out, sizeof(double) * (size_t)nsl * S, hipMemcpyDeviceToHost, h->stream));
    W_TRY(sync_reset(h));
    for (int u : act) {
        double cbest = 0.0;
        int best = u * R;
        for (int hc = 0; hc < R; ++hc) {
            double ch = 0.0;
            for (int gi = 0; gi < S; ++gi) {
                const double e = w->h_amp[(size_t)(u * R + hc) * S + gi];
                if (std::isnan(e))
                    return h->device_fail("window: amplified power iteration failed (barrier timeout or non-finite rows)");
                if (e > ch) ch = e;
            }
            if (hc == 0 || ch < cbest) {
                cbest = ch;
                best = u * R + hc;
            }
        }
        st[(size_t)u].best = best;
    }
    return SK_OK;
}

// Doubling loop of Algorithm "AeroSketch: Update" (k = 2, 4, ...) for many
// levels at once: every doubling step runs the simul_iter calls of all the
// levels still doubling as one batch (amp_r candidates per level when
// amplified), and the dumps of the batch run together at the end.  Each
// level's threshold is its theta.  The levels are independent, so this
// equals running their loops one after the other.
static sk_status doubling_batch(sketch_t h, const std::vector<DJob>& in) {
    WindowState* w = h->win;
    const int R = w->amp_r;
    const bool amplified = R > 1 || w->amp_s > 0;
    const size_t cap = (size_t)std::max(1, w->nslots / R);
    sk_status rc;
    for (size_t c0 = 0; c0 < in.size(); c0 += cap) {
        std::vector<DState> st;
        for (size_t a = c0; a < std::min(in.size(), c0 + cap); ++a) {
            const WinLevel& l = w->lv[(size_t)in[a].j];
            int kmax = std::min(w->ell, w->d);
            if (kmax > l.sub->fill) kmax = (int)l.sub->fill;
            if (kmax < 1) continue;
            st.push_back(DState{in[a].j, 1, kmax, 0, 0, in[a].ts, false});
        }
        std::vector<int> act;
        for (size_t u = 0; u < st.size(); ++u) act.push_back((int)u);
        std::vector<DumpJob> dumps;
        std::vector<SiJob> sj;
        while (!act.empty()) {
            sj.clear();
            for (int u : act) {
                DState& x = st[(size_t)u];
                x.k = std::min(1 << x.s, x.kmax);
                const uint64_t base = 0x200u + 32u * (uint64_t)w->lv[(size_t)x.j].rlevel + (uint64_t)x.s;
                for (int hc = 0; hc < R; ++hc)
                    sj.push_back(SiJob{x.j, x.k, u * R + hc, base + 0x1000u * (uint64_t)hc, x.ts});
            }
            if ((rc = simul_iter_batch(h, sj))) return rc;
            if (amplified) {
                if ((rc = amplify_pick(h, st, act))) return rc;
            } else {
                for (int u : act) st[(size_t)u].best = u;
            }
            std::vector<int> next;
            for (int u : act) {
                DState& x = st[(size_t)u];
                const double theta = w->lv[(size_t)x.j].theta;
                const double* est = w->h_slam + (size_t)x.best * w->kmax;
                if (est[x.k - 1] < theta || x.k == x.kmax) {
                    int xi = 0;
                    while (xi < x.k && est[xi] >= theta) ++xi;
                    if (xi > 0) dumps.push_back(DumpJob{x.j, x.best, xi, x.ts, nullptr, nullptr});
                    x.done = true;
                } else {
                    x.s += 1;
                    next.push_back(u);
                }
            }
            act.swap(next);
        }
        if ((rc = dump_batch(h, dumps))) return rc;
    }
    return SK_OK;
}

static void expire(WindowState* w, WinLevel& l, int64_t i) {
    const size_t cap = 4 * (size_t)w->ell;  // 8 / eps with eps = 2 / ell
    while (!l.q.empty() && (l.q.size() > cap || l.q.front().t <= i - w->N)) {
        const WinEntry& e = l.q.front();
        if (e.t > i - w->N && e.t > l.dropped_t) l.dropped_t = e.t;
        l.q.pop_front();
    }
}

sk_status window_create(sketch_t h) {
    const sketch_config& cfg = h->cfg;
    if (cfg.d > kWinDmax) return fail(SK_EINVAL, "sketch_create: window sketches support d <= 4096");
    WindowState* w = new WindowState();
    h->win = w;
    h->ld = round_up(cfg.d, 64);
    w->d = cfg.d;
    w->ell = cfg.ell;
    w->q = cfg.q;
    w->N = cfg.window_N;
    w->ld = h->ld;
    w->seed = cfg.seed;
    w->stream = cfg.stream_id;
    w->kmax = std::min(cfg.ell, cfg.d);
    w->steps = (int)std::ceil(std::log2((double)cfg.d)) + 1;
    w->attp = cfg.kind == SK_ATTP;
    w->p5 = cfg.kind == SK_P5;
    w->m = w->p5 ? cfg.sites : 0;
    int L = w->p5 ? cfg.sites : w->attp ? 1 : (int)std::ceil(std::log2(cfg.R));
    w->L = L < 1 ? 1 : L;
    if (w->attp || w->p5) w->N = INT64_MAX;
    const double eps = 2.0 / cfg.ell;
    const int d = w->d, ell = w->ell, lk = w->kmax, n2 = 2 * ell;
    w->lv.resize((size_t)w->L);
    for (int j = 0; j < w->L; ++j) {
        WinLevel& l = w->lv[(size_t)j];
        l.theta = (w->attp || w->p5) ? 0.0 : std::ldexp(1.0, j) * eps * (double)w->N;
        // P5 site j draws as an ATTP sketch with stream word 4096 stream + j
        l.rstream = w->p5 ? cfg.stream_id * 4096u + (uint64_t)j : cfg.stream_id;
        l.rlevel = w->p5 ? 0 : j;
        sketch_config sc = cfg;
        sc.kind = SK_PERSISTENT;
        sc.amplify_r = 1;
        sc.amplify_s = 0;
        sc.state_dtype = SK_F64;
        sc.proj_dtype = SK_F64;
        sc.oversample = 0;
        sc.sites = 0;
        sc.stream_id = w->p5 ? l.rstream * 64u + 1u : cfg.stream_id * 64u + (uint64_t)j + 1u;
        sc.hip_stream = h->stream;
        sc.use_given_stream = 1;
        sk_status rc = sketch_create(&sc, &l.sub);
        if (rc) return rc;
        if (w->p5) continue;  // a site's snapshots go to the coordinator
        // ATTP's store starts small and doubles as snapshots accumulate
        l.pcap = w->attp ? 4 * (int64_t)lk : (4 * (int64_t)ell + 4) * lk;
        l.rcap = 4 * (int64_t)ell + 2;
        W_TRY(h->dalloc((void**)&l.Zp, sizeof(double) * (size_t)l.pcap * w->ld));
        W_TRY(h->dalloc((void**)&l.Wp, sizeof(double) * (size_t)l.pcap * w->ld));
        W_TRY(h->dalloc((void**)&l.Rp, sizeof(double) * (size_t)l.rcap * w->ld));
    }
    auto A = [&](double** p, size_t n) { return h->dalloc((void**)p, sizeof(double) * (n ? n : 1)); };
    W_TRY(A(&w->pi_out, (size_t)w->L));
    // simul_iter slots: amp_r per doubling level, up to 64 (at least amp_r)
    w->amp_r = cfg.amplify_r;
    w->amp_s = cfg.amplify_s;
    w->nslots = std::max(w->amp_r, std::min(64, w->L * w->amp_r));
    {
        const size_t ns = (size_t)w->nslots, zs = (size_t)d * lk, ys = (size_t)n2 * lk, ks = (size_t)lk * lk;
        for (double** p : {&w->sK, &w->sZ}) W_TRY(A(p, ns * zs));
        if (d <= 8 * w->ell) W_TRY(A(&w->sQ, ns * zs));  // the d-side form's second iterate
        for (double** p : {&w->sY, &w->sCQ, &w->sCZ}) W_TRY(A(p, ns * ys));
        for (double** p : {&w->sW, &w->sX, &w->sM, &w->sU, &w->sw1, &w->sw2}) W_TRY(A(p, ns * ks));
        W_TRY(A(&w->slam, ns * lk));
        if (w->amp_s > 0) {
            W_TRY(A(&w->sR, ns * (size_t)n2 * w->ld));
            W_TRY(A(&w->amp_out, ns * (size_t)w->amp_s));
            W_TRY(hipHostMalloc((void**)&w->h_amp, sizeof(double) * ns * (size_t)w->amp_s, hipHostMallocDefault));
        }
    }
    W_TRY(h->dalloc((void**)&w->info, 64));
    W_TRY(hipMemset(w->info, 0, 64));
    // query: d x d restore and eigen-solve, snapshot chunks of `chunk` directions
    const int64_t N32 = round_up(d, 32);
    w->chunk = 1024;
    W_TRY(A(&w->Bq, (size_t)d * d));
    W_TRY(A(&w->Eq, (size_t)(N32 * N32)));
    W_TRY(A(&w->Vq, (size_t)(N32 * N32)));
    W_TRY(A(&w->Uq, (size_t)d * d));
    W_TRY(A(&w->lamq, (size_t)d));
    W_TRY(A(&w->Zs, (size_t)w->chunk * w->ld));
    W_TRY(A(&w->Ws, (size_t)w->chunk * w->ld));
    W_TRY(A(&w->S, (size_t)w->chunk * w->chunk));
    W_TRY(A(&w->T2, (size_t)d * w->chunk));
    W_TRY(A(&w->Rs, (size_t)(4 * ell + 2) * w->ld));
    W_TRY(A(&w->Xq, (size_t)ell * w->ld));
    W_TRY(A(&w->Xq2, (size_t)ell * w->ld));
    W_TRY(h->dalloc((void**)&w->ent, sizeof(int32_t) * (size_t)w->chunk));
    W_TRY(A(&w->ubuf, (size_t)(N32 / 32) * 1024));
    W_TRY(A(&w->part, 256));
    W_TRY(A(&w->stats, 16));
    W_TRY(h->dalloc((void**)&w->ctrl, 64 * sizeof(int32_t)));
    W_TRY(A(&w->pi_part, (size_t)kPiBatch * 2 * win_pi_groups(d) * (n2 + 1)));
    W_TRY(A(&w->pg, (size_t)w->L * n2 * n2));
    W_TRY(A(&w->pu, (size_t)w->L * (n2 + 1)));
    W_TRY(h->dalloc((void**)&w->pi_bars, sizeof(unsigned) * 2 * (size_t)kPiBatch));
    // split-K partials: the single products, and up to 128 x 64 x 64 per
    // product of a batch over the slots
    w->gpart_cap = std::max<int64_t>((int64_t)1 << 21, (int64_t)w->nslots * 128 * 64 * 64);
    W_TRY(A(&w->gpart, (size_t)w->gpart_cap));
    w->acap = (size_t)8 << 20;
    W_TRY(h->dalloc((void**)&w->darena, w->acap));
    W_TRY(hipHostMalloc((void**)&w->harena, w->acap, hipHostMallocDefault));
    W_TRY(hipEventCreateWithFlags(&w->done, hipEventDisableTiming));
    W_TRY(hipHostMalloc((void**)&w->h_pi, sizeof(double) * (size_t)w->L, hipHostMallocDefault));
    W_TRY(hipHostMalloc((void**)&w->h_slam, sizeof(double) * (size_t)w->nslots * lk, hipHostMallocDefault));
    if (w->p5) {
        W_TRY(A(&w->Bc, (size_t)d * d));
        W_TRY(hipMemset(w->Bc, 0, sizeof(double) * (size_t)d * d));
        w->p5rows.resize((size_t)w->m);
        w->qent.reserve((size_t)w->chunk);
    }
    return SK_OK;
}

void window_destroy(sketch_t h) {
    WindowState* w = h->win;
    if (!w) return;
    for (WinLevel& l : w->lv)
        if (l.sub) sketch_destroy(l.sub);
    if (w->harena) (void)hipHostFree(w->harena);
    if (w->done) (void)hipEventDestroy(w->done);
    if (w->h_pi) (void)hipHostFree(w->h_pi);
    if (w->h_slam) (void)hipHostFree(w->h_slam);
    if (w->h_amp) (void)hipHostFree(w->h_amp);
    if (w->h_norms) (void)hipHostFree(w->h_norms);
    delete w;
    h->win = nullptr;
}

sk_status window_update(sketch_t h, const char* rows, int64_t n, int64_t ld, int dtype) {
    WindowState* w = h->win;
    const int d = w->d;
    if (n > w->norms_cap) {
        W_TRY(hipStreamSynchronize(h->stream));
        int64_t cap = std::max<int64_t>(n, 4096);
        if (w->h_norms) (void)hipHostFree(w->h_norms);
        w->h_norms = nullptr;
        W_TRY(h->dalloc((void**)&w->norms, sizeof(double) * (size_t)cap));
        W_TRY(hipHostMalloc((void**)&w->h_norms, sizeof(double) * (size_t)cap, hipHostMallocDefault));
        w->norms_cap = cap;
    }
    W_TRY(launch_rownorm(rows, ld, dtype, n, d, w->norms, h->stream));
    W_TRY(hipMemcpyAsync(w->h_norms, w->norms, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, h->stream));
    W_TRY(sync_reset(h));
    const int64_t es = dtype_size(dtype);
    std::vector<sketch_t> owners;
    std::vector<Task> tasks;
    std::vector<PiDesc> pis;
    std::vector<int> pj;
    std::vector<DJob> dj;
    for (int64_t e = 0; e < n; ++e) {
        const int64_t i = w->T + 1;
        w->T = i;
        const char* row = rows + e * ld * es;
        owners.clear();
        tasks.clear();
        pis.clear();
        pj.clear();
        if (w->attp) {
            // theta_i = eps ||A_i||_F^2 before the row's update
            w->fro2 += w->h_norms[e];
            w->lv[0].theta = (2.0 / w->ell) * w->fro2;
        }
        for (int j = 0; j < w->L; ++j) {
            WinLevel& l = w->lv[(size_t)j];
            if (!w->attp) expire(w, l, i);
            if (!w->attp && w->h_norms[e] >= l.theta) {
                const int64_t slot = l.rtail;
                l.rtail = (l.rtail + 1) % l.rcap;
                W_TRY(launch_rows_to_f64(row, ld, dtype, l.Rp + slot * w->ld, w->ld, 1, d, h->stream));
                WinEntry en{};
                en.kind = 1;
                en.s = l.last_t + 1;
                en.t = i;
                en.slot = slot;
                l.q.push_back(en);
                l.last_t = i;
                l.nraw += 1;
            } else {
                plan_rows(l.sub, 1, row, ld, dtype, nullptr, nullptr, nullptr, owners, tasks);
                pj.push_back(j);
            }
        }
        if (!tasks.empty()) {
            sk_status rc = execute_batched(h, owners, tasks, dtype);
            if (rc) return rc;
        }
        if (pj.empty()) continue;
        for (int j : pj) {
            const WinLevel& l = w->lv[(size_t)j];
            PiDesc p{};
            p.C = level_C(l);
            p.out = w->pi_out + j;
            p.ldc = l.sub->ld;
            p.r = (int)l.sub->fill;
            p.d = d;
            p.steps = w->steps;
            p.seed = w->seed;
            p.stream = l.rstream;
            p.c2 = (uint64_t)i;
            p.c3 = 0x100u + (uint64_t)l.rlevel;
            pis.push_back(p);
        }
        if (sk_status prc = launch_pis_gram(h, pj, pis)) return prc;
        W_TRY(hipMemcpyAsync(w->h_pi, w->pi_out, sizeof(double) * (size_t)w->L, hipMemcpyDeviceToHost, h->stream));
        W_TRY(sync_reset(h));
        for (int j : pj)
            if (std::isnan(w->h_pi[j]))
                return h->device_fail("window: power iteration failed (barrier timeout or non-finite rows)");
        dj.clear();
        for (int j : pj)
            if (w->h_pi[j] >= w->lv[(size_t)j].theta / 2.0) dj.push_back(DJob{j, i});
        if (!dj.empty()) {
            sk_status rc = doubling_batch(h, dj);
            if (rc) return rc;
        }
    }
    return SK_OK;
}

sk_status window_advance_impl(sketch_t h, int64_t t_now) {
    WindowState* w = h->win;
    if (t_now < w->T) return fail(SK_EINVAL, "window_advance: time moves backwards");
    w->T = t_now;
    for (WinLevel& l : w->lv)
        while (!l.q.empty() && l.q.front().t <= t_now - w->N) l.q.pop_front();
    return SK_OK;
}

// eigen-decomposition of the d x d matrix Bq into Uq / lamq
static sk_status eig_d(sketch_t h) {
    WindowState* w = h->win;
    const int d = w->d;
    if (d <= jacobi_lds_max()) {
        SmallDesc sd{};
        sd.A = w->Bq;
        sd.lda = d;
        sd.X = w->Uq;
        sd.ldx = d;
        sd.lam = w->lamq;
        sd.n = d;
        sd.work = w->Eq;
        sd.work2 = w->Vq;
        sd.info = w->info;
        return small_eig(h, sd);
    }
    CoopEig a{};
    a.Ain = w->Bq;
    a.ldin = d;
    a.n = d;
    a.A = w->Eq;
    a.V = w->Vq;
    a.U = w->Uq;
    a.lu = d;
    a.lam = w->lamq;
    a.info = w->info;
    a.ubuf = w->ubuf;
    a.part = w->part;
    a.ctrl = w->ctrl;
    a.stats = w->stats;
    a.bar = (uint32_t*)(w->ctrl + 8);
    W_TRY(launch_jacobi_coop(a, h->stream));
    return SK_OK;
}

// The query of Algorithm "AeroSketch: Query" over entries with lb < t <= ub:
// the window (T - N, T] on the valid level, or for ATTP (0, ub] on its one
// level, where the residual's Gram enters only at the current time (past
// residuals are not kept).
static sk_status query_range(sketch_t h, int64_t lb, int64_t ub, const double** out);

static sk_status p5_query(sketch_t h, const double** out);

sk_status window_query(sketch_t h, const double** out) {
    WindowState* w = h->win;
    if (w->p5) return p5_query(h, out);
    if (w->attp) return query_range(h, 0, w->T, out);
    return query_range(h, w->T - w->N, w->T, out);
}

sk_status window_query_at(sketch_t h, int64_t t, const double** out) {
    WindowState* w = h->win;
    if (!w->attp) return fail(SK_EUNSUPPORTED, "sketch_query_at: not an ATTP sketch");
    if (t < 0 || t > w->T) return fail(SK_EINVAL, "sketch_query_at: t outside [0, current time]");
    return query_range(h, 0, t, out);
}

static sk_status query_range(sketch_t h, int64_t lb, int64_t ub, const double** out) {
    WindowState* w = h->win;
    const int d = w->d, ell = w->ell;
    const int64_t T = w->T, ld = w->ld;
    int j = w->L - 1;
    for (int c = 0; c < w->L; ++c)
        if (w->lv[(size_t)c].dropped_t <= lb) {
            j = c;
            break;
        }
    WinLevel& l = w->lv[(size_t)j];
    const double* C = level_C(l);
    const int r = (ub == T) ? (int)l.sub->fill : 0;
    sk_status rc;
    W_TRY(sync_reset(h));
    // B = C^T C + sum over the snapshots in (lb, ub] of Z W + W^T Z^T - Z (W Z) Z^T
    if (r > 0) {
        if ((rc = gemm1(h, gd(C, (int)l.sub->ld, true, C, (int)l.sub->ld, false, w->Bq, d, d, d, r)))) return rc;
    } else {
        W_TRY(hipMemsetAsync(w->Bq, 0, sizeof(double) * (size_t)d * d, h->stream));
    }
    std::vector<const WinEntry*> snaps, raws;
    for (const WinEntry& e : l.q) {
        if (!(lb < e.t && e.t <= ub)) continue;
        (e.kind == 0 ? snaps : raws).push_back(&e);
    }
    size_t si = 0;
    std::vector<int32_t> ent;
    while (si < snaps.size()) {
        int D = 0;
        ent.clear();
        for (; si < snaps.size() && D + snaps[si]->xi <= w->chunk; ++si) {
            const WinEntry& e = *snaps[si];
            W_TRY(hipMemcpyAsync(w->Zs + (int64_t)D * ld, l.Zp + e.slot * ld, sizeof(double) * (size_t)e.xi * ld,
                                 hipMemcpyDeviceToDevice, h->stream));
            W_TRY(hipMemcpyAsync(w->Ws + (int64_t)D * ld, l.Wp + e.slot * ld, sizeof(double) * (size_t)e.xi * ld,
                                 hipMemcpyDeviceToDevice, h->stream));
            for (int c = 0; c < e.xi; ++c) ent.push_back((int32_t)si);
            D += e.xi;
        }
        W_TRY(hipMemcpyAsync(w->ent, ent.data(), sizeof(int32_t) * ent.size(), hipMemcpyHostToDevice, h->stream));
        const int li = (int)ld;
        if ((rc = gemm1(h, gd(w->Zs, li, true, w->Ws, li, false, w->Bq, d, d, d, D, 1.0, 1.0)))) return rc;
        if ((rc = gemm1(h, gd(w->Ws, li, true, w->Zs, li, false, w->Bq, d, d, d, D, 1.0, 1.0)))) return rc;
        if ((rc = gemm1(h, gd(w->Ws, li, false, w->Zs, li, true, w->S, w->chunk, D, D, d)))) return rc;
        W_TRY(launch_blockmask(w->S, w->chunk, D, w->ent, h->stream));
        if ((rc = gemm1(h, gd(w->Zs, li, true, w->S, w->chunk, false, w->T2, w->chunk, d, D, D)))) return rc;
        if ((rc = gemm1(h, gd(w->T2, w->chunk, false, w->Zs, li, false, w->Bq, d, d, d, D, -1.0, 1.0)))) return rc;
        W_TRY(sync_reset(h));  // the host entry list of this chunk is reused
    }
    // eigen-decomposition and the shrink by lambda_ell (the query's final step)
    if ((rc = eig_d(h))) return rc;
    W_TRY(launch_shrink_rows(w->Uq, d, w->lamq, d, ell, w->Xq, ld, d, h->stream));
    if (!raws.empty()) {
        // FD over [B_hat; raw rows]: f_ell of B_hat^T B_hat + R^T R
        int nr = 0;
        for (const WinEntry* e : raws) {
            W_TRY(hipMemcpyAsync(w->Rs + (int64_t)nr * ld, l.Rp + e->slot * ld, sizeof(double) * (size_t)ld,
                                 hipMemcpyDeviceToDevice, h->stream));
            ++nr;
        }
        const int li = (int)ld;
        if ((rc = gemm1(h, gd(w->Xq, li, true, w->Xq, li, false, w->Bq, d, d, d, ell)))) return rc;
        if ((rc = gemm1(h, gd(w->Rs, li, true, w->Rs, li, false, w->Bq, d, d, d, nr, 1.0, 1.0)))) return rc;
        if ((rc = eig_d(h))) return rc;
        W_TRY(launch_shrink_rows(w->Uq, d, w->lamq, d, ell, w->Xq, ld, d, h->stream));
    }
    W_TRY(sync_reset(h));
    for (const WinLevel& lv : w->lv) {
        int32_t inf[2] = {0, 0};
        W_TRY(hipMemcpy(inf, lv.sub->host.info, sizeof(inf), hipMemcpyDeviceToHost));
        if (inf[0] != 0) return h->device_fail("window: FD reduce eigen-solver did not converge");
    }
    *out = w->Xq;
    return SK_OK;
}

const int32_t* window_info_ptr(sketch_t h) { return h->win->info; }
int64_t window_time(sketch_t h) { return h->win->T; }
int32_t window_levels(sketch_t h) { return h->win->L; }

sk_status window_level_stats(sketch_t h, int32_t level, int64_t* st) {
    WindowState* w = h->win;
    if (level < 0 || level >= w->L) return fail(SK_EINVAL, "window_level_stats: bad level");
    const WinLevel& l = w->lv[(size_t)level];
    st[0] = l.ndumps;
    st[1] = l.nraw;
    st[2] = l.ndirs;
    st[3] = l.sub->fill;
    st[4] = (int64_t)l.q.size();
    st[5] = l.sub->shrinks;
    return SK_OK;
}

// ---------------------------------------------------------------- P5
// Algorithm "P5" with m simulated sites on one GPU.  The counter protocol
// depends on the rows' squared norms alone, so one pass on the host over
// the block's norms fixes, for every row, its site's timestamp and the
// site's threshold (eps / m) Fhat_j when the row arrives (every site holds
// the last broadcast value).  Given those thresholds the sites are
// independent, so their rows go through in lockstep: step t takes the t-th
// row of every site in the block -- one batched FD ingest (with the reduces
// that fall due), one launch of all the sites' power iterations, one
// transfer of the estimates -- and the rare doubling steps and dumps run
// site by site.  This yields what processing the rows one at a time does.
sk_status p5_update_impl(sketch_t h, const int32_t* site, const char* rows, int64_t n, int64_t ld, int dtype) {
    WindowState* w = h->win;
    const int d = w->d, m = w->m;
    if (n > w->norms_cap) {
        W_TRY(hipStreamSynchronize(h->stream));
        int64_t cap = std::max<int64_t>(n, 4096);
        if (w->h_norms) (void)hipHostFree(w->h_norms);
        w->h_norms = nullptr;
        W_TRY(h->dalloc((void**)&w->norms, sizeof(double) * (size_t)cap));
        W_TRY(hipHostMalloc((void**)&w->h_norms, sizeof(double) * (size_t)cap, hipHostMallocDefault));
        w->norms_cap = cap;
    }
    W_TRY(launch_rownorm(rows, ld, dtype, n, d, w->norms, h->stream));
    W_TRY(hipMemcpyAsync(w->h_norms, w->norms, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, h->stream));
    W_TRY(sync_reset(h));
    // the counter protocol (Update lines on F_j; the coordinator's
    // Receive_Update on F_j and its broadcast)
    const double eps = 2.0 / w->ell;
    for (auto& v : w->p5rows) v.clear();
    std::vector<int> act;
    for (int64_t e = 0; e < n; ++e) {
        const int j = site[e];
        WinLevel& l = w->lv[(size_t)j];
        const double nrm = w->h_norms[e];
        l.clock += 1;
        l.F += nrm;
        if (l.F >= (eps / m) * w->Fb) {
            w->Fhat += l.F;
            l.F = 0.0;
            w->fmsgs += 1;
            w->words += 1;
            if (++w->nmsg >= m) {
                w->nmsg = 0;
                w->bcasts += 1;
                w->words += m;
                w->Fb = w->Fhat;
            }
        }
        const double theta = (eps / m) * w->Fb;
        if (theta == 0.0 && !(nrm > 0.0)) continue;  // a zero row before the first broadcast sends nothing
        auto& v = w->p5rows[(size_t)j];
        if (v.empty()) act.push_back(j);
        v.push_back(P5Row{e, l.clock, theta, theta == 0.0});
    }
    w->T += n;
    std::sort(act.begin(), act.end());
    const int64_t es = dtype_size(dtype);
    std::vector<sketch_t> owners;
    std::vector<Task> tasks;
    std::vector<PiDesc> pis;
    std::vector<int> pj;
    std::vector<const P5Row*> pr;
    std::vector<DJob> dj;
    sk_status rc;
    for (size_t t = 0; !act.empty(); ++t) {
        owners.clear();
        tasks.clear();
        pis.clear();
        pj.clear();
        pr.clear();
        size_t keep = 0;
        for (size_t a = 0; a < act.size(); ++a) {
            const int j = act[a];
            const auto& v = w->p5rows[(size_t)j];
            if (t >= v.size()) continue;
            act[keep++] = j;
            const P5Row& r = v[t];
            WinLevel& l = w->lv[(size_t)j];
            const char* row = rows + r.e * ld * es;
            if (r.raw) {
                // the row goes to the coordinator as it is
                if (w->rawn == 4 * w->ell + 2 && (rc = p5_flush(h))) return rc;
                W_TRY(launch_rows_to_f64(row, ld, dtype, w->Rs + (int64_t)w->rawn * w->ld, w->ld, 1, d, h->stream));
                w->rawn += 1;
                l.nraw += 1;
                w->raws += 1;
                w->words += d;
                continue;
            }
            plan_rows(l.sub, 1, row, ld, dtype, nullptr, nullptr, nullptr, owners, tasks);
            pj.push_back(j);
            pr.push_back(&r);
        }
        act.resize(keep);
        if (!tasks.empty() && (rc = execute_batched(h, owners, tasks, dtype))) return rc;
        if (pj.empty()) continue;
        for (size_t u = 0; u < pj.size(); ++u) {
            const WinLevel& l = w->lv[(size_t)pj[u]];
            PiDesc p{};
            p.C = level_C(l);
            p.out = w->pi_out + pj[u];
            p.ldc = l.sub->ld;
            p.r = (int)l.sub->fill;
            p.d = d;
            p.steps = w->steps;
            p.seed = w->seed;
            p.stream = l.rstream;
            p.c2 = (uint64_t)pr[u]->i;
            p.c3 = 0x100u + (uint64_t)l.rlevel;
            pis.push_back(p);
        }
        if ((rc = launch_pis_gram(h, pj, pis))) return rc;
        W_TRY(hipMemcpyAsync(w->h_pi, w->pi_out, sizeof(double) * (size_t)w->L, hipMemcpyDeviceToHost, h->stream));
        W_TRY(sync_reset(h));
        for (int j : pj)
            if (std::isnan(w->h_pi[j]))
                return h->device_fail("P5: power iteration failed (barrier timeout or non-finite rows)");
        dj.clear();
        for (size_t u = 0; u < pj.size(); ++u) {
            const int j = pj[u];
            WinLevel& l = w->lv[(size_t)j];
            l.theta = pr[u]->theta;
            if (w->h_pi[j] >= l.theta / 2.0) dj.push_back(DJob{j, pr[u]->i});
        }
        if (!dj.empty() && (rc = doubling_batch(h, dj))) return rc;
    }
    if ((rc = p5_flush(h))) return rc;
    W_TRY(sync_reset(h));
    return SK_OK;
}

void p5_counters(sketch_t h, int64_t* st) {
    const WindowState* w = h->win;
    int64_t red = 0;
    for (const WinLevel& l : w->lv) red += l.sub->shrinks;
    st[0] = w->fmsgs;
    st[1] = w->bcasts;
    st[2] = w->smsgs;
    st[3] = w->sdirs;
    st[4] = w->raws;
    st[5] = w->words;
    st[6] = red;
    st[7] = w->T;
}

static sk_status p5_check_sites(sketch_t h) {
    for (const WinLevel& lv : h->win->lv) {
        int32_t inf[2] = {0, 0};
        W_TRY(hipMemcpy(inf, lv.sub->host.info, sizeof(inf), hipMemcpyDeviceToHost));
        if (inf[0] != 0) return h->device_fail("P5: FD reduce eigen-solver did not converge");
    }
    return SK_OK;
}

sk_status p5_coordinator_impl(sketch_t h, double* fhat, void* gram, int on_device) {
    WindowState* w = h->win;
    sk_status rc;
    if ((rc = p5_flush(h))) return rc;
    if (fhat) *fhat = w->Fhat;
    if (gram) {
        const size_t nb = sizeof(double) * (size_t)w->d * w->d;
        W_TRY(hipMemcpyAsync(gram, w->Bc, nb, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    }
    W_TRY(sync_reset(h));
    return p5_check_sites(h);
}

// The coordinator's Query: B's eigen-decomposition, shrunk by its ell-th
// eigenvalue.
static sk_status p5_query(sketch_t h, const double** out) {
    WindowState* w = h->win;
    const int d = w->d;
    sk_status rc;
    if ((rc = p5_flush(h))) return rc;
    W_TRY(hipMemcpyAsync(w->Bq, w->Bc, sizeof(double) * (size_t)d * d, hipMemcpyDeviceToDevice, h->stream));
    if ((rc = eig_d(h))) return rc;
    W_TRY(launch_shrink_rows(w->Uq, d, w->lamq, d, w->ell, w->Xq, w->ld, d, h->stream));
    W_TRY(sync_reset(h));
    if ((rc = p5_check_sites(h))) return rc;
    *out = w->Xq;
    return SK_OK;
}
