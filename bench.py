"""Benchmark of the FD sketch-update hot path on one MI355X.

Workload (default): the tight-error persistent stream -- d = 4096, ell = 256,
n = 200,000 rows in FP32, power-law spectrum s_i = i^-0.8 over rank 1024 plus
N(0, 1e-3) noise, seed 1.  A step is one pass of the hot path over the whole
stream: row ingest, every FD shrink that falls due (randomized: Philox Omega,
bf16 MFMA projection, FP64 Gram / CholeskyQR / Rayleigh-Ritz / Jacobi core,
rebuild) and the final query.  Rows are resident in HBM before timing starts.

Printed (one JSON line): rows/s of the randomized mixed-precision path, the
exact-SVD FD path on the same GPU (timed on a prefix of the stream), their
covariance errors (matched-error check), the dominant kernel's roofline and
the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector (and matrix) peak
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows", type=int, default=200_000)
    ap.add_argument("--d", type=int, default=4096)
    ap.add_argument("--ell", type=int, default=256)
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--exact-rows", type=int, default=0,
                    help="rows on which the exact-SVD FD path is timed and the errors compared (0: all)")
    ap.add_argument("--no-exact", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-err", action="store_true",
                    help="skip the covariance-error evaluation (torch eigvalsh) of the timed sketch")
    ap.add_argument("--cpu-shrinks", type=int, default=1,
                    help="shrinks of the CPU oracle sample")
    ap.add_argument("--workload", choices=["persistent", "small", "window", "sites", "serving", "copy", "attp",
                                           "p5", "cod"],
                    default="persistent",
                    help="persistent: the tight-error single stream (default); small: the FP64 exact "
                         "small stream; window: the sliding-window stream; sites: 64 CSR sites with "
                         "tree merges; serving: many concurrent streams with Poisson bursts; copy: a "
                         "plain device copy of known size (HBM reference and counter calibration); attp: "
                         "the ATTP stream; p5: continuous distributed tracking over the sites' rows; cod: "
                         "approximate matrix multiplication over a sliding window (Uniform Random pairs)")
    ap.add_argument("--window-rows", type=int, default=200_000, help="rows of the window stream")
    ap.add_argument("--site-rows", type=int, default=100_000, help="rows per site")
    ap.add_argument("--attp-rows", type=int, default=10_000, help="rows of the ATTP stream")
    ap.add_argument("--sites", type=int, default=64)
    ap.add_argument("--p5-rows", type=int, default=2000, help="rows per site (on average) of the p5 workload")
    ap.add_argument("--cod-pairs", type=int, default=10_000, help="pairs of the cod stream")
    ap.add_argument("--cod-ell", type=int, default=32, help="ell of the cod workload")
    ap.add_argument("--streams", type=int, default=512)
    ap.add_argument("--bursts", type=int, default=2000, help="bursts per load point")
    ap.add_argument("--loads", default="0.25,0.5,0.75,0.9",
                    help="offered loads as fractions of the measured saturation rate")
    ap.add_argument("--row-cap", type=int, default=4096, help="rows of one stream per serving tick")
    ap.add_argument("--shrink-cap", type=int, default=1,
                    help="shrinks of one stream per serving tick (more for ell < 64)")
    ap.add_argument("--pool-rows", type=int, default=4096, help="resident rows per stream")
    return ap.parse_args()


def make_stream(n, d, rank, seed, device):
    """Rows = (g * s) V^T + noise, generated on the GPU (inputs only)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    G = torch.randn(d, rank, device=device, generator=gen, dtype=torch.float64)
    V, _ = torch.linalg.qr(G)
    V = V.float()
    s = torch.arange(1, rank + 1, device=device, dtype=torch.float32) ** -0.8
    A = torch.empty(n, d, device=device, dtype=torch.float32)
    chunk = 16384
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        g = torch.randn(r1 - r0, rank, device=device, generator=gen) * s
        A[r0:r1] = g @ V.T + math.sqrt(1e-3) * torch.randn(r1 - r0, d, device=device, generator=gen)
    return A


def gram_f64(A, chunk=16384):
    import torch
    d = A.shape[1]
    G = torch.zeros(d, d, device=A.device, dtype=torch.float64)
    for r0 in range(0, A.shape[0], chunk):
        X = A[r0:r0 + chunk].double()
        G += X.T @ X
    return G


def cov_err(AtA, B):
    import torch
    Bd = B.double()
    D = AtA - Bd.T @ Bd
    D = (D + D.T) / 2
    ev = torch.linalg.eigvalsh(D)
    return float(ev.abs().max())


def measured_traffic(kernel, source):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a copy of known size), or None
    when the kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, source), "rb").read()
    except OSError:
        return None
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _site_oracle_job(job):
    """CPU-baseline job: the FP64 oracle over the first m rows of one site."""
    import oracle
    import synth
    site, m, d, ell = job
    ip, ix, vv = synth.streams.sparse_sites(m, d=d, density=0.01, seed=4, site=site)
    Xd = synth.streams.csr_to_dense(ip, ix, vv, d)
    o = oracle.FD(d, ell, "rand", k=ell, q=1, seed=4, stream=site)
    o.update(Xd)
    return m


def _serving_oracle_job(job):
    """CPU-baseline job: the FP64 oracle over two shrinks' worth of rows of
    one serving stream (its own low-rank-plus-noise model)."""
    import numpy as np
    import oracle
    import synth
    i, d, ell = job
    r = min(2 * ell, d)
    m = 2 * ell + ell + 1
    A = synth.lowrank_rows(m, d, 1.0 - np.arange(r) / r, 0.1, seed=1000 + i)
    o = oracle.FD(d, ell, "rand", k=ell, q=1, seed=5, stream=i)
    o.update(A)
    return m


def oracle_pool(fn, jobs, procs):
    """Runs fn over jobs on `procs` processes (fresh interpreters, so the GPU
    state of this process is not shared); returns (seconds, rows)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        t = time.perf_counter()
        rows = sum(pool.map(fn, jobs))
        tc = time.perf_counter() - t
    return tc, rows


def tri_flops(n):
    """Dense arithmetic of the tridiagonal reduction (FP64 flops): a symmetric
    product and a rank-2 update per column, 4 n^3 / 3 in all."""
    return 4.0 * n ** 3 / 3.0


def tri_product_bytes(n):
    """Bytes the blocked reduction reads per launch for its products with the
    panel-start matrix (column j reads the (n - j - 1)^2 trailing block once,
    FP64), about 8 n^3 / 3; the once-per-panel trailing updates add little."""
    return 8.0 * sum((n - j - 1) ** 2 for j in range(n - 1))


def jacobi_flops(n, sweeps):
    """Arithmetic of the block Jacobi solver per solve (FP64 flops): per block
    step, one 31-step rotation sweep of every 32 x 32 pair sub-problem and the
    32 x 32 block rotations of A (two products per sandwich tile, upper tiles)
    and of V."""
    N = (n + 31) // 32 * 32
    nb, npair = N // 16, N // 32
    inner = npair * 31 * (32 * 32 * 6 + 32 * 16 * 6)
    sandwich = (npair * (npair + 1) // 2) * 2 * (2 * 32 ** 3)
    vtiles = (N // 32) * npair * (2 * 32 ** 3)
    return sweeps * (nb - 1) * (inner + sandwich + vtiles)


def serving_streams(n_streams, pool_rows, seed, device):
    """Per stream: d ~ U{128..2048}, ell ~ U{16..256}; rows from its own
    low-rank-plus-noise model: rank r = min(2 ell, d), scales 1 - (i-1)/r on
    an orthonormal basis, plus N(0, 0.1^2) noise; pool_rows resident rows."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    ds = rng.choice([128, 256, 512, 1024, 2048], size=n_streams)
    ells = rng.choice([16, 32, 64, 128, 256], size=n_streams)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    pools = []
    for d, ell in zip(ds.tolist(), ells.tolist()):
        r = min(2 * ell, d)
        V, _ = torch.linalg.qr(torch.randn(d, r, device=device, generator=gen))
        sc = 1.0 - torch.arange(r, device=device, dtype=torch.float32) / r
        g = torch.randn(pool_rows, r, device=device, generator=gen) * sc
        pools.append((g @ V.T + 0.1 * torch.randn(pool_rows, d, device=device, generator=gen)).contiguous())
    return ds.tolist(), ells.tolist(), pools


def burst_schedule(n_bursts, n_streams, rate, pool_rows, seed):
    """(arrival offset s, stream, rows, pool offset): Poisson arrivals at the
    aggregate rate (bursts/s; None: all at time 0), stream uniform, burst
    size floor(exp(U[0, ln 4097))) in [1, 4096]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_bursts):
        if rate:
            t += rng.exponential(1.0 / rate)
        b = int(min(4096, max(1, np.floor(np.exp(rng.uniform(0.0, np.log(4097.0)))))))
        b = min(b, pool_rows)
        out.append((t, int(rng.integers(n_streams)), b, int(rng.integers(0, pool_rows - b + 1))))
    return out


def serve(srv, ids, pools, sched):
    """Drives the serving loop through a schedule; returns (latencies,
    rows, seconds from first arrival to last completion)."""
    import numpy as np
    t0 = srv.now() + 0.01
    i, outstanding, lat, rows = 0, 0, [], 0
    last_done = t0
    while i < len(sched) or outstanding:
        now = srv.now()
        while i < len(sched) and t0 + sched[i][0] <= now:
            ta, s, b, off = sched[i]
            srv.submit(ids[s], pools[s][off:off + b], arrival=t0 + ta)
            i += 1
            outstanding += 1
        srv.tick()
        for c in srv.poll():
            lat.append(c["done"] - c["arrival"])
            rows += c["rows"]
            last_done = max(last_done, c["done"])
            outstanding -= 1
            if len(lat) % 20000 == 0:
                print(f"[bench] {len(lat)} of {len(sched)} bursts done", file=sys.stderr, flush=True)
    return np.asarray(lat), rows, last_done - t0


def serving_main(args):
    import numpy as np
    import torch
    from paper_2601_02019_amd import Server

    dev = torch.device("cuda:0")
    t0 = time.time()
    ds, ells, pools = serving_streams(args.streams, args.pool_rows, 3, dev)
    torch.cuda.synchronize()
    print(f"[bench] {args.streams} stream pools generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    srv = Server(max_inflight=2, max_rows_per_tick=args.row_cap, max_shrinks_per_tick=args.shrink_cap)
    ids = [srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=1, seed=5,
                    stream_id=i) for i, (d, ell) in enumerate(zip(ds, ells))]
    st = srv.stats()
    print(f"[bench] admitted {st['admitted']} streams, {st['bytes_in_use'] / 2**20:.0f} MiB of state",
          file=sys.stderr, flush=True)
    # warm-up, then saturation: every burst queued at once
    serve(srv, ids, pools, burst_schedule(max(64, args.bursts // 10), args.streams, None,
                                          args.pool_rows, 100))
    sched = burst_schedule(args.bursts, args.streams, None, args.pool_rows, 101)
    torch.cuda.synchronize()
    lat, rows, secs = serve(srv, ids, pools, sched)
    sat_rows = rows / secs
    sat_bursts = len(sched) / secs
    print(f"[bench] saturation: {sat_rows:.0f} rows/s, {sat_bursts:.1f} bursts/s over {secs:.1f}s",
          file=sys.stderr, flush=True)
    points = []
    for j, f in enumerate(float(x) for x in args.loads.split(",")):
        sched = burst_schedule(args.bursts, args.streams, f * sat_bursts, args.pool_rows, 200 + j)
        lat, rows, secs = serve(srv, ids, pools, sched)
        pt = {"load": f, "offered_bursts_per_s": f * sat_bursts, "rows_per_s": rows / secs,
              "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
              "bursts": len(sched)}
        points.append(pt)
        print(f"[bench] load {f}: {pt}", file=sys.stderr, flush=True)
    st = srv.stats()
    finite = all(bool(torch.isfinite(srv.query(ids[i], torch.float32)).all()) for i in range(0, len(ids), 37))
    srv.close()
    cpu = None
    if not args.no_cpu:
        # the oracle on a pool of processes over the host cores, one stream
        # each (the first streams of the set with ell <= 128, so that a sample
        # stays within seconds), two shrinks' worth of rows per stream
        procs = max(1, min(os.cpu_count() or 1, 16))
        jobs = [(i, d, ell) for i, (d, ell) in enumerate(zip(ds, ells)) if ell <= 128][:procs]
        tc, rows_c = oracle_pool(_serving_oracle_job, jobs, procs)
        cpu = {"value": rows_c / tc, "unit": "rows/s", "cores": procs, "kind": "oracle",
               "sample": f"{len(jobs)} serving streams with ell <= 128, 3 ell + 1 rows each, one process per "
                         f"stream, randomized shrink k=ell q=1, FP64 plain C, {tc:.1f}s",
               "cpu": cpu_model(), "nproc": os.cpu_count()}
    hi = points[-1] if points else None
    out = {
        "metric": "rows/sec sketch update at matched cov-err vs exact-SVD FD; batched p99 lat",
        "value": sat_rows, "unit": "rows/s", "n_gpus": 1, "steps": len(points), "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16 (FP64 core)", "data": "synthetic",
        "config": {"workload": "batched serving: %d concurrent streams, d ~ U{128..2048}, ell ~ "
                               "U{16..256}, rank 2 ell low-rank + noise, log-uniform bursts 1-4096 "
                               "rows, Poisson arrivals; randomized shrink, bf16 projection, q=1"
                               % args.streams,
                   "streams": args.streams, "bursts_per_point": args.bursts, "row_cap": args.row_cap,
                   "shrink_cap": args.shrink_cap},
        "saturation": {"rows_per_s": sat_rows, "bursts_per_s": sat_bursts},
        "latency": points,
        "p99_ms_at_highest_load": hi["p99_ms"] if hi else None,
        "server": {"ticks": st["ticks"], "batches": st["batches"], "state_MiB": st["bytes_in_use"] / 2**20},
        "sketches_finite": finite,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def base_line(args, value, unit, ms_per_step, workload, extra):
    out = {
        "metric": "rows/sec sketch update at matched cov-err vs exact-SVD FD; batched p99 lat",
        "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": extra.pop("dtype"), "data": "synthetic", "config": {"workload": workload},
    }
    out.update(extra)
    print(json.dumps(out))


def small_main(args):
    """Persistent stream, exact FP64 shrink: n = 10,000, d = 256, ell = 32."""
    import numpy as np
    import torch
    import synth
    from paper_2601_02019_amd import Sketch
    n, d, ell = 10_000, 256, 32
    A = synth.persistent_small(n, d, seed=0)
    At = torch.from_numpy(A).cuda()
    for _ in range(args.warmup):
        s = Sketch(d, ell)
        s.update(At)
        s.query()
        s.close()
    times = []
    for _ in range(args.steps):
        s = Sketch(d, ell)
        s.profile("all")
        B, t = timed(lambda: (s.update(At), s.query())[1])
        times.append(t)
        prof = s.profile_read()
        s.close()
    ms = 1e3 * float(np.median(times))
    AtA = A.T @ A
    Bn = B.cpu().numpy()
    err = float(np.max(np.abs(np.linalg.eigvalsh(AtA - Bn.T @ Bn)))) / float(np.trace(AtA))
    cpu = None
    if not args.no_cpu:
        import oracle
        o = oracle.FD(d, ell)
        t = time.perf_counter()
        o.update(A)
        o.query()
        tc = time.perf_counter() - t
        cpu = {"value": n / tc, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole stream ({n} rows, {o.shrinks} exact shrinks), FP64 plain C, one "
                         f"thread, {tc:.1f}s", "cpu": cpu_model(), "nproc": os.cpu_count()}
    stages = {k: v for k, v in prof.items() if v[0] > 0}
    base_line(args, n / (ms / 1e3), "rows/s", ms,
              "persistent stream, exact FP64 shrink: n=10000, d=256, ell=32, rank-20 signal "
              "10*0.8^i + N(0, 0.1^2)",
              {"dtype": "f64", "us_per_shrink": 1e3 * ms / 302, "cov_err_rel": err, "bound_rel": 1 / ell,
               "cpu_baseline": cpu, "stage_ms_per_step": {k: v[1] for k, v in stages.items()}})


def window_main(args):
    """Sliding window: d = 1024, ell = 128, N = 100,000, FP32 rows, queries
    every 10,000 rows; the first --window-rows rows of the stream."""
    import numpy as np
    import torch
    import synth
    from paper_2601_02019_amd import Sketch
    d, ell, N, R = 1024, 128, 100_000, 64.0
    n = args.window_rows
    t0 = time.time()
    A = synth.window_stream(n, d=d, seed=2)
    At = torch.from_numpy(A).cuda()
    print(f"[bench] window stream {n} x {d} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    w = Sketch(d, ell, kind="window", shrink="rand", window_N=N, R=R, q=1, seed=9, stream_id=0)
    # warm-up on a separate sketch
    ww = Sketch(d, ell, kind="window", shrink="rand", window_N=N, R=R, q=1, seed=9, stream_id=1)
    ww.update(At[:2000])
    ww.query()
    ww.close()
    upd, qry, errs = 0.0, [], []
    for r0 in range(0, n, 10_000):
        blk = At[r0:r0 + 10_000]
        _, t = timed(lambda: w.update(blk))
        upd += t
        B, tq = timed(lambda: w.query(torch.float64))
        qry.append(tq)
        lo = max(0, r0 + blk.shape[0] - N)
        W = At[lo:r0 + blk.shape[0]].double()
        G = W.T @ W
        D = G - B.T @ B
        errs.append(float(torch.linalg.eigvalsh((D + D.T) / 2).abs().max() / torch.trace(G)))
        print(f"[bench] window rows {r0 + blk.shape[0]}: update {t:.2f}s query {1e3 * tq:.0f} ms "
              f"err {errs[-1]:.2e}", file=sys.stderr, flush=True)
    lv = w.info()["levels"]
    stats = [w.window_stats(j) for j in range(lv)]
    w.close()
    cpu = None
    if not args.no_cpu:
        import oracle
        m = 600  # about 20-30 s of the FP64 oracle
        print(f"[bench] CPU oracle on the first {m} rows", file=sys.stderr, flush=True)
        o = oracle.Window(d, ell, N, R, q=1, seed=9, stream=0, fd="rand")
        t = time.perf_counter()
        o.update(A[:m].astype(np.float64))
        tc = time.perf_counter() - t
        cpu = {"value": m / tc, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": f"first {m} rows of the window stream, FP64 plain C, one thread, {tc:.1f}s", "cpu": cpu_model(), "nproc": os.cpu_count()}
    base_line(args, n / upd, "rows/s", None,
              "sliding window: d=1024, ell=128, N=100000, FP32 rows, rank-64 spectrum 0.95^j rotating "
              "by a Givens sweep every 50000 rows; first %d rows, query every 10000" % n,
              {"dtype": "f32 rows, f64 state", "rows": n, "update_s": upd,
               "query_ms_median": 1e3 * float(np.median(qry)), "query_ms_max": 1e3 * float(np.max(qry)),
               "cov_err_rel_max": max(errs), "bound_rel_25_over_ell": 25.0 / ell,
               "level_stats": stats, "cpu_baseline": cpu})


def attp_main(args):
    """ATTP persistent sketch (Algorithm "ATTP Sketch using AeroSketch"): the
    shape of the paper's ATTP experiment, a Random Noisy stream (D_ii =
    1 - (i-1)/d, noise 1/zeta, zeta = 10) with d = 500 and T = --attp-rows
    rows; ell = 64 (eps = 1/32), randomized FD reduce, FP64.  After the
    stream, the sketches of 20 past times t = T/20, 2T/20, ..., T are queried."""
    import numpy as np
    import torch
    import synth
    from paper_2601_02019_amd import Sketch
    d, ell, n = 500, 64, args.attp_rows
    A = synth.random_noisy(n, d, seed=5)
    At = torch.from_numpy(A).cuda()
    warm = Sketch(d, ell, kind="attp", shrink="rand", q=1, seed=3, stream_id=1)
    warm.update(At[:500])
    warm.query_at(250)
    warm.close()
    s = Sketch(d, ell, kind="attp", shrink="rand", q=1, seed=3, stream_id=0)
    _, tu = timed(lambda: s.update(At))
    times = [n * (i + 1) // 20 for i in range(20)]
    qms, errs = [], []
    for t in times:
        B, tq = timed(lambda: s.query_at(t))
        qms.append(1e3 * tq)
        Ap = At[:t]
        G = Ap.T @ Ap
        D = G - B.T @ B
        errs.append(float(torch.linalg.eigvalsh((D + D.T) / 2).abs().max() / torch.trace(G)))
    st = s.window_stats(0)
    s.close()
    print(f"[bench] attp: update {tu:.2f}s, queries {np.median(qms):.1f} ms, max err {max(errs):.3e}",
          file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        import oracle
        m = 600
        o = oracle.ATTP(d, ell, q=1, seed=3, stream=0, fd="rand")
        tc0 = time.perf_counter()
        o.update(A[:m])
        tc = time.perf_counter() - tc0
        cpu = {"value": m / tc, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": f"first {m} rows of the ATTP stream, FP64 plain C, one thread, {tc:.1f}s",
               "cpu": cpu_model(), "nproc": os.cpu_count()}
    base_line(args, n / tu, "rows/s", None,
              "ATTP persistent sketch: Random Noisy stream d=500, T=%d rows, ell=64 (eps=1/32), randomized "
              "FD reduce, FP64; sketches of 20 past times queried" % n,
              {"dtype": "f64", "rows": n, "update_s": tu, "query_ms_median": float(np.median(qms)),
               "cov_err_rel_max_over_times": max(errs), "bound_rel_10_over_ell": 10.0 / ell,
               "snapshots": st["dumps"], "dumped_directions": st["dirs"], "cpu_baseline": cpu})


def sites_main(args):
    """64 logical sites, each 100,000 CSR rows (d = 2048, 1 % density, values
    N(0,1) * j^-0.5), ell = 128 per site; every 10,000 rows per site the
    coordinator re-merges the current site sketches by a binary tree."""
    import numpy as np
    import torch
    from paper_2601_02019_amd import Sketch, sketch_update_csr_batch
    d, ell, S, n = 2048, 128, args.sites, args.site_rows
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(4)
    w = torch.arange(1, d + 1, device=dev, dtype=torch.float32) ** -0.5
    t0 = time.time()
    sites = []
    for s in range(S):
        ips, ixs, vvs = [torch.zeros(1, dtype=torch.int64, device=dev)], [], []
        base = 0
        for r0 in range(0, n, 10_000):
            m = min(10_000, n - r0)
            mask = torch.rand(m, d, device=dev, generator=gen) < 0.01
            cnt = mask.sum(1)
            idx = mask.nonzero()[:, 1].to(torch.int32)
            vals = torch.randn(idx.shape[0], device=dev, generator=gen) * w[idx.long()]
            ips.append(base + torch.cumsum(cnt, 0))
            base += int(cnt.sum())
            ixs.append(idx)
            vvs.append(vals)
        sites.append((torch.cat(ips).contiguous(), torch.cat(ixs).contiguous(), torch.cat(vvs).contiguous()))
    torch.cuda.synchronize()
    nnz = sum(int(x[1].shape[0]) for x in sites)
    print(f"[bench] {S} sites x {n} CSR rows ({nnz / (S * n):.1f} nnz/row) in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    def run():
        sk = [Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=1, seed=4, stream_id=s)
              for s in range(S)]
        coord = None
        t_upd = t_mrg = 0.0
        for r0 in range(0, n, 10_000):
            m = min(10_000, n - r0)
            chunk = [(x[0][r0:r0 + m + 1].contiguous(), x[1], x[2]) for x in sites]
            _, t = timed(lambda: sketch_update_csr_batch(sk, chunk))
            t_upd += t
            if coord is not None:
                coord.close()
            coord = Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=1, seed=4,
                           stream_id=1000 + r0 // 10_000)
            _, t = timed(lambda: coord.merge_tree(sk))
            t_mrg += t
        B = coord.query()
        coord.close()
        for x in sk:
            x.close()
        return B, t_upd, t_mrg

    if args.warmup:  # load the kernels on a small piece of the work
        wk = [Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=1, seed=4, stream_id=s)
              for s in range(2)]
        sketch_update_csr_batch(wk, [(x[0][:1001].contiguous(), x[1], x[2]) for x in sites[:2]])
        wc = Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=1, seed=4, stream_id=99)
        wc.merge_tree(wk)
        wc.query()
        for x in wk + [wc]:
            x.close()
    B, t_upd, t_mrg = run()
    total = t_upd + t_mrg
    # error of the final merged sketch against the union of all site rows
    G = torch.zeros(d, d, device=dev, dtype=torch.float64)
    for ip, ix, vv in sites:
        for r0 in range(0, n, 20_000):
            m = min(20_000, n - r0)
            X = torch.zeros(m, d, device=dev, dtype=torch.float64)
            a, b = int(ip[r0]), int(ip[r0 + m])
            rows = torch.repeat_interleave(torch.arange(m, device=dev), (ip[r0 + 1:r0 + m + 1] - ip[r0:r0 + m]))
            X[rows, ix[a:b].long()] = vv[a:b].double()
            G += X.T @ X
    D = G - B.double().T @ B.double()
    err = float(torch.linalg.eigvalsh((D + D.T) / 2).abs().max() / torch.trace(G))
    cpu = None
    if not args.no_cpu:
        # the oracle on a pool of processes over the host cores, one site each
        m = 2 * ell + 2 * (ell + 1)
        procs = max(1, min(S, os.cpu_count() or 1, 16))
        tc, rows = oracle_pool(_site_oracle_job, [(site, m, d, ell) for site in range(procs)], procs)
        cpu = {"value": rows / tc, "unit": "rows/s", "cores": procs, "kind": "oracle",
               "sample": f"first {m} rows of each of {procs} sites densified ({procs} processes, one site "
                         f"each, randomized shrinks k={ell}), FP64 plain C, {tc:.1f}s",
               "cpu": cpu_model(), "nproc": os.cpu_count()}
    base_line(args, S * n / total, "rows/s", None,
              "distributed sites on one GPU: %d sites x %d CSR rows, d=2048, 1%% density, values N(0,1) "
              "j^-0.5, ell=128 per site, tree merge every 10000 rows per site" % (S, n),
              {"dtype": "f32 state + bf16 projection (FP64 core)", "update_s": t_upd, "merge_s": t_mrg,
               "update_rows_per_s": S * n / t_upd, "cov_err_rel_merged": err, "bound_rel": 1 / ell,
               "cpu_baseline": cpu})


def p5_main(args):
    """Continuous distributed tracking (Algorithm "P5") on the distributed
    workload's shape: --sites sites (64), d = 2048, ell = 128, rows with 1 %
    density and values N(0,1) j^-0.5 (stored dense, FP32 on the device), each
    row at a site drawn uniformly; --p5-rows rows per site on average.  The
    rows go in blocks of 16,384; the coordinator is queried at the end."""
    import numpy as np
    import torch
    from paper_2601_02019_amd import Sketch
    d, ell, S = 2048, 128, args.sites
    n = S * args.p5_rows
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    w = torch.arange(1, d + 1, device=dev, dtype=torch.float32) ** -0.5
    A = torch.empty(n, d, device=dev, dtype=torch.float32)
    for r0 in range(0, n, 16_384):
        m = min(16_384, n - r0)
        mask = torch.rand(m, d, device=dev, generator=gen) < 0.01
        A[r0:r0 + m] = torch.randn(m, d, device=dev, generator=gen) * w * mask
    site = np.random.default_rng(5).integers(0, S, size=n).astype(np.int32)
    torch.cuda.synchronize()
    warm = Sketch(d, ell, kind="p5", shrink="rand", q=1, seed=5, stream_id=1, sites=S)
    warm.p5_update(A[:4096], site[:4096])
    warm.query()
    warm.close()
    s = Sketch(d, ell, kind="p5", shrink="rand", q=1, seed=5, stream_id=0, sites=S)
    upd = 0.0
    for r0 in range(0, n, 16_384):
        m = min(16_384, n - r0)
        _, t = timed(lambda: s.p5_update(A[r0:r0 + m], site[r0:r0 + m]))
        upd += t
        print(f"[bench] p5 rows {r0 + m}: {t:.2f}s", file=sys.stderr, flush=True)
    B, tq = timed(lambda: s.query(torch.float64))
    st = s.p5_stats()
    fhat, Bc = s.p5_coordinator()
    s.close()
    G = gram_f64(A)
    tot = float(torch.trace(G))
    D = G - B.T @ B
    err = float(torch.linalg.eigvalsh((D + D.T) / 2).abs().max() / tot)
    D = G - Bc
    err_c = float(torch.linalg.eigvalsh((D + D.T) / 2).abs().max() / tot)
    print(f"[bench] p5: update {upd:.2f}s, query {1e3 * tq:.0f} ms, err {err:.3e} (coordinator {err_c:.3e}), "
          f"{st}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        import oracle
        Ah = A.double().cpu().numpy()
        o = oracle.P5(d, ell, S, q=1, seed=5, stream=0, fd="rand")
        done, tc = 0, 0.0
        while done < n and tc < 20.0:
            m = min(256, n - done)
            t = time.perf_counter()
            o.update(Ah[done:done + m], site[done:done + m])
            tc += time.perf_counter() - t
            done += m
        cpu = {"value": done / tc, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": f"first {done} rows of the P5 stream (about 20 s), FP64 plain C, one thread, {tc:.1f}s",
               "cpu": cpu_model(), "nproc": os.cpu_count()}
    base_line(args, n / upd, "rows/s", None,
              "P5 continuous distributed tracking: %d sites, %d rows (d=2048, 1%% density, values N(0,1) "
              "j^-0.5, dense FP32 on the device), each at a uniformly drawn site; ell=128, randomized FD "
              "reduce at the sites" % (S, n),
              {"dtype": "f32 rows, f64 state", "rows": n, "update_s": upd, "query_ms": 1e3 * tq,
               "cov_err_rel": err, "cov_err_rel_coordinator": err_c, "bound_rel_eps": 2.0 / ell,
               "fhat_over_fro2": fhat / tot, "messages": st,
               "words_over_raw_rows": st["words"] / float(n * d), "cpu_baseline": cpu})


def cod_main(args):
    """Approximate matrix multiplication over a sliding window (Algorithm
    "AeroSketchCOD Framework") on the paper's AMM setting: Uniform Random
    pairs (entries in (0, 1]), d_x = 300, d_y = 500, N = 5,000, T = --cod-pairs
    (10,000); ell = --cod-ell (eps = 2 / ell) and theta = eps N min ||x|| ||y||
    (at most eps ||X_W||_F ||Y_W||_F for every window).  Queried every 1,000
    pairs; the error is taken against the exact window product."""
    import numpy as np
    import torch
    from paper_2601_02019_amd import Sketch
    dx, dy, N, n, ell = 300, 500, 5000, args.cod_pairs, args.cod_ell
    rng = np.random.default_rng(6)
    X = 1.0 - rng.random((n, dx))
    Y = 1.0 - rng.random((n, dy))
    nx = np.sqrt(np.sum(X ** 2, axis=1))
    ny = np.sqrt(np.sum(Y ** 2, axis=1))
    theta = (2.0 / ell) * N * float(np.min(nx * ny))
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    warm = Sketch(dx, ell, kind="cod", window_N=N, q=1, seed=6, stream_id=1, d_y=dy, theta=theta)
    warm.cod_update(Xt[:300], Yt[:300])
    warm.cod_query()
    warm.close()
    s = Sketch(dx, ell, kind="cod", window_N=N, q=1, seed=6, stream_id=0, d_y=dy, theta=theta)
    upd, qms, errs = 0.0, [], []
    for r0 in range(0, n, 1000):
        m = min(1000, n - r0)
        _, t = timed(lambda: s.cod_update(Xt[r0:r0 + m], Yt[r0:r0 + m]))
        upd += t
        (A, B), tq = timed(lambda: s.cod_query())
        qms.append(1e3 * tq)
        lo = max(0, r0 + m - N)
        W = Xt[lo:r0 + m].T @ Yt[lo:r0 + m]
        fro = float(torch.linalg.norm(Xt[lo:r0 + m]) * torch.linalg.norm(Yt[lo:r0 + m]))
        errs.append(float(torch.linalg.matrix_norm(W - A @ B.T, ord=2)) / fro)
        print(f"[bench] cod pairs {r0 + m}: update {t:.2f}s query {1e3 * tq:.0f} ms err {errs[-1]:.2e}",
              file=sys.stderr, flush=True)
    st = s.window_stats(0)
    s.close()
    cpu = None
    if not args.no_cpu:
        import oracle
        o = oracle.COD(dx, dy, ell, N=N, theta=theta, q=1, seed=6, stream=0)
        done, tc = 0, 0.0
        while done < n and tc < 20.0:
            m = min(50, n - done)
            t = time.perf_counter()
            o.update(X[done:done + m], Y[done:done + m])
            tc += time.perf_counter() - t
            done += m
        cpu = {"value": done / tc, "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"first {done} pairs of the stream (about 20 s), FP64 plain C, one thread, {tc:.1f}s",
               "cpu": cpu_model(), "nproc": os.cpu_count()}
    base_line(args, n / upd, "pairs/s", None,
              "AMM over a sliding window (AeroSketchCOD): Uniform Random pairs, d_x=300, d_y=500, N=5000, "
              "T=%d, ell=%d, theta = eps N min|x||y|, FP64; query every 1000 pairs" % (n, ell),
              {"dtype": "f64", "pairs": n, "update_s": upd, "query_ms_median": float(np.median(qms)),
               "err_rel_max": max(errs), "bound_rel_eps": 2.0 / ell, "theta": theta, "snapshots": st["dumps"],
               "reduces": st["shrinks"], "cpu_baseline": cpu})


def copy_main(args):
    """A plain device-to-device copy of 1 GiB, args.steps times: the measured
    HBM rate, and a kernel of known traffic for calibrating the FETCH_SIZE /
    WRITE_SIZE counters (2^30 bytes read and 2^30 written per launch)."""
    import torch
    n = 1 << 28
    src = torch.ones(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(max(1, args.warmup)):
        dst.copy_(src)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gbs = 2 * 4 * n / (ms / 1e3) / 1e9
    base_line(args, gbs, "GB/s", ms, "device copy of 2^30 bytes (read + write)",
              {"dtype": "f32", "bytes_per_launch": 2 * 4 * n, "frac_of_8TBs": gbs / PEAK_HBM_GBS})


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (--gpus {args.gpus} "
              f"requested). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload != "persistent":
        return {"serving": serving_main, "small": small_main, "window": window_main,
                "sites": sites_main, "copy": copy_main, "attp": attp_main, "p5": p5_main,
                "cod": cod_main}[args.workload](args)
    import torch
    from paper_2601_02019_amd import Sketch

    dev = torch.device("cuda:0")
    d, ell, n = args.d, args.ell, args.rows
    t0 = time.time()
    A = make_stream(n, d, 1024, 1, dev)
    torch.cuda.synchronize()
    print(f"[bench] stream {n} x {d} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    # ---------------- randomized mixed-precision path (the timed hot path)
    sk = Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=args.q, seed=7,
                stream_id=1)
    for w in range(args.warmup):
        sk.update(A)
        sk.query()
        print(f"[bench] warmup step {w} done", file=sys.stderr, flush=True)
    sk.profile("all")
    torch.cuda.synchronize()
    times, fills = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.update(A)
        fills.append(sk.info()["fill"])  # host-planned: no device round trip
        B = sk.query()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        print(f"[bench] step {k}: {times[-1]:.3f}s", file=sys.stderr, flush=True)
    prof = sk.profile_read()
    sk.close()
    ms_per_step = 1e3 * float(sorted(times)[len(times) // 2])  # median step
    rows_per_s = n / (ms_per_step / 1e3)

    # dominant kernel: the stage with the largest event-timed total
    stages = {k: v for k, v in prof.items() if v[0] > 0}
    dom = max(stages, key=lambda k: stages[k][1])
    dom_calls, dom_ms = stages[dom]
    avg_ms = dom_ms / dom_calls
    roofline = None
    if dom == "eig_reduce":
        # Householder reduction of the k x k Rayleigh-Ritz matrix of every
        # shrink (k = ell) and of the query's r x r buffer Gram (r = the fill
        # at the query, when r >= ell): orders from 160 up run on ceil(n / 16)
        # workgroups with one exchange per column
        orders = [ell] * (dom_calls - len([f for f in fills if f >= ell])) + [f for f in fills if f >= ell]
        flops = sum(tri_flops(n_) for n_ in orders) / dom_calls
        achieved = flops / (avg_ms / 1e3) / 1e12
        multi = ell >= 160
        kern = "k_tri_reduce_x" if multi else ("k_tri_reduce_blk" if ell > 128 else "k_tri_reduce")
        src = "paper_2601_02019_amd/csrc/k_trix.hip" if multi else "paper_2601_02019_amd/csrc/k_tri.hip"
        roofline = {"bound": "alu",
                    "kernel": "%s (FP64 Householder tridiagonalisation, n=%d, %s)"
                    % (kern, ell, "%d workgroups, one exchange per column" % ((ell + 15) // 16) if multi
                       else "one workgroup"),
                    "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64_TFLOPS,
                    "traffic": measured_traffic(kern, src),
                    "avg_launch_ms": avg_ms, "launches": dom_calls, "algorithmic_flops_per_launch": flops,
                    "us_per_column": 1e3 * avg_ms / max(1.0, sum(n_ - 2 for n_ in orders) / dom_calls),
                    "fallbacks_to_jacobi": prof.get("eig_fallbacks", (0, 0.0))[1]}
    else:
        roofline = {"bound": "unknown", "kernel": dom, "avg_launch_ms": avg_ms}

    # ---------------- exact-SVD FD on the same GPU and the matched-error check:
    # both paths over the same rows (the whole stream unless --exact-rows)
    exact = None
    pre = min(args.exact_rows, n) if args.exact_rows > 0 else n
    if not args.no_exact:
        Ap = A[:pre]
        ex = Sketch(d, ell, shrink="exact", state_dtype="f32", seed=7, stream_id=1)
        ra = Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", q=args.q, seed=7,
                    stream_id=1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ex.update(Ap)
        Be = ex.query()
        torch.cuda.synchronize()
        te = time.perf_counter() - t
        ra.update(Ap)
        Br = ra.query()
        AtA = gram_f64(Ap)
        ee, er = cov_err(AtA, Be), cov_err(AtA, Br)
        fro2 = float(torch.trace(AtA))
        exact = {"rows_per_s": pre / te, "timed_rows": pre,
                 "cov_err_rel_exact": ee / fro2, "cov_err_rel_rand": er / fro2,
                 "rand_over_exact_err": er / ee, "matched": bool(er <= 1.05 * ee), "bound_rel": 1.0 / ell,
                 "eig_solver": "tridiagonal (multi-workgroup reduction) for 2 ell <= 512"}
        print(f"[bench] exact path: {exact}", file=sys.stderr, flush=True)
        ex.close()
        ra.close()

    # full-stream error of the timed sketch
    err_full = None
    if not args.no_err:
        AtA = gram_f64(A)
        fro2 = float(torch.trace(AtA))
        # the sketch saw the stream (warmup + steps) times: compare with that many copies
        passes = args.warmup + args.steps
        err_full = cov_err(passes * AtA, B) / (passes * fro2)

    # ---------------- CPU baseline: the FP64 oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        import oracle
        rows_cpu = 2 * ell + (args.cpu_shrinks - 1) * (ell + 1)
        Ah = A[:rows_cpu].double().cpu().numpy()
        o = oracle.FD(d, ell, "rand", k=ell, q=args.q, seed=7, stream=1)
        t = time.perf_counter()
        o.update(Ah)
        tc = time.perf_counter() - t
        cpu = {"value": rows_cpu / tc, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": f"first {rows_cpu} rows of the d={d} stream ({o.shrinks} randomized "
                         f"shrinks, k={ell}, q={args.q}), FP64 plain C, one thread, {tc:.1f}s",
               "cpu": cpu_model(), "nproc": os.cpu_count()}

    # row ingest: FP32 rows read once, written once into the FP32 buffer
    ingest = None
    if "ingest" in stages:
        ing_bytes = float(n) * d * (4 + 4) * args.steps
        ing_s = stages["ingest"][1] / 1e3
        ingest = {"gbs": ing_bytes / ing_s / 1e9, "frac_of_hbm_peak": ing_bytes / ing_s / 1e9 / PEAK_HBM_GBS,
                  "launches": stages["ingest"][0], "bytes_per_step": ing_bytes / args.steps}

    out = {
        "metric": "rows/sec sketch update at matched cov-err vs exact-SVD FD; batched p99 lat",
        "value": rows_per_s, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16 (FP64 core)",
        "data": "synthetic",
        "config": {"workload": "persistent stream, tight error: n=%d, d=%d, ell=%d, FP32 rows, "
                               "power-law spectrum i^-0.8 over rank 1024 + N(0,1e-3); randomized "
                               "shrink k=ell, q=%d, bf16 projection" % (n, d, ell, args.q),
                   "rows": n, "d": d, "ell": ell, "q": args.q},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "exact_fd_same_gpu": exact,
        "cov_err_rel_full_stream": err_full,
        "stage_ms_per_step": {k: v[1] / args.steps for k, v in stages.items()},
        "ingest": ingest,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
