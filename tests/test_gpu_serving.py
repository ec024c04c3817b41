"""GPU tests of the serving loop (server_* in the C ABI): a result is the
same alone and in the mix (bitwise), admission by memory budget with reuse of
released sketches, and latency accounting against a fake clock."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gram, note, rel_fro

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2601_02019_amd as sk
    return sk


def _bursts(n_rows, rng, max_burst):
    sizes = []
    while sum(sizes) < n_rows:
        b = int(np.exp(rng.uniform(0.0, np.log(max_burst + 1))))
        sizes.append(max(1, min(b, n_rows - sum(sizes))))
    return sizes


STREAMS = [  # (d, ell, shrink, state, proj)
    (128, 16, "rand", "f32", "bf16"),
    (256, 32, "rand", "f32", "bf16"),
    (512, 16, "rand", "f32", "bf16"),
    (128, 64, "rand", "f32", "bf16"),
    (256, 16, "exact", "f64", "f64"),
    (384, 32, "rand", "f64", "f64"),
    (128, 32, "rand", "f32", "f32"),
    (200, 8, "exact", "f32", "f64"),
]


@pytest.mark.parametrize("row_cap,inflight,shrink_cap", [(0, 2, 0), (96, 1, 0), (200, 3, 0), (0, 2, 1)])
def test_mix_equals_alone_bitwise(row_cap, inflight, shrink_cap):
    sk = _lib()
    rng = np.random.default_rng(7)
    note(f"serving mix row_cap={row_cap} inflight={inflight}")
    data, bursts = [], []
    for i, (d, ell, *_rest) in enumerate(STREAMS):
        n = int(rng.integers(4 * ell, 1200))
        A = synth.lowrank_rows(n, d, np.linspace(1.0, 0.1, min(2 * ell, d)), 0.1, seed=100 + i)
        dt = torch.float64 if STREAMS[i][3] == "f64" else torch.float32
        data.append(torch.from_numpy(A).to("cuda", dt))
        bursts.append(_bursts(n, rng, 300))
    srv = sk.Server(max_inflight=inflight, max_rows_per_tick=row_cap, max_shrinks_per_tick=shrink_cap)
    ids = []
    for i, (d, ell, shr, st, pj) in enumerate(STREAMS):
        ids.append(srv.open(d, ell, shrink=shr, state_dtype=st, proj_dtype=pj, seed=11, stream_id=i))
    # interleave submissions and ticks, streams in random order
    pos = [0] * len(STREAMS)
    nb = [0] * len(STREAMS)
    tickets = 0
    while any(nb[i] < len(bursts[i]) for i in range(len(STREAMS))):
        for i in rng.permutation(len(STREAMS)):
            if nb[i] < len(bursts[i]) and rng.uniform() < 0.6:
                b = bursts[i][nb[i]]
                srv.submit(ids[i], data[i][pos[i]:pos[i] + b].contiguous())
                pos[i] += b
                nb[i] += 1
                tickets += 1
        srv.tick()
    srv.drain()
    done = srv.poll()
    assert len(done) == tickets
    assert srv.stats()["pending_bursts"] == 0
    for i, (d, ell, shr, st, pj) in enumerate(STREAMS):
        alone = sk.Sketch(d, ell, shrink=shr, state_dtype=st, proj_dtype=pj, seed=11, stream_id=i)
        alone.update(data[i])
        Ba = alone.query()
        Bm = srv.query(ids[i])
        assert torch.equal(Ba, Bm), (i, STREAMS[i])
        alone.close()
        if shr == "exact" and st == "f64":
            fd = oracle.FD(d, ell)
            fd.update(data[i].double().cpu().numpy())
            assert rel_fro(gram(Bm), gram(fd.query())) <= 1e-9
        if shr == "rand" and st == "f64" and pj == "f64":
            fd = oracle.FD(d, ell, mode="rand", k=ell, q=1, seed=11, stream=i)
            fd.update(data[i].double().cpu().numpy())
            assert rel_fro(gram(Bm), gram(fd.query())) <= 1e-9
    srv.close()


def test_admission_budget_fifo_and_reuse():
    sk = _lib()
    d, ell = 256, 32
    probe = sk.Server()
    probe.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16")
    one = probe.stats()["bytes_in_use"]
    probe.close()
    assert one > 0
    srv = sk.Server(memory_budget=2 * one + one // 2)
    a = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=0)
    b = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=1)
    c = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=2)
    st = srv.stats()
    assert (st["admitted"], st["waiting"], st["bytes_in_use"]) == (2, 1, 2 * one)
    rows = [torch.from_numpy(synth.lowrank_rows(700, d, np.linspace(1, 0.1, 40), 0.1, seed=s)).float().cuda()
            for s in range(3)]
    for sid, r in zip((a, b, c), rows):
        srv.submit(sid, r[:400].contiguous())
        srv.submit(sid, r[400:].contiguous())
    srv.drain()
    done = srv.poll()
    assert sorted(x["stream"] for x in done) == [a, a, b, b]  # c still waits
    assert srv.stats()["pending_bursts"] == 2
    with pytest.raises(sk.SketchError):
        srv.query(c)
    Ba = srv.query(a)
    srv.close_stream(a)
    srv.drain()
    st = srv.stats()
    assert (st["admitted"], st["waiting"], st["closed"], st["bytes_in_use"]) == (2, 0, 1, 2 * one)
    done = srv.poll()
    assert sorted(x["stream"] for x in done) == [c, c]
    # c runs in a's reused memory: same result as a fresh sketch
    alone = sk.Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=2)
    alone.update(rows[2])
    assert torch.equal(alone.query(), srv.query(c))
    alone0 = sk.Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=0)
    alone0.update(rows[0])
    assert torch.equal(alone0.query(), Ba)
    # a stream that alone exceeds the budget is refused
    with pytest.raises(sk.SketchError) as e:
        srv.open(4096, 256, shrink="rand", state_dtype="f32", proj_dtype="bf16")
    assert e.value.code == sk.SK_ENOMEM
    # a closed stream takes no more bursts
    with pytest.raises(sk.SketchError) as e:
        srv.submit(a, rows[0][:5].contiguous())
    assert e.value.code == sk.SK_ESTATE
    srv.close()


def test_waiting_stream_close_reports_dropped_bursts():
    sk = _lib()
    d, ell = 128, 16
    probe = sk.Server()
    probe.open(d, ell)
    one = probe.stats()["bytes_in_use"]
    probe.close()
    srv = sk.Server(memory_budget=one)
    a = srv.open(d, ell)
    b = srv.open(d, ell)
    t = srv.submit(b, torch.ones(10, d, dtype=torch.float64, device="cuda"), arrival=0.0)
    srv.close_stream(b)
    done = srv.poll()
    assert len(done) == 1 and done[0]["ticket"] == t and done[0]["done"] == -1.0
    assert srv.stats()["waiting"] == 0
    srv.submit(a, torch.ones(10, d, dtype=torch.float64, device="cuda"))
    srv.drain()
    assert len(srv.poll()) == 1
    srv.close()


def test_latency_accounting_fake_clock():
    sk = _lib()
    clock = [0.0]
    srv = sk.Server(max_inflight=1, max_rows_per_tick=128, clock=lambda: clock[0])
    d, ell = 128, 16
    sid = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16")
    A = torch.randn(600, d, device="cuda")
    clock[0] = 1.0
    t1 = srv.submit(sid, A[:100].contiguous(), arrival=0.5)
    t2 = srv.submit(sid, A[100:150].contiguous(), arrival=1.0)
    assert srv.now() == 1.0
    clock[0] = 2.0
    assert srv.tick() == 2          # 100 rows of the first burst, 28 of the second
    clock[0] = 3.5
    srv.drain()                     # one more tick: the second burst's last 22 rows
    assert srv.stats()["ticks"] == 2
    got = {c["ticket"]: c for c in srv.poll()}
    assert got[t1]["launched"] == 2.0 and got[t1]["done"] == 3.5 and got[t1]["arrival"] == 0.5
    assert got[t2]["launched"] == 2.0 and got[t2]["done"] == 3.5 and got[t2]["rows"] == 50
    # a 300-row burst under a 128-row cap spans three ticks
    t3 = srv.submit(sid, A[150:450].contiguous(), arrival=4.0)
    for c in (10.0, 11.0, 12.0):
        clock[0] = c
        assert srv.tick() == 1
    clock[0] = 13.0
    torch.cuda.synchronize()  # poll does not wait: let the last tick finish first
    got = {c["ticket"]: c for c in srv.poll()}
    assert got[t3]["launched"] == 10.0 and got[t3]["done"] == 13.0 and got[t3]["rows"] == 300
    assert srv.stats()["ticks"] == 5
    srv.close()


def test_real_clock_latency_is_ordered():
    sk = _lib()
    srv = sk.Server()
    ids = [srv.open(256, 32, shrink="rand", state_dtype="f32", proj_dtype="bf16", stream_id=i)
           for i in range(4)]
    A = torch.randn(2000, 256, device="cuda")
    for k in range(8):
        for sid in ids:
            srv.submit(sid, A[k * 200:(k + 1) * 200].contiguous())
        srv.tick()
    srv.drain()
    done = srv.poll()
    assert len(done) == 32
    for c in done:
        assert c["arrival"] <= c["launched"] + 1e-6
        assert c["launched"] <= c["done"] + 1e-3
        assert c["done"] - c["arrival"] < 30.0


def test_serving_argument_errors():
    sk = _lib()
    srv = sk.Server()
    with pytest.raises(sk.SketchError) as e:
        srv.open(64, 8, kind="window", window_N=10, R=2.0)
    assert e.value.code == sk.SK_EUNSUPPORTED
    with pytest.raises(sk.SketchError) as e:
        srv.open(64, 1)
    assert e.value.code == sk.SK_EINVAL
    with pytest.raises(sk.SketchError) as e:
        sk.server_submit(srv.handle, 99, torch.ones(2, 64, device="cuda"), 0.0)
    assert e.value.code == sk.SK_EINVAL
    srv.close()


def test_reused_sketch_does_not_inherit_a_failed_solve():
    """A released sketch that recorded a failed eigen-solve (injected from the
    host, no kernel fails) is reset before reuse, so the next stream of the
    same shape queries cleanly; a sketch whose failure was reported (sticky)
    is freed instead of reused."""
    sk = _lib()
    d, ell = 128, 16
    A = torch.from_numpy(synth.lowrank_rows(200, d, np.linspace(1.0, 0.1, 20), 0.1, seed=5)).to("cuda", torch.float32)
    srv = sk.Server(max_inflight=1)
    # 1. failure recorded but never observed: the stream is closed, its sketch idles
    a = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=0)
    srv.submit(a, A)
    srv.drain()
    srv.debug_fail_solver(a)
    srv.close_stream(a)
    srv.drain()
    srv.tick()
    b = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=0)
    srv.submit(b, A)
    srv.drain()
    assert srv.stats()["admitted"] == 1
    Bb = srv.query(b)  # no SK_EDEVICE from the previous stream's record
    alone = sk.Sketch(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=0)
    alone.update(A)
    assert torch.equal(alone.query(), Bb)
    alone.close()
    # 2. failure observed: the handle turns sticky and is not reused
    srv.debug_fail_solver(b)
    with pytest.raises(sk.SketchError) as e:
        srv.query(b)
    assert e.value.code == sk.SK_EDEVICE
    srv.close_stream(b)
    srv.drain()
    srv.tick()
    c = srv.open(d, ell, shrink="rand", state_dtype="f32", proj_dtype="bf16", seed=1, stream_id=0)
    srv.submit(c, A)
    srv.drain()
    assert torch.equal(srv.query(c), Bb)
    srv.close()


def test_debug_fail_solver_makes_the_sketch_sticky():
    sk = _lib()
    s = sk.Sketch(64, 8, shrink="exact")
    s.update(torch.randn(40, 64, dtype=torch.float64, device="cuda"))
    s.query()
    sk.sketch_debug_fail_solver(s.handle)
    with pytest.raises(sk.SketchError) as e:
        s.sync()
    assert e.value.code == sk.SK_EDEVICE
    with pytest.raises(sk.SketchError) as e:
        s.query()
    assert e.value.code == sk.SK_EDEVICE
    s.close()
