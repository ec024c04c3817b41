"""GPU parity of the sliding-window sketch (Algorithm "ML-AeroSketch")
against the FP64 window oracle, through the C ABI.

Every decision of the method (raw row or not, power-iteration estimate
against theta/2, the doubling loop, the number of dumped directions) is taken
in FP64 on both sides from the same Philox draws, so the decision traces agree
(checked through the per-level counters) and the queried sketches agree to
1e-9 in relative Frobenius norm of B^T B.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gram, note, rel_fro

pytestmark = pytest.mark.gpu


def normed_rows(n, d, R, seed, rank=6):
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, rank), 0.05, seed=seed)
    nrm = np.linalg.norm(A, axis=1, keepdims=True)
    return A / nrm * np.sqrt(rng.uniform(1.0, R, size=(n, 1)))


def make(d, ell, N, R, fd, q=1, seed=0, stream=0):
    from paper_2601_02019_amd import Sketch
    return Sketch(d, ell, kind="window", shrink=fd, window_N=N, R=R, q=q, seed=seed, stream_id=stream)


def compare(o, g, levels):
    Bo, lo = o.query()
    Bg = g.query()
    for j in range(levels):
        so, sg = o.stats(j), g.window_stats(j)
        for key in ("dumps", "raw", "dirs", "fill", "queue", "shrinks"):
            assert so[key] == sg[key], (j, key, so, sg)
    return rel_fro(gram(Bg), gram(Bo))


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_window_matches_oracle_through_time(fd):
    d, ell, N, R = 24, 8, 300, 8.0
    note(f"window {fd} d={d} ell={ell} N={N}")
    A = normed_rows(1000, d, R, seed=10)
    o = oracle.Window(d, ell, N, R, q=1, seed=3, stream=5, fd=fd)
    g = make(d, ell, N, R, fd, seed=3, stream=5)
    At = torch.from_numpy(A).cuda()
    for t0 in range(0, 1000, 250):
        o.update(A[t0:t0 + 250])
        g.update(At[t0:t0 + 250])
        assert compare(o, g, o.levels) <= 1e-9


def test_window_with_raw_rows_and_advance():
    d, ell, N, R = 20, 6, 40, 64.0
    A = normed_rows(400, d, R, seed=11)
    o = oracle.Window(d, ell, N, R, q=1, seed=1, stream=2)
    g = make(d, ell, N, R, "exact", seed=1, stream=2)
    o.update(A)
    g.update(torch.from_numpy(A).cuda())
    assert sum(o.stats(j)["raw"] for j in range(o.levels)) > 0
    assert compare(o, g, o.levels) <= 1e-9
    o.advance(420)
    g.advance(420)
    assert compare(o, g, o.levels) <= 1e-9


def test_window_without_dumps_equals_persistent_fd():
    d, ell = 32, 8
    A = synth.lowrank_rows(300, d, np.geomspace(2, 0.2, 10), 0.05, seed=1)
    g = make(d, ell, 10**9, 2.0, "exact")
    g.update(torch.from_numpy(A).cuda())
    assert g.window_stats(0)["dumps"] == 0
    fd = oracle.FD(d, ell)
    fd.update(A)
    assert rel_fro(gram(g.query()), gram(fd.query())) <= 1e-9


def test_window_large_d_uses_multiworkgroup_eigensolver():
    # d > 128: the d x d restore of the query is solved by the cooperative solver
    d, ell, N, R = 160, 8, 200, 4.0
    A = normed_rows(500, d, R, seed=12, rank=10)
    o = oracle.Window(d, ell, N, R, q=1, seed=4, stream=1, fd="rand")
    g = make(d, ell, N, R, "rand", seed=4, stream=1)
    o.update(A)
    g.update(torch.from_numpy(A).cuda())
    assert compare(o, g, o.levels) <= 1e-9


def test_window_rotating_subspace_stream():
    # the sliding-window workload's structure at a small size: geometric
    # spectrum over a rotating subspace, rows stored as FP32
    d, ell, N = 64, 8, 500
    A = synth.window_stream(1500, d=d, rank=16, period=400, seed=2).astype(np.float32)
    R = float(np.max(np.sum(A.astype(np.float64) ** 2, axis=1))) + 1.0
    o = oracle.Window(d, ell, N, R, q=1, seed=9, stream=3, fd="rand")
    g = make(d, ell, N, R, "rand", seed=9, stream=3)
    o.update(A.astype(np.float64))
    g.update(torch.from_numpy(A).cuda())
    assert compare(o, g, o.levels) <= 1e-9


def test_window_d512_ell32():
    # a larger window: d = 512, ell = 32, three levels, randomized FD reduce,
    # queried twice (the d x d restore runs on the cooperative eigen-solver)
    d, ell, N, R = 512, 32, 600, 8.0
    A = normed_rows(1200, d, R, seed=13, rank=12)
    note(f"window rand d={d} ell={ell} N={N}")
    o = oracle.Window(d, ell, N, R, q=1, seed=6, stream=2, fd="rand")
    g = make(d, ell, N, R, "rand", seed=6, stream=2)
    At = torch.from_numpy(A).cuda()
    for t0 in (0, 600):
        o.update(A[t0:t0 + 600])
        g.update(At[t0:t0 + 600])
        assert compare(o, g, o.levels) <= 1e-9
    assert sum(o.stats(j)["dumps"] for j in range(o.levels)) > 100
    g.close()


def test_window_advance_backwards_is_rejected():
    from paper_2601_02019_amd import SketchError
    g = make(8, 4, 10, 2.0, "exact")
    g.update(torch.ones(5, 8, dtype=torch.float64, device="cuda") * 0.1)
    from paper_2601_02019_amd import SK_EINVAL
    with pytest.raises(SketchError) as e:
        g.advance(3)
    assert e.value.code == SK_EINVAL
    assert g.info()["rows_seen"] == 5  # state unchanged
    g.close()
