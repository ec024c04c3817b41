"""GPU parity of the ATTP persistent sketch (Algorithm "ATTP Sketch using
AeroSketch") against the FP64 ATTP oracle, through the C ABI.

Every decision (power-iteration estimate against theta_i / 2, the doubling
loop, the number of dumped directions) is taken in FP64 on both sides from
the same Philox draws, so the counters agree exactly and the sketches of
past times agree to 1e-9 in relative Frobenius norm of B^T B.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gram, note, rel_fro

pytestmark = pytest.mark.gpu


def unit_rows(n, d, R, seed, rank=6):
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, rank), 0.05, seed=seed)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A * np.sqrt(rng.uniform(1.0, R, size=(n, 1)))


def growing_rows(n, d, seed):
    """Rows in random directions whose squared norms grow by 1.5 per row:
    most rows are dumped (many snapshots, the store grows)."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    return U * np.sqrt(1.5 ** np.arange(1, n + 1))[:, None]


def make(d, ell, fd, seed, stream):
    from paper_2601_02019_amd import Sketch
    return Sketch(d, ell, kind="attp", shrink=fd, q=1, seed=seed, stream_id=stream)


def compare(o, g, times):
    so, sg = o.stats(), g.window_stats(0)
    assert (so["snapshots"], so["dirs"], so["fill"], so["shrinks"]) == \
        (sg["dumps"], sg["dirs"], sg["fill"], sg["shrinks"]), (so, sg)
    worst = 0.0
    for t in times:
        Bo = o.query_at(t)
        Bg = g.query_at(t)
        Go = gram(Bo)
        if np.linalg.norm(Go) == 0:
            assert torch.count_nonzero(Bg) == 0
            continue
        worst = max(worst, rel_fro(gram(Bg), Go))
    return worst


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_attp_matches_oracle_at_past_times(fd):
    d, ell, n = 24, 8, 600
    A = unit_rows(n, d, 8.0, seed=31, rank=10)
    note(f"attp {fd} d={d} ell={ell} n={n}")
    o = oracle.ATTP(d, ell, q=1, seed=3, stream=2, fd=fd)
    g = make(d, ell, fd, 3, 2)
    At = torch.from_numpy(A).cuda()
    for t0 in (0, 250):
        o.update(A[t0:t0 + 250])
        g.update(At[t0:t0 + 250])
        assert compare(o, g, [0, 1, 17, 131, t0 + 250]) <= 1e-9
    o.update(A[500:])
    g.update(At[500:])
    assert compare(o, g, [1, 77, 249, 250, 433, 599, 600]) <= 1e-9
    g.close()


def test_attp_many_snapshots_grow_the_store():
    d, ell, n = 40, 8, 70
    A = growing_rows(n, d, seed=5)
    o = oracle.ATTP(d, ell, q=1, seed=1, stream=9, fd="rand")
    g = make(d, ell, "rand", 1, 9)
    o.update(A)
    g.update(torch.from_numpy(A).cuda())
    note(f"attp growing rows: {o.stats()}")
    assert o.stats()["dirs"] > 4 * ell   # beyond the store's first capacity
    assert compare(o, g, [1, 2, 10, 33, 50, 69, 70]) <= 1e-9
    g.close()


def test_attp_large_d_restore_on_the_cooperative_solver():
    d, ell, n = 160, 16, 400
    A = unit_rows(n, d, 8.0, seed=37, rank=10)
    o = oracle.ATTP(d, ell, q=1, seed=4, stream=1, fd="rand")
    g = make(d, ell, "rand", 4, 1)
    o.update(A)
    g.update(torch.from_numpy(A).cuda())
    assert compare(o, g, [100, 399, 400]) <= 1e-9
    g.close()


def test_attp_argument_errors():
    import paper_2601_02019_amd as sk
    g = make(8, 4, "exact", 0, 0)
    g.update(torch.ones(5, 8, dtype=torch.float64, device="cuda"))
    with pytest.raises(sk.SketchError) as e:
        g.query_at(6)
    assert e.value.code == sk.SK_EINVAL
    with pytest.raises(sk.SketchError) as e:
        g.advance(10)
    assert e.value.code == sk.SK_EUNSUPPORTED
    assert g.info()["rows_seen"] == 5
    # the current-time query equals sketch_query
    assert torch.equal(g.query_at(5), g.query())
    p = sk.Sketch(8, 4)
    with pytest.raises(sk.SketchError) as e:
        p.query_at(0)
    assert e.value.code == sk.SK_EUNSUPPORTED
    g.close()
    p.close()
