"""GPU parity of the P5 sketch (continuous distributed tracking, Algorithm
"P5") against the FP64 P5 oracle, through the C ABI.

The counter protocol is decided in FP64 on both sides from the rows' squared
norms, and each site's decisions (power-iteration estimate against
theta / 2, the doubling loop, the dumped directions) from the same Philox
draws, so every counter agrees exactly; the coordinator's Fhat agrees to
1e-12 and its B, and the query's B^T B, to 1e-9 in relative Frobenius norm.
The GPU runs the sites' steps in lockstep; the oracle takes the rows one at
a time.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import gram, note, rel_fro

pytestmark = pytest.mark.gpu

SITE_KEYS = [("dumps", "snapshots"), ("raw", "raw"), ("dirs", "dirs"), ("fill", "fill"), ("shrinks", "shrinks")]


def stream(n, d, seed, rank=10, lo=0.5, hi=2.0):
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, rank), 0.05, seed=seed)
    return A * np.sqrt(rng.uniform(lo, hi, size=(n, 1)))


def sites_of(n, m, seed):
    return np.random.default_rng(seed + 7).integers(0, m, size=n).astype(np.int32)


def make(d, ell, m, fd, seed, stream_id, amplify=(1, 0)):
    from paper_2601_02019_amd import Sketch
    return Sketch(d, ell, kind="p5", shrink=fd, q=1, seed=seed, stream_id=stream_id, sites=m, amplify=amplify)


def compare(o, g, m):
    so, sg = o.stats(), g.p5_stats()
    assert so == sg, (so, sg)
    for j in range(m):
        a, b = o.site(j), g.window_stats(j)
        for kg, ko in SITE_KEYS:
            assert b[kg] == a[ko], (j, kg, a, b)
    fo = o.fhat
    fg, Bg = g.p5_coordinator()
    assert abs(fg - fo) <= 1e-12 * fo
    Bo = o.gram()
    worst = rel_fro(Bg.cpu().numpy(), Bo)
    worst = max(worst, rel_fro(gram(g.query()), gram(o.query())))
    return worst


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_p5_matches_oracle(fd):
    d, ell, m, n = 32, 8, 4, 900
    note(f"p5 {fd} d={d} ell={ell} m={m} n={n}")
    A = stream(n, d, seed=1)
    S = sites_of(n, m, 1)
    o = oracle.P5(d, ell, m, q=1, seed=2, stream=3, fd=fd)
    g = make(d, ell, m, fd, 2, 3)
    At = torch.from_numpy(A).cuda()
    for a, b in [(0, 1), (1, 250), (250, 251), (251, 900)]:
        o.update(A[a:b], S[a:b])
        g.p5_update(At[a:b], S[a:b])
        assert compare(o, g, m) <= 1e-9
    st = o.stats()
    assert st["raw"] == m - 1 and st["snapshots"] > 10 and st["shrinks"] > 10 and st["broadcasts"] > 5
    g.close()


def test_p5_many_sites_larger_d_fp32_rows():
    # d = 160: the query's d x d eigen-solve runs on the cooperative solver;
    # rows stored as FP32 on the device (the oracle gets the same values)
    d, ell, m, n = 160, 16, 12, 2400
    note(f"p5 rand d={d} ell={ell} m={m} n={n}")
    A = stream(n, d, seed=4, rank=24).astype(np.float32)
    S = sites_of(n, m, 4)
    o = oracle.P5(d, ell, m, q=1, seed=7, stream=1, fd="rand")
    g = make(d, ell, m, "rand", 7, 1)
    o.update(A.astype(np.float64), S)
    g.p5_update(torch.from_numpy(A).cuda(), S)
    assert compare(o, g, m) <= 1e-9
    assert o.stats()["snapshots"] > 20
    g.close()


def test_p5_skewed_sites_and_zero_rows():
    # one site takes most rows (long lockstep tail), some rows are zero
    d, ell, m, n = 24, 6, 5, 700
    A = stream(n, d, seed=6)
    rng = np.random.default_rng(6)
    A[rng.random(n) < 0.05] = 0.0
    A[:3] = 0.0  # zero rows before the first broadcast send nothing
    S = np.where(rng.random(n) < 0.7, 2, rng.integers(0, m, size=n)).astype(np.int32)
    o = oracle.P5(d, ell, m, q=1, seed=1, stream=9, fd="exact")
    g = make(d, ell, m, "exact", 1, 9)
    o.update(A, S)
    g.p5_update(torch.from_numpy(A).cuda(), S)
    assert compare(o, g, m) <= 1e-9
    g.close()


def test_p5_with_amplification():
    d, ell, m, n = 32, 8, 3, 600
    A = stream(n, d, seed=9)
    S = sites_of(n, m, 9)
    o = oracle.P5(d, ell, m, q=1, seed=5, stream=2, fd="rand", amplify=(3, 2))
    g = make(d, ell, m, "rand", 5, 2, amplify=(3, 2))
    o.update(A, S)
    g.p5_update(torch.from_numpy(A).cuda(), S)
    assert compare(o, g, m) <= 1e-9
    assert o.stats()["snapshots"] > 0
    g.close()


def test_p5_argument_errors_leave_the_state_unchanged():
    import paper_2601_02019_amd as sk
    d, ell, m = 16, 4, 3
    g = make(d, ell, m, "exact", 0, 0)
    A = torch.from_numpy(stream(50, d, seed=3)).cuda()
    g.p5_update(A, sites_of(50, m, 3))
    before = g.p5_stats()
    with pytest.raises(sk.SketchError) as e:
        g.p5_update(A[:2], np.array([0, 3], dtype=np.int32))
    assert e.value.code == sk.SK_EINVAL
    with pytest.raises(sk.SketchError) as e:
        g.update(A[:2])
    assert e.value.code == sk.SK_EUNSUPPORTED
    with pytest.raises(sk.SketchError) as e:
        g.query_at(10)
    assert e.value.code == sk.SK_EUNSUPPORTED
    assert g.p5_stats() == before
    p = sk.Sketch(d, ell)
    with pytest.raises(sk.SketchError) as e:
        p.p5_update(A[:1], [0])
    assert e.value.code == sk.SK_EUNSUPPORTED
    g.close()
    p.close()
