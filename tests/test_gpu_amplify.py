"""GPU parity of the probability amplification of the dump step (Algorithm
"Probability Amplification" in place of the simul_iter call of Algorithm
"AeroSketch: Update") against the FP64 oracle, through the C ABI.

Candidate h of a doubling step draws its test matrix from its own Philox
counters and every power iteration on a candidate's residual from its own
start vector, on both sides; the estimates are compared in FP64, so the kept
candidates, hence the decision traces, agree (per-level counters) and the
queried sketches agree to 1e-9 in relative Frobenius norm of B^T B.  With a
single candidate the amplified step is the plain step, bit for bit.
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


def window(d, ell, N, R, fd, seed, stream, amplify):
    from paper_2601_02019_amd import Sketch
    return Sketch(d, ell, kind="window", shrink=fd, window_N=N, R=R, q=1, seed=seed, stream_id=stream,
                  amplify=amplify)


def attp(d, ell, fd, seed, stream, amplify):
    from paper_2601_02019_amd import Sketch
    return Sketch(d, ell, kind="attp", shrink=fd, q=1, seed=seed, stream_id=stream, amplify=amplify)


def compare_window(o, g):
    Bo, _ = o.query()
    Bg = g.query()
    for j in range(o.levels):
        so, sg = o.stats(j), g.window_stats(j)
        for key in ("dumps", "raw", "dirs", "fill", "queue", "shrinks"):
            assert so[key] == sg[key], (j, key, so, sg)
    return rel_fro(gram(Bg), gram(Bo))


@pytest.mark.parametrize("fd,amp", [("exact", (2, 3)), ("rand", (3, 2)), ("exact", (2, 0))])
def test_amplified_window_matches_oracle(fd, amp):
    d, ell, N, R = 24, 8, 300, 8.0
    note(f"amplified window {fd} amplify={amp} d={d} ell={ell} N={N}")
    A = normed_rows(900, d, R, seed=21)
    o = oracle.Window(d, ell, N, R, q=1, seed=3, stream=5, fd=fd, amplify=amp)
    g = window(d, ell, N, R, fd, 3, 5, amp)
    At = torch.from_numpy(A).cuda()
    for t0 in range(0, 900, 300):
        o.update(A[t0:t0 + 300])
        g.update(At[t0:t0 + 300])
        assert compare_window(o, g) <= 1e-9
    assert sum(o.stats(j)["dumps"] for j in range(o.levels)) > 0
    g.close()


def test_one_candidate_is_the_plain_window_bit_for_bit():
    d, ell, N, R = 32, 8, 250, 8.0
    A = torch.from_numpy(normed_rows(700, d, R, seed=22)).cuda()
    plain = window(d, ell, N, R, "exact", 1, 2, (1, 0))
    amp = window(d, ell, N, R, "exact", 1, 2, (1, 3))
    plain.update(A)
    amp.update(A)
    assert sum(plain.window_stats(j)["dumps"] for j in range(plain.info()["levels"])) > 0
    assert torch.equal(plain.query(), amp.query())
    plain.close()
    amp.close()


def test_amplified_window_rotating_subspace_larger_d():
    # d = 160: the residual power iterations span several slabs and the
    # candidates' eigen-solves and the query restore run on the cooperative solver
    d, ell, N = 160, 16, 400
    A = synth.window_stream(1000, d=d, rank=16, period=300, seed=4, dtype=np.float64)
    R = float(np.max(np.sum(A ** 2, axis=1))) + 1.0
    note(f"amplified window rand amplify=(4, 2) d={d} ell={ell} N={N}")
    o = oracle.Window(d, ell, N, R, q=1, seed=8, stream=1, fd="rand", amplify=(4, 2))
    g = window(d, ell, N, R, "rand", 8, 1, (4, 2))
    o.update(A)
    g.update(torch.from_numpy(A).cuda())
    assert compare_window(o, g) <= 1e-9
    g.close()


def test_amplified_attp_matches_oracle_at_past_times():
    d, ell, n = 24, 8, 500
    rng = np.random.default_rng(31)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, 10), 0.05, seed=31)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    A *= np.sqrt(rng.uniform(1.0, 8.0, size=(n, 1)))
    o = oracle.ATTP(d, ell, q=1, seed=3, stream=2, fd="rand", amplify=(3, 3))
    g = attp(d, ell, "rand", 3, 2, (3, 3))
    o.update(A)
    g.update(torch.from_numpy(A).cuda())
    so, sg = o.stats(), g.window_stats(0)
    assert (so["snapshots"], so["dirs"], so["fill"], so["shrinks"]) == \
        (sg["dumps"], sg["dirs"], sg["fill"], sg["shrinks"]), (so, sg)
    assert so["snapshots"] > 0
    for t in [1, 50, 199, 333, 500]:
        Go = gram(o.query_at(t))
        Bg = g.query_at(t)
        if np.linalg.norm(Go) == 0:
            assert torch.count_nonzero(Bg) == 0
        else:
            assert rel_fro(gram(Bg), Go) <= 1e-9, t
    g.close()


def test_amplification_rejected_for_persistent_sketches():
    import paper_2601_02019_amd as sk
    with pytest.raises(sk.SketchError) as e:
        sk.Sketch(8, 4, amplify=(2, 1))
    assert e.value.code == sk.SK_EINVAL
