"""GPU parity of the approximate-matrix-multiplication window (Algorithm
"AeroSketchCOD Framework") against the FP64 COD oracle, through the C ABI.

Every decision (power-iteration estimate against theta / 2, the doubling
loop, the directions dumped, expiry) is taken in FP64 on both sides from the
same Philox draws, so the counters agree exactly; the restored product M_W
and the query's A* B*^T agree to 1e-9 in relative Frobenius norm.  The GPU
computes the reduce and the power iteration in the buffers' row space and
every product with M = A^T B through A and B; the oracle forms M.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import note, rel_fro

pytestmark = pytest.mark.gpu


def pairs(n, dx, dy, seed, kind="uniform", rank=6):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return 1.0 - rng.random((n, dx)), 1.0 - rng.random((n, dy))
    G = rng.standard_normal((n, rank))
    X = G @ rng.standard_normal((rank, dx)) + 0.05 * rng.standard_normal((n, dx))
    Y = G @ rng.standard_normal((rank, dy)) + 0.05 * rng.standard_normal((n, dy))
    return X, Y


def make(dx, dy, ell, N, theta, seed=0, stream=0, q=1):
    from paper_2601_02019_amd import Sketch
    return Sketch(dx, ell, kind="cod", window_N=N, q=q, seed=seed, stream_id=stream, d_y=dy, theta=theta)


def compare(o, g):
    so, sg = o.stats(), g.window_stats(0)
    assert (so["snapshots"], so["dirs"], so["fill"], so["queue"], so["reduces"]) == \
        (sg["dumps"], sg["dirs"], sg["fill"], sg["queue"], sg["shrinks"]), (so, sg)
    Mo = o.product()
    err = rel_fro(g.cod_product().cpu().numpy(), Mo)
    Ao, Bo = o.query()
    Ag, Bg = g.cod_query()
    Po = Ao @ Bo.T
    err = max(err, rel_fro((Ag @ Bg.T).cpu().numpy(), Po))
    return err


@pytest.mark.parametrize("blocks", [[200], [1, 59, 60, 80]])
def test_cod_uniform_matches_oracle(blocks):
    dx, dy, ell, N, theta = 12, 16, 4, 60, 20.0
    X, Y = pairs(sum(blocks), dx, dy, seed=0)
    note(f"cod uniform dx={dx} dy={dy} ell={ell} N={N} blocks={blocks}")
    o = oracle.COD(dx, dy, ell, N=N, theta=theta, q=1, seed=1, stream=2)
    g = make(dx, dy, ell, N, theta, seed=1, stream=2)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    t0 = 0
    for b in blocks:
        o.update(X[t0:t0 + b], Y[t0:t0 + b])
        g.cod_update(Xt[t0:t0 + b], Yt[t0:t0 + b])
        t0 += b
        assert compare(o, g) <= 1e-9
    assert o.stats()["snapshots"] > 10 and o.stats()["reduces"] > 10
    g.close()


def test_cod_lowrank_larger_dims_fp32_rows():
    dx, dy, ell, N, n = 40, 24, 8, 200, 700
    X, Y = pairs(n, dx, dy, seed=5, kind="lowrank", rank=10)
    X, Y = X.astype(np.float32), Y.astype(np.float32)
    fro = np.sqrt(np.sum(X.astype(np.float64) ** 2, 1) * np.sum(Y.astype(np.float64) ** 2, 1))
    theta = (2.0 / ell) * N * float(np.median(fro))
    note(f"cod lowrank dx={dx} dy={dy} ell={ell} N={N} theta={theta:.3g}")
    o = oracle.COD(dx, dy, ell, N=N, theta=theta, q=1, seed=3, stream=7)
    g = make(dx, dy, ell, N, theta, seed=3, stream=7)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    for t0 in range(0, n, 175):
        o.update(X[t0:t0 + 175].astype(np.float64), Y[t0:t0 + 175].astype(np.float64))
        g.cod_update(Xt[t0:t0 + 175], Yt[t0:t0 + 175])
        assert compare(o, g) <= 1e-9
    assert o.stats()["snapshots"] > 0
    g.close()


def test_cod_without_dumps_and_small_dx():
    # dx = 3 < ell: the reduce keeps the whole product; theta out of reach
    dx, dy, ell, N, n = 3, 20, 6, 10 ** 6, 150
    X, Y = pairs(n, dx, dy, seed=9)
    o = oracle.COD(dx, dy, ell, N=N, theta=1e12, q=1, seed=0, stream=0)
    g = make(dx, dy, ell, N, 1e12)
    o.update(X, Y)
    g.cod_update(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda())
    assert compare(o, g) <= 1e-9
    assert o.stats()["snapshots"] == 0 and o.stats()["reduces"] > 5
    g.close()


def test_cod_host_inputs_and_errors():
    import paper_2601_02019_amd as sk
    dx, dy, ell, N, theta = 10, 8, 4, 40, 10.0
    X, Y = pairs(90, dx, dy, seed=2)
    o = oracle.COD(dx, dy, ell, N=N, theta=theta)
    g = make(dx, dy, ell, N, theta)
    o.update(X, Y)
    g.cod_update(X, Y)  # host numpy arrays: staged by the library
    assert compare(o, g) <= 1e-9
    with pytest.raises(sk.SketchError) as e:
        g.update(torch.from_numpy(X).cuda())
    assert e.value.code == sk.SK_EUNSUPPORTED
    with pytest.raises(sk.SketchError) as e:
        g.query()
    assert e.value.code == sk.SK_EUNSUPPORTED
    p = sk.Sketch(dx, ell)
    with pytest.raises(sk.SketchError) as e:
        p.cod_update(X[:2], Y[:2])
    assert e.value.code == sk.SK_EUNSUPPORTED
    g.close()
    p.close()
