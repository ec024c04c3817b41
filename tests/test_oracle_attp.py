"""Pins of the ATTP oracle (Algorithm "ATTP Sketch using AeroSketch").

Each expected value comes from the paper or from exact arithmetic, never from
the oracle itself:

  - the threshold schedule theta_i = eps ||A_i||_F^2 with eps = 2 / ell
    (closed form over the rows);
  - before the first FD reduce no mass is lost: the restored matrix of the
    current time is exactly A^T A (the restore identity of Algorithm
    "AeroSketch: Query" plus the residual);
  - a stream along one direction with growing weights dumps every row
    whole, so the sketch of EVERY time t is exactly A_t^T A_t (this
    separates "timestamp <= t" from "< t" in the historical query);
  - history does not change: the sketch of time t is the same when queried
    at any later time, and equals the snapshot part of a second sketch fed
    only the first t rows;
  - each update without an FD reduce removes either nothing or at least
    xi theta_i from the residual (every dumped direction carries at least
    theta of C'^T C'; appendix, proof of Theorem "ATTP", space analysis);
  - the space bound sum xi <= (2 / eps) log(2 ||A_T||_F^2 / eps) for rows
    with ||a_1||^2 >= 1 (same proof);
  - the restored matrix never exceeds A_t^T A_t in the PSD order, and the
    historical error stays within (1/ell + 4 eps) ||A_t||_F^2 (Term 1 +
    Term 2 of the proof) plus the final shrink's lambda_ell;
  - the final shrink leaves the spectral error max(|lambda_ell|,
    |lambda_d|) of the restored matrix (query-shrink identity).
"""
import numpy as np
import pytest

import oracle
import synth


def unit_rows(n, d, R, seed, rank=6):
    """Low-rank rows rescaled to squared norms in [1, R]."""
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, rank), 0.05, seed=seed)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A * np.sqrt(rng.uniform(1.0, R, size=(n, 1)))


def rel(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))


def test_theta_follows_the_stream_norm():
    d, ell = 12, 6
    A = unit_rows(40, d, 9.0, seed=1)
    a = oracle.ATTP(d, ell)
    for i in range(40):
        a.update(A[i:i + 1])
        expect = (2.0 / ell) * float(np.sum(A[:i + 1] ** 2))
        assert abs(a.theta - expect) <= 1e-14 * expect


def test_no_loss_before_the_first_reduce():
    d, ell = 14, 8
    A = unit_rows(2 * ell - 1, d, 16.0, seed=2, rank=9)
    a = oracle.ATTP(d, ell, q=1, seed=3, stream=1)
    for i in range(A.shape[0]):
        a.update(A[i:i + 1])
        At = A[:i + 1]
        assert rel(a.gram_at(i + 1), At.T @ At) <= 1e-12
    assert a.stats()["shrinks"] == 0
    assert a.stats()["snapshots"] > 0


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_one_direction_is_exact_at_every_time(fd):
    # a_i = c_i e with c_i^2 = 1.5^i: each row carries about a third of
    # ||A_i||_F^2, more than theta_i = ||A_i||_F^2 / 4 at ell = 8, so every
    # row is dumped whole and every past time is restored exactly
    d, ell, n = 10, 8, 40
    rng = np.random.default_rng(5)
    e = rng.standard_normal(d)
    e /= np.linalg.norm(e)
    A = np.sqrt(1.5 ** np.arange(1, n + 1))[:, None] * e[None, :]
    a = oracle.ATTP(d, ell, q=1, seed=1, stream=4, fd=fd)
    a.update(A)
    assert a.stats()["snapshots"] == n
    for t in range(0, n + 1):
        At = A[:t]
        G = a.gram_at(t)
        ref = At.T @ At
        if t == 0:
            assert np.count_nonzero(G) == 0
            continue
        assert rel(G, ref) <= 1e-10, t
        B = a.query_at(t)
        assert rel(B.T @ B, ref) <= 1e-10, t


def test_history_does_not_change_and_matches_a_shorter_stream():
    d, ell, n, t = 16, 4, 300, 137
    A = unit_rows(n, d, 8.0, seed=7)
    full = oracle.ATTP(d, ell, q=1, seed=2, stream=3)
    full.update(A[:200])
    G200 = full.gram_at(t)
    full.update(A[200:])
    assert np.array_equal(full.gram_at(t), G200)
    short = oracle.ATTP(d, ell, q=1, seed=2, stream=3)
    short.update(A[:t])
    C = short.buffer()
    assert rel(full.gram_at(t), short.gram_at(t) - C.T @ C) <= 1e-12
    snaps_full = [s for s in full.snapshots() if s["t"] <= t]
    snaps_short = short.snapshots()
    assert [(s["xi"], s["s"], s["t"]) for s in snaps_full] == [(s["xi"], s["s"], s["t"]) for s in snaps_short]


def test_dumps_remove_at_least_xi_theta():
    d, ell, n = 16, 8, 150
    A = unit_rows(n, d, 6.0, seed=11, rank=5)
    a = oracle.ATTP(d, ell, q=1, seed=9, stream=2)
    prev_C = np.zeros((0, d))
    seen_dump = 0
    for i in range(n):
        st0 = a.stats()
        a.update(A[i:i + 1])
        st1 = a.stats()
        C = a.buffer()
        if st1["shrinks"] == st0["shrinks"]:
            before = float(np.sum(prev_C ** 2)) + float(np.sum(A[i] ** 2))
            removed = before - float(np.sum(C ** 2))
            if st1["snapshots"] == st0["snapshots"]:
                assert abs(removed) <= 1e-10 * before
            else:
                xi = a.snapshots()[-1]["xi"]
                assert removed >= xi * a.theta * (1 - 1e-9)
                seen_dump += 1
        prev_C = C
    assert seen_dump > 5


def test_space_bound():
    d, ell, n = 24, 8, 1500
    A = unit_rows(n, d, 10.0, seed=13, rank=12)
    a = oracle.ATTP(d, ell, q=1, seed=4, stream=6)
    a.update(A)
    eps = 2.0 / ell
    fro2 = float(np.sum(A ** 2))
    dirs = a.stats()["dirs"]
    assert 0 < dirs <= (2.0 / eps) * np.log(2.0 * fro2 / eps)


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_psd_order_and_historical_error_bound(fd):
    d, ell, n = 48, 32, 1500
    A = unit_rows(n, d, 4.0, seed=17, rank=20)
    a = oracle.ATTP(d, ell, q=1, seed=5, stream=7, fd=fd)
    a.update(A)
    assert a.stats()["shrinks"] > 10
    eps = 2.0 / ell
    for t in (50, 300, 777, 1200, n):
        At = A[:t]
        AtA = At.T @ At
        fro2 = float(np.trace(AtA))
        G = a.gram_at(t)
        lam = np.linalg.eigvalsh(AtA - (G + G.T) / 2)
        assert lam.min() >= -1e-9 * fro2, t
        assert lam.max() <= (1.0 / ell + 4 * eps) * fro2, t
        B = a.query_at(t)
        err = np.abs(np.linalg.eigvalsh(AtA - B.T @ B)).max()
        lg = np.linalg.eigvalsh((G + G.T) / 2)[::-1]
        assert err <= (1.0 / ell + 4 * eps) * fro2 + max(lg[ell - 1], 0.0) + 1e-9 * fro2, t
        assert err <= 10.0 / ell * fro2


def test_query_shrink_identity():
    d, ell = 20, 6
    A = unit_rows(400, d, 5.0, seed=19, rank=14)
    a = oracle.ATTP(d, ell, q=1, seed=8, stream=1)
    a.update(A)
    for t in (120, 400):
        G = a.gram_at(t)
        G = (G + G.T) / 2
        lam = np.linalg.eigvalsh(G)[::-1]
        B = a.query_at(t)
        gap = np.abs(np.linalg.eigvalsh(G - B.T @ B)).max()
        assert abs(gap - max(abs(lam[ell - 1]), abs(lam[-1]))) <= 1e-9 * abs(lam[0])


def test_bad_times_are_rejected():
    a = oracle.ATTP(6, 3)
    a.update(np.ones((4, 6)))
    with pytest.raises(RuntimeError):
        a.gram_at(5)
    with pytest.raises(RuntimeError):
        a.query_at(-1)


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_reduce_then_dump_is_the_composition_of_the_keyed_steps(fd):
    # the row that fills the buffer: FD reduce (exact, or the persistent
    # randomized shrink keyed (seed, 64 stream + 1) with shrink count 0),
    # rows ell - 1 .. 2 ell - 1 zeroed, then the dump step at theta_i with the
    # level-0 counters, composed here by hand from the oracle's own steps
    d, ell, seed, stream = 18, 5, 6, 3
    A = unit_rows(2 * ell, d, 3.0, seed=23, rank=12)
    a = oracle.ATTP(d, ell, q=1, seed=seed, stream=stream, fd=fd)
    a.update(A[:-1])
    Cprev = a.buffer()
    ns = a.stats()["snapshots"]
    a.update(A[-1:])
    X = np.vstack([Cprev, A[-1:]])
    if fd == "exact":
        X = oracle.shrink_exact(X, ell)
    else:
        X = oracle.shrink_rand(X, ell, ell, 1, seed, stream * 64 + 1, 0)
    X = X[: ell - 1]
    theta = (2.0 / ell) * float(np.sum(A ** 2))
    out = oracle.aero_dump(X, theta, ell=ell, q=1, seed=seed, stream=stream, level=0, i=2 * ell)
    assert np.allclose(a.buffer(), out["C"], rtol=0, atol=1e-12 * np.abs(X).max())
    assert a.stats()["snapshots"] == ns + (1 if out["xi"] > 0 else 0)
