"""Pins of the sliding-window oracle (ML-AeroSketch) on the CPU.

What fixes each expected value:
  - with thresholds far above any row or sketch mass nothing is dumped or
    stored raw, so the level is plain FD (pinned separately);
  - the restore identity of the error analysis (the snapshot (Z, Z^T C'^T C')
    restores C'^T C' exactly) makes the restored Gram equal A^T A whenever
    no FD reduce has happened;
  - the query's shrink is f_ell of the restored Gram, whose spectral distance
    is max(|lambda_ell|, |lambda_d|) (proof of the window theorem);
  - the residual lemma ||C^T C||_2 <= 4 theta and the final window bound
    (25/2) eps ||A_W||_F^2 hold with high probability.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import cov_err, f_ell, rel_fro


def normed_rows(n, d, R, seed, rank=6):
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, rank), 0.05, seed=seed)
    nrm = np.linalg.norm(A, axis=1, keepdims=True)
    target = np.sqrt(rng.uniform(1.0, R, size=(n, 1)))
    return A / nrm * target


def test_window_without_dumps_is_plain_fd():
    d, ell, n = 20, 4, 150
    A = synth.lowrank_rows(n, d, np.geomspace(2, 0.2, 10), 0.05, seed=1)
    w = oracle.Window(d, ell, N=10**9, R=2.0, q=1)
    w.update(A)
    st = w.stats(0)
    assert st["dumps"] == 0 and st["raw"] == 0
    B, lvl = w.query()
    fd = oracle.FD(d, ell)
    fd.update(A)
    Bf = fd.query()
    assert lvl == 0
    assert rel_fro(B.T @ B, Bf.T @ Bf) < 1e-10


@pytest.mark.parametrize("q", [0, 1, 2])
def test_restore_identity_before_any_reduce(q):
    d, ell, N = 16, 8, 100
    rng = np.random.default_rng(q)
    base = rng.standard_normal(d)
    A = np.array([base * rng.uniform(0.8, 1.2) + 0.2 * rng.standard_normal(d) for _ in range(12)])
    A *= np.sqrt(3.0) / np.linalg.norm(A, axis=1, keepdims=True)
    w = oracle.Window(d, ell, N=N, R=4.0, q=q, seed=3)
    w.update(A)
    st = w.stats(0)
    assert st["shrinks"] == 0
    assert st["dumps"] >= 1, st   # the snapshot path ran
    for lvl in range(w.levels):
        G = w.level_gram(lvl)
        assert rel_fro(G, A.T @ A) < 1e-10


def test_query_shrink_identity_no_raw_rows():
    d, ell, N = 24, 6, 400
    A = normed_rows(600, d, R=4.0, seed=5)
    w = oracle.Window(d, ell, N=N, R=4.0, q=1, seed=1)
    w.update(A)
    B, lvl = w.query()
    assert w.stats(lvl)["raw"] == 0
    G = w.level_gram(lvl)
    assert rel_fro(B.T @ B, f_ell(G, ell)) < 1e-9
    lam = np.linalg.eigvalsh((G + G.T) / 2)[::-1]
    gap = np.max(np.abs(np.linalg.eigvalsh(G - B.T @ B)))
    assert abs(gap - max(abs(lam[ell - 1]), abs(lam[-1]))) < 1e-9 * abs(lam[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_window_error_bound_and_residual_lemma(seed):
    d, ell, N, R = 24, 8, 300, 8.0
    eps = 2.0 / ell
    A = normed_rows(1000, d, R=R, seed=10 + seed)
    w = oracle.Window(d, ell, N=N, R=R, q=1, seed=seed)
    for t0 in range(0, 1000, 100):
        w.update(A[t0:t0 + 100])
        T = t0 + 100
        AW = A[max(0, T - N):T]
        B, lvl = w.query()
        fa = np.linalg.norm(AW) ** 2
        assert cov_err(AW, B) <= 12.5 * eps * fa
        assert np.linalg.eigvalsh(B.T @ B).min() >= -1e-9 * fa


def test_advance_expires_snapshots_and_residual_is_bounded():
    d, ell, N, R = 20, 6, 200, 4.0
    A = normed_rows(700, d, R=R, seed=3)
    w = oracle.Window(d, ell, N=N, R=R, q=1, seed=2)
    w.update(A)
    w.advance(700 + N)
    for lvl in range(w.levels):
        st = w.stats(lvl)
        assert st["queue"] == 0
        G = w.level_gram(lvl)
        theta = 2 ** lvl * (2.0 / ell) * N
        # only the residual C remains; Lemma: ||C^T C||_2 <= 4 theta
        assert np.max(np.linalg.eigvalsh(G)) <= 4 * theta


def test_advance_backwards_is_rejected():
    w = oracle.Window(8, 4, N=10, R=2.0)
    w.update(np.ones((5, 8)) * 0.1)
    with pytest.raises(RuntimeError):
        w.advance(3)
