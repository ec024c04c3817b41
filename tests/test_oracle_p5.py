"""Pins of the P5 oracle (continuous distributed tracking, Algorithm "P5",
Sec. 4.3; Theorem "dist" and its proof in the appendix).

Every expected value comes from what the algorithm and the mathematics fix,
never from the oracle's own output:

  - the protocol conserves mass: Fhat plus every site's unsent counter is
    ||A||_F^2; the coordinator broadcasts exactly at every m-th counter
    message; every site holds the last broadcast value; a site's counter
    stays below (eps / m) of it (or is zero) after every row;
  - between two broadcasts Fhat grows by a factor >= 1 + eps (the proof's
    round argument), which bounds the number of broadcasts by
    1 + log_{1+eps}(||A||_F^2 / Fhat_1);
  - the coordinator's B and the sites' residuals decompose A^T A up to the FD
    reduces' losses: with the exact shrink, A^T A - B - sum_j C_j^T C_j is
    positive semidefinite with norm <= ||A||_F^2 / ell (the restore of a
    snapshot is exact);
  - Theorem "dist": ||A^T A - B||_2 <= eps ||A||_F^2; each site's residual
    satisfies ||C_j||_2^2 <= 4 theta_j; the query adds at most lambda_ell(B);
  - one site on a stream whose every row sends its counter is the ATTP
    sketch keyed (seed, 4096 stream): the same decisions, and B is ATTP's
    restored matrix without the residual;
  - before the first broadcast the rows reach the coordinator as they are.
"""
import numpy as np
import pytest

import oracle
import synth


def stream(n, d, seed, rank=10, lo=0.5, hi=2.0):
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.geomspace(3, 0.3, rank), 0.05, seed=seed)
    return A * np.sqrt(rng.uniform(lo, hi, size=(n, 1)))


def sites_of(n, m, seed):
    return np.random.default_rng(seed + 7).integers(0, m, size=n).astype(np.int32)


def test_protocol_conserves_mass_and_broadcasts_every_m_messages():
    d, ell, m, n = 16, 6, 5, 400
    A = stream(n, d, seed=1, lo=0.01, hi=5.0)
    S = sites_of(n, m, 1)
    p = oracle.P5(d, ell, m, q=1, seed=2, stream=3)
    eps = 2.0 / ell
    total = 0.0
    for e in range(n):
        p.update(A[e:e + 1], S[e:e + 1])
        total += float(A[e] @ A[e])
        st = p.stats()
        sites = [p.site(j) for j in range(m)]
        unsent = sum(s["F"] for s in sites)
        assert abs(p.fhat + unsent - total) <= 1e-12 * total
        assert st["broadcasts"] == st["fmsgs"] // m
        views = {s["Fhat"] for s in sites}
        assert len(views) == 1
        (view,) = views
        assert view <= p.fhat
        if st["broadcasts"] == 0:
            assert view == 0.0
        for s in sites:
            assert s["F"] == 0.0 or s["F"] < (eps / m) * s["Fhat"]
            assert s["theta"] == (eps / m) * s["Fhat"]
    st = p.stats()
    assert st["T"] == n and st["broadcasts"] > 3
    assert st["words"] == st["fmsgs"] + m * st["broadcasts"] + d * st["raw"] + 2 * d * st["dirs"]


def test_fhat_grows_by_one_plus_eps_per_round():
    d, ell, m, n = 12, 4, 3, 600
    A = stream(n, d, seed=2, lo=0.1, hi=3.0)
    S = sites_of(n, m, 2)
    p = oracle.P5(d, ell, m, q=0, seed=1, stream=1)
    eps = 2.0 / ell
    seen = []
    for e in range(n):
        before = p.stats()["broadcasts"]
        p.update(A[e:e + 1], S[e:e + 1])
        if p.stats()["broadcasts"] > before:
            seen.append(p.fhat)
    assert len(seen) >= 5
    for a, b in zip(seen, seen[1:]):
        assert b >= (1 + eps) * a * (1 - 1e-12)
    total = float(np.sum(A ** 2))
    assert len(seen) <= 1 + np.log(total / seen[0]) / np.log(1 + eps) + 1e-9
    assert p.stats()["fmsgs"] <= m * (len(seen) + 1)


@pytest.mark.parametrize("seed", range(3))
def test_coordinator_and_residuals_decompose_the_gram(seed):
    d, ell, m, n = 24, 6, 4, 500
    A = stream(n, d, seed=10 + seed)
    S = sites_of(n, m, seed)
    p = oracle.P5(d, ell, m, q=1, seed=seed, stream=2, fd="exact")
    p.update(A, S)
    total = float(np.sum(A ** 2))
    CC = sum(p.site(j)["C"].T @ p.site(j)["C"] for j in range(m))
    D = A.T @ A - p.gram() - CC
    w = np.linalg.eigvalsh((D + D.T) / 2)
    assert w.min() >= -1e-10 * total
    assert w.max() <= total / ell * (1 + 1e-12)
    assert p.stats()["shrinks"] > 0 and p.stats()["dirs"] > 0


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_theorem_error_bound_and_residual_thresholds(fd):
    d, ell, m, n = 32, 8, 4, 800
    A = stream(n, d, seed=5)
    S = sites_of(n, m, 5)
    p = oracle.P5(d, ell, m, q=1, seed=4, stream=6, fd=fd)
    p.update(A, S)
    eps = 2.0 / ell
    total = float(np.sum(A ** 2))
    AtA = A.T @ A
    B = p.gram()
    assert np.linalg.norm(AtA - B, 2) <= eps * total
    for j in range(m):
        s = p.site(j)
        if s["fill"]:
            assert np.linalg.norm(s["C"], 2) ** 2 <= 4 * s["theta"]
    Q = p.query()
    lam = np.linalg.eigvalsh(B)[::-1]
    assert np.linalg.norm(B - Q.T @ Q, 2) <= lam[ell - 1] * (1 + 1e-9) + 1e-12 * total
    assert np.linalg.norm(AtA - Q.T @ Q, 2) <= (eps + 1.0 / ell) * total


def test_query_is_the_shrunk_eigendecomposition_of_b():
    d, ell, m, n = 20, 5, 3, 300
    A = stream(n, d, seed=8)
    p = oracle.P5(d, ell, m, q=1, seed=1, stream=1)
    p.update(A, sites_of(n, m, 8))
    B = p.gram()
    lam, V = np.linalg.eigh((B + B.T) / 2)
    lam, V = lam[::-1], V[:, ::-1]
    keep = np.maximum(lam[:ell] - lam[ell - 1], 0.0)
    G = (V[:, :ell] * keep) @ V[:, :ell].T
    Q = p.query()
    assert np.linalg.norm(Q.T @ Q - G) <= 1e-10 * np.linalg.norm(B)


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_one_site_with_every_counter_sent_is_attp(fd):
    # squared norms grow by 1.5 per row: |a_i|^2 >= eps * ||A_{i-1}||_F^2, so
    # every row sends its counter and theta follows eps ||A_i||_F^2 exactly
    d, ell, n = 24, 8, 90
    rng = np.random.default_rng(3)
    U = rng.standard_normal((n, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    A = U * np.sqrt(1.5 ** np.arange(n))[:, None]
    p = oracle.P5(d, ell, 1, q=1, seed=5, stream=2, fd=fd)
    a = oracle.ATTP(d, ell, q=1, seed=5, stream=2 * 4096, fd=fd)
    p.update(A, np.zeros(n, dtype=np.int32))
    a.update(A)
    st, sa, s0 = p.stats(), a.stats(), p.site(0)
    assert st["fmsgs"] == n and st["broadcasts"] == n and st["raw"] == 0
    assert (s0["snapshots"], s0["dirs"], s0["fill"], s0["shrinks"], s0["simul_iters"]) == \
        (sa["snapshots"], sa["dirs"], sa["fill"], sa["shrinks"], sa["simul_iters"])
    assert sa["snapshots"] > 5
    C = a.buffer()
    G = a.gram_at(n) - C.T @ C
    assert np.linalg.norm(p.gram() - G) <= 1e-12 * np.linalg.norm(G)
    assert np.array_equal(s0["C"], C)


def test_rows_before_the_first_broadcast_arrive_as_they_are():
    d, ell, m = 10, 4, 6
    A = stream(40, d, seed=9)
    S = sites_of(40, m, 9)
    p = oracle.P5(d, ell, m, q=1, seed=0, stream=0)
    p.update(A[:m - 1], S[:m - 1])
    st = p.stats()
    assert st["raw"] == m - 1 and st["broadcasts"] == 0 and st["snapshots"] == 0
    G = A[:m - 1].T @ A[:m - 1]
    assert np.linalg.norm(p.gram() - G) <= 1e-14 * np.linalg.norm(G)
    assert all(p.site(j)["fill"] == 0 for j in range(m))
    p.update(A[m - 1:], S[m - 1:])
    assert p.stats()["raw"] == m - 1 and p.stats()["broadcasts"] >= 1


def test_amplification_with_one_candidate_is_the_plain_protocol():
    d, ell, m, n = 16, 6, 3, 300
    A = stream(n, d, seed=12)
    S = sites_of(n, m, 12)
    p0 = oracle.P5(d, ell, m, q=1, seed=3, stream=3, fd="rand")
    p1 = oracle.P5(d, ell, m, q=1, seed=3, stream=3, fd="rand", amplify=(1, 2))
    p0.update(A, S)
    p1.update(A, S)
    assert p0.stats() == p1.stats() and p0.stats()["dirs"] > 0
    assert np.array_equal(p0.gram(), p1.gram())


def test_bad_parameters_are_rejected():
    with pytest.raises(ValueError):
        oracle.P5(8, 4, 0)
    with pytest.raises(ValueError):
        oracle.P5(8, 4, 4097)
    with pytest.raises(ValueError):
        oracle.P5(8, 4, 2, amplify=(0, 1))
    p = oracle.P5(8, 4, 2)
    with pytest.raises(Exception):
        p.update(np.ones((2, 8)), np.array([0, 2]))
