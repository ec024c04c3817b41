"""Pins of the AeroSketchCOD oracle (approximate matrix multiplication over a
sliding window, Algorithm "AeroSketchCOD Framework", Sec. 4.2; Theorem
"sw-amm" and its proof in the appendix).

Every expected value comes from a definition, a library routine or a bound,
never from the oracle's own output:

  - the co-occurring-directions reduce is the product's SVD shrunk by its
    ell-th singular value (numpy SVD), split evenly between the factors, with
    the reduce's error sigma_ell <= ||A~||_F ||B~||_F / ell;
  - with theta out of reach nothing is dumped and the sketch is the plain COD
    stream: a numpy recurrence of SVD shrinks at the reduce cadence (a reduce
    at 2 ell rows leaves ell - 1), queried by one more shrink;
  - with no reduce and no expiry the restored product is sum x_i y_i^T
    exactly (snapshot restore + residual = the product before the dump);
  - a single pair: no power-iteration firing below theta / 2, firing without
    a dump in [theta / 2, theta), one direction dumped at or above theta,
    with Z, H the pair's unit vectors;
  - snapshots older than N pairs are gone; the residual's top singular value
    stays <= 4 theta; the window error bound of the theorem's proof.
"""
import numpy as np
import pytest

import oracle


def shrink(M, ell):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    delta = s[ell - 1] if s.shape[0] >= ell else 0.0
    return (U * np.maximum(s - delta, 0.0)) @ Vt


def pairs(n, dx, dy, seed, kind="uniform", rank=6):
    rng = np.random.default_rng(seed)
    if kind == "uniform":  # the paper's Uniform Random AMM data: entries in (0, 1]
        return 1.0 - rng.random((n, dx)), 1.0 - rng.random((n, dy))
    G = rng.standard_normal((n, rank))
    X = G @ rng.standard_normal((rank, dx)) + 0.05 * rng.standard_normal((n, dx))
    Y = G @ rng.standard_normal((rank, dy)) + 0.05 * rng.standard_normal((n, dy))
    return X, Y


@pytest.mark.parametrize("dx,dy,ell", [(12, 9, 4), (30, 20, 8), (5, 7, 4), (3, 40, 6)])
def test_reduce_is_the_shrunk_svd_of_the_product(dx, dy, ell):
    rng = np.random.default_rng(dx + dy)
    A = rng.standard_normal((2 * ell, dx))
    B = rng.standard_normal((2 * ell, dy))
    A2, B2 = oracle.cod_reduce(A, B, ell)
    M = A.T @ B
    assert np.linalg.norm(A2.T @ B2 - shrink(M, ell)) <= 1e-10 * np.linalg.norm(M)
    # at most ell - 1 non-zero rows; the factors are balanced: A' A'^T = B' B'^T diagonal
    assert np.all(A2[ell - 1:] == 0) and np.all(B2[ell - 1:] == 0)
    Ga, Gb = A2 @ A2.T, B2 @ B2.T
    assert np.allclose(Ga, Gb, atol=1e-10 * np.abs(Ga).max())
    assert np.allclose(Ga, np.diag(np.diag(Ga)), atol=1e-10 * np.abs(Ga).max())
    s = np.linalg.svd(M, compute_uv=False)
    if s.shape[0] >= ell:
        assert np.linalg.norm(M - A2.T @ B2, 2) <= s[ell - 1] * (1 + 1e-10)
        assert s[ell - 1] <= np.linalg.norm(A) * np.linalg.norm(B) / ell


def test_without_dumps_the_sketch_is_the_cod_stream():
    dx, dy, ell, n = 14, 10, 5, 230
    X, Y = pairs(n, dx, dy, seed=3, kind="lowrank")
    c = oracle.COD(dx, dy, ell, N=10 ** 9, theta=1e12, q=1, seed=1, stream=1)
    c.update(X, Y)
    st = c.stats()
    assert st["snapshots"] == 0 and st["simul_iters"] == 0
    M = np.zeros((dx, dy))
    rows = 0
    for i in range(n):
        M += np.outer(X[i], Y[i])
        rows += 1
        if rows == 2 * ell:
            M = shrink(M, ell)
            rows = ell - 1
    assert st["reduces"] > 10 and st["fill"] == rows
    assert np.linalg.norm(c.product() - M) <= 1e-9 * np.linalg.norm(M)
    A, B = c.query()
    assert np.linalg.norm(A @ B.T - shrink(M, ell)) <= 1e-9 * np.linalg.norm(M)


@pytest.mark.parametrize("seed", range(3))
def test_restore_plus_residual_is_the_exact_product(seed):
    # fewer than 2 ell pairs: no reduce; N beyond the stream: no expiry
    dx, dy, ell, n = 16, 12, 12, 23
    X, Y = pairs(n, dx, dy, seed=seed, kind="lowrank", rank=4)
    theta = 0.3 * np.linalg.norm(X[:4]) * np.linalg.norm(Y[:4])
    c = oracle.COD(dx, dy, ell, N=1000, theta=theta, q=1, seed=seed, stream=2)
    c.update(X, Y)
    assert c.stats()["reduces"] == 0 and c.stats()["snapshots"] > 0
    W = X.T @ Y
    assert np.linalg.norm(c.product() - W) <= 1e-10 * np.linalg.norm(W)
    for s in c.snapshots():
        Z, H = s["Z"], s["H"]
        assert np.allclose(Z.T @ Z, np.eye(s["xi"]), atol=1e-10)
        assert np.allclose(H.T @ H, np.eye(s["xi"]), atol=1e-10)


def test_a_single_pair_fires_and_dumps_by_its_singular_value():
    dx, dy, ell = 8, 6, 4
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal((1, dx)), rng.standard_normal((1, dy))
    sv = np.linalg.norm(x) * np.linalg.norm(y)
    # below theta / 2: no power-iteration firing
    c = oracle.COD(dx, dy, ell, N=100, theta=2.2 * sv)
    c.update(x, y)
    assert c.stats()["simul_iters"] == 0 and c.stats()["snapshots"] == 0
    # in [theta / 2, theta): the doubling runs (k = 1, the cap) and dumps nothing
    c = oracle.COD(dx, dy, ell, N=100, theta=1.5 * sv)
    c.update(x, y)
    assert c.stats()["simul_iters"] == 2 and c.stats()["snapshots"] == 0
    # at or above theta: one direction, the pair's unit vectors, restore = x y^T
    c = oracle.COD(dx, dy, ell, N=100, theta=0.9 * sv)
    c.update(x, y)
    (s,) = c.snapshots()
    assert s["xi"] == 1 and s["t"] == 1 and s["s"] == 1
    z, h = s["Z"][:, 0], s["H"][:, 0]
    assert abs(abs(z @ x[0]) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)
    assert abs(abs(h @ y[0]) - np.linalg.norm(y)) <= 1e-12 * np.linalg.norm(y)
    A, B = c.buffers()
    assert np.linalg.norm(A.T @ B) <= 1e-12 * sv
    assert np.linalg.norm(c.product() - x.T @ y) <= 1e-12 * sv


def test_expiry_residual_and_window_bound():
    dx, dy, ell, N, n = 20, 15, 8, 150, 600
    X, Y = pairs(n, dx, dy, seed=11)
    eps = 2.0 / ell
    fro = np.sqrt(np.sum(X ** 2, axis=1) * np.sum(Y ** 2, axis=1))
    theta = eps * N * float(fro.min())  # theta <= eps ||X_W||_F ||Y_W||_F
    c = oracle.COD(dx, dy, ell, N=N, theta=theta, q=1, seed=4, stream=9)
    for t0 in range(0, n, 100):
        c.update(X[t0:t0 + 100], Y[t0:t0 + 100])
        T = t0 + 100
        for s in c.snapshots():
            assert T - N < s["t"] <= T
        A, B = c.buffers()
        assert np.linalg.norm(A.T @ B, 2) <= 4 * theta
        Xw, Yw = X[max(0, T - N):T], Y[max(0, T - N):T]
        bound = np.linalg.norm(Xw) * np.linalg.norm(Yw)
        As, Bs = c.query()
        assert np.linalg.norm(Xw.T @ Yw - As @ Bs.T, 2) <= 3 * bound / ell + 24 * theta
    assert c.stats()["snapshots"] > 20 and c.stats()["reduces"] > 20


def test_bad_parameters_are_rejected():
    with pytest.raises(ValueError):
        oracle.COD(0, 4, 4, 10, 1.0)
    with pytest.raises(ValueError):
        oracle.COD(4, 4, 1, 10, 1.0)
    with pytest.raises(ValueError):
        oracle.COD(4, 4, 4, 10, 0.0)
