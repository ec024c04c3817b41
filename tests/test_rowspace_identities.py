"""The row-space forms of Algorithm "Power Iteration" and Algorithm
"Simultaneous Iteration" that the GPU window and AMM engines run, checked in
numpy FP64 against the plain iterations on the d side (the oracle's order).

For a buffer C (r x d) with Gram G = C C^T:
  - power iteration: x <- C^T C x / |x| from x0, estimate |C x|^2 / |x|^2,
    equals y <- G y / sqrt(y^T G y) from y = C x0 / |x0|, estimate |y|^2;
  - simul_iter: with the iterate K = C^T T, C K = G T, K^T K = T^T G T and
    K X^T = C^T (T X^T); only C Omega and the final C^T (T U) touch C;
  - the AMM form: M = A^T B, C v = R^T (P v) with P, R the two buffers and
    K = P^T S: C^T C K = P^T (G_R G_P S), K^T K = S^T G_P S.
These are identities of exact arithmetic; FP64 agreement to 1e-10 on
well-conditioned inputs pins each derivation (a dropped factor, a wrong
Gram or a transposed operand breaks it by orders of magnitude).
"""
import numpy as np
import pytest


def cholqr(K, passes):
    for _ in range(passes):
        L = np.linalg.cholesky(K.T @ K)
        K = K @ np.linalg.inv(L).T
    return K


def pi_cols(C, x0, steps):
    x = x0.copy()
    for _ in range(steps):
        x = C.T @ (C @ (x / np.linalg.norm(x)))
    return float(np.sum((C @ x) ** 2) / np.sum(x ** 2))


def pi_rows(G, u0, n0, steps):
    y = u0 / np.sqrt(n0)
    for _ in range(steps):
        v = G @ y
        y = v / np.sqrt(y @ v)
    return float(y @ y)


def si_cols(Cf, Ct, Om, q):
    """simul_iter on the d side: Cf applies C, Ct applies C^T."""
    K = Om
    for it in range(q + 1):
        if it > 0:
            K = cholqr(K, 1)
        K = Ct(Cf(K))
    K = cholqr(K, 2)
    CQ = Cf(K)
    lam, U = np.linalg.eigh(CQ.T @ CQ)
    lam, U = lam[::-1], U[:, ::-1]
    return lam, K @ U


def si_rows(C, G, Om, q):
    """the window engine's row-space form: K = C^T T."""
    T = C @ Om
    for _ in range(q):
        X = np.linalg.inv(np.linalg.cholesky(T.T @ G @ T))
        T = T @ X.T
        T = G @ T
    for _ in range(2):
        X = np.linalg.inv(np.linalg.cholesky(T.T @ G @ T))
        T = T @ X.T
    GT = G @ T
    lam, U = np.linalg.eigh(GT.T @ GT)
    lam, U = lam[::-1], U[:, ::-1]
    return lam, C.T @ (T @ U)


def si_rows_amm(P, R, Om, q):
    """the AMM engine's row-space form: K = P^T S, C v = R^T (P v)."""
    GP, GR = P @ P.T, R @ R.T
    S = GR @ (P @ Om)
    for _ in range(q):
        X = np.linalg.inv(np.linalg.cholesky(S.T @ GP @ S))
        S = S @ X.T
        S = GR @ (GP @ S)
    for _ in range(2):
        X = np.linalg.inv(np.linalg.cholesky(S.T @ GP @ S))
        S = S @ X.T
    GS = GP @ S
    lam, U = np.linalg.eigh(GS.T @ (GR @ GS))
    lam, U = lam[::-1], U[:, ::-1]
    return lam, P.T @ (S @ U)


def buffer(r, d, seed, decay=0.8):
    rng = np.random.default_rng(seed)
    s = decay ** np.arange(r)
    Q1, _ = np.linalg.qr(rng.standard_normal((r, r)))
    Q2, _ = np.linalg.qr(rng.standard_normal((d, r)))
    return (Q1 * s) @ Q2.T


@pytest.mark.parametrize("r,d,steps", [(8, 40, 7), (30, 200, 9), (64, 64, 8)])
def test_power_iteration_row_space(r, d, steps):
    C = buffer(r, d, seed=r + d)
    x0 = np.random.default_rng(1).standard_normal(d)
    a = pi_cols(C, x0, steps)
    b = pi_rows(C @ C.T, C @ x0, x0 @ x0, steps)
    assert abs(a - b) <= 1e-12 * a
    # and it is a Rayleigh quotient: at most the top eigenvalue of C^T C
    assert b <= np.linalg.eigvalsh(C @ C.T)[-1] * (1 + 1e-12)


@pytest.mark.parametrize("r,d,k,q", [(16, 60, 4, 1), (32, 150, 8, 1), (24, 90, 6, 2)])
def test_simul_iter_row_space(r, d, k, q):
    C = buffer(r, d, seed=3 * r + k)
    Om = np.random.default_rng(k).standard_normal((d, k))
    la, Za = si_cols(lambda K: C @ K, lambda Y: C.T @ Y, Om, q)
    lb, Zb = si_rows(C, C @ C.T, Om, q)
    assert np.allclose(la, lb, rtol=1e-10, atol=1e-12 * la[0])
    # the directions agree up to sign
    for j in range(k):
        assert abs(abs(Za[:, j] @ Zb[:, j]) - 1.0) <= 1e-8
    assert np.allclose(Zb.T @ Zb, np.eye(k), atol=1e-10)


@pytest.mark.parametrize("left", [True, False])
def test_amm_simul_iter_row_space(left):
    r, dx, dy, k, q = 20, 50, 70, 5, 1
    A = buffer(r, dx, seed=11)
    B = buffer(r, dy, seed=12, decay=0.85)
    P, R = (A, B) if left else (B, A)
    Om = np.random.default_rng(5).standard_normal((P.shape[1], k))
    # d side: C = M^T (left) or M (right); C K = R^T (P K), C^T Y = P^T (R Y)
    la, Za = si_cols(lambda K: R.T @ (P @ K), lambda Y: P.T @ (R @ Y), Om, q)
    lb, Zb = si_rows_amm(P, R, Om, q)
    assert np.allclose(la, lb, rtol=1e-9, atol=1e-12 * la[0])
    for j in range(k):
        assert abs(abs(Za[:, j] @ Zb[:, j]) - 1.0) <= 1e-7
    # the estimates are the squared singular values of M = A^T B
    s = np.linalg.svd(A.T @ B, compute_uv=False)
    assert np.all(lb <= s[0] ** 2 * (1 + 1e-10))


def test_a_dropped_gram_factor_is_caught():
    # planted mistake: the Rayleigh-Ritz matrix formed as (G_P S)^T G_R S
    # (one G_P dropped) instead of (G_P S)^T G_R (G_P S)
    r, dx, dy, k, q = 20, 50, 70, 5, 1
    A, B = buffer(r, dx, seed=11), buffer(r, dy, seed=12, decay=0.85)
    Om = np.random.default_rng(5).standard_normal((dx, k))
    la, _ = si_cols(lambda K: B.T @ (A @ K), lambda Y: A.T @ (B @ Y), Om, q)
    GP, GR = A @ A.T, B @ B.T
    S = GR @ (A @ Om)
    for _ in range(q):
        S = S @ np.linalg.inv(np.linalg.cholesky(S.T @ GP @ S)).T
        S = GR @ (GP @ S)
    for _ in range(2):
        S = S @ np.linalg.inv(np.linalg.cholesky(S.T @ GP @ S)).T
    Mbad = (GP @ S).T @ (GR @ S)
    lam_bad = np.linalg.eigvalsh((Mbad + Mbad.T) / 2)[::-1]
    assert not np.allclose(la, lam_bad, rtol=1e-3)
