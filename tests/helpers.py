"""Shared test helpers: the plain definitions used to pin the oracle.

f_ell(X) = sum_i max(lambda_i - lambda_ell, 0) v_i v_i^T (lambda_ell := 0 when X
has fewer than ell eigenvalues), written with numpy's LAPACK eigh.  This is
the Gram-domain form of the FD shrink (Sec. 2.3) and of the query shrink
(the final step of Algorithm "AeroSketch: Query").
"""
import numpy as np


def f_ell(X, ell):
    w, V = np.linalg.eigh((X + X.T) / 2)
    w = w[::-1]
    V = V[:, ::-1]
    de = w[ell - 1] if w.shape[0] >= ell else 0.0
    return (V * np.maximum(w - de, 0.0)) @ V.T


def blocks(n, ell):
    """Row ranges that fill the FD buffer: 2*ell rows first, then ell+1 rows
    per shrink; the remainder is the tail."""
    out = []
    pos = 0
    while True:
        sz = 2 * ell if pos == 0 else ell + 1
        if pos + sz > n:
            break
        out.append((pos, pos + sz))
        pos += sz
    return out, (pos, n)


def fd_gram_recurrence(A, ell):
    """Exact FD as the Gram recurrence G_b = f_ell(G_{b-1} + A_b^T A_b); the
    query returns f_ell(G + A_tail^T A_tail) when the buffer holds >= ell rows."""
    d = A.shape[1]
    G = np.zeros((d, d))
    bl, (t0, t1) = blocks(A.shape[0], ell)
    for a, b in bl:
        G = f_ell(G + A[a:b].T @ A[a:b], ell)
    G = G + A[t0:t1].T @ A[t0:t1]
    fill = (ell - 1 if bl else 0) + (t1 - t0)
    if fill >= ell:
        G = f_ell(G, ell)
    return G


def nystrom(H, Om, q):
    """Nystrom approximation of PSD H with test matrix Om and q power steps:
    H S (S^T H S)^+ S^T H with S = H^q Om."""
    S = Om.copy()
    for _ in range(q):
        S = H @ S
    HS = H @ S
    core = S.T @ HS
    return HS @ np.linalg.pinv((core + core.T) / 2, rcond=1e-13) @ HS.T


def rel_fro(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))


def cov_err(A, B):
    """Spectral covariance error ||A^T A - B^T B||_2."""
    D = A.T @ A - B.T @ B
    return float(np.max(np.abs(np.linalg.eigvalsh((D + D.T) / 2))))
