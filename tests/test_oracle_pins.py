"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names what fixes the expected value: a library routine (numpy's
Philox bit generator, LAPACK eigh / svd / qr), a closed form, an invariant of
Frequent Directions, or a special case that reduces to a textbook algorithm
(Misra-Gries counting on one-hot rows).
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from helpers import blocks, cov_err, f_ell, fd_gram_recurrence, nystrom, rel_fro


# --------------------------------------------------------------- Philox -----
@pytest.mark.parametrize("key", [(0, 0), (1, 2), (2**63 + 5, 12345), (2**64 - 1, 7)])
def test_philox_matches_numpy_bitgen(key):
    # numpy's Philox is Philox4x64-10; it increments the counter before each
    # block, so its n-th block is the block of counter n (n >= 1).
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([0, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(4 * 6)
    for c in range(1, 7):
        blk = oracle.philox4x64_10([c, 0, 0, 0], key)
        assert np.array_equal(blk, raw[4 * (c - 1):4 * c])


def test_philox_counter_words_matches_numpy():
    # a counter that carries into the higher words: numpy's state counter
    # [2^64-1, 5, 6, 7] incremented once is [0, 6, 6, 7]
    key = (99, 101)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([2**64 - 1, 5, 6, 7], dtype=np.uint64))
    raw = bg.random_raw(4)
    assert np.array_equal(oracle.philox4x64_10([0, 6, 6, 7], key), raw)


def test_gauss_is_standard_normal():
    z = oracle.omega(7, 3, 0, 20000, 8).ravel()
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the cos and sin halves of Box-Muller are uncorrelated
    a, b = z[0::2], z[1::2]
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01


def test_omega_layout_is_prefix_stable_and_keyed():
    a = oracle.omega(5, 9, 3, 17, 11)
    b = oracle.omega(5, 9, 3, 17, 6)
    assert np.array_equal(a[:, :6], b)
    c = oracle.omega(5, 9, 4, 17, 6)      # another shrink
    e = oracle.omega(5, 10, 3, 17, 6)     # another stream
    assert not np.allclose(b, c) and not np.allclose(b, e)


# ---------------------------------------------------------- linear algebra --
@pytest.mark.parametrize("m,d", [(8, 5), (5, 8), (16, 16), (30, 64), (64, 20)])
def test_jacobi_rows_matches_lapack_svd(m, d):
    rng = np.random.default_rng(m * 100 + d)
    X = rng.standard_normal((m, d)) @ np.diag(np.logspace(0, -3, d))
    R, sig = oracle.jacobi_rows(X)
    ref = np.linalg.svd(X, compute_uv=False)
    r = min(m, d)
    assert np.allclose(sig[:r], ref, rtol=1e-12, atol=1e-13 * ref[0])
    assert np.allclose(sig[r:], 0, atol=1e-12 * ref[0])
    # rotations are orthogonal: the d x d Gram is preserved
    assert rel_fro(R.T @ R, X.T @ X) < 1e-13
    # rows are mutually orthogonal
    G = R @ R.T
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < 1e-12 * ref[0] ** 2


@pytest.mark.parametrize("n", [1, 2, 7, 32, 65])
def test_sym_eig_matches_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V = oracle.sym_eig(A)
    ref = np.linalg.eigvalsh(A)[::-1]
    assert np.allclose(w, ref, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-12)
    assert np.allclose(A @ V, V * w, atol=1e-11 * np.abs(ref).max())


def test_sym_eig_degenerate_spectrum():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.array([5, 5, 5, 2, 2, 0, 0, 0, 0, -1, -1, -3], dtype=float)
    A = (Q * lam) @ Q.T
    w, V = oracle.sym_eig(A)
    assert np.allclose(w, lam, atol=1e-12)
    assert np.allclose((V * w) @ V.T, A, atol=1e-12)


@pytest.mark.parametrize("m,k,rank", [(10, 4, 4), (40, 12, 12), (32, 16, 5)])
def test_qr_householder(m, k, rank):
    rng = np.random.default_rng(m + k)
    K = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, k))
    Q = oracle.qr(K)
    assert np.allclose(Q.T @ Q, np.eye(k), atol=1e-13)
    # range(K) is contained in range(Q)
    assert np.allclose(Q @ (Q.T @ K), K, atol=1e-12 * np.abs(K).max())
    if rank == k:
        Qn, _ = np.linalg.qr(K)
        assert np.allclose(np.abs(Q.T @ Qn), np.eye(k), atol=1e-10)


def test_power_iteration_converges_to_top_eigenvalue():
    rng = np.random.default_rng(3)
    C = rng.standard_normal((20, 30)) @ np.diag(np.linspace(3, 0.1, 30))
    top = np.linalg.eigvalsh(C.T @ C)[-1]
    s, v = oracle.power_iteration(C, rng.standard_normal(30), 200)
    assert abs(s - top) < 1e-9 * top
    assert abs(np.linalg.norm(v) - 1) < 1e-12


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_power_iteration_after_a_given_number_of_steps_is_the_spectral_closed_form(steps):
    # s steps of x <- C^T C x / |C^T C x| from x0 give x_s ~ V diag(lambda^s) V^T x0,
    # and the returned estimate is the Rayleigh quotient x_s^T C^T C x_s
    rng = np.random.default_rng(steps)
    C = rng.standard_normal((6, 9))
    x0 = rng.standard_normal(9)
    lam, V = np.linalg.eigh(C.T @ C)
    xs = V @ (lam ** steps * (V.T @ x0))
    xs /= np.linalg.norm(xs)
    expect = xs @ (C.T @ C) @ xs
    s, v = oracle.power_iteration(C, x0, steps)
    assert abs(s - expect) < 1e-12 * lam[-1]
    assert abs(abs(v @ xs) - 1.0) < 1e-12


# ------------------------------------------------------------- exact FD -----
@pytest.mark.parametrize("d,ell,n", [(40, 6, 100), (16, 4, 57), (12, 8, 80), (64, 16, 300),
                                     (8, 8, 40), (30, 3, 31)])
def test_exact_fd_equals_gram_recurrence(d, ell, n):
    A = synth.lowrank_rows(n, d, 5 * 0.7 ** np.arange(min(d, 12)), 0.05, seed=d + ell + n)
    fd = oracle.FD(d, ell)
    fd.update(A)
    B = fd.query()
    G = fd_gram_recurrence(A, ell)
    assert rel_fro(B.T @ B, G) < 1e-11
    bl, _ = blocks(n, ell)
    assert fd.shrinks == len(bl)


def test_exact_fd_brute_force_tiny():
    # every prefix length of tiny streams: all block boundaries enumerated
    rng = np.random.default_rng(11)
    for d in (2, 3, 4, 6):
        for ell in (1, 2, 3):
            A = rng.standard_normal((12, d))
            for n in range(0, 13):
                fd = oracle.FD(d, ell)
                fd.update(A[:n])
                B = fd.query()
                G = fd_gram_recurrence(A[:n], ell)
                assert np.allclose(B.T @ B, G, atol=1e-11 * max(1.0, np.abs(G).max())), (d, ell, n)


def test_exact_fd_is_misra_gries_on_one_hot_rows():
    # One-hot rows keep every Gram diagonal, so FD reduces to a counting
    # algorithm: at each shrink subtract the ell-th largest count (clamped).
    rng = np.random.default_rng(5)
    d, ell = 24, 5
    cols = rng.choice(d, size=400, p=np.linspace(2, 0.1, d) / np.linspace(2, 0.1, d).sum())
    A = np.eye(d)[cols]
    fd = oracle.FD(d, ell)
    fd.update(A)
    B = fd.query()
    c = np.zeros(d, dtype=np.int64)
    r = 0
    for j in cols:
        c[j] += 1
        r += 1
        if r == 2 * ell:
            de = np.sort(c)[::-1][ell - 1]
            c = np.maximum(c - de, 0)
            r = ell - 1
    if r >= ell:
        c = np.maximum(c - np.sort(c)[::-1][ell - 1], 0)
    assert np.allclose(B.T @ B, np.diag(c.astype(float)), atol=1e-10)


def test_exact_fd_zero_error_below_rank_ell():
    A = synth.lowrank_rows(500, 50, np.linspace(3, 1, 7), 0.0, seed=9)
    fd = oracle.FD(50, 8)
    fd.update(A)
    B = fd.query()
    assert cov_err(A, B) <= 1e-11 * np.linalg.norm(A) ** 2


def test_exact_fd_short_stream_is_f_ell():
    A = synth.lowrank_rows(13, 20, np.linspace(3, 1, 20), 0.1, seed=2)
    fd = oracle.FD(20, 7)
    fd.update(A)
    assert fd.shrinks == 0
    B = fd.query()
    assert rel_fro(B.T @ B, f_ell(A.T @ A, 7)) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_exact_fd_psd_order_and_bound(seed):
    rng = np.random.default_rng(seed)
    d, ell = 48, 8
    A = rng.standard_normal((600, d)) * np.linspace(3, 0.2, d)
    fd = oracle.FD(d, ell)
    fd.update(A)
    B = fd.query()
    D = A.T @ A - B.T @ B
    lam = np.linalg.eigvalsh(D)
    fa, fb = np.linalg.norm(A) ** 2, np.linalg.norm(B) ** 2
    assert lam.min() >= -1e-10 * fa                     # B^T B <= A^T A
    assert lam.max() <= (fa - fb) / ell * (1 + 1e-12)   # sharper FD bound
    assert lam.max() <= fa / ell


# -------------------------------------------------------- randomized FD -----
@pytest.mark.parametrize("d,ell,q", [(40, 6, 0), (40, 6, 1), (12, 8, 1), (64, 10, 2)])
def test_rand_fd_full_rank_k_equals_exact(d, ell, q):
    A = synth.lowrank_rows(200, d, 4 * 0.8 ** np.arange(min(d, 15)), 0.1, seed=d * ell)
    k = min(2 * ell, d)
    ex = oracle.FD(d, ell)
    ra = oracle.FD(d, ell, "rand", k=k, q=q, seed=1, stream=2)
    ex.update(A)
    ra.update(A)
    Be, Br = ex.query(), ra.query()
    assert rel_fro(Br.T @ Br, Be.T @ Be) < 1e-9


def test_rand_fd_k_above_rank_equals_exact():
    A = synth.lowrank_rows(300, 60, np.linspace(4, 1, 9), 0.0, seed=4)
    ex = oracle.FD(60, 10)
    ra = oracle.FD(60, 10, "rand", k=10, q=1, seed=3, stream=0)
    ex.update(A)
    ra.update(A)
    Be, Br = ex.query(), ra.query()
    assert rel_fro(Br.T @ Br, Be.T @ Be) < 1e-9


@pytest.mark.parametrize("q", [0, 1])
def test_rand_fd_equals_nystrom_recurrence(q):
    # Gram-domain definition: G_b = f_ell(Nys_b), Nys_b the Nystrom
    # approximation of H_b = G_{b-1} + A_b^T A_b with the shrink's Omega.
    d, ell, k, seed, stream = 24, 5, 5, 7, 1
    A = synth.lowrank_rows(120, d, 3 * 0.85 ** np.arange(d), 0.05, seed=13)
    ra = oracle.FD(d, ell, "rand", k=k, q=q, seed=seed, stream=stream)
    ra.update(A)
    G = np.zeros((d, d))
    bl, (t0, t1) = blocks(A.shape[0], ell)
    for b, (a0, a1) in enumerate(bl):
        H = G + A[a0:a1].T @ A[a0:a1]
        G = f_ell(nystrom(H, oracle.omega(seed, stream, b, d, k), q), ell)
    Gq = G + A[t0:t1].T @ A[t0:t1]
    if (ell - 1) + (t1 - t0) >= ell:
        Gq = f_ell(Gq, ell)
    Br = ra.query()
    assert rel_fro(Br.T @ Br, Gq) < 1e-8


def test_rand_fd_more_power_steps_approach_exact():
    d, ell = 80, 10
    A = synth.lowrank_rows(400, d, np.arange(1, 41) ** -0.5, 0.05, seed=21)
    ex = oracle.FD(d, ell)
    ex.update(A)
    Ge = ex.query()
    errs = []
    for q in (0, 2, 8, 32):
        ra = oracle.FD(d, ell, "rand", k=ell, q=q, seed=2, stream=0)
        ra.update(A)
        Br = ra.query()
        errs.append(rel_fro(Br.T @ Br, Ge.T @ Ge))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rand_fd_psd_order_and_bound(q):
    rng = np.random.default_rng(40 + q)
    d, ell = 48, 8
    A = rng.standard_normal((500, d)) * np.linspace(3, 0.2, d)
    ra = oracle.FD(d, ell, "rand", k=ell, q=q, seed=q, stream=0)
    ra.update(A)
    B = ra.query()
    lam = np.linalg.eigvalsh(A.T @ A - B.T @ B)
    fa = np.linalg.norm(A) ** 2
    assert lam.min() >= -1e-10 * fa
    assert lam.max() <= fa / ell


def test_rand_shrink_musco_musco_per_vector_bound():
    # Simultaneous Iteration theorem (Sec. 2.2), guarantee 3, as a frequency:
    # |u_i^T G u_i - z_i^T G z_i| <= eps_SI sigma_{k+1}^2 for most draws.
    d, m, k, q = 120, 40, 10, 4
    rng = np.random.default_rng(8)
    ok = 0
    trials = 30
    for t in range(trials):
        X = rng.standard_normal((m, d)) * (np.arange(1, d + 1) ** -0.6)
        G = X @ X.T
        w = np.linalg.eigvalsh(G)[::-1]
        Om = oracle.omega(t, 0, 0, d, k)
        K = X @ Om
        for _ in range(q):
            K = X @ (X.T @ K)
        Q = oracle.qr(K)
        wm, U = oracle.sym_eig(Q.T @ G @ Q)
        ok += np.all(np.abs(w[:k] - wm) <= 0.4 * w[k])
    assert ok >= 0.9 * trials


# ---------------------------------------------------------------- merge -----
def test_merge_into_empty_is_query():
    A = synth.lowrank_rows(200, 30, np.linspace(4, 1, 12), 0.1, seed=1)
    src = oracle.FD(30, 6)
    src.update(A)
    dst = oracle.FD(30, 6)
    dst.merge(src)
    Bs, Bd = src.query(), dst.query()
    assert rel_fro(Bd.T @ Bd, Bs.T @ Bs) < 1e-12


def test_merge_decomposability_bound():
    rng = np.random.default_rng(2)
    d, ell = 40, 8
    parts = [rng.standard_normal((300, d)) * np.linspace(2, 0.3, d) for _ in range(4)]
    sk = []
    for p in parts:
        s = oracle.FD(d, ell)
        s.update(p)
        sk.append(s)
    dst = oracle.FD(d, ell)
    for s in sk:
        dst.merge(s)
    B = dst.query()
    A = np.vstack(parts)
    D = A.T @ A - B.T @ B
    lam = np.linalg.eigvalsh(D)
    assert lam.min() >= -1e-10 * np.linalg.norm(A) ** 2
    # errors of disjoint parts add: sum ||A_i||_F^2 / ell, plus the merge's own
    # shrinks which are bounded by the same total mass
    assert lam.max() <= 2 * np.linalg.norm(A) ** 2 / ell
