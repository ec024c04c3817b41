"""Pins of the window oracle's dump step, its identities and its counters.

Each expected value here comes from the paper or from arithmetic that is
exact, never from the oracle itself:

  - the dump step of Algorithm "AeroSketch: Update" on hand-built buffers
    whose C^T C spectrum is chosen around theta / 2 and theta: whether the
    power iteration fires (estimate >= theta / 2), how many doubling steps
    simul_iter takes, how many directions are dumped (estimate >= theta),
    and the snapshot itself (Z spans the top eigenvectors of C^T C, computed
    by LAPACK; W = Z^T C^T C; residual C - C Z Z^T);
  - exact ties at theta / 2 and theta with exactly representable values
    (rows e_1, theta = 2), which separate ">=" from ">";
  - between two FD reduces no mass is lost: the restored Gram grows by
    exactly a_i^T a_i per row (error analysis of the sliding-window
    theorem); at a reduce the loss is the FD loss, PSD with its top
    eigenvalue ell-fold;
  - the trace identity tr(B) = |C|_F^2 + sum |C'_j Z_j|_F^2, and every
    dumped direction carries at least theta of C'^T C';
  - the count of dumped directions in the window is at most
    4/eps + 16 ell (appendix, time-complexity lemma);
  - the window's FD reduce in randomized mode is the persistent randomized
    shrink with the per-level Philox key (seed, 64 stream + level + 1);
  - the window error bound (25/2) eps |A_W|_F^2 at an ell where it is below
    |A_W|_F^2, on a stream whose top direction holds most of the mass.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import cov_err, rel_fro


def designed_buffer(spec, d, seed):
    """r x d buffer C = diag(sqrt(spec)) V^T with orthonormal V (d x r), so
    C^T C has eigenvalues spec with eigenvectors V."""
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((d, len(spec))))
    return np.sqrt(np.asarray(spec, dtype=np.float64))[:, None] * V.T, V


def proj(Z):
    return Z @ Z.T


# ------------------------------------------------------------------ dump step
def test_dump_not_fired_below_half_theta():
    theta = 10.0
    C, _ = designed_buffer([0.45 * theta, 0.2 * theta, 0.1 * theta], 16, 1)
    out = oracle.aero_dump(C, theta, ell=8, q=1, seed=3)
    assert out["pi"] <= 0.45 * theta * (1 + 1e-12)
    assert out["nsi"] == 0 and out["xi"] == 0
    assert np.array_equal(out["C"], C)


def test_dump_fired_at_half_theta_but_nothing_dumped_below_theta():
    # the power iteration fires (its estimate is close to 0.8 theta >= theta/2),
    # one simul_iter at k = 2 finds its 2nd estimate below theta and no
    # direction reaching theta: nothing is dumped, C is unchanged
    theta = 10.0
    C, _ = designed_buffer([0.8 * theta, 0.05 * theta, 0.01 * theta], 16, 2)
    out = oracle.aero_dump(C, theta, ell=8, q=1, seed=3)
    assert 0.5 * theta <= out["pi"] <= 0.8 * theta * (1 + 1e-12)
    assert out["nsi"] == 1
    assert out["xi"] == 0
    assert np.array_equal(out["C"], C)


@pytest.mark.parametrize("q", [1, 2])
def test_dump_single_direction_stops_at_k2(q):
    theta = 10.0
    spec = np.array([8.0, 0.5, 0.2, 0.1]) * theta
    C, V = designed_buffer(spec, 16, 3)
    out = oracle.aero_dump(C, theta, ell=8, q=q, seed=5, level=1, i=7)
    assert out["nsi"] == 1 and out["xi"] == 1
    Z = out["Z"]
    assert np.allclose(Z.T @ Z, np.eye(1), atol=1e-12)
    # k = 2 < rank: the Ritz vector converges at the rate (lambda_3 / lambda_1)^(q+1)
    assert np.linalg.norm(proj(Z) - proj(V[:, :1])) < 10 * (spec[2] / spec[0]) ** (q + 1)
    G = C.T @ C
    assert rel_fro(out["W"], Z.T @ G) < 1e-12
    assert rel_fro(out["C"], C - C @ Z @ Z.T) < 1e-12


def test_dump_doubling_to_the_rank_dumps_exactly_the_directions_above_theta():
    # k = 2: both estimates >= theta, so k doubles to 4 = rank, where the
    # Ritz values are exact: xi = #{lambda >= theta} = 3
    theta = 10.0
    spec = np.array([8.0, 4.0, 2.0, 0.25]) * theta
    C, V = designed_buffer(spec, 16, 4)
    out = oracle.aero_dump(C, theta, ell=8, q=2, seed=6)
    assert out["nsi"] == 2
    assert out["xi"] == 3
    Z = out["Z"]
    assert np.allclose(Z.T @ Z, np.eye(3), atol=1e-12)
    assert np.linalg.norm(proj(Z) - proj(V[:, :3])) < 1e-10
    G = C.T @ C
    assert rel_fro(out["W"], Z.T @ G) < 1e-12
    Cn = out["C"]
    assert rel_fro(Cn, C - C @ Z @ Z.T) < 1e-12
    lam = np.sort(np.linalg.eigvalsh(Cn.T @ Cn))[::-1]
    assert abs(lam[0] - 0.25 * theta) < 1e-9 * theta and abs(lam[1]) < 1e-9 * theta
    # Ritz values of the dumped directions are the eigenvalues >= theta
    assert np.allclose(np.sort(np.diag(out["W"] @ Z))[::-1], spec[:3], rtol=1e-10)


def test_dump_falls_through_at_the_cap_and_dumps_everything_above_theta():
    # rank 3 = min(ell, d, r): every k keeps its k-th estimate >= theta, the
    # loop ends at the cap and all three directions go (reading: the
    # fall-through still dumps)
    theta = 10.0
    spec = np.array([4.0, 3.0, 2.0]) * theta
    C, V = designed_buffer(spec, 16, 5)
    out = oracle.aero_dump(C, theta, ell=8, q=1, seed=7)
    assert out["nsi"] == 2 and out["xi"] == 3
    assert np.linalg.norm(out["C"]) < 1e-6 * np.linalg.norm(C)


def test_dump_cap_is_ell_when_the_buffer_has_more_rows():
    # ell = 2 caps k at 2: one simul_iter, both directions >= theta dumped
    theta = 10.0
    spec = np.array([6.0, 5.0, 4.0, 0.5]) * theta
    C, V = designed_buffer(spec, 16, 8)
    out = oracle.aero_dump(C, theta, ell=2, q=2, seed=9)
    assert out["nsi"] == 1 and out["xi"] == 2


def test_dump_power_iteration_runs_ceil_log2_d_plus_one_steps():
    # the start vector is Philox draw (coordinate, 0, i, 0x100 + level); after
    # ceil(log2 d) + 1 steps the estimate is the spectral closed form
    theta, d, level, i, seed, stream = 1e6, 20, 2, 9, 4, 5
    C, _ = designed_buffer([5.0, 4.0, 3.5, 1.0], d, 12)
    out = oracle.aero_dump(C, theta, ell=8, q=1, seed=seed, stream=stream, level=level, i=i)
    x0 = oracle.omega(seed, stream, i, d, 1, tag=0x100 + level)[:, 0]
    lam, V = np.linalg.eigh(C.T @ C)
    steps = int(np.ceil(np.log2(d))) + 1
    xs = V @ (lam ** steps * (V.T @ x0))
    xs /= np.linalg.norm(xs)
    assert abs(out["pi"] - xs @ (C.T @ C) @ xs) < 1e-12 * lam[-1]
    assert out["nsi"] == 0


def test_threshold_ties_are_inclusive():
    # theta_0 = 2^0 * (2 / ell) * N = 2 exactly (ell = 4, N = 4); rows e_1:
    # after one row the power-iteration estimate is 1 = theta / 2 exactly
    # (fires: simul_iter runs, nothing reaches theta); after two rows C^T C
    # = 2 e_1 e_1^T, the estimate 2 = theta is dumped; a row with
    # |a|^2 = 2 = theta is stored raw
    d, ell = 4, 4
    e1 = np.zeros((1, d))
    e1[0, 0] = 1.0
    w = oracle.Window(d, ell, N=4, R=2.0, q=1, seed=1)
    w.update(e1)
    c = w.counters(0)
    assert c["simul_iters"] == 1 and c["dumps"] == 0 and c["raw"] == 0
    w.update(e1)
    c = w.counters(0)
    assert c["simul_iters"] == 2 and c["dumps"] == 1 and c["dirs"] == 1
    assert np.linalg.norm(w.buffer(0)) == 0.0
    a = np.zeros((1, d))
    a[0, 1] = a[0, 2] = 1.0
    w.update(a)
    assert w.counters(0)["raw"] == 1


def test_dump_uses_the_level_and_time_streams():
    # the snapshot depends on (level, i) through the Philox counters: other
    # levels / times give another (equally valid) basis of the same span
    theta = 10.0
    spec = np.array([8.0, 0.5, 0.2, 0.1]) * theta
    C, _ = designed_buffer(spec, 12, 11)
    a = oracle.aero_dump(C, theta, ell=8, q=1, seed=5, level=0, i=3)
    b = oracle.aero_dump(C, theta, ell=8, q=1, seed=5, level=1, i=3)
    c = oracle.aero_dump(C, theta, ell=8, q=1, seed=5, level=0, i=4)
    assert a["xi"] == b["xi"] == c["xi"] == 1
    assert a["pi"] != b["pi"] and a["pi"] != c["pi"]
    assert np.linalg.norm(proj(a["Z"]) - proj(b["Z"])) < 10 * (spec[2] / spec[0]) ** 2


# ------------------------------------------------------- identities on a stream
def concentrated_rows(n, d, seed, R=4.0):
    """Rows with |a|^2 in [1, R] concentrated in a few directions, so that the
    level buffers dump often."""
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(n, d, np.array([3.0, 1.5, 0.6]), 0.05, seed=seed)
    return A / np.linalg.norm(A, axis=1, keepdims=True) * np.sqrt(rng.uniform(1.0, R, (n, 1)))


@pytest.mark.parametrize("fd", ["exact", "rand"])
def test_lossless_between_reduces_and_fd_loss_at_reduces(fd):
    d, ell, N = 12, 6, 10**6
    A = concentrated_rows(60, d, 1)
    # theta_j = 2^j (2 / ell) N is huge for N = 10^6: lower it through R
    # instead by a short window whose expiry never triggers (i - N < 1)
    w = oracle.Window(d, ell, N=60, R=4.0, q=1, seed=2, fd=fd)
    prev = [np.zeros((d, d)) for _ in range(w.levels)]
    prev_shr = [0] * w.levels
    dumps = 0
    for i in range(A.shape[0]):
        a = A[i:i + 1]
        w.update(a)
        for lvl in range(w.levels):
            G = w.level_gram(lvl)
            c = w.counters(lvl)
            expect = prev[lvl] + a.T @ a
            if c["shrinks"] == prev_shr[lvl]:
                # no reduce: dumps and raw rows keep every bit of mass
                assert rel_fro(G, expect) < 1e-12
            else:
                D = expect - G
                ev = np.sort(np.linalg.eigvalsh((D + D.T) / 2))[::-1]
                assert ev[-1] >= -1e-10 * ev[0]          # PSD loss
                if fd == "exact":                        # min(lambda, delta): ell-fold top
                    assert np.allclose(ev[:ell], ev[0], rtol=1e-9)
            prev[lvl], prev_shr[lvl] = G, c["shrinks"]
            dumps += c["dumps"]
    assert dumps > 0


def test_trace_identity_and_dumped_mass_at_least_theta():
    d, ell, N = 16, 6, 80
    A = concentrated_rows(400, d, 3)
    w = oracle.Window(d, ell, N=N, R=4.0, q=1, seed=4)
    ndumps = 0
    for t0 in range(0, 400, 20):
        w.update(A[t0:t0 + 20])
        T = t0 + 20
        for lvl in range(w.levels):
            theta = 2 ** lvl * (2.0 / ell) * N
            G = w.level_gram(lvl)
            C = w.buffer(lvl)
            tr = np.sum(C * C)
            for e in w.entries(lvl):
                if not (T - N < e["t"] <= T):
                    continue
                if e["kind"] == "dump":
                    ritz = np.diag(e["W"] @ e["Z"])       # |C' z_c|^2 for each dumped z_c
                    assert np.all(ritz >= theta * (1 - 1e-12))
                    assert np.allclose(e["Z"].T @ e["Z"], np.eye(e["xi"]), atol=1e-12)
                    tr += ritz.sum()
                    ndumps += 1
                else:
                    tr += e["a"] @ e["a"]
            assert abs(np.trace(G) - tr) <= 1e-11 * max(tr, 1.0)
    assert ndumps > 10


def test_dumped_directions_in_window_within_the_count_bound():
    d, ell, N = 16, 4, 200
    eps = 2.0 / ell
    A = concentrated_rows(1500, d, 5, R=8.0)
    w = oracle.Window(d, ell, N=N, R=8.0, q=1, seed=6)
    peak = 0
    for t0 in range(0, 1500, 25):
        w.update(A[t0:t0 + 25])
        T = t0 + 25
        for lvl in range(w.levels):
            k = sum(e["xi"] for e in w.entries(lvl) if e["kind"] == "dump" and T - N < e["t"] <= T)
            assert k <= 4.0 / eps + 16 * ell
            peak = max(peak, k)
    assert peak > 0


def test_randomized_reduce_is_the_persistent_shrink_with_the_level_key():
    # thresholds above any mass (large N): every level is plain FD with the
    # randomized shrink keyed (seed, 64 stream + level + 1), the persistent
    # randomized oracle with that stream id
    d, ell, seed, stream = 24, 5, 9, 3
    A = synth.lowrank_rows(140, d, np.geomspace(2, 0.2, 12), 0.05, seed=7)
    A *= np.sqrt(1.5) / np.linalg.norm(A, axis=1, keepdims=True)
    w = oracle.Window(d, ell, N=10**9, R=4.0, q=1, seed=seed, stream=stream, fd="rand")
    w.update(A)
    assert w.levels == 2
    for lvl in range(2):
        c = w.counters(lvl)
        assert c["dumps"] == 0 and c["raw"] == 0 and c["shrinks"] > 3
        fd = oracle.FD(d, ell, "rand", k=ell, q=1, seed=seed, stream=64 * stream + lvl + 1)
        fd.update(A)
        assert fd.shrinks == c["shrinks"]
        Cw, Cf = w.buffer(lvl), fd.buffer()
        assert np.array_equal(Cw, Cf)
    # and not the key of another level or the unshifted stream id
    other = oracle.FD(d, ell, "rand", k=ell, q=1, seed=seed, stream=stream)
    other.update(A)
    assert not np.allclose(w.buffer(0).T @ w.buffer(0), other.buffer().T @ other.buffer(), rtol=1e-6)


@pytest.mark.parametrize("seed", [0, 1])
def test_window_error_bound_where_it_is_informative(seed):
    # ell = 40: (25/2) eps = 25 / ell = 0.625 < 1, on rows whose top direction
    # holds ~95 % of the mass -- a sketch that lost that direction fails
    d, ell, N, R = 64, 40, 400, 4.0
    rng = np.random.default_rng(seed)
    A = synth.lowrank_rows(1200, d, np.array([8.0, 0.5, 0.25]), 0.02, seed=20 + seed)
    A = A / np.linalg.norm(A, axis=1, keepdims=True) * np.sqrt(rng.uniform(1.0, R, (1200, 1)))
    w = oracle.Window(d, ell, N=N, R=R, q=1, seed=seed)
    worst = 0.0
    for t0 in range(0, 1200, 200):
        w.update(A[t0:t0 + 200])
        T = t0 + 200
        AW = A[max(0, T - N):T]
        B, _ = w.query()
        fa = np.linalg.norm(AW) ** 2
        assert np.max(np.linalg.eigvalsh(AW.T @ AW)) > 0.8 * fa
        err = cov_err(AW, B) / fa
        worst = max(worst, err)
        assert err <= 25.0 / ell
    assert worst < 25.0 / ell
