"""Pins of the probability amplification of the dump step (Algorithm
"Probability Amplification", replacing the simul_iter call of Algorithm
"AeroSketch: Update"; analysis in the appendix on the amplified estimation).

Each expected value comes from the algorithm's definition, from exact
arithmetic or from pinned building blocks (Philox, power iteration), never
from the amplified code path itself:

  - with one candidate the amplified step is the plain dump step, bit for bit
    (whatever the number of power iterations);
  - the candidate kept is the one with the smallest estimate (the first on
    ties), and its reported estimate is the largest of the s power
    iterations on its own residual C - C Z Z^T from the documented start
    vectors;
  - candidate 0 is the plain simul_iter: on a buffer whose doubling ends at
    its first step, its estimate is the power iteration of the plain dump's
    residual;
  - every estimate of the kept candidate is a Rayleigh quotient of its
    residual, so it never exceeds the residual's top squared singular value;
  - after an amplified dump the residual satisfies |C|_2^2 <= 4 theta
    (the amplified estimation's guarantee), and a window built with
    amplification keeps the window error bound.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import cov_err


def designed(spec, d, seed):
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((d, len(spec))))
    return np.sqrt(np.asarray(spec, dtype=np.float64))[:, None] * V.T


def start_vector(seed, stream, i, g, h, level, step, d):
    tag = 0x100000 + 0x10000 * g + 0x1000 * h + 32 * level + step
    return oracle.omega(seed, stream, i, d, 1, tag=tag)[:, 0]


@pytest.mark.parametrize("s", [0, 3])
def test_one_candidate_is_the_plain_dump(s):
    d, ell = 24, 8
    C = designed([9.0, 6.0, 2.5, 0.4, 0.1, 0.05], d, seed=1)
    theta = 4.0
    plain = oracle.aero_dump(C, theta, ell, q=1, seed=3, stream=2, level=1, i=17)
    amp = oracle.aero_dump(C, theta, ell, q=1, seed=3, stream=2, level=1, i=17, amplify=(1, s))
    assert plain["xi"] > 0
    assert amp["xi"] == plain["xi"]
    assert np.array_equal(amp["Z"], plain["Z"])
    assert np.array_equal(amp["W"], plain["W"])
    assert np.array_equal(amp["C"], plain["C"])
    assert amp["amp_h"] == (0 if s > 0 else -1)  # (1, 0) is the plain step itself


@pytest.mark.parametrize("seed", range(6))
def test_kept_candidate_minimises_its_residual_estimate(seed):
    d, ell, r_, s_ = 32, 8, 3, 2
    rng = np.random.default_rng(seed)
    spec = np.sort(rng.uniform(0.05, 10.0, size=7))[::-1]
    C = designed(spec, d, seed=100 + seed)
    theta = float(spec[2]) * 0.9
    out = oracle.aero_dump(C, theta, ell, q=0, seed=11, stream=5, level=0, i=9, amplify=(r_, s_))
    c = out["amp_c"]
    h = out["amp_h"]
    assert 0 <= h < r_
    assert h == int(np.argmin(c))  # np.argmin returns the first minimum
    # the kept candidate's estimate from its own residual (the returned buffer)
    R = out["C"]
    steps = int(np.ceil(np.log2(d))) + 1
    step = out["nsi"] // r_  # the doubling step of the dump (every step runs r candidates)
    est = [oracle.power_iteration(R, start_vector(11, 5, 9, g, h, 0, step, d), steps)[0] for g in range(s_)]
    assert abs(c[h] - max(est)) <= 1e-12 * max(1.0, max(est))
    # a Rayleigh quotient never exceeds the top squared singular value
    top = np.linalg.norm(R, 2) ** 2
    assert c[h] <= top * (1 + 1e-12) + 1e-300
    # the residual is C - C Z Z^T for the returned Z
    Z = out["Z"]
    assert np.allclose(R, C - (C @ Z) @ Z.T, atol=1e-12 * np.abs(C).max())


def test_candidate_zero_is_the_plain_simul_iter():
    # two rows: the doubling ends at its first step (k = 2 = rows), so the
    # amplified step and the plain call both run step 1
    d, ell, s_ = 20, 8, 3
    C = designed([7.0, 3.0], d, seed=4)
    theta = 5.0
    plain = oracle.aero_dump(C, theta, ell, q=1, seed=2, stream=1, level=2, i=40)
    amp = oracle.aero_dump(C, theta, ell, q=1, seed=2, stream=1, level=2, i=40, amplify=(2, s_))
    assert plain["nsi"] == 1 and amp["nsi"] == 2
    steps = int(np.ceil(np.log2(d))) + 1
    est0 = [oracle.power_iteration(plain["C"], start_vector(2, 1, 40, g, 0, 2, 1, d), steps)[0] for g in range(s_)]
    assert abs(amp["amp_c"][0] - max(est0)) <= 1e-12 * max(1.0, max(est0))
    if amp["amp_h"] == 0:
        assert np.array_equal(amp["C"], plain["C"]) and amp["xi"] == plain["xi"]


def test_amplified_residual_meets_the_four_theta_guarantee():
    d, ell = 40, 16
    fired = 0
    for seed in range(10):
        rng = np.random.default_rng(1000 + seed)
        spec = np.sort(rng.uniform(0.01, 6.0, size=12))[::-1]
        C = designed(spec, d, seed=2000 + seed)
        theta = float(rng.uniform(1.0, 4.0))
        out = oracle.aero_dump(C, theta, ell, q=1, seed=seed, stream=7, level=0, i=seed + 1, amplify=(2, 4))
        if out["pi"] >= theta / 2:
            fired += 1
            assert np.linalg.norm(out["C"], 2) ** 2 <= 4 * theta
    assert fired >= 5


def test_window_with_amplification_keeps_the_window_bound():
    d, ell, N, n = 24, 8, 300, 700
    A = synth.window_stream(n, d, rank=6, seed=8)
    fro_max = float(np.max(np.sum(A ** 2, axis=1)))
    R = max(2.0, 2 * fro_max)
    w = oracle.Window(d, ell, N, R, q=1, seed=3, stream=4, amplify=(2, 3))
    plain = oracle.Window(d, ell, N, R, q=1, seed=3, stream=4)
    w.update(A)
    plain.update(A)
    Aw = A[-N:]
    err = cov_err(Aw, w.query()[0])
    assert err <= 25.0 / ell * float(np.sum(Aw ** 2))
    # the amplified window dumped through more simul_iter calls
    st_amp = [w.counters(j)["simul_iters"] for j in range(w.levels)]
    st_pl = [plain.counters(j)["simul_iters"] for j in range(plain.levels)]
    assert sum(st_amp) >= 2 * sum(st_pl) > 0


def test_attp_with_one_candidate_is_the_plain_attp():
    d, ell = 16, 6
    rng = np.random.default_rng(5)
    A = synth.lowrank_rows(200, d, np.geomspace(4, 0.4, 6), 0.05, seed=5)
    A *= np.sqrt(rng.uniform(1.0, 4.0, size=(200, 1)))
    a1 = oracle.ATTP(d, ell, q=1, seed=2, stream=3, amplify=(1, 2))
    a0 = oracle.ATTP(d, ell, q=1, seed=2, stream=3)
    a1.update(A)
    a0.update(A)
    assert a1.stats()["snapshots"] == a0.stats()["snapshots"] > 0
    assert np.array_equal(a1.gram_at(150), a0.gram_at(150))


def test_bad_amplification_parameters_are_rejected():
    with pytest.raises(ValueError):
        oracle.Window(8, 4, 10, 2.0, amplify=(0, 1))
    with pytest.raises(ValueError):
        oracle.ATTP(8, 4, amplify=(2, 17))
