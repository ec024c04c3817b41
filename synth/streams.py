"""Workload generators (inputs only).

Every generator is deterministic in its seed.  numpy's ``Generator`` on the
Philox bit generator is used for every draw; orthonormal bases come from a
QR factorisation of a Gaussian matrix.
"""
from dataclasses import dataclass

import numpy as np


def _rng(seed, sub=0):
    return np.random.Generator(np.random.Philox(key=np.array([seed, sub], dtype=np.uint64)))


def orthonormal(d, r, rng):
    """Random d x r matrix with orthonormal columns."""
    g = rng.standard_normal((d, r))
    q, rr = np.linalg.qr(g)
    q = q * np.sign(np.diag(rr))[None, :]
    return q


@dataclass
class StreamSpec:
    """A low-rank-plus-noise row model: a = sum_i g_i s_i v_i^T + noise_std * z."""
    d: int
    spectrum: np.ndarray      # population singular values s_i (per-row scales)
    basis: np.ndarray         # d x r orthonormal
    noise_std: float

    def rows(self, n, rng, dtype=np.float64):
        r = self.spectrum.shape[0]
        g = rng.standard_normal((n, r)) * self.spectrum[None, :]
        a = g @ self.basis.T
        if self.noise_std > 0:
            a += self.noise_std * rng.standard_normal((n, self.d))
        return a.astype(dtype, copy=False)


def lowrank_rows(n, d, spectrum, noise_std, seed, dtype=np.float64):
    rng = _rng(seed, 0)
    spec = np.asarray(spectrum, dtype=np.float64)
    V = orthonormal(d, spec.shape[0], rng)
    return StreamSpec(d, spec, V, noise_std).rows(n, _rng(seed, 1), dtype)


def persistent_small(n=10_000, d=256, seed=0, dtype=np.float64):
    """Persistent stream, exact FP64 workload: rank-20 signal with singular
    values 10 * 0.8^i in a random orthonormal basis plus N(0, 0.1^2) noise."""
    spec = 10.0 * 0.8 ** np.arange(20)
    return lowrank_rows(n, d, spec, 0.1, seed, dtype)


def persistent_tight_spec(d=4096, rank=1024, seed=1):
    """Power-law spectrum s_i = i^-0.8 over rank 1024 plus N(0, 1e-3) noise
    (1e-3 read as the variance, as in N(0, 0.1^2) of the small workload)."""
    rng = _rng(seed, 0)
    spec = np.arange(1, rank + 1, dtype=np.float64) ** -0.8
    V = orthonormal(d, rank, rng)
    return StreamSpec(d, spec, V, float(np.sqrt(1e-3)))


def persistent_tight(n, d=4096, rank=1024, seed=1, dtype=np.float32):
    return persistent_tight_spec(d, rank, seed).rows(n, _rng(seed, 1), dtype)


def random_noisy(n, d, seed, zeta=10.0, rank=None, dtype=np.float64):
    """The paper's Random Noisy model A = S D U + N / zeta with
    D_ii = 1 - (i-1)/rank (rank defaults to d)."""
    r = d if rank is None else rank
    spec = 1.0 - np.arange(r, dtype=np.float64) / r
    return lowrank_rows(n, d, spec, 1.0 / zeta, seed, dtype)


def givens_sweep(V, angles):
    """Rotate the rows of V (d x r) by Givens rotations on coordinate pairs
    (i, i+1), i = 0 .. d-2, in order."""
    V = V.copy()
    for i, th in enumerate(angles):
        c, s = np.cos(th), np.sin(th)
        a, b = V[i].copy(), V[i + 1].copy()
        V[i] = c * a - s * b
        V[i + 1] = s * a + c * b
    return V


def window_stream(n, d=1024, rank=64, ratio=0.95, period=50_000, seed=2, dtype=np.float32,
                  start=0):
    """Sliding-window workload: rank-64 signal with geometric spectrum 0.95^j,
    no noise; the basis rotates by a random Givens sweep every ``period`` rows.
    Rows [start, start + n) of the infinite stream are returned."""
    rng0 = _rng(seed, 0)
    V = orthonormal(d, rank, rng0)
    spec = ratio ** np.arange(rank, dtype=np.float64)
    out = np.empty((n, d), dtype=dtype)
    epoch = 0
    pos = 0
    while pos < start + n:
        e_end = (epoch + 1) * period
        lo, hi = max(pos, start), min(e_end, start + n)
        if hi > lo:
            rr = _rng(seed, 1000 + epoch)
            skip = lo - epoch * period
            if skip:
                rr.standard_normal((skip, rank))
            g = rr.standard_normal((hi - lo, rank)) * spec[None, :]
            out[lo - start:hi - start] = (g @ V.T).astype(dtype)
        pos = e_end
        V = givens_sweep(V, _rng(seed, 2000 + epoch).uniform(0, 2 * np.pi, d - 1))
        epoch += 1
    return out


def serving_streams(count=512, seed=3):
    """Batched-serving population: per stream d in {128..2048}, ell in
    {16..256}, rank min(2 ell, d) with the Random Noisy scales 1 - (i-1)/r and
    noise 1/zeta (zeta = 10)."""
    rng = _rng(seed, 0)
    ds = rng.choice([128, 256, 512, 1024, 2048], size=count)
    ells = rng.choice([16, 32, 64, 128, 256], size=count)
    specs = []
    for s in range(count):
        d, ell = int(ds[s]), int(ells[s])
        r = min(2 * ell, d)
        srng = _rng(seed, 10 + s)
        V = orthonormal(d, r, srng)
        spec = 1.0 - np.arange(r, dtype=np.float64) / r
        specs.append((d, ell, StreamSpec(d, spec, V, 0.1)))
    return specs


def bursts(count_streams, n_bursts, rate, seed=3):
    """Poisson arrivals (aggregate rate per second) of bursts of
    floor(exp(U[0, ln 4097))) rows, each for a uniformly drawn stream."""
    rng = _rng(seed, 1)
    gaps = rng.exponential(1.0 / rate, n_bursts)
    t = np.cumsum(gaps)
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(4097.0), n_bursts))).astype(np.int64)
    sizes = np.clip(sizes, 1, 4096)
    sid = rng.integers(0, count_streams, n_bursts)
    return t, sid, sizes


def sparse_sites(n_rows, d=2048, density=0.01, seed=4, site=0):
    """Sparse CSR rows of one site: each entry present with probability
    ``density``; values N(0,1) * j^-0.5 for column j = 1..d.
    Returns (indptr int64, indices int32, values float32)."""
    rng = _rng(seed, 100 + site)
    nnz_row = rng.binomial(d, density, n_rows)
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(nnz_row, out=indptr[1:])
    idx = np.empty(indptr[-1], dtype=np.int32)
    for i in range(n_rows):
        k = nnz_row[i]
        if k:
            idx[indptr[i]:indptr[i + 1]] = np.sort(rng.choice(d, size=k, replace=False))
    w = (np.arange(1, d + 1, dtype=np.float64) ** -0.5)
    vals = (rng.standard_normal(indptr[-1]) * w[idx]).astype(np.float32)
    return indptr, idx, vals


def csr_to_dense(indptr, idx, vals, d):
    n = indptr.shape[0] - 1
    out = np.zeros((n, d), dtype=np.float64)
    for i in range(n):
        out[i, idx[indptr[i]:indptr[i + 1]]] = vals[indptr[i]:indptr[i + 1]]
    return out
