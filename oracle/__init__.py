"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  The C sources
cite the paper section each function follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SKETCH_ORACLE_LIB selects another build of the same sources (the mutation
# tests load deliberately broken copies through it)
_LIBPATH = os.environ.get("SKETCH_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.o_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.o_gauss4.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _u64p, _dp]
    lib.o_omega.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                            ctypes.c_int, ctypes.c_int, _dp]
    lib.o_jacobi_rows.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
    lib.o_sym_eig.argtypes = [_dp, ctypes.c_int, _dp, _dp]
    lib.o_qr_householder.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp]
    lib.o_fd_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.o_fd_create.restype = ctypes.c_void_p
    lib.o_fd_destroy.argtypes = [ctypes.c_void_p]
    lib.o_fd_update.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int64, ctypes.c_int64]
    lib.o_fd_query.argtypes = [ctypes.c_void_p, _dp]
    lib.o_fd_buffer.argtypes = [ctypes.c_void_p, _dp]
    lib.o_fd_buffer.restype = ctypes.c_int64
    lib.o_fd_fill.argtypes = [ctypes.c_void_p]
    lib.o_fd_fill.restype = ctypes.c_int64
    lib.o_fd_shrinks.argtypes = [ctypes.c_void_p]
    lib.o_fd_shrinks.restype = ctypes.c_int64
    lib.o_fd_merge.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.o_shrink_exact.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.o_shrink_rand.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint64]
    lib.o_power_iteration.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                      ctypes.c_int, _dp]
    lib.o_power_iteration.restype = ctypes.c_double
    lib.o_win_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.o_win_create.restype = ctypes.c_void_p
    lib.o_win_create2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
    lib.o_win_create2.restype = ctypes.c_void_p
    lib.o_win_destroy.argtypes = [ctypes.c_void_p]
    lib.o_win_update.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int64, ctypes.c_int64]
    lib.o_win_advance.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.o_win_query.argtypes = [ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_int)]
    lib.o_win_levels.argtypes = [ctypes.c_void_p]
    lib.o_win_stats.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p]
    lib.o_win_level_gram.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
    lib.o_win_counters.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p]
    lib.o_win_entry.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, _i64p, _dp, _dp, _dp]
    lib.o_win_buffer.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
    lib.o_aero_dump.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int64, ctypes.c_int64, _dp, _dp,
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _dp]
    lib.o_aero_dump_amp.argtypes = lib.o_aero_dump.argtypes + [ctypes.c_int, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int)]
    lib.o_win_set_amplify.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.o_attp_set_amplify.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.o_attp_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_int]
    lib.o_attp_create.restype = ctypes.c_void_p
    lib.o_attp_destroy.argtypes = [ctypes.c_void_p]
    lib.o_attp_update.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int64, ctypes.c_int64]
    lib.o_attp_gram_at.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp]
    lib.o_attp_query_at.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp]
    lib.o_attp_stats.argtypes = [ctypes.c_void_p, _i64p]
    lib.o_attp_theta.argtypes = [ctypes.c_void_p]
    lib.o_attp_theta.restype = ctypes.c_double
    lib.o_attp_snapshot.argtypes = [ctypes.c_void_p, ctypes.c_int64, _i64p, _dp, _dp]
    lib.o_attp_buffer.argtypes = [ctypes.c_void_p, _dp]
    lib.o_p5_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                ctypes.c_uint64, ctypes.c_int]
    lib.o_p5_create.restype = ctypes.c_void_p
    lib.o_p5_set_amplify.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.o_p5_destroy.argtypes = [ctypes.c_void_p]
    lib.o_p5_update.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), _dp, ctypes.c_int64,
                                ctypes.c_int64]
    lib.o_p5_gram.argtypes = [ctypes.c_void_p, _dp]
    lib.o_p5_query.argtypes = [ctypes.c_void_p, _dp]
    lib.o_p5_stats.argtypes = [ctypes.c_void_p, _i64p]
    lib.o_p5_fhat.argtypes = [ctypes.c_void_p]
    lib.o_p5_fhat.restype = ctypes.c_double
    lib.o_p5_site.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _i64p, _dp]
    lib.o_simul_iter.argtypes = [_dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _dp, _dp]
    lib.o_cod_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.o_cod_create.restype = ctypes.c_void_p
    lib.o_cod_destroy.argtypes = [ctypes.c_void_p]
    lib.o_cod_update.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int64, _dp, ctypes.c_int64, ctypes.c_int64]
    lib.o_cod_product.argtypes = [ctypes.c_void_p, _dp]
    lib.o_cod_query.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.o_cod_stats.argtypes = [ctypes.c_void_p, _i64p]
    lib.o_cod_buffers.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.o_cod_snapshot.argtypes = [ctypes.c_void_p, ctypes.c_int64, _i64p, _dp, _dp, _dp, _dp]
    lib.o_cod_reduce.argtypes = [_dp, _dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def philox4x64_10(ctr, key):
    """Philox4x64-10 block for a 4-word counter and a 2-word key."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.o_philox4x64_10(c.ctypes.data_as(_u64p), k.ctypes.data_as(_u64p), out.ctypes.data_as(_u64p))
    return out


def gauss4(seed, stream, ctr):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    out = np.zeros(4)
    lib.o_gauss4(seed, stream, c.ctypes.data_as(_u64p), _p(out))
    return out


def omega(seed, stream, b, d, k, tag=0):
    """Gaussian test matrix (d x k) of shrink ``b``."""
    lib = _load()
    out = np.zeros((d, k))
    lib.o_omega(seed, stream, b, tag, d, k, _p(out))
    return out


def jacobi_rows(X):
    """One-sided Jacobi on the rows of X: returns (rotated rows sorted, sigma)."""
    lib = _load()
    X = _f64(X).copy()
    m, d = X.shape
    sig = np.zeros(m)
    _check(lib.o_jacobi_rows(_p(X), m, d, d, _p(sig)), "jacobi_rows")
    return X, sig


def sym_eig(A):
    lib = _load()
    A = _f64(A).copy()
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    _check(lib.o_sym_eig(_p(A), n, _p(w), _p(V)), "sym_eig")
    return w, V


def qr(K):
    lib = _load()
    K = _f64(K)
    m, k = K.shape
    Q = np.zeros((m, k))
    _check(lib.o_qr_householder(_p(K), m, k, _p(Q)), "qr")
    return Q


def shrink_exact(X, ell):
    lib = _load()
    X = _f64(X).copy()
    m, d = X.shape
    _check(lib.o_shrink_exact(_p(X), m, d, d, ell), "shrink_exact")
    return X


def shrink_rand(X, ell, k, q, seed, stream, b):
    lib = _load()
    X = _f64(X).copy()
    m, d = X.shape
    _check(lib.o_shrink_rand(_p(X), m, d, d, ell, k, q, seed, stream, b), "shrink_rand")
    return X


def aero_dump(C, theta, ell, q=1, seed=0, stream=0, level=0, i=1, amplify=(1, 0)):
    """The window's dump step on the buffer C (r x d).  Returns a dict with
    the power-iteration estimate ``pi``, the simul_iter call count ``nsi``,
    ``xi``, the snapshot ``Z`` (d x xi) and ``W`` (xi x d) and the residual
    buffer ``C`` (C - C Z Z^T).  ``amplify = (r, s)`` runs Algorithm
    "Probability Amplification" in place of each simul_iter call; then
    ``amp_c`` holds the r candidates' squared residual estimates of the last
    amplified step and ``amp_h`` the candidate kept."""
    lib = _load()
    C = _f64(np.atleast_2d(C)).copy()
    r, d = C.shape
    Z = np.zeros((d, ell))
    W = np.zeros((ell, d))
    xi, nsi, pi = ctypes.c_int(0), ctypes.c_int(0), np.zeros(1)
    ar, as_ = amplify
    amp_c = np.full(16, np.nan)
    amp_h = ctypes.c_int(-1)
    _check(lib.o_aero_dump_amp(d, ell, q, seed, stream, level, float(theta), _p(C), r, i, _p(Z), _p(W),
                               ctypes.byref(xi), ctypes.byref(nsi), _p(pi), int(ar), int(as_), _p(amp_c),
                               ctypes.byref(amp_h)), "aero_dump")
    x = xi.value
    return {"pi": float(pi[0]), "nsi": nsi.value, "xi": x, "Z": Z[:, :x].copy(), "W": W[:x].copy(), "C": C,
            "amp_c": amp_c[:ar].copy(), "amp_h": amp_h.value}


def power_iteration(C, x0, steps):
    lib = _load()
    C = _f64(C)
    m, d = C.shape
    x0 = _f64(x0)
    v = np.zeros(d)
    s = lib.o_power_iteration(_p(C), m, d, d, _p(x0), steps, _p(v))
    return s, v


class FD:
    """Frequent Directions, exact (mode 'exact') or randomized (mode 'rand')."""

    def __init__(self, d, ell, mode="exact", k=0, q=1, seed=0, stream=0):
        lib = _load()
        m = {"exact": 0, "rand": 1}[mode]
        self._h = lib.o_fd_create(d, ell, m, k, q, seed, stream)
        if not self._h:
            raise ValueError("bad FD parameters")
        self.d, self.ell = d, ell

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.o_fd_destroy(self._h)
            self._h = None

    def update(self, rows):
        rows = _f64(np.atleast_2d(rows))
        if rows.shape[0] == 0:
            return
        _check(_lib.o_fd_update(self._h, _p(rows), rows.shape[0], rows.shape[1]), "fd_update")

    def query(self):
        out = np.zeros((self.ell, self.d))
        _check(_lib.o_fd_query(self._h, _p(out)), "fd_query")
        return out

    def buffer(self):
        r = _lib.o_fd_fill(self._h)
        out = np.zeros((max(r, 1), self.d))
        _lib.o_fd_buffer(self._h, _p(out))
        return out[:r]

    @property
    def fill(self):
        return _lib.o_fd_fill(self._h)

    @property
    def shrinks(self):
        return _lib.o_fd_shrinks(self._h)

    def merge(self, other):
        _check(_lib.o_fd_merge(self._h, other._h), "fd_merge")


class Window:
    """ML-AeroSketch over a sliding window of N rows."""

    def __init__(self, d, ell, N, R, q=1, seed=0, stream=0, fd="exact", amplify=(1, 0)):
        lib = _load()
        self._h = lib.o_win_create2(d, ell, N, float(R), q, seed, stream, {"exact": 0, "rand": 1}[fd])
        if not self._h:
            raise ValueError("bad window parameters")
        if lib.o_win_set_amplify(self._h, int(amplify[0]), int(amplify[1])) != 0:
            raise ValueError("bad amplification parameters")
        self.d, self.ell, self.N = d, ell, N

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.o_win_destroy(self._h)
            self._h = None

    @property
    def levels(self):
        return _lib.o_win_levels(self._h)

    def update(self, rows):
        rows = _f64(np.atleast_2d(rows))
        if rows.shape[0] == 0:
            return
        _check(_lib.o_win_update(self._h, _p(rows), rows.shape[0], rows.shape[1]), "win_update")

    def advance(self, t_now):
        _check(_lib.o_win_advance(self._h, t_now), "win_advance")

    def query(self):
        out = np.zeros((self.ell, self.d))
        lvl = ctypes.c_int(0)
        _check(_lib.o_win_query(self._h, _p(out), ctypes.byref(lvl)), "win_query")
        return out, lvl.value

    def stats(self, level):
        st = np.zeros(6, dtype=np.int64)
        _check(_lib.o_win_stats(self._h, level, st.ctypes.data_as(_i64p)), "win_stats")
        keys = ["dumps", "raw", "dirs", "fill", "queue", "shrinks"]
        return dict(zip(keys, st.tolist()))

    def level_gram(self, level):
        G = np.zeros((self.d, self.d))
        _check(_lib.o_win_level_gram(self._h, level, _p(G)), "win_level_gram")
        return G

    def counters(self, level):
        st = np.zeros(8, dtype=np.int64)
        _check(_lib.o_win_counters(self._h, level, st.ctypes.data_as(_i64p)), "win_counters")
        keys = ["dumps", "raw", "dirs", "fill", "queue", "shrinks", "simul_iters", "dropped_t"]
        return dict(zip(keys, st.tolist()))

    def entries(self, level):
        """Queue of a level, oldest first: dicts with kind ('dump'/'raw'), s,
        t and Z, W (dumps) or a (raw rows)."""
        out = []
        q = self.counters(level)["queue"]
        meta = np.zeros(4, dtype=np.int64)
        for e in range(q):
            _check(_lib.o_win_entry(self._h, level, e, meta.ctypes.data_as(_i64p), None, None, None),
                   "win_entry")
            xi = int(meta[1])
            Z, W, a = np.zeros((self.d, max(xi, 1))), np.zeros((max(xi, 1), self.d)), np.zeros(self.d)
            _check(_lib.o_win_entry(self._h, level, e, meta.ctypes.data_as(_i64p), _p(Z), _p(W), _p(a)),
                   "win_entry")
            if meta[0] == 0:
                out.append({"kind": "dump", "xi": xi, "s": int(meta[2]), "t": int(meta[3]),
                            "Z": Z[:, :xi].copy(), "W": W[:xi].copy()})
            else:
                out.append({"kind": "raw", "s": int(meta[2]), "t": int(meta[3]), "a": a})
        return out

    def buffer(self, level):
        C = np.zeros((2 * self.ell, self.d))
        r = _lib.o_win_buffer(self._h, level, _p(C))
        if r < 0:
            raise RuntimeError("oracle win_buffer failed")
        return C[:r].copy()


class ATTP:
    """ATTP persistent sketch (Algorithm "ATTP Sketch using AeroSketch")."""

    def __init__(self, d, ell, q=1, seed=0, stream=0, fd="exact", amplify=(1, 0)):
        lib = _load()
        self._h = lib.o_attp_create(d, ell, q, seed, stream, {"exact": 0, "rand": 1}[fd])
        if not self._h:
            raise ValueError("bad ATTP parameters")
        if lib.o_attp_set_amplify(self._h, int(amplify[0]), int(amplify[1])) != 0:
            raise ValueError("bad amplification parameters")
        self.d, self.ell = d, ell

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.o_attp_destroy(self._h)
            self._h = None

    def update(self, rows):
        rows = _f64(np.atleast_2d(rows))
        if rows.shape[0] == 0:
            return
        _check(_lib.o_attp_update(self._h, _p(rows), rows.shape[0], rows.shape[1]), "attp_update")

    def gram_at(self, t):
        G = np.zeros((self.d, self.d))
        _check(_lib.o_attp_gram_at(self._h, t, _p(G)), "attp_gram_at")
        return G

    def query_at(self, t):
        out = np.zeros((self.ell, self.d))
        _check(_lib.o_attp_query_at(self._h, t, _p(out)), "attp_query_at")
        return out

    def stats(self):
        st = np.zeros(6, dtype=np.int64)
        _check(_lib.o_attp_stats(self._h, st.ctypes.data_as(_i64p)), "attp_stats")
        return dict(zip(["snapshots", "dirs", "fill", "shrinks", "simul_iters", "T"], st.tolist()))

    @property
    def theta(self):
        return _lib.o_attp_theta(self._h)

    def snapshots(self):
        out = []
        meta = np.zeros(3, dtype=np.int64)
        for e in range(self.stats()["snapshots"]):
            _check(_lib.o_attp_snapshot(self._h, e, meta.ctypes.data_as(_i64p), None, None), "attp_snapshot")
            xi = int(meta[0])
            Z, W = np.zeros((self.d, xi)), np.zeros((xi, self.d))
            _check(_lib.o_attp_snapshot(self._h, e, meta.ctypes.data_as(_i64p), _p(Z), _p(W)), "attp_snapshot")
            out.append({"xi": xi, "s": int(meta[1]), "t": int(meta[2]), "Z": Z, "W": W})
        return out

    def buffer(self):
        C = np.zeros((2 * self.ell, self.d))
        r = _lib.o_attp_buffer(self._h, _p(C))
        return C[:r].copy()


class P5:
    """Continuous distributed tracking (Algorithm "P5"): m sites and a
    coordinator, messages delivered at once."""

    STATS = ["fmsgs", "broadcasts", "snapshots", "dirs", "raw", "words", "shrinks", "T"]
    SITE = ["T", "fill", "shrinks", "snapshots", "dirs", "raw", "simul_iters"]

    def __init__(self, d, ell, m, q=1, seed=0, stream=0, fd="exact", amplify=(1, 0)):
        lib = _load()
        self._h = lib.o_p5_create(d, ell, m, q, seed, stream, {"exact": 0, "rand": 1}[fd])
        if not self._h:
            raise ValueError("bad P5 parameters")
        if lib.o_p5_set_amplify(self._h, int(amplify[0]), int(amplify[1])) != 0:
            raise ValueError("bad amplification parameters")
        self.d, self.ell, self.m = d, ell, m

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.o_p5_destroy(self._h)
            self._h = None

    def update(self, rows, sites):
        rows = _f64(np.atleast_2d(rows))
        sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int32).reshape(-1))
        if rows.shape[0] != sites.shape[0]:
            raise ValueError("one site per row")
        if rows.shape[0] == 0:
            return
        _check(_lib.o_p5_update(self._h, sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(rows),
                                rows.shape[0], rows.shape[1]), "p5_update")

    def gram(self):
        G = np.zeros((self.d, self.d))
        _check(_lib.o_p5_gram(self._h, _p(G)), "p5_gram")
        return G

    def query(self):
        out = np.zeros((self.ell, self.d))
        _check(_lib.o_p5_query(self._h, _p(out)), "p5_query")
        return out

    def stats(self):
        st = np.zeros(8, dtype=np.int64)
        _check(_lib.o_p5_stats(self._h, st.ctypes.data_as(_i64p)), "p5_stats")
        return dict(zip(self.STATS, st.tolist()))

    @property
    def fhat(self):
        return _lib.o_p5_fhat(self._h)

    def site(self, j):
        f3 = np.zeros(3)
        st = np.zeros(7, dtype=np.int64)
        C = np.zeros((2 * self.ell, self.d))
        _check(_lib.o_p5_site(self._h, j, _p(f3), st.ctypes.data_as(_i64p), _p(C)), "p5_site")
        out = dict(zip(self.SITE, st.tolist()))
        out.update(F=float(f3[0]), Fhat=float(f3[1]), theta=float(f3[2]), C=C[:out["fill"]].copy())
        return out


class COD:
    """AeroSketchCOD over a sliding window of N pairs, one level with dump
    threshold theta (Algorithm "AeroSketchCOD Framework")."""

    STATS = ["snapshots", "dirs", "fill", "reduces", "simul_iters", "queue", "T"]

    def __init__(self, dx, dy, ell, N, theta, q=1, seed=0, stream=0):
        lib = _load()
        self._h = lib.o_cod_create(dx, dy, ell, int(N), float(theta), q, seed, stream)
        if not self._h:
            raise ValueError("bad COD parameters")
        self.dx, self.dy, self.ell = dx, dy, ell

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.o_cod_destroy(self._h)
            self._h = None

    def update(self, X, Y):
        X = _f64(np.atleast_2d(X))
        Y = _f64(np.atleast_2d(Y))
        if X.shape[0] != Y.shape[0]:
            raise ValueError("X and Y need the same number of rows")
        if X.shape[0] == 0:
            return
        _check(_lib.o_cod_update(self._h, _p(X), X.shape[1], _p(Y), Y.shape[1], X.shape[0]), "cod_update")

    def product(self):
        M = np.zeros((self.dx, self.dy))
        _check(_lib.o_cod_product(self._h, _p(M)), "cod_product")
        return M

    def query(self):
        A = np.zeros((self.dx, self.ell))
        B = np.zeros((self.dy, self.ell))
        _check(_lib.o_cod_query(self._h, _p(A), _p(B)), "cod_query")
        return A, B

    def stats(self):
        st = np.zeros(7, dtype=np.int64)
        _check(_lib.o_cod_stats(self._h, st.ctypes.data_as(_i64p)), "cod_stats")
        return dict(zip(self.STATS, st.tolist()))

    def buffers(self):
        A = np.zeros((2 * self.ell, self.dx))
        B = np.zeros((2 * self.ell, self.dy))
        r = _lib.o_cod_buffers(self._h, _p(A), _p(B))
        return A[:r].copy(), B[:r].copy()

    def snapshots(self):
        out = []
        meta = np.zeros(3, dtype=np.int64)
        for e in range(self.stats()["queue"]):
            _check(_lib.o_cod_snapshot(self._h, e, meta.ctypes.data_as(_i64p), None, None, None, None), "cod_snap")
            xi = int(meta[0])
            Z, ZM = np.zeros((self.dx, xi)), np.zeros((xi, self.dy))
            MH, H = np.zeros((self.dx, xi)), np.zeros((self.dy, xi))
            _check(_lib.o_cod_snapshot(self._h, e, meta.ctypes.data_as(_i64p), _p(Z), _p(ZM), _p(MH), _p(H)),
                   "cod_snap")
            out.append({"xi": xi, "s": int(meta[1]), "t": int(meta[2]), "Z": Z, "ZM": ZM, "MH": MH, "H": H})
        return out


def cod_reduce(A, B, ell):
    """The co-occurring-directions reduce of row buffers A (r x dx), B (r x dy)."""
    _load()
    A = np.ascontiguousarray(A, dtype=np.float64).copy()
    B = np.ascontiguousarray(B, dtype=np.float64).copy()
    _check(_lib.o_cod_reduce(_p(A), _p(B), A.shape[0], A.shape[1], B.shape[1], ell), "cod_reduce")
    return A, B
