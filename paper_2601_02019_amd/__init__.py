"""MI355X (gfx950) Frequent-Directions sketches with a randomized shrink.

Python front end over the C ABI in include/sketch.h.  The functions below
have the C names and only marshal arguments; the ``Sketch`` class wraps a
handle for convenience.  Device rows are torch tensors on the sketch's GPU;
host rows may be numpy arrays or CPU tensors.
"""
import atexit
import ctypes
import sys
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import (  # noqa: F401
    SK_BF16, SK_EDEVICE, SK_EINVAL, SK_ENOMEM, SK_ESHAPE, SK_ESTATE, SK_EUNSUPPORTED, SK_F32,
    SK_ATTP, SK_COD, SK_P5, SK_F64, SK_OK, SK_PERSISTENT, SK_SHRINK_EXACT, SK_SHRINK_RAND, SK_WINDOW, SketchError,
    sk_completion, sk_server_config, sk_server_stats, sketch_config, sketch_info_t,
)

_TORCH_DT = {torch.float64: SK_F64, torch.float32: SK_F32, torch.bfloat16: SK_BF16}
_NP_DT = {np.dtype(np.float64): SK_F64, np.dtype(np.float32): SK_F32}
_NAME_DT = {"f64": SK_F64, "f32": SK_F32, "bf16": SK_BF16}


# Live owning wrappers.  They are closed from an atexit hook, which runs
# before the interpreter tears down modules and before the HIP runtime's own
# exit handlers: a handle destroyed later (from __del__ during finalisation)
# would synchronise streams and free memory while the runtime, and any
# profiler attached to it, are already shutting down.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    objs = list(_LIVE)
    # servers first: they own their streams' sketches
    for o in sorted(objs, key=lambda o: 0 if isinstance(o, Server) else 1):
        try:
            o.close()
        except Exception:
            pass


def _finalizing():
    return sys.is_finalizing()


def _dt(x):
    if isinstance(x, int):
        return x
    return _NAME_DT[x]


def sketch_config_init():
    cfg = sketch_config()
    _lib.check(_lib.load().sketch_config_init(ctypes.byref(cfg)), "sketch_config_init")
    return cfg


def sketch_create(cfg):
    h = ctypes.c_void_p()
    _lib.check(_lib.load().sketch_create(ctypes.byref(cfg), ctypes.byref(h)), "sketch_create")
    return h


def _rows_arg(rows):
    """(pointer, n, ld, dtype, on_device, keepalive) for a 2-D row block."""
    if isinstance(rows, torch.Tensor):
        if rows.dim() != 2:
            raise ValueError("rows must be 2-D")
        if rows.stride(1) != 1:
            rows = rows.contiguous()
        dt = _TORCH_DT[rows.dtype]
        return rows.data_ptr(), rows.shape[0], rows.stride(0), dt, int(rows.is_cuda), rows
    a = np.asarray(rows)
    if a.ndim != 2:
        raise ValueError("rows must be 2-D")
    if a.dtype not in _NP_DT:
        a = a.astype(np.float64)
    a = np.ascontiguousarray(a)
    return a.ctypes.data, a.shape[0], a.shape[1], _NP_DT[a.dtype], 0, a


def sketch_update(h, rows):
    ptr, n, ld, dt, dev, keep = _rows_arg(rows)
    _lib.check(_lib.load().sketch_update(h, ctypes.c_void_p(ptr), n, ld, dt, dev), "sketch_update")
    return keep


def sketch_update_csr(h, indptr, indices, values):
    on_dev = isinstance(indptr, torch.Tensor) and indptr.is_cuda
    if on_dev:
        ip, ix, vv = indptr.contiguous(), indices.contiguous(), values.contiguous()
        assert ip.dtype == torch.int64 and ix.dtype == torch.int32 and vv.dtype == torch.float32
        ptrs = (ip.data_ptr(), ix.data_ptr(), vv.data_ptr())
        keep = (ip, ix, vv)
    else:
        ip = np.ascontiguousarray(indptr, dtype=np.int64)
        ix = np.ascontiguousarray(indices, dtype=np.int32)
        vv = np.ascontiguousarray(values, dtype=np.float32)
        ptrs = (ip.ctypes.data, ix.ctypes.data, vv.ctypes.data)
        keep = (ip, ix, vv)
    n = (ip.shape[0] - 1)
    _lib.check(_lib.load().sketch_update_csr(h, *(ctypes.c_void_p(p) for p in ptrs), n, int(on_dev)),
               "sketch_update_csr")
    return keep


def sketch_query(h, out):
    """Writes the ell x d sketch into ``out`` (torch tensor, CUDA or CPU, or
    a numpy array), float64 or float32, contiguous."""
    if isinstance(out, torch.Tensor):
        assert out.is_contiguous()
        dt = _TORCH_DT[out.dtype]
        _lib.check(_lib.load().sketch_query(h, ctypes.c_void_p(out.data_ptr()), dt, int(out.is_cuda)),
                   "sketch_query")
    else:
        assert out.flags["C_CONTIGUOUS"]
        _lib.check(_lib.load().sketch_query(h, ctypes.c_void_p(out.ctypes.data), _NP_DT[out.dtype], 0),
                   "sketch_query")
    return out


def sketch_query_at(h, t, out):
    """ATTP sketches: writes the ell x d sketch of the first t rows into
    ``out`` (as sketch_query)."""
    if isinstance(out, torch.Tensor):
        assert out.is_contiguous()
        _lib.check(_lib.load().sketch_query_at(h, int(t), ctypes.c_void_p(out.data_ptr()), _TORCH_DT[out.dtype],
                                               int(out.is_cuda)), "sketch_query_at")
    else:
        assert out.flags["C_CONTIGUOUS"]
        _lib.check(_lib.load().sketch_query_at(h, int(t), ctypes.c_void_p(out.ctypes.data), _NP_DT[out.dtype], 0),
                   "sketch_query_at")
    return out


def window_advance(h, t_now):
    _lib.check(_lib.load().window_advance(h, int(t_now)), "window_advance")


def p5_update(h, rows, sites):
    """Rows arrive in order, row e at site sites[e] (Algorithm "P5")."""
    ptr, n, ld, dt, dev, keep = _rows_arg(rows)
    st = np.ascontiguousarray(np.asarray(sites, dtype=np.int32).reshape(-1))
    if st.shape[0] != n:
        raise ValueError("p5_update: one site per row")
    _lib.check(_lib.load().p5_update(h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.c_void_p(ptr),
                                     n, ld, dt, dev), "p5_update")
    return keep


def p5_stats(h):
    st = (ctypes.c_int64 * 8)()
    _lib.check(_lib.load().p5_stats(h, st), "p5_stats")
    keys = ["fmsgs", "broadcasts", "snapshots", "dirs", "raw", "words", "shrinks", "T"]
    return dict(zip(keys, list(st)))


def p5_coordinator(h, gram=None):
    """(Fhat, B): B into ``gram`` (a d x d FP64 CUDA tensor) when given."""
    f = ctypes.c_double()
    ptr = ctypes.c_void_p(gram.data_ptr()) if gram is not None else None
    if gram is not None:
        assert gram.is_cuda and gram.dtype == torch.float64 and gram.is_contiguous()
    _lib.check(_lib.load().p5_coordinator(h, ctypes.byref(f), ptr, 1), "p5_coordinator")
    return f.value, gram


def cod_update(h, X, Y):
    """Pairs (row e of X, row e of Y) arrive in order (Algorithm "AeroSketchCOD Framework")."""
    px, n, ldx, dt, dev, kx = _rows_arg(X)
    py, ny, ldy, dty, devy, ky = _rows_arg(Y)
    if n != ny or dt != dty or dev != devy:
        raise ValueError("cod_update: X and Y need the same rows, dtype and memory")
    _lib.check(_lib.load().cod_update(h, ctypes.c_void_p(px), ldx, ctypes.c_void_p(py), ldy, n, dt, dev),
               "cod_update")
    return kx, ky


def cod_query(h, A_out, B_out):
    for t in (A_out, B_out):
        assert t.is_cuda and t.is_contiguous() and t.dtype in (torch.float64, torch.float32)
    _lib.check(_lib.load().cod_query(h, ctypes.c_void_p(A_out.data_ptr()), ctypes.c_void_p(B_out.data_ptr()),
                                     _TORCH_DT[A_out.dtype], 1), "cod_query")
    return A_out, B_out


def cod_product(h, M_out):
    assert M_out.is_cuda and M_out.is_contiguous() and M_out.dtype == torch.float64
    _lib.check(_lib.load().cod_product(h, ctypes.c_void_p(M_out.data_ptr()), 1), "cod_product")
    return M_out


def window_stats(h, level):
    st = (ctypes.c_int64 * 6)()
    _lib.check(_lib.load().window_stats(h, level, st), "window_stats")
    keys = ["dumps", "raw", "dirs", "fill", "queue", "shrinks"]
    return dict(zip(keys, list(st)))


def _handles(srcs):
    arr = (ctypes.c_void_p * len(srcs))()
    for i, s in enumerate(srcs):
        arr[i] = s.value if isinstance(s, ctypes.c_void_p) else s.handle.value
    return arr


def sketch_merge(dst, srcs):
    _lib.check(_lib.load().sketch_merge(dst, _handles(srcs), len(srcs)), "sketch_merge")


def sketch_merge_tree(dst, srcs):
    _lib.check(_lib.load().sketch_merge_tree(dst, _handles(srcs), len(srcs)), "sketch_merge_tree")


def sketch_sync(h):
    _lib.check(_lib.load().sketch_sync(h), "sketch_sync")


def sketch_destroy(h):
    _lib.check(_lib.load().sketch_destroy(h), "sketch_destroy")


def sketch_debug_fail_solver(h):
    _lib.check(_lib.load().sketch_debug_fail_solver(h), "sketch_debug_fail_solver")


def server_debug_fail_solver(s, sid):
    _lib.check(_lib.load().server_debug_fail_solver(s, sid), "server_debug_fail_solver")


def sketch_last_error():
    return _lib.load().sketch_last_error().decode(errors="replace")


def sketch_info(h):
    info = sketch_info_t()
    _lib.check(_lib.load().sketch_info(h, ctypes.byref(info)), "sketch_info")
    return {f: getattr(info, f) for f, _ in sketch_info_t._fields_}


def sketch_set_memory_budget(nbytes):
    _lib.check(_lib.load().sketch_set_memory_budget(int(nbytes)), "sketch_set_memory_budget")


def sketch_memory_in_use():
    return _lib.load().sketch_memory_in_use()


def sketch_update_batch(sketches, rows_list, dtype=None, _entry="sketch_update_batch"):
    """Batched update: rows_list[i] is a contiguous CUDA tensor (n_i x d_i)."""
    n = len(sketches)
    hs = _handles(sketches)
    ptrs = (ctypes.c_void_p * n)()
    ns = (ctypes.c_int64 * n)()
    dt = None
    for i, r in enumerate(rows_list):
        assert isinstance(r, torch.Tensor) and r.is_cuda and r.is_contiguous()
        ptrs[i] = r.data_ptr()
        ns[i] = r.shape[0]
        dt = _TORCH_DT[r.dtype] if dt is None else dt
    if dtype is not None:
        dt = _dt(dtype)
    _lib.check(getattr(_lib.load(), _entry)(hs, ptrs, ns, n, SK_F32 if dt is None else dt), _entry)


def sketch_update_batch_noalloc(sketches, rows_list, dtype=None):
    """sketch_update_batch through the entry point that allocates nothing (task
    records in the library's static device array)."""
    sketch_update_batch(sketches, rows_list, dtype, _entry="sketch_update_batch_noalloc")


def sketch_update_csr_batch(sketches, csr_list):
    """Batched CSR update: csr_list[i] = (indptr int64, indices int32, values
    float32), contiguous CUDA tensors; sketch i takes indptr.shape[0] - 1 rows."""
    n = len(sketches)
    hs = _handles(sketches)
    ip, ix, vv = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
    ns = (ctypes.c_int64 * n)()
    for i, (a, b, c) in enumerate(csr_list):
        assert a.is_cuda and a.dtype == torch.int64 and b.dtype == torch.int32 and c.dtype == torch.float32
        assert a.is_contiguous() and b.is_contiguous() and c.is_contiguous()
        ip[i], ix[i], vv[i] = a.data_ptr(), b.data_ptr(), c.data_ptr()
        ns[i] = a.shape[0] - 1
    _lib.check(_lib.load().sketch_update_csr_batch(hs, ip, ix, vv, ns, n), "sketch_update_csr_batch")


def sketch_profile_enable(h, stages="all"):
    """Event-times the given stages (names of _lib.SK_STAGE, or "all")."""
    if stages == "all":
        mask = _lib.SK_STAGE_ALL
    elif isinstance(stages, int):
        mask = stages
    else:
        mask = 0
        for st in stages:
            mask |= _lib.SK_STAGE[st]
    _lib.check(_lib.load().sketch_profile_enable(h, mask), "sketch_profile_enable")


def sketch_profile_read(h):
    """{stage: (calls, total_ms)} plus solver counters (calls = 0)."""
    buf = (_lib.sketch_stage_time * 64)()
    n = ctypes.c_int32(0)
    _lib.check(_lib.load().sketch_profile_read(h, buf, 64, ctypes.byref(n)), "sketch_profile_read")
    return {buf[i].name.decode(): (buf[i].calls, buf[i].total_ms) for i in range(min(n.value, 64))}


def make_config(d, ell, kind="persistent", shrink="exact", state_dtype="f64", proj_dtype="f64", q=1,
                oversample=0, window_N=0, R=1.0, seed=0, stream_id=0, device=0, amplify=(1, 0), sites=0,
                d_y=0, theta=0.0):
    cfg = sketch_config_init()
    cfg.d, cfg.ell = d, ell
    cfg.kind = {"persistent": SK_PERSISTENT, "window": SK_WINDOW, "attp": SK_ATTP, "p5": SK_P5, "cod": SK_COD}[kind]
    cfg.shrink = {"exact": SK_SHRINK_EXACT, "rand": SK_SHRINK_RAND}[shrink]
    cfg.state_dtype = _dt(state_dtype)
    cfg.proj_dtype = _dt(proj_dtype)
    cfg.q, cfg.oversample = q, oversample
    cfg.window_N, cfg.R = int(window_N), float(R)
    cfg.seed, cfg.stream_id, cfg.device = seed, stream_id, device
    cfg.amplify_r, cfg.amplify_s = int(amplify[0]), int(amplify[1])
    cfg.sites = int(sites)
    cfg.d_y, cfg.theta = int(d_y), float(theta)
    return cfg


# ------------------------------------------------------------------ serving
def server_config_init():
    cfg = sk_server_config()
    _lib.check(_lib.load().server_config_init(ctypes.byref(cfg)), "server_config_init")
    return cfg


def server_create(cfg):
    h = ctypes.c_void_p()
    _lib.check(_lib.load().server_create(ctypes.byref(cfg), ctypes.byref(h)), "server_create")
    return h


def server_open(s, cfg):
    sid = ctypes.c_int64()
    _lib.check(_lib.load().server_open(s, ctypes.byref(cfg), ctypes.byref(sid)), "server_open")
    return sid.value


def server_submit(s, sid, rows, arrival):
    assert isinstance(rows, torch.Tensor) and rows.is_cuda and rows.is_contiguous() and rows.dim() == 2
    t = ctypes.c_int64()
    _lib.check(_lib.load().server_submit(s, sid, ctypes.c_void_p(rows.data_ptr()), rows.shape[0],
                                         _TORCH_DT[rows.dtype], float(arrival), ctypes.byref(t)),
               "server_submit")
    return t.value


def server_tick(s):
    n = ctypes.c_int32()
    _lib.check(_lib.load().server_tick(s, ctypes.byref(n)), "server_tick")
    return n.value


_POLL_FIELDS = [f for f, _ in sk_completion._fields_]


def server_poll(s, max_n=1024, buf=None):
    if buf is None:
        buf = (sk_completion * max_n)()
    n = ctypes.c_int32()
    _lib.check(_lib.load().server_poll(s, buf, len(buf), ctypes.byref(n)), "server_poll")
    return [{f: getattr(buf[i], f) for f in _POLL_FIELDS} for i in range(n.value)]


def server_drain(s):
    _lib.check(_lib.load().server_drain(s), "server_drain")


def server_query(s, sid, out):
    assert isinstance(out, torch.Tensor) and out.is_contiguous()
    _lib.check(_lib.load().server_query(s, sid, ctypes.c_void_p(out.data_ptr()), _TORCH_DT[out.dtype],
                                        int(out.is_cuda)), "server_query")
    return out


def server_close(s, sid):
    _lib.check(_lib.load().server_close(s, sid), "server_close")


def server_stats(s):
    st = sk_server_stats()
    _lib.check(_lib.load().server_stats(s, ctypes.byref(st)), "server_stats")
    return {f: getattr(st, f) for f, _ in sk_server_stats._fields_}


def server_now(s):
    return _lib.load().server_now(s)


def server_destroy(s):
    _lib.check(_lib.load().server_destroy(s), "server_destroy")


class Server:
    """Owning wrapper of a serving loop.  Keeps each submitted tensor alive
    until its burst has been reported complete by ``poll``.  ``clock``: an
    optional Python callable returning seconds (a fake clock for tests).
    ``stream``: a torch stream for all of the server's work (default: the
    current one), or False for a stream of the server's own."""

    def __init__(self, device=0, max_inflight=2, memory_budget=0, max_rows_per_tick=0, clock=None,
                 stream=None, max_shrinks_per_tick=0):
        cfg = server_config_init()
        cfg.device, cfg.max_inflight = device, max_inflight
        cfg.memory_budget, cfg.max_rows_per_tick = int(memory_budget), int(max_rows_per_tick)
        cfg.max_shrinks_per_tick = int(max_shrinks_per_tick)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        if stream is not False:
            # all work on the torch stream, ordered after the tensors' producers
            cfg.hip_stream = ctypes.c_void_p(stream.cuda_stream)
            cfg.use_given_stream = 1
        self._clock = None
        if clock is not None:
            self._clock = _lib.CLOCK_FN(lambda ctx: float(clock()))
            cfg.clock = self._clock
        self.device = device
        self.handle = server_create(cfg)
        _LIVE.add(self)
        self._rows = {}
        self._shape = {}
        self._pollbuf = (sk_completion * 1024)()

    def open(self, d, ell, **kw):
        sid = server_open(self.handle, make_config(d, ell, device=self.device, **kw))
        self._shape[sid] = (d, ell)
        return sid

    def submit(self, sid, rows, arrival=None):
        if arrival is None:
            arrival = self.now()
        t = server_submit(self.handle, sid, rows, arrival)
        self._rows[t] = rows
        return t

    def tick(self):
        return server_tick(self.handle)

    def poll(self):
        out = []
        while True:
            got = server_poll(self.handle, buf=self._pollbuf)
            for c in got:
                self._rows.pop(c["ticket"], None)
            out.extend(got)
            if len(got) < len(self._pollbuf):
                return out

    def drain(self):
        server_drain(self.handle)

    def query(self, sid, dtype=torch.float64):
        d, ell = self._shape[sid]
        out = torch.empty((ell, d), dtype=dtype, device=f"cuda:{self.device}")
        return server_query(self.handle, sid, out)

    def close_stream(self, sid):
        server_close(self.handle, sid)

    def debug_fail_solver(self, sid):
        server_debug_fail_solver(self.handle, sid)

    def stats(self):
        return server_stats(self.handle)

    def now(self):
        return server_now(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            server_destroy(self.handle)
            self.handle = None
            self._rows.clear()

    def __del__(self):
        if _finalizing():  # the atexit hook has closed every live handle
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Sketch:
    """Owning wrapper of one sketch handle."""

    def __init__(self, d, ell, kind="persistent", shrink="exact", state_dtype="f64",
                 proj_dtype="f64", q=1, oversample=0, window_N=0, R=1.0, seed=0, stream_id=0,
                 device=0, stream=None, amplify=(1, 0), sites=0, d_y=0, theta=0.0):
        cfg = make_config(d, ell, kind, shrink, state_dtype, proj_dtype, q, oversample, window_N, R,
                          seed, stream_id, device, amplify, sites, d_y, theta)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        if stream is not False:
            # order the sketch's work on the torch stream (handle 0 is the
            # default stream, which the C ABI takes only with this flag)
            cfg.hip_stream = ctypes.c_void_p(stream.cuda_stream)
            cfg.use_given_stream = 1
        self.d, self.ell, self.d_y = d, ell, d_y
        self.device = device
        self.handle = sketch_create(cfg)
        _LIVE.add(self)
        self._keep = []

    def update(self, rows):
        keep = sketch_update(self.handle, rows)
        if isinstance(rows, torch.Tensor) and rows.is_cuda:
            self._keep.append(keep)
            if len(self._keep) > 64:
                self.sync()
        return self

    def update_csr(self, indptr, indices, values):
        keep = sketch_update_csr(self.handle, indptr, indices, values)
        if isinstance(indptr, torch.Tensor) and indptr.is_cuda:
            self._keep.append(keep)
        return self

    def query(self, dtype=torch.float64, out=None):
        if out is None:
            out = torch.empty((self.ell, self.d), dtype=dtype, device=f"cuda:{self.device}")
        sketch_query(self.handle, out)
        self._keep.clear()
        return out

    def query_at(self, t, dtype=torch.float64, out=None):
        if out is None:
            out = torch.empty((self.ell, self.d), dtype=dtype, device=f"cuda:{self.device}")
        sketch_query_at(self.handle, t, out)
        self._keep.clear()
        return out

    def advance(self, t_now):
        window_advance(self.handle, t_now)

    def window_stats(self, level):
        return window_stats(self.handle, level)

    def p5_update(self, rows, sites):
        p5_update(self.handle, rows, sites)  # returns once the rows are processed
        return self

    def p5_stats(self):
        return p5_stats(self.handle)

    def cod_update(self, X, Y):
        cod_update(self.handle, X, Y)  # returns once the pairs are processed
        return self

    def cod_query(self, dtype=torch.float64):
        A = torch.empty((self.d, self.ell), dtype=dtype, device=f"cuda:{self.device}")
        B = torch.empty((self.d_y, self.ell), dtype=dtype, device=f"cuda:{self.device}")
        return cod_query(self.handle, A, B)

    def cod_product(self):
        M = torch.empty((self.d, self.d_y), dtype=torch.float64, device=f"cuda:{self.device}")
        return cod_product(self.handle, M)

    def p5_coordinator(self):
        g = torch.empty((self.d, self.d), dtype=torch.float64, device=f"cuda:{self.device}")
        f, _ = p5_coordinator(self.handle, g)
        return f, g

    def merge(self, srcs):
        sketch_merge(self.handle, srcs)

    def merge_tree(self, srcs):
        sketch_merge_tree(self.handle, srcs)

    def sync(self):
        sketch_sync(self.handle)
        self._keep.clear()

    def info(self):
        return sketch_info(self.handle)

    def profile(self, stages="all"):
        sketch_profile_enable(self.handle, stages)

    def profile_read(self):
        return sketch_profile_read(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            sketch_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        if _finalizing():  # the atexit hook has closed every live handle
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
