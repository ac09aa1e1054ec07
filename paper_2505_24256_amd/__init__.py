"""MI355X (gfx950) sparse Zippel reconstruction over F_p.

Thin ctypes binding of ``libzippel_hip.so`` (C ABI in ``include/zippel.h``).
Every step of the reconstruction runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch is used for device memory and streams.
The library must be built (``paper_2505_24256_amd.build.build()``); importing
the binding on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzippel_hip.so")

ZR_OK, ZR_EINVAL, ZR_ENOTPRIME, ZR_ESINGULAR, ZR_EDEGEN = 0, -1, -2, -3, -4
ZR_EPROBE, ZR_ENORM, ZR_ENOMEM, ZR_EDEVICE, ZR_EBLACKBOX = -5, -6, -7, -8, -9

# every symbol include/zippel.h declares
EXPORTS = [
    "zr_strerror", "zr_last_error", "zr_poly_free", "zr_thiele_nodes", "zr_schedule", "zr_is_prime", "zippel_reconstruct",
    "zippel_balanced_reconstruct", "vandermonde_solve_batch", "zr_copy_h2d", "zr_copy_d2h", "zr_copy_d2d",
    "zr_recorder_create", "zr_recorder_destroy", "zr_recorder_rewind", "zr_recorder_set_replay",
    "zr_recorder_blackbox", "zr_timing_enable", "zr_timing_reset", "zr_timing_get", "zr_last_counters",
    "zr_microbench", "zippel_reconstruct_batch", "zr_autotune", "zr_tuning_get", "zr_tuning_set",
    "zr_server_create", "zr_server_destroy", "zr_server_submit", "zr_server_step", "zr_server_poll",
    "zr_server_get_stats", "zr_server_finished", "zr_batch_graphs", "zr_solve_variant", "zr_thiele_slices",
    "zr_vandermonde_solve", "zr_vandermonde_solve_noalloc", "zippel_reconstruct_rational", "zr_qpoly_free",
    "zr_skeleton_solve", "zippel_reconstruct_multi", "zippel_reconstruct_adaptive",
]
MB_KINDS = {"mad_u64_u32": 0, "mul_lo_u32": 1, "mul_hi_u32": 2, "add_u32": 3, "mac192": 4, "shoup": 5, "copy": 6,
            "lds_read": 7, "lds_bcast": 8}


class ZippelError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = lib().zr_strerror(code).decode() if _LIB is not None else str(code)
        detail = lib().zr_last_error().decode() if _LIB is not None else ""
        super().__init__(f"{what}: status {code} ({msg}){'; ' + detail if detail else ''}")
        self.code = code


class ZrPoints(ctypes.Structure):
    _fields_ = [("nvars", ctypes.c_uint32), ("k", ctypes.c_uint32), ("i_first", ctypes.c_uint64),
                ("ni", ctypes.c_uint64), ("nj", ctypes.c_uint64), ("y", ctypes.POINTER(ctypes.c_uint64)),
                ("anchor", ctypes.POINTER(ctypes.c_uint64)), ("xk", ctypes.POINTER(ctypes.c_uint64)),
                ("p", ctypes.c_uint64), ("nexpr", ctypes.c_uint32)]


class ZrPoly(ctypes.Structure):
    _fields_ = [("nvars", ctypes.c_uint32), ("nterms", ctypes.c_uint64), ("exps", ctypes.POINTER(ctypes.c_uint16)),
                ("coeffs", ctypes.POINTER(ctypes.c_uint64))]


class ZrQPoly(ctypes.Structure):
    _fields_ = [("nvars", ctypes.c_uint32), ("nterms", ctypes.c_uint64), ("nwords", ctypes.c_uint32),
                ("nprimes", ctypes.c_uint32), ("exps", ctypes.POINTER(ctypes.c_uint16)),
                ("num", ctypes.POINTER(ctypes.c_uint64)), ("neg", ctypes.POINTER(ctypes.c_uint8)),
                ("den", ctypes.POINTER(ctypes.c_uint64))]


class ZrParams(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint64), ("nvars", ctypes.c_uint32), ("deg", ctypes.c_void_p),
                ("deg_den", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("y", ctypes.c_void_p),
                ("anchor", ctypes.c_void_p), ("nodes", ctypes.c_void_p), ("nnodes", ctypes.c_void_p),
                ("nprobes", ctypes.c_uint32), ("probes", ctypes.c_void_p), ("last_stage", ctypes.c_uint32),
                ("first_stage", ctypes.c_uint32), ("start", ctypes.c_void_p)]


class ZrBandChoice(ctypes.Structure):
    _fields_ = [("packed", ctypes.c_uint32), ("min_chunk", ctypes.c_uint32)]


NBANDS = 5


class ZrServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "completed", "failed", "steps", "footprint",
                                               "peak_footprint", "active", "pending", "peak_active")]


class ZrCounters(ctypes.Structure):
    _fields_ = [("mulmods", ctypes.c_uint64), ("solve_mulmods", ctypes.c_uint64), ("vsolve_terms", ctypes.c_uint64),
                ("stages", ctypes.c_uint32), ("max_t", ctypes.c_uint64), ("dot_products", ctypes.c_uint64),
                ("chain_steps", ctypes.c_uint64)]


BLACKBOX_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ZrPoints), ctypes.c_void_p,
                               ctypes.c_void_p)

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_2505_24256_amd.build.build())")
        # PyTorch ships its own copy of the HIP runtime; loading it first makes
        # the library bind to that same copy (one runtime per process)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, vp, sz, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        L.zr_strerror.restype = ctypes.c_char_p
        L.zr_last_error.restype = ctypes.c_char_p
        L.zr_last_error.argtypes = []
        L.zr_strerror.argtypes = [i32]
        L.zr_poly_free.argtypes = [ctypes.POINTER(ZrPoly)]
        L.zr_poly_free.restype = None
        L.zr_thiele_nodes.restype = u32
        L.zr_thiele_nodes.argtypes = [u32, u32]
        L.zr_schedule.argtypes = [u64, u32, vp, u64, u32, vp, vp, vp, vp]
        L.zr_is_prime.argtypes = [u64]
        L.zippel_reconstruct.argtypes = [ctypes.POINTER(ZrParams), vp, vp, vp, ctypes.POINTER(ZrPoly)]
        L.zippel_balanced_reconstruct.argtypes = [ctypes.POINTER(ZrParams), vp, vp, vp, ctypes.POINTER(ZrPoly),
                                                  ctypes.POINTER(ZrPoly)]
        L.vandermonde_solve_batch.argtypes = [sz, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.zr_thiele_slices.argtypes = [u64, u32, u32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.zr_vandermonde_solve.argtypes = [u64, u32, u32, vp, vp, vp, vp, vp]
        L.zr_vandermonde_solve_noalloc.argtypes = [u64, u32, u32, vp, vp, vp, vp, vp]
        L.zippel_reconstruct_rational.argtypes = [ctypes.POINTER(ZrParams), vp, u32, vp, vp, vp,
                                                  ctypes.POINTER(ZrQPoly)]
        L.zr_qpoly_free.argtypes = [ctypes.POINTER(ZrQPoly)]
        L.zr_qpoly_free.restype = None
        L.zr_skeleton_solve.argtypes = [u64, u32, u32, vp, vp, vp, vp, vp, vp]
        L.zippel_reconstruct_multi.argtypes = [ctypes.POINTER(ZrParams), u32, vp, vp, vp, vp, ctypes.POINTER(ZrPoly)]
        L.zippel_reconstruct_adaptive.argtypes = [ctypes.POINTER(ZrParams), u32, vp, vp, vp, ctypes.POINTER(ZrPoly),
                                                  vp]
        L.zippel_reconstruct_batch.argtypes = [u32, ctypes.POINTER(ZrParams), vp, vp, vp, ctypes.POINTER(ZrPoly),
                                               vp]
        L.zr_autotune.argtypes = [u64, vp, ctypes.POINTER(ZrBandChoice)]
        L.zr_solve_variant.argtypes = [i32]
        L.zr_batch_graphs.argtypes = [i32]
        L.zr_batch_graphs.restype = None
        L.zr_server_create.argtypes = [ctypes.POINTER(vp), u64, u64, u32, vp]
        L.zr_server_destroy.argtypes = [vp]
        L.zr_server_destroy.restype = None
        L.zr_server_submit.argtypes = [vp, ctypes.POINTER(ZrParams), i32, u64, vp, vp, ctypes.POINTER(u64)]
        L.zr_server_step.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]
        L.zr_server_poll.argtypes = [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(ZrPoly), ctypes.POINTER(ZrPoly)]
        L.zr_server_get_stats.argtypes = [vp, ctypes.POINTER(ZrServerStats)]
        L.zr_server_finished.argtypes = [vp, ctypes.POINTER(u64), u32]
        L.zr_server_finished.restype = u32
        L.zr_tuning_get.argtypes = [ctypes.POINTER(ZrBandChoice)]
        L.zr_tuning_set.argtypes = [ctypes.POINTER(ZrBandChoice)]
        for n in ("zr_copy_h2d", "zr_copy_d2h", "zr_copy_d2d"):
            getattr(L, n).argtypes = [vp, vp, sz, vp]
        L.zr_recorder_create.argtypes = [ctypes.POINTER(vp), vp, vp]
        L.zr_recorder_destroy.argtypes = [vp]
        L.zr_recorder_destroy.restype = None
        L.zr_recorder_rewind.argtypes = [vp]
        L.zr_recorder_rewind.restype = None
        L.zr_recorder_set_replay.argtypes = [vp, i32]
        L.zr_recorder_set_replay.restype = None
        L.zr_timing_enable.argtypes = [i32]
        L.zr_timing_enable.restype = None
        L.zr_timing_reset.restype = None
        L.zr_timing_get.restype = u64
        L.zr_timing_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]
        L.zr_last_counters.argtypes = [ctypes.POINTER(ZrCounters)]
        L.zr_last_counters.restype = None
        L.zr_microbench.argtypes = [i32, u32, u32, u64, vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        _LIB = L
    return _LIB


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None or a.size == 0 else a.ctypes.data


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def is_prime(n: int) -> bool:
    return bool(lib().zr_is_prime(n))


def thiele_nodes(deg_num: int, deg_den: int) -> int:
    return int(lib().zr_thiele_nodes(deg_num, deg_den))


def schedule(p: int, nnodes: Sequence[int], seed: int, nprobes: int = 0):
    """The library's seeded schedule: (y, anchor, nodes_concat, probes)."""
    nv = len(nnodes)
    cnt = _u32(nnodes)
    y = np.zeros(nv, np.uint64)
    a = np.zeros(nv, np.uint64)
    nodes = np.zeros(max(int(cnt.sum()), 1), np.uint64)
    pr = np.zeros(max(nprobes * nv, 1), np.uint64)
    st = lib().zr_schedule(p, nv, _ptr(cnt), seed, nprobes, y.ctypes.data, a.ctypes.data, nodes.ctypes.data,
                           pr.ctypes.data)
    if st != ZR_OK:
        raise ZippelError(st, "zr_schedule")
    return y, a, nodes[:int(cnt.sum())], pr[:nprobes * nv].reshape(nprobes, nv)


# ---------------------------------------------------------------------------
# black boxes

class HostBlackBox:
    """Wraps a host evaluator ``f(k, i_first, ni, y, anchor, xk) -> uint64[nj*ni]``
    (e.g. ``synth.BlackBox.eval``) as a device black box: values are computed on
    the host and copied to the device buffer the library provides."""

    def __init__(self, fn: Callable, nvars: int, with_prime: bool = False):
        self.fn = fn
        self.nvars = nvars
        self.with_prime = with_prime  # fn(p, k, ...) instead of fn(k, ...): boxes asked modulo several primes
        self.calls = 0
        self.error: Optional[BaseException] = None
        self._cb = BLACKBOX_FN(self._call)

    def _call(self, ctx, pts_ptr, d_vals, stream):
        try:
            pts = pts_ptr.contents
            nv = pts.nvars
            y = np.ctypeslib.as_array(pts.y, shape=(nv,)).copy() if nv else np.zeros(0, np.uint64)
            a = np.ctypeslib.as_array(pts.anchor, shape=(nv,)).copy()
            xk = np.ctypeslib.as_array(pts.xk, shape=(pts.nj,)).copy()
            args = (pts.k, pts.i_first, pts.ni, y, a, xk)
            vals = _u64(self.fn(pts.p, *args) if self.with_prime else self.fn(*args)).reshape(-1)
            if vals.size != pts.ni * pts.nj * max(pts.nexpr, 1):
                return 11
            st = lib().zr_copy_h2d(d_vals, vals.ctypes.data, vals.nbytes, stream)
            self.calls += 1
            return 0 if st == ZR_OK else 12
        except BaseException as e:  # noqa: BLE001 - reported through the status code
            self.error = e
            return 13

    @property
    def fn_ptr(self):
        return ctypes.cast(self._cb, ctypes.c_void_p)

    ctx = None


class Recorder:
    """Record a black box's outputs once on the device, then replay them."""

    def __init__(self, inner):
        self.inner = inner
        h = ctypes.c_void_p()
        st = lib().zr_recorder_create(ctypes.byref(h), inner.fn_ptr, inner.ctx)
        if st != ZR_OK:
            raise ZippelError(st, "zr_recorder_create")
        self.handle = h

    def replay(self, on: bool = True):
        lib().zr_recorder_set_replay(self.handle, 1 if on else 0)

    @property
    def fn_ptr(self):
        return ctypes.cast(lib().zr_recorder_blackbox, ctypes.c_void_p)

    @property
    def ctx(self):
        return self.handle

    def close(self):
        if self.handle:
            lib().zr_recorder_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


# ---------------------------------------------------------------------------
# reconstruction

def _take(poly: ZrPoly, nvars: int):
    n = poly.nterms
    if n:
        e = np.ctypeslib.as_array(poly.exps, shape=(n * nvars,)).reshape(n, nvars).copy()
        c = np.ctypeslib.as_array(poly.coeffs, shape=(n,)).copy()
    else:
        e = np.zeros((0, nvars), np.uint16)
        c = np.zeros(0, np.uint64)
    lib().zr_poly_free(ctypes.byref(poly))
    return e, c


class _ParamsHolder:
    def __init__(self, p, deg, deg_den, sched, seed, nprobes, last_stage):
        self.deg = _u32(deg)
        self.deg_den = _u32(deg_den) if deg_den is not None else None
        self.s = ZrParams()
        self.s.p = p
        self.s.nvars = len(deg)
        self.s.deg = _ptr(self.deg)
        self.s.deg_den = _ptr(self.deg_den)
        self.s.seed = seed
        self.s.last_stage = last_stage
        if sched is not None:
            self.y = _u64(sched.y)
            self.anchor = _u64(sched.anchor)
            self.nodes = _u64(sched.nodes_concat())
            self.nnodes = _u32(sched.counts())
            self.probes = _u64(sched.probes).reshape(-1)
            self.s.y = _ptr(self.y)
            self.s.anchor = _ptr(self.anchor)
            self.s.nodes = self.nodes.ctypes.data
            self.s.nnodes = _ptr(self.nnodes)
            self.s.nprobes = sched.probes.shape[0] if nprobes is None else nprobes
            self.s.probes = _ptr(self.probes)
        else:
            self.s.nprobes = nprobes or 0


def _box_args(box):
    """Any object with ``fn_ptr`` (a zr_blackbox_fn) and ``ctx`` attributes."""
    if hasattr(box, "fn_ptr") and hasattr(box, "ctx"):
        return box.fn_ptr, box.ctx
    raise TypeError("black box must expose fn_ptr and ctx (HostBlackBox, Recorder, ...)")


def reconstruct(p: int, deg: Sequence[int], box, sched=None, seed: int = 0, nprobes: Optional[int] = None,
                last_stage: int = 0, stream=None, first_stage: int = 0, start=None):
    """Polynomial Zippel on the GPU.  Returns (exps [nterms][nvars] uint16, coefs uint64).

    With first_stage = k >= 2 the reconstruction resumes at stage k from
    start = (exps, coefs), the result of stage k-1 (what this function returns
    with last_stage = k-1 on the same schedule)."""
    h = _ParamsHolder(p, deg, None, sched, seed, nprobes, last_stage)
    if first_stage > 1:
        if start is None:
            raise ValueError("first_stage >= 2 needs the previous stage's result as start=(exps, coefs)")
        h.start_exps = np.ascontiguousarray(np.asarray(start[0], dtype=np.uint16).reshape(-1, len(deg)))
        h.start_coefs = _u64(start[1])
        h.start = ZrPoly(len(deg), len(h.start_coefs),
                         h.start_exps.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                         h.start_coefs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        h.s.first_stage = first_stage
        h.s.start = ctypes.cast(ctypes.pointer(h.start), ctypes.c_void_p)
    out = ZrPoly()
    fn, ctx = _box_args(box)
    st = lib().zippel_reconstruct(ctypes.byref(h.s), fn, ctx, _stream(stream), ctypes.byref(out))
    if st != ZR_OK:
        err = getattr(box, "error", None)
        raise ZippelError(st, f"zippel_reconstruct{' (' + repr(err) + ')' if err else ''}")
    return _take(out, len(deg))


def balanced_reconstruct(p: int, deg_num: Sequence[int], deg_den: Sequence[int], box, sched=None, seed: int = 0,
                         nprobes: Optional[int] = None, last_stage: int = 0, stream=None):
    """Balanced Zippel on the GPU.  Returns ((exps, coefs) of num, (exps, coefs) of den), den(0) = 1."""
    h = _ParamsHolder(p, deg_num, deg_den, sched, seed, nprobes, last_stage)
    on, od = ZrPoly(), ZrPoly()
    fn, ctx = _box_args(box)
    st = lib().zippel_balanced_reconstruct(ctypes.byref(h.s), fn, ctx, _stream(stream), ctypes.byref(on),
                                           ctypes.byref(od))
    if st != ZR_OK:
        raise ZippelError(st, "zippel_balanced_reconstruct")
    return _take(on, len(deg_num)), _take(od, len(deg_num))


def reconstruct_adaptive(p: int, caps: Sequence[int], box, sched=None, seed: int = 0, confirm: int = 1,
                         nprobes: Optional[int] = None, stream=None):
    """Polynomial Zippel without degree bounds (zippel_reconstruct_adaptive):
    caps[v] limits the nodes of x_v to caps[v] + confirm.  Returns
    (exps, coefs, degrees found per variable)."""
    h = _ParamsHolder(p, caps, None, sched, seed, nprobes, 0)
    out = ZrPoly()
    found = np.zeros(len(caps), dtype=np.uint32)
    fn, ctx = _box_args(box)
    st = lib().zippel_reconstruct_adaptive(ctypes.byref(h.s), confirm, fn, ctx, _stream(stream), ctypes.byref(out),
                                           found.ctypes.data)
    if st != ZR_OK:
        err = getattr(box, "error", None)
        raise ZippelError(st, f"zippel_reconstruct_adaptive{' (' + repr(err) + ')' if err else ''}")
    e, c = _take(out, len(caps))
    return e, c, [int(d) for d in found]


def reconstruct_multi(p: int, degs: Sequence[Sequence[int]], box, sched=None, seed: int = 0,
                      nprobes: Optional[int] = None, stream=None):
    """Several polynomials sampled together (zippel_reconstruct_multi):
    degs[e] the degree bounds of expression e; the box returns all of them per
    point.  Returns [(exps, coefs)] per expression."""
    degs = np.ascontiguousarray(np.asarray(degs, dtype=np.uint32))
    E, nv = degs.shape
    h = _ParamsHolder(p, degs.max(axis=0), None, sched, seed, nprobes, 0)
    outs = (ZrPoly * E)()
    fn, ctx = _box_args(box)
    st = lib().zippel_reconstruct_multi(ctypes.byref(h.s), E, degs.ctypes.data, fn, ctx, _stream(stream), outs)
    if st != ZR_OK:
        err = getattr(box, "error", None)
        raise ZippelError(st, f"zippel_reconstruct_multi{' (' + repr(err) + ')' if err else ''}")
    return [_take(outs[e], nv) for e in range(E)]


def rational_from_words(raw):
    """(exps, num words [t][nw], den words [t][nw], neg [t], primes) -> (exps, [(num, den)], primes)."""
    e, num, den, neg, used = raw

    def big(row):
        return sum(int(w) << (64 * i) for i, w in enumerate(row))
    return e, [(-big(num[l]) if neg[l] else big(num[l]), big(den[l])) for l in range(len(neg))], used


def reconstruct_rational(p: int, deg: Sequence[int], box, primes: Sequence[int], sched=None, seed: int = 0,
                         nprobes: Optional[int] = None, stream=None, raw: bool = False):
    """Polynomial with rational coefficients (zippel_reconstruct_rational):
    Zippel modulo p, then the further primes in order until one confirms.
    Returns (exps [nterms][nvars] uint16, [(num, den)] as Python ints, primes
    used); with raw=True the magnitudes as uint64 word arrays [nterms][nwords]
    and the signs instead (rational_from_words converts)."""
    h = _ParamsHolder(p, deg, None, sched, seed, nprobes, 0)
    pr = _u64(primes)
    out = ZrQPoly()
    fn, ctx = _box_args(box)
    st = lib().zippel_reconstruct_rational(ctypes.byref(h.s), _ptr(pr) if len(pr) else None, len(pr), fn, ctx,
                                           _stream(stream), ctypes.byref(out))
    if st != ZR_OK:
        err = getattr(box, "error", None)
        raise ZippelError(st, f"zippel_reconstruct_rational{' (' + repr(err) + ')' if err else ''}")
    n, nv, nw = out.nterms, len(deg), out.nwords
    try:
        if n:
            e = np.ctypeslib.as_array(out.exps, shape=(n * nv,)).reshape(n, nv).copy()
            num = np.ctypeslib.as_array(out.num, shape=(n * nw,)).reshape(n, nw).copy()
            den = np.ctypeslib.as_array(out.den, shape=(n * nw,)).reshape(n, nw).copy()
            neg = np.ctypeslib.as_array(out.neg, shape=(n,)).copy()
        else:
            e = np.zeros((0, nv), np.uint16)
            num = den = np.zeros((0, max(nw, 1)), np.uint64)
            neg = np.zeros(0, np.uint8)
        words = (e, num, den, neg, int(out.nprimes))
        return words if raw else rational_from_words(words)
    finally:
        lib().zr_qpoly_free(ctypes.byref(out))


def skeleton_solve(p: int, exps, y, vals, stream=None):
    """Coefficients modulo p of the terms exps [t][nvars] from samples
    vals[i-1] at x_v = y_v^i, i = 1..t (zr_skeleton_solve).  Returns (a [t], status)."""
    import torch
    exps = np.ascontiguousarray(np.asarray(exps, dtype=np.uint16))
    t, nv = exps.shape
    y = _u64(y)
    dev = torch.device("cuda")
    d_v = torch.from_numpy(np.concatenate([_u64(vals), np.zeros(1, np.uint64)]).view(np.int64)).to(dev)
    d_o = torch.zeros_like(d_v)
    d_s = torch.zeros(1, dtype=torch.int32, device=dev)
    st = lib().zr_skeleton_solve(p, nv, t, exps.ctypes.data, _ptr(y), d_v.data_ptr(), d_o.data_ptr(),
                                 d_s.data_ptr(), _stream(stream))
    if st != ZR_OK:
        raise ZippelError(st, "zr_skeleton_solve")
    torch.cuda.synchronize()
    return d_o.cpu().numpy().view(np.uint64)[:t].copy(), int(d_s.cpu().item())


class _Dispatch:
    """One zr_blackbox_fn for a batch whose boxes have different callbacks:
    ctx carries the instance index."""

    def __init__(self, boxes):
        self.fns = [(BLACKBOX_FN(ctypes.cast(b.fn_ptr, ctypes.c_void_p).value), b.ctx) for b in boxes]
        self._cb = BLACKBOX_FN(self._call)

    def _call(self, ctx, pts, d_vals, stream):
        fn, c = self.fns[ctx or 0]
        return fn(c, pts, d_vals, stream)


def reconstruct_batch(p: int, items: Sequence[dict], stream=None):
    """Batched polynomial Zippel on the GPU (zippel_reconstruct_batch).  Each
    item is a dict with keys deg, box and optionally sched, seed, nprobes,
    last_stage.  Returns a list of (exps, coefs) or ZippelError per instance."""
    n = len(items)
    holders = [_ParamsHolder(p, it["deg"], None, it.get("sched"), it.get("seed", 0), it.get("nprobes"),
                             it.get("last_stage", 0)) for it in items]
    params = (ZrParams * max(n, 1))(*[h.s for h in holders])
    boxes = [it["box"] for it in items]
    fptrs = {ctypes.cast(b.fn_ptr, ctypes.c_void_p).value for b in boxes}
    if len(fptrs) == 1:
        fn = boxes[0].fn_ptr
        ctxs = (ctypes.c_void_p * max(n, 1))(*[b.ctx for b in boxes])
        disp = None
    else:
        disp = _Dispatch(boxes)
        fn = ctypes.cast(disp._cb, ctypes.c_void_p)
        ctxs = (ctypes.c_void_p * max(n, 1))(*range(n))
    outs = (ZrPoly * max(n, 1))()
    status = np.zeros(max(n, 1), np.int32)
    st = lib().zippel_reconstruct_batch(n, params, fn, ctxs, _stream(stream), outs, status.ctypes.data)
    if st != ZR_OK:
        raise ZippelError(st, "zippel_reconstruct_batch")
    res = []
    for i in range(n):
        if status[i] != ZR_OK:
            res.append(ZippelError(int(status[i]), f"instance {i}"))
        else:
            res.append(_take(outs[i], len(items[i]["deg"])))
    del disp
    return res


def autotune(p: int, stream=None):
    """Measure the per-band choices of the batched solve on this device; returns them."""
    tab = (ZrBandChoice * NBANDS)()
    st = lib().zr_autotune(p, _stream(stream), tab)
    if st != ZR_OK:
        raise ZippelError(st, "zr_autotune")
    return [(t.packed, t.min_chunk) for t in tab]


SOLVE_VARIANTS = {"waves": 0, "producer_consumer": 1}
DEFAULT_SOLVE_VARIANT = "producer_consumer"


def solve_variant(variant=DEFAULT_SOLVE_VARIANT):
    """Select the dot-product pass of the one-system solve (zr_solve_variant):
    "waves" or "producer_consumer" (the default), both on the integer vector ALU."""
    st = lib().zr_solve_variant(SOLVE_VARIANTS[variant])
    if st != ZR_OK:
        raise ZippelError(st, "zr_solve_variant")


def batch_graphs(on: bool):
    """Capture each stage's batched solve into one hipGraph (zr_batch_graphs)."""
    lib().zr_batch_graphs(1 if on else 0)


def tuning_get():
    tab = (ZrBandChoice * NBANDS)()
    tuned = lib().zr_tuning_get(tab)
    return bool(tuned), [(t.packed, t.min_chunk) for t in tab]


def tuning_set(choices):
    tab = (ZrBandChoice * NBANDS)(*[ZrBandChoice(int(a), int(b)) for a, b in choices])
    st = lib().zr_tuning_set(tab)
    if st != ZR_OK:
        raise ZippelError(st, "zr_tuning_set")


class Server:
    """Request loop with continuous batching (zr_server_*).  submit() queues a
    request (polynomial, or balanced when deg_den is given); step() admits what
    fits and advances every active request by one stage; poll() returns the
    result once finished."""

    def __init__(self, p: int, hbm_budget: int = 8 << 30, max_active: int = 256, stream=None):
        self.p = p
        h = ctypes.c_void_p()
        st = lib().zr_server_create(ctypes.byref(h), p, hbm_budget, max_active, _stream(stream))
        if st != ZR_OK:
            raise ZippelError(st, "zr_server_create")
        self.handle = h
        self._keep = {}

    def submit(self, deg, box, sched=None, seed: int = 0, nprobes: Optional[int] = None, deg_den=None,
               expected_terms: int = 0, last_stage: int = 0) -> int:
        h = _ParamsHolder(self.p, deg, deg_den, sched, seed, nprobes, last_stage)
        fn, ctx = _box_args(box)
        rid = ctypes.c_uint64()
        st = lib().zr_server_submit(self.handle, ctypes.byref(h.s), 1 if deg_den is not None else 0, expected_terms,
                                    fn, ctx, ctypes.byref(rid))
        if st != ZR_OK:
            raise ZippelError(st, "zr_server_submit")
        self._keep[rid.value] = (box, len(deg), deg_den is not None)  # the box must outlive the request
        return rid.value

    def step(self):
        a, p, f = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        st = lib().zr_server_step(self.handle, ctypes.byref(a), ctypes.byref(p), ctypes.byref(f))
        if st != ZR_OK:
            raise ZippelError(st, "zr_server_step")
        return a.value, p.value, f.value

    def poll(self, rid: int):
        """None while pending or active; else (status, num, den) with num/den as
        (exps, coefs) (den None for polynomial requests, both None on failure)."""
        status = ctypes.c_int32()
        num, den = ZrPoly(), ZrPoly()
        r = lib().zr_server_poll(self.handle, rid, ctypes.byref(status), ctypes.byref(num), ctypes.byref(den))
        if r == 1:
            return None
        if r != 0:
            raise ZippelError(r, "zr_server_poll")
        _, nv, bal = self._keep.pop(rid)
        if status.value != ZR_OK:
            lib().zr_poly_free(ctypes.byref(num))
            lib().zr_poly_free(ctypes.byref(den))
            return status.value, None, None
        n = _take(num, nv)
        d = _take(den, nv) if bal else None
        if not bal:
            lib().zr_poly_free(ctypes.byref(den))
        return status.value, n, d

    def finished(self, cap: int = 4096):
        """Ids of the requests that finished since the previous call."""
        out = []
        buf = (ctypes.c_uint64 * cap)()
        while True:
            n = lib().zr_server_finished(self.handle, buf, cap)
            out.extend(buf[:n])
            if n < cap:
                return out

    def stats(self):
        s = ZrServerStats()
        lib().zr_server_get_stats(self.handle, ctypes.byref(s))
        return {n: getattr(s, n) for n, _ in ZrServerStats._fields_}

    def close(self):
        if self.handle:
            lib().zr_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def vandermonde_solve_batch(p: int, systems: List[Tuple[np.ndarray, np.ndarray]], stream=None):
    """Solve sum_l a_l m_l^i = v_i (i = 1..t) for a list of (m [t], rhs [R][t]) on
    the GPU.  Returns (list of a [R][t] arrays, status array)."""
    import torch
    nsys = len(systems)
    t = np.array([len(m) for m, _ in systems], dtype=np.uint64)
    def nrhs(m, r):
        r = np.asarray(r)
        if r.ndim == 2:
            return r.shape[0]
        return r.size // len(m) if len(m) else 0

    R = np.array([nrhs(m, r) for m, r in systems], dtype=np.uint32)
    sys_off = np.zeros(nsys + 1, np.uint64)
    sys_off[1:] = np.cumsum(t)
    rhs_off = np.zeros(nsys + 1, np.uint64)
    rhs_off[1:] = np.cumsum(t * R.astype(np.uint64))
    mono = np.concatenate([_u64(m) for m, _ in systems] + [np.zeros(1, np.uint64)])
    rhs = np.concatenate([_u64(r).reshape(-1) for _, r in systems] + [np.zeros(1, np.uint64)])
    dev = torch.device("cuda")
    d_sys_off = torch.from_numpy(sys_off.view(np.int64)).to(dev)
    d_rhs_off = torch.from_numpy(rhs_off.view(np.int64)).to(dev)
    d_mono = torch.from_numpy(mono.view(np.int64)).to(dev)
    d_rhs = torch.from_numpy(rhs.view(np.int64)).to(dev)
    d_out = torch.zeros_like(d_rhs)
    d_status = torch.zeros(max(nsys, 1), dtype=torch.int32, device=dev)
    s = _stream(stream)
    st = lib().vandermonde_solve_batch(nsys, p, d_sys_off.data_ptr(), sys_off.ctypes.data, d_mono.data_ptr(),
                                       R.ctypes.data, d_rhs_off.data_ptr(), rhs_off.ctypes.data, d_rhs.data_ptr(),
                                       d_out.data_ptr(), d_status.data_ptr(), s)
    if st != ZR_OK:
        raise ZippelError(st, "vandermonde_solve_batch")
    torch.cuda.synchronize()
    out = d_out.cpu().numpy().view(np.uint64)
    res = [out[int(rhs_off[i]):int(rhs_off[i + 1])].reshape(int(R[i]), int(t[i])) for i in range(nsys)]
    return res, d_status.cpu().numpy()[:nsys]


def vandermonde_solve(p: int, m, rhs, stream=None):
    """One system sum_l a_l m_l^i = v_i (i = 1..t) through the one-system solve
    (zr_vandermonde_solve): m [t], rhs [R][t].  Returns (a [R][t], status)."""
    import torch
    m = _u64(m)
    t = len(m)
    rhs = _u64(rhs).reshape(-1, t) if t else np.zeros((0, 0), np.uint64)
    R = rhs.shape[0]
    dev = torch.device("cuda")
    d_m = torch.from_numpy(np.concatenate([m, np.zeros(1, np.uint64)]).view(np.int64)).to(dev)
    d_r = torch.from_numpy(np.concatenate([rhs.reshape(-1), np.zeros(1, np.uint64)]).view(np.int64)).to(dev)
    d_o = torch.zeros_like(d_r)
    d_s = torch.zeros(1, dtype=torch.int32, device=dev)
    st = lib().zr_vandermonde_solve(p, t, R, d_m.data_ptr(), d_r.data_ptr(), d_o.data_ptr(), d_s.data_ptr(),
                                    _stream(stream))
    if st != ZR_OK:
        raise ZippelError(st, "zr_vandermonde_solve")
    torch.cuda.synchronize()
    out = d_o.cpu().numpy().view(np.uint64)[:R * t].reshape(R, t)
    return out, int(d_s.cpu().item())


def vandermonde_solve_noalloc(p: int, d_mono, d_rhs, d_out, d_status, t: int, R: int, stream=None) -> int:
    """zr_vandermonde_solve_noalloc on caller-owned device tensors (d_mono [t],
    d_rhs and d_out [R][t] of int64 holding the u64 values, d_status int32 [1]).
    Asynchronous on `stream`; returns the call's status."""
    return int(lib().zr_vandermonde_solve_noalloc(p, t, R, d_mono.data_ptr(), d_rhs.data_ptr(), d_out.data_ptr(),
                                                  d_status.data_ptr(), _stream(stream)))


def thiele_slices(p: int, x, f, stream=None):
    """Per-slice Thiele reconstruction on the GPU (zr_thiele_slices): x [nk]
    nodes, f [nk][T] samples.  Returns (A [nk+1][T], B [nk+1][T], degA [T],
    degB [T], status [T]); column i holds slice i, entries of failed slices
    are unspecified."""
    import torch
    x = _u64(x)
    f = _u64(f).reshape(len(x), -1) if len(x) else np.zeros((0, 0), np.uint64)
    nk, T = f.shape
    dev = torch.device("cuda")
    d_x = torch.from_numpy(np.concatenate([x, np.zeros(1, np.uint64)]).view(np.int64)).to(dev)
    d_f = torch.from_numpy(np.concatenate([f.reshape(-1), np.zeros(1, np.uint64)]).view(np.int64)).to(dev)
    d_a = torch.zeros((nk + 1) * max(T, 1), dtype=torch.int64, device=dev)
    d_b = torch.zeros_like(d_a)
    d_i = torch.zeros(3 * max(T, 1), dtype=torch.int32, device=dev)
    st = lib().zr_thiele_slices(p, T, nk, d_x.data_ptr(), d_f.data_ptr(), d_a.data_ptr(), d_b.data_ptr(),
                                d_i.data_ptr(), d_i.data_ptr() + 4 * max(T, 1), d_i.data_ptr() + 8 * max(T, 1),
                                _stream(stream))
    if st != ZR_OK:
        raise ZippelError(st, "zr_thiele_slices")
    torch.cuda.synchronize()
    a = d_a.cpu().numpy().view(np.uint64)[:(nk + 1) * T].reshape(nk + 1, T)
    b = d_b.cpu().numpy().view(np.uint64)[:(nk + 1) * T].reshape(nk + 1, T)
    i = d_i.cpu().numpy().reshape(3, max(T, 1))[:, :T]
    return a, b, i[0], i[1], i[2]


# ---------------------------------------------------------------------------
# timing and counters

def timing(enable: bool = True, dots_only: bool = False):
    """Kernel timing (zr_timing_enable): every named launch, or with
    dots_only only the solve's dot-product launches ("vs_dots")."""
    lib().zr_timing_enable((2 if dots_only else 1) if enable else 0)


def timing_reset():
    lib().zr_timing_reset()


def timing_get(name: str) -> Tuple[int, float]:
    ms = ctypes.c_double()
    n = lib().zr_timing_get(name.encode(), ctypes.byref(ms))
    return int(n), float(ms.value)


def last_counters() -> dict:
    c = ZrCounters()
    lib().zr_last_counters(ctypes.byref(c))
    return {k: int(getattr(c, k)) for k, _ in ZrCounters._fields_}


def microbench(kind: str, blocks: int = 2048, iters: int = 4096, nbytes: int = 1 << 30, stream=None):
    """(ms, ops) of one timed launch of a throughput probe (see include/zippel_microbench.h)."""
    ms = ctypes.c_double()
    ops = ctypes.c_double()
    st = lib().zr_microbench(MB_KINDS[kind], blocks, iters, nbytes, _stream(stream), ctypes.byref(ms),
                             ctypes.byref(ops))
    if st != 0:
        raise ZippelError(st, f"zr_microbench({kind})")
    return ms.value, ops.value
