"""ORACLE — test infrastructure only.

ctypes binding of ``zippel_oracle.c``: a plain CPU Zippel / balanced Zippel
reconstruction in 128-bit integer arithmetic, written from the paper.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it; the
product library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, EINVAL, ENOTPRIME, ESINGULAR, EDEGEN, EPROBE, ENORM, ENOMEM, EBLACKBOX = 0, -1, -2, -3, -4, -5, -6, -7, -9

BB_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                         ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                         ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"oracle status {code} {what}")
        self.code = code


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "zippel_oracle.c")
    out = lib_path()
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(out + ".tmp", out)
    return out


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            build()
        L = ctypes.CDLL(lib_path())
        u64, u32, i32, vp, sz = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
        for name in ("or_mul", "or_add", "or_sub", "or_pow"):
            getattr(L, name).restype = u64
            getattr(L, name).argtypes = [u64, u64, u64]
        L.or_inv.restype = u64
        L.or_inv.argtypes = [u64, u64]
        L.or_is_prime.restype = ctypes.c_int
        L.or_is_prime.argtypes = [u64]
        L.or_gauss_solve.argtypes = [u64, sz, vp, sz, vp, vp]
        L.or_gauss_vandermonde.argtypes = [u64, sz, vp, sz, vp, vp]
        L.or_master.argtypes = [u64, sz, vp, vp]
        L.or_master.restype = None
        L.or_vandermonde_solve.argtypes = [u64, sz, vp, sz, vp, vp, ctypes.c_int]
        L.or_vandermonde_solve_rows.argtypes = [u64, sz, vp, sz, vp, sz, vp, vp, ctypes.c_int]
        L.or_vandermonde_apply.argtypes = [u64, sz, vp, vp, u64, sz, vp]
        L.or_vandermonde_apply.restype = None
        L.or_newton.argtypes = [u64, sz, vp, vp, vp]
        L.or_thiele.argtypes = [u64, sz, vp, vp, vp, vp, vp, vp]
        L.or_poly_eval.restype = u64
        L.or_poly_eval.argtypes = [u64, u32, u64, vp, vp, vp]
        L.or_zippel.argtypes = [u64, u32, vp, vp, vp, vp, vp, u32, vp, u32, vp, vp, ctypes.c_int, vp]
        L.or_balanced_zippel.argtypes = [u64, u32, vp, vp, vp, vp, vp, vp, u32, vp, u32, vp, vp, ctypes.c_int,
                                         vp, vp]
        L.or_dense_newton.argtypes = [u64, u32, vp, vp, vp, vp, vp, vp, vp]
        L.or_poly_nterms.restype = u64
        L.or_poly_nterms.argtypes = [vp]
        L.or_poly_exps.restype = vp
        L.or_poly_exps.argtypes = [vp]
        L.or_poly_coefs.restype = vp
        L.or_poly_coefs.argtypes = [vp]
        L.or_poly_free.argtypes = [vp]
        L.or_poly_free.restype = None
        L.or_max_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


# --- field -----------------------------------------------------------------

def mul(a: int, b: int, p: int) -> int: return lib().or_mul(a, b, p)
def add(a: int, b: int, p: int) -> int: return lib().or_add(a, b, p)
def sub(a: int, b: int, p: int) -> int: return lib().or_sub(a, b, p)
def power(a: int, e: int, p: int) -> int: return lib().or_pow(a, e, p)
def inv(a: int, p: int) -> int: return lib().or_inv(a, p)
def is_prime(n: int) -> bool: return bool(lib().or_is_prime(n))
def max_threads() -> int: return lib().or_max_threads()


# --- linear algebra ----------------------------------------------------------

def gauss_solve(p: int, A, B) -> np.ndarray:
    A = _u64(A)
    B = _u64(B)
    n = A.shape[0]
    nrhs = B.shape[1]
    X = np.zeros((n, nrhs), dtype=np.uint64)
    st = lib().or_gauss_solve(p, n, _ptr(A), nrhs, _ptr(B), _ptr(X))
    if st != OK:
        raise OracleError(st, "gauss_solve")
    return X


def gauss_vandermonde(p: int, m, rhs) -> np.ndarray:
    m = _u64(m)
    rhs = _u64(rhs).reshape(-1, len(m))
    out = np.zeros_like(rhs)
    st = lib().or_gauss_vandermonde(p, len(m), _ptr(m), rhs.shape[0], _ptr(rhs), _ptr(out))
    if st != OK:
        raise OracleError(st, "gauss_vandermonde")
    return out


def master(p: int, m) -> np.ndarray:
    m = _u64(m)
    M = np.zeros(len(m) + 1, dtype=np.uint64)
    lib().or_master(p, len(m), _ptr(m), _ptr(M))
    return M


def vandermonde_solve(p: int, m, rhs, nthreads: int = 0) -> np.ndarray:
    """Solve sum_l a_l m_l^i = v_i (i = 1..t) for each row of rhs [R][t]."""
    m = _u64(m)
    rhs = _u64(rhs).reshape(-1, len(m)) if len(m) else _u64(rhs).reshape(-1, 0)
    out = np.zeros_like(rhs)
    st = lib().or_vandermonde_solve(p, len(m), _ptr(m), rhs.shape[0], _ptr(rhs), _ptr(out), nthreads)
    if st != OK:
        raise OracleError(st, "vandermonde_solve")
    return out


def vandermonde_solve_rows(p: int, m, rhs, rows, nthreads: int = 0) -> np.ndarray:
    m = _u64(m)
    rhs = _u64(rhs).reshape(-1, len(m))
    rows = _u64(rows)
    out = np.zeros((rhs.shape[0], len(rows)), dtype=np.uint64)
    st = lib().or_vandermonde_solve_rows(p, len(m), _ptr(m), rhs.shape[0], _ptr(rhs), len(rows), _ptr(rows),
                                         _ptr(out), nthreads)
    if st != OK:
        raise OracleError(st, "vandermonde_solve_rows")
    return out


def vandermonde_apply(p: int, m, a, i_first: int, ni: int) -> np.ndarray:
    m = _u64(m)
    a = _u64(a)
    out = np.zeros(ni, dtype=np.uint64)
    lib().or_vandermonde_apply(p, len(m), _ptr(m), _ptr(a), i_first, ni, _ptr(out))
    return out


def newton(p: int, x, f) -> np.ndarray:
    x = _u64(x)
    f = _u64(f)
    c = np.zeros(len(x), dtype=np.uint64)
    st = lib().or_newton(p, len(x), _ptr(x), _ptr(f), _ptr(c))
    if st != OK:
        raise OracleError(st, "newton")
    return c


def thiele(p: int, x, f) -> Tuple[np.ndarray, np.ndarray]:
    """Shortest confirmed continued fraction -> (A, B) with lowest nonzero B coefficient 1."""
    x = _u64(x)
    f = _u64(f)
    n = len(x)
    A = np.zeros(n + 1, dtype=np.uint64)
    B = np.zeros(n + 1, dtype=np.uint64)
    da = ctypes.c_int32()
    db = ctypes.c_int32()
    st = lib().or_thiele(p, n, _ptr(x), _ptr(f), _ptr(A), _ptr(B), ctypes.addressof(da), ctypes.addressof(db))
    if st != OK:
        raise OracleError(st, "thiele")
    return A[:da.value + 1].copy(), B[:db.value + 1].copy()


def poly_eval(p: int, exps, coefs, pt) -> int:
    exps = np.ascontiguousarray(np.asarray(exps, dtype=np.uint16))
    coefs = _u64(coefs)
    pt = _u64(pt)
    nv = exps.shape[1] if exps.ndim == 2 else len(pt)
    return lib().or_poly_eval(p, nv, len(coefs), _ptr(exps), _ptr(coefs), _ptr(pt))


# --- reconstruction ----------------------------------------------------------

def _take_poly(handle: int, nvars: int):
    L = lib()
    n = L.or_poly_nterms(handle)
    if n:
        e = np.ctypeslib.as_array(ctypes.cast(L.or_poly_exps(handle), ctypes.POINTER(ctypes.c_uint16)),
                                  shape=(n * nvars,)).reshape(n, nvars).copy()
        c = np.ctypeslib.as_array(ctypes.cast(L.or_poly_coefs(handle), ctypes.POINTER(ctypes.c_uint64)),
                                  shape=(n,)).copy()
    else:
        e = np.zeros((0, nvars), dtype=np.uint16)
        c = np.zeros(0, dtype=np.uint64)
    L.or_poly_free(handle)
    return e, c


def _bb_args(box):
    """box: a synth.BlackBox (C evaluator, fast path) or a Python callable
    (k, i_first, ni, y, anchor, xk) -> values[nj*ni]."""
    if hasattr(box, "c_function_address"):
        return ctypes.c_void_p(box.c_function_address()), ctypes.c_void_p(box.ctx()), None
    nvars_holder = {}

    def cb(ctx, nvars, k, i_first, ni, y, anchor, nj, xk, vals):
        try:
            yy = np.ctypeslib.as_array(ctypes.cast(y, ctypes.POINTER(ctypes.c_uint64)), shape=(nvars,)).copy()
            aa = np.ctypeslib.as_array(ctypes.cast(anchor, ctypes.POINTER(ctypes.c_uint64)),
                                       shape=(nvars,)).copy()
            xx = np.ctypeslib.as_array(ctypes.cast(xk, ctypes.POINTER(ctypes.c_uint64)), shape=(nj,)).copy()
            res = np.asarray(box(k, i_first, ni, yy, aa, xx), dtype=np.uint64).reshape(-1)
            out = np.ctypeslib.as_array(ctypes.cast(vals, ctypes.POINTER(ctypes.c_uint64)), shape=(nj * ni,))
            out[:] = res
            return 0
        except Exception:  # noqa: BLE001 - report through the status code
            return 1

    fn = BB_FN(cb)
    return ctypes.cast(fn, ctypes.c_void_p), ctypes.c_void_p(0), fn


def zippel(p: int, deg: Sequence[int], schedule, box, last_stage: int = 0, nprobes: Optional[int] = None,
           nthreads: int = 0):
    """Polynomial Zippel.  Returns (exps [nterms][nvars] uint16, coefs uint64), lex order."""
    nvars = len(deg)
    deg_a = _u32(deg)
    y = _u64(schedule.y)
    anc = _u64(schedule.anchor)
    nodes = _u64(schedule.nodes_concat())
    cnt = _u32(schedule.counts())
    probes = _u64(schedule.probes).reshape(-1)
    npr = schedule.probes.shape[0] if nprobes is None else nprobes
    fn, ctx, keep = _bb_args(box)
    out = ctypes.c_void_p()
    st = lib().or_zippel(p, nvars, _ptr(deg_a), _ptr(y), _ptr(anc), _ptr(nodes), _ptr(cnt), npr, _ptr(probes),
                         last_stage, fn, ctx, nthreads, ctypes.addressof(out))
    del keep
    if st != OK:
        raise OracleError(st, "zippel")
    return _take_poly(out.value, nvars)


def balanced_zippel(p: int, deg_num: Sequence[int], deg_den: Sequence[int], schedule, box, last_stage: int = 0,
                    nprobes: Optional[int] = None, nthreads: int = 0):
    """Balanced Zippel for P/Q.  Returns ((exps, coefs) of N, (exps, coefs) of D), D(0) = 1."""
    nvars = len(deg_num)
    dn = _u32(deg_num)
    dd = _u32(deg_den)
    y = _u64(schedule.y)
    anc = _u64(schedule.anchor)
    nodes = _u64(schedule.nodes_concat())
    cnt = _u32(schedule.counts())
    probes = _u64(schedule.probes).reshape(-1)
    npr = schedule.probes.shape[0] if nprobes is None else nprobes
    fn, ctx, keep = _bb_args(box)
    on = ctypes.c_void_p()
    od = ctypes.c_void_p()
    st = lib().or_balanced_zippel(p, nvars, _ptr(dn), _ptr(dd), _ptr(y), _ptr(anc), _ptr(nodes), _ptr(cnt), npr,
                                  _ptr(probes), last_stage, fn, ctx, nthreads, ctypes.addressof(on),
                                  ctypes.addressof(od))
    del keep
    if st != OK:
        raise OracleError(st, "balanced_zippel")
    return _take_poly(on.value, nvars), _take_poly(od.value, nvars)


def dense_newton(p: int, deg: Sequence[int], schedule, box) -> np.ndarray:
    """Full coefficient tensor from the black box on the node grid (brute force)."""
    nvars = len(deg)
    deg_a = _u32(deg)
    total = int(np.prod([d + 1 for d in deg]))
    coef = np.zeros(total, dtype=np.uint64)
    anc = _u64(schedule.anchor)
    nodes = _u64(schedule.nodes_concat())
    cnt = _u32(schedule.counts())
    fn, ctx, keep = _bb_args(box)
    st = lib().or_dense_newton(p, nvars, _ptr(deg_a), _ptr(anc), _ptr(nodes), _ptr(cnt), fn, ctx, _ptr(coef))
    del keep
    if st != OK:
        raise OracleError(st, "dense_newton")
    return coef.reshape([d + 1 for d in deg])
