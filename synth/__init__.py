"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module produces *inputs* only: the prime, the hidden polynomials or
rational functions that play the role of the black box, the sampling schedule
(the random points the method draws, passed into both implementations), and
a host black-box evaluator (``blackbox.c``).  It contains none of the
reconstruction method's arithmetic (no Vandermonde solve, no Newton or Thiele
interpolation).

Randomness: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), a counter-based generator: output i of a
stream with seed s is mix(s + (i+1)*gamma).  Uniform integers in [lo, hi) use
rejection: draw u, accept iff u < floor(2^64/n)*n with n = hi-lo, return
lo + u mod n.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1

PRIME_SEED = 20250530


def _mix_np(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        return z ^ (z >> np.uint64(31))


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


class SplitMix64:
    """Stream of SplitMix64 outputs; ``next()`` and ``block(n)`` consume in order."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        return _mix(self.state)

    def block(self, n: int) -> np.ndarray:
        """The next n outputs as a uint64 array (vectorised, same stream)."""
        if n <= 0:
            return np.zeros(0, dtype=np.uint64)
        idx = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            st = np.uint64(self.state) + idx * np.uint64(_GAMMA)
        self.state = (self.state + n * _GAMMA) & _MASK
        return _mix_np(st)

    def uniform(self, lo: int, hi: int) -> int:
        n = hi - lo
        assert n >= 1
        lim = ((1 << 64) // n) * n
        while True:
            u = self.next()
            if lim == (1 << 64) or u < lim:
                return lo + u % n

    def uniform_block(self, lo: int, hi: int, count: int) -> np.ndarray:
        """``count`` draws of ``uniform(lo, hi)``, identical to calling it in a loop:
        raw outputs are drawn in bulk, rejected ones skipped in order, and the
        stream is left just after the last raw output consumed."""
        n = hi - lo
        assert n >= 1
        lim = ((1 << 64) // n) * n
        if count <= 0:
            return np.zeros(0, dtype=np.uint64)
        if n == (1 << 64):
            return self.block(count)
        if lim == (1 << 64):
            return np.uint64(lo) + self.block(count) % np.uint64(n)
        rate = lim / float(1 << 64)
        parts = []
        got = 0
        while got < count:
            need = count - got
            m = int(need / rate * 1.02) + 64
            raw = self.block(m)
            idx = np.flatnonzero(raw < np.uint64(lim))
            if len(idx) >= need:
                last = int(idx[need - 1])
                parts.append(np.uint64(lo) + raw[idx[:need]] % np.uint64(n))
                # give back the raw outputs after the last one used
                self.state = (self.state - (m - last - 1) * _GAMMA) & _MASK
                got = count
            else:
                parts.append(np.uint64(lo) + raw[idx] % np.uint64(n))
                got += len(idx)
        return np.concatenate(parts)


# --------------------------------------------------------------------------
# primes (input generation: the prime is an input to the method)

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 with the first twelve prime bases."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def make_prime(seed: int = PRIME_SEED) -> int:
    """Smallest prime >= an odd seeded value in [2^62, 2^63)."""
    g = SplitMix64(seed)
    x = g.uniform(1 << 62, 1 << 63) | 1
    while not is_prime(x):
        x += 2
        if x >= (1 << 63):
            x = (1 << 62) + 1
    return x


# --------------------------------------------------------------------------
# hidden polynomials

@dataclass
class SparsePoly:
    """Polynomial over F_p: exps [nterms][nvars] (uint16), coefs [nterms] (uint64), lex-sorted."""
    p: int
    nvars: int
    exps: np.ndarray
    coefs: np.ndarray

    @property
    def nterms(self) -> int:
        return int(self.coefs.shape[0])

    def sorted(self) -> "SparsePoly":
        if self.nterms == 0:
            return self
        order = np.lexsort(self.exps.T[::-1])
        return SparsePoly(self.p, self.nvars, np.ascontiguousarray(self.exps[order]),
                          np.ascontiguousarray(self.coefs[order]))

    def as_dict(self):
        return {tuple(int(x) for x in e): int(c) for e, c in zip(self.exps, self.coefs)}

    def degrees(self) -> List[int]:
        if self.nterms == 0:
            return [0] * self.nvars
        return [int(x) for x in self.exps.max(axis=0)]


def _distinct_exponents(g: SplitMix64, nvars: int, nterms: int, draw_row) -> np.ndarray:
    seen = {}
    rows = []
    while len(rows) < nterms:
        e = draw_row()
        key = bytes(e.astype(np.uint16).tobytes())
        if key in seen:
            continue
        seen[key] = True
        rows.append(e)
    return np.array(rows, dtype=np.uint16).reshape(nterms, nvars)


def random_poly(p: int, nvars: int, deg: Sequence[int] | int, nterms: int, seed: int) -> SparsePoly:
    """t distinct exponent vectors uniform in prod [0, D_v], coefficients uniform in [1, p)."""
    if isinstance(deg, int):
        deg = [deg] * nvars
    space = 1
    for d in deg:
        space *= d + 1
    assert nterms <= space, "more terms than monomials"
    g = SplitMix64(seed)
    if nterms * 4 > space:
        # dense regime: draw a random subset of all monomials by index
        idx = []
        seen = set()
        while len(idx) < nterms:
            u = g.uniform(0, space)
            if u not in seen:
                seen.add(u)
                idx.append(u)
        exps = np.zeros((nterms, nvars), dtype=np.uint16)
        for r, u in enumerate(idx):
            for v in range(nvars - 1, -1, -1):
                exps[r, v] = u % (deg[v] + 1)
                u //= deg[v] + 1
    else:
        # draw candidate rows in bulk; first occurrences in stream order win
        # (rows compared through their mixed-radix index, which fits in 64 bits)
        radix = np.array([d + 1 for d in deg], dtype=object)
        assert space < (1 << 63)
        kept = []
        seen_keys = np.zeros(0, dtype=np.int64)
        bulk = max(1024, nterms * 2)
        total = 0
        while total < nterms:
            cols = [g.uniform_block(0, deg[v] + 1, bulk) for v in range(nvars)]
            cand = np.stack(cols, axis=1).astype(np.uint16)
            key = np.zeros(bulk, dtype=np.int64)
            for v in range(nvars):
                key = key * int(radix[v]) + cand[:, v].astype(np.int64)
            _, first = np.unique(key, return_index=True)
            first.sort()
            first = first[~np.isin(key[first], seen_keys)]
            first = first[:nterms - total]
            kept.append(cand[first])
            seen_keys = np.concatenate([seen_keys, key[first]])
            total += len(first)
        exps = np.concatenate(kept).reshape(nterms, nvars)
    coefs = g.uniform_block(1, p, nterms)
    return SparsePoly(p, nvars, exps, coefs).sorted()


@dataclass
class QPoly:
    """Polynomial with rational coefficients num[l]/den[l] (Python ints, den > 0,
    gcd 1), exponents as in SparsePoly: the black box of a reconstruction over
    several primes.  ``mod(p)`` is its image over F_p."""
    nvars: int
    exps: np.ndarray
    num: List[int]
    den: List[int]

    @property
    def nterms(self) -> int:
        return int(self.exps.shape[0])

    def mod(self, p: int) -> SparsePoly:
        c = np.array([(a % p) * pow(b, -1, p) % p for a, b in zip(self.num, self.den)], dtype=np.uint64)
        return SparsePoly(p, self.nvars, self.exps.copy(), c)


def random_qpoly(nvars: int, deg: Sequence[int] | int, nterms: int, bits: int, seed: int) -> QPoly:
    """Exponents as random_poly (distinct, uniform in prod [0, D_v]); numerators
    uniform in (-2^bits, 2^bits) without 0, denominators uniform in [1, 2^bits),
    each fraction reduced.  Draws: the exponent stream of seed, then per term a
    numerator magnitude, its sign and a denominator from seed + 1, in 64-bit
    words (low word first)."""
    shape = random_poly(3, nvars, deg, nterms, seed)  # exponents only (F_3 coefficients unused)
    g = SplitMix64(seed + 1)
    words = (bits + 63) // 64

    def draw(lo: int) -> int:
        while True:
            x = 0
            for w in range(words):
                x |= g.next() << (64 * w)
            x &= (1 << bits) - 1
            if x >= lo:
                return x
    num, den = [], []
    for _ in range(nterms):
        a = draw(1)
        if g.next() & 1:
            a = -a
        b = draw(1)
        d = math.gcd(a, b)
        num.append(a // d)
        den.append(b // d)
    return QPoly(nvars, shape.exps, num, den)


def prime_list(count: int, seed: int = PRIME_SEED) -> List[int]:
    """count distinct primes in (2^62, 2^63): make_prime(seed), make_prime(seed + 1), ..."""
    out: List[int] = []
    j = 0
    while len(out) < count:
        q = make_prime(seed + j)
        if q not in out:
            out.append(q)
        j += 1
    return out


def _simplex_row(g: SplitMix64, nvars: int, total: int) -> np.ndarray:
    """Uniform exponent vector with sum <= total (stars and bars: a uniform
    nvars-subset of {0..total+nvars-1} gives the bar positions)."""
    npos = total + nvars
    chosen = set()
    while len(chosen) < nvars:
        chosen.add(g.uniform(0, npos))
    bars = sorted(chosen)
    e = np.empty(nvars, dtype=np.uint16)
    prev = -1
    for v, b in enumerate(bars):
        e[v] = b - prev - 1
        prev = b
    return e


def random_poly_total_degree(p: int, nvars: int, total: int, nterms: int, seed: int,
                             with_constant_one: bool = False) -> SparsePoly:
    """t distinct exponents uniform over {e : sum(e) <= total}; coefficients in [1, p).
    With ``with_constant_one`` the zero monomial is included with coefficient 1."""
    g = SplitMix64(seed)
    rows = []
    seen = set()
    if with_constant_one:
        z = np.zeros(nvars, dtype=np.uint16)
        rows.append(z)
        seen.add(z.tobytes())
    while len(rows) < nterms:
        e = _simplex_row(g, nvars, total)
        key = e.tobytes()
        if key in seen:
            continue
        seen.add(key)
        rows.append(e)
    exps = np.array(rows, dtype=np.uint16).reshape(nterms, nvars)
    coefs = g.uniform_block(1, p, nterms)
    if with_constant_one:
        coefs[0] = 1
    return SparsePoly(p, nvars, exps, coefs).sorted()


# --------------------------------------------------------------------------
# sampling schedule (the random points the method draws; an input to both sides)

@dataclass
class Schedule:
    """y_v (Zippel bases), anchors c_v, per-variable extra nodes c_v^(1..J_v), probe points."""
    p: int
    y: np.ndarray          # [nvars]
    anchor: np.ndarray     # [nvars]
    nodes: List[np.ndarray]  # nodes[v] has J_v entries, all distinct and != anchor[v]
    probes: np.ndarray     # [nprobes][nvars]

    def nodes_concat(self) -> np.ndarray:
        if not self.nodes:
            return np.zeros(0, dtype=np.uint64)
        return np.concatenate([np.asarray(n, dtype=np.uint64) for n in self.nodes]).astype(np.uint64)

    def counts(self) -> np.ndarray:
        return np.array([len(n) for n in self.nodes], dtype=np.uint32)


def make_schedule(p: int, nvars: int, nnodes: Sequence[int], seed: int, nprobes: int = 0) -> Schedule:
    """Draw order: y_1..y_n in [2, p-1); c_1..c_n in [1, p); for each variable k its
    nodes in [1, p), redrawing any value equal to c_k or to an earlier node of k;
    finally nprobes points, each n values in [1, p)."""
    g = SplitMix64(seed)
    y = np.array([g.uniform(2, p - 1) for _ in range(nvars)], dtype=np.uint64)
    anchor = np.array([g.uniform(1, p) for _ in range(nvars)], dtype=np.uint64)
    nodes = []
    for k in range(nvars):
        used = {int(anchor[k])}
        lst = []
        while len(lst) < nnodes[k]:
            x = g.uniform(1, p)
            if x in used:
                continue
            used.add(x)
            lst.append(x)
        nodes.append(np.array(lst, dtype=np.uint64))
    probes = np.array([[g.uniform(1, p) for _ in range(nvars)] for _ in range(nprobes)],
                      dtype=np.uint64).reshape(nprobes, nvars)
    return Schedule(p, y, anchor, nodes, probes)


def thiele_nodes_needed(dnum: int, dden: int) -> int:
    """Nodes beyond the anchor for a univariate rational function of type at most
    (dnum, dden): the continued fraction needs m = max(2a-1, 2b) + 1 samples and one
    more sample confirms it."""
    m = max(2 * dnum - 1, 2 * dden, 0)
    return m + 1


# --------------------------------------------------------------------------
# workload configurations (shapes of the paper's sparse workloads, synthetic)

@dataclass
class PolyWorkload:
    name: str
    p: int
    hidden: SparsePoly
    deg: List[int]
    schedule: Schedule


@dataclass
class RationalWorkload:
    name: str
    p: int
    num: SparsePoly
    den: SparsePoly
    deg_num: List[int]
    deg_den: List[int]
    schedule: Schedule


POLY_CONFIGS = {
    # name: (nvars, per-variable degree bound, nterms)
    "cfg1_n3_d10_t50": (3, 10, 50),
    "cfg2_n6_d30_t1e4": (6, 30, 10_000),
    "cfg3_n8_d40_t5e5": (8, 40, 500_000),
}


def poly_workload(name: str, nvars: int, deg: int, nterms: int, poly_seed: int,
                  sched_seed: int, nprobes: int = 2, p: Optional[int] = None) -> PolyWorkload:
    p = make_prime() if p is None else p
    hidden = random_poly(p, nvars, deg, nterms, poly_seed)
    degs = [deg] * nvars
    sched = make_schedule(p, nvars, degs, sched_seed, nprobes)
    return PolyWorkload(name, p, hidden, degs, sched)


def config_workload(idx: int, nprobes: int = 2) -> PolyWorkload:
    """Polynomial configurations 1-3: hidden-polynomial seed = idx, schedule seed = 1000+idx."""
    name = list(POLY_CONFIGS)[idx - 1]
    n, d, t = POLY_CONFIGS[name]
    return poly_workload(name, n, d, t, idx, 1000 + idx, nprobes)


def stage_result(poly: SparsePoly, anchor, L: int):
    """f(x_1..x_L, anchor_{L+1}..anchor_n) of a hidden polynomial: the known
    answer of reconstruction stage L.  Exponents beyond L set to 0, terms with
    equal prefixes summed mod p, zero sums dropped, lexicographic order.
    Returns (exps [nterms][nvars] uint16, coefs uint64)."""
    p = poly.p
    c = poly.coefs.astype(object)
    for v in range(L, poly.nvars):
        tab = [1]
        for _ in range(int(poly.exps[:, v].max()) if poly.nterms else 0):
            tab.append(tab[-1] * int(anchor[v]) % p)
        tab = np.array(tab, dtype=object)
        c = c * tab[poly.exps[:, v].astype(np.int64)] % p
    if poly.nterms == 0:
        return np.zeros((0, poly.nvars), dtype=np.uint16), np.zeros(0, dtype=np.uint64)
    pre = poly.exps[:, :L]
    starts = np.flatnonzero(np.r_[True, np.any(pre[1:] != pre[:-1], axis=1)])
    sums = np.add.reduceat(c, starts) % p
    keep = np.array([int(x) != 0 for x in sums], dtype=bool)
    e = np.zeros((int(keep.sum()), poly.nvars), dtype=np.uint16)
    e[:, :L] = pre[starts[keep]]
    return e, np.array([int(x) for x in sums[keep]], dtype=np.uint64)


def batch_workload(count: int = 4096, seed: int = 4, tmin: int = 10, tmax: int = 20_000, deg: int = 30,
                   nmin: int = 3, nmax: int = 8, nprobes: int = 2, p: Optional[int] = None) -> List[PolyWorkload]:
    """Many independent instances sharing p: n uniform in [nmin, nmax], t
    log-uniform in [tmin, tmax] (capped by the number of monomials), per-variable
    degree bound `deg`; instance i uses hidden-polynomial seed seed*10^6 + i and
    schedule seed seed*10^6 + 500000 + i."""
    p = make_prime() if p is None else p
    return [batch_instance(i, n, t, seed, deg, nprobes, p)
            for i, (n, t) in enumerate(batch_shapes(count, seed, tmin, tmax, deg, nmin, nmax))]


def batch_shapes(count: int = 4096, seed: int = 4, tmin: int = 10, tmax: int = 20_000, deg: int = 30,
                 nmin: int = 3, nmax: int = 8) -> List[Tuple[int, int]]:
    """(n, t) of each instance of batch_workload, without building the polynomials."""
    g = SplitMix64(seed * 7919 + 1)
    out = []
    for _ in range(count):
        n = nmin + int(g.uniform(0, nmax - nmin + 1))
        u = g.next() / 2.0 ** 64
        t = int(round(math.exp(math.log(tmin) + u * (math.log(tmax) - math.log(tmin)))))
        out.append((n, max(1, min(t, (deg + 1) ** n))))
    return out


def batch_instance(i: int, n: int, t: int, seed: int = 4, deg: int = 30, nprobes: int = 2,
                   p: Optional[int] = None) -> PolyWorkload:
    """Instance i of batch_workload (with its (n, t) from batch_shapes)."""
    return poly_workload(f"b{i}", n, deg, t, seed * 1_000_000 + i, seed * 1_000_000 + 500_000 + i, nprobes,
                         make_prime() if p is None else p)


def rational_workload(nvars: int, total_deg: int, tnum: int, tden: int, seed: int,
                      nprobes: int = 2, p: Optional[int] = None,
                      name: str = "rational") -> RationalWorkload:
    """P/Q with Q(0)=1; exponents uniform over the total-degree simplex; per-variable
    bounds = total_deg for both."""
    p = make_prime() if p is None else p
    num = random_poly_total_degree(p, nvars, total_deg, tnum, seed * 2 + 1)
    den = random_poly_total_degree(p, nvars, total_deg, tden, seed * 2 + 2, with_constant_one=True)
    dn = [total_deg] * nvars
    dd = [total_deg] * nvars
    J = [thiele_nodes_needed(a, b) for a, b in zip(dn, dd)]
    sched = make_schedule(p, nvars, J, 1000 + seed, nprobes)
    return RationalWorkload(name, p, num, den, dn, dd, sched)


def loguniform_int(g: SplitMix64, lo: int, hi: int) -> int:
    u = g.uniform(0, 1 << 53) / float(1 << 53)
    return int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))


# --------------------------------------------------------------------------
# host black box (C, OpenMP): evaluates a hidden polynomial or P/Q at the
# structured Zippel points or at explicit points

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _PolyDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint64), ("nvars", ctypes.c_uint32), ("nterms", ctypes.c_uint32),
                ("exps", ctypes.c_void_p), ("coefs", ctypes.c_void_p)]


class _BoxDesc(ctypes.Structure):
    _fields_ = [("num", _PolyDesc), ("den", _PolyDesc), ("rational", ctypes.c_int32),
                ("nthreads", ctypes.c_int32)]


def lib_path() -> str:
    return os.path.join(_HERE, "libzsynth.so")


def dev_lib_path() -> str:
    return os.path.join(_HERE, "libzsynth_hip.so")


def build(verbose: bool = False) -> str:
    import subprocess
    src = os.path.join(_HERE, "blackbox.c")
    out = lib_path()
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(out + ".tmp", out)
    dsrc = os.path.join(_HERE, "devbox.hip")
    dout = dev_lib_path()
    cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           "-o", dout + ".tmp", dsrc]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(dout + ".tmp", dout)
    return out


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            build()
        L = ctypes.CDLL(lib_path())
        L.zs_eval_points.restype = ctypes.c_int
        L.zs_eval_points.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_void_p]
        L.zs_group_stage.restype = ctypes.c_uint64
        L.zs_group_stage.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _LIB = L
    return _LIB


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class BlackBox:
    """Evaluates a hidden polynomial (or P/Q) mod p.

    ``eval(k, i_first, ni, y, anchor, xk)`` returns values at the nj*ni points
    (jj, ii): x_v = y_v^(i_first+ii) for v < k, x_k = xk[jj], x_v = anchor_v for
    v > k (k is 1-based), laid out [jj][ii].
    """

    def __init__(self, num: SparsePoly, den: Optional[SparsePoly] = None, nthreads: int = 0):
        self.num = num
        self.den = den
        self.p = num.p
        self.nvars = num.nvars
        self._keep = []
        self.desc = _BoxDesc()
        self.desc.num = self._pd(num)
        if den is not None:
            self.desc.den = self._pd(den)
            self.desc.rational = 1
        else:
            self.desc.rational = 0
        self.desc.nthreads = nthreads
        self.calls = 0

    def _pd(self, poly: SparsePoly) -> _PolyDesc:
        e = _arr(poly.exps, np.uint16)
        c = _arr(poly.coefs, np.uint64)
        self._keep += [e, c]
        return _PolyDesc(poly.p, poly.nvars, poly.nterms, e.ctypes.data, c.ctypes.data)

    def ctx(self) -> int:
        return ctypes.addressof(self.desc)

    def eval(self, k: int, i_first: int, ni: int, y, anchor, xk) -> np.ndarray:
        y = _arr(y, np.uint64)
        anchor = _arr(anchor, np.uint64)
        xk = _arr(xk, np.uint64)
        out = np.zeros(len(xk) * ni, dtype=np.uint64)
        rc = lib().zs_eval_points(ctypes.addressof(self.desc), self.nvars, k, i_first, ni,
                                  y.ctypes.data, anchor.ctypes.data, len(xk), xk.ctypes.data,
                                  out.ctypes.data)
        self.calls += 1
        if rc != 0:
            raise ZeroDivisionError("black box: denominator vanishes at a requested point")
        return out

    def at(self, point) -> int:
        """Value at one explicit point."""
        pt = _arr(point, np.uint64)
        n = self.nvars
        return int(self.eval(n, 1, 1, pt[:n - 1] if n > 1 else np.zeros(1, np.uint64),
                             np.zeros(n, np.uint64), pt[n - 1:n])[0])

    @staticmethod
    def c_function_address() -> int:
        return ctypes.cast(lib().zs_eval_points, ctypes.c_void_p).value


# --------------------------------------------------------------------------
# device black box: the same values as BlackBox, computed on the GPU for the
# structured Zippel points (large workloads); small requests use the host.

class _ZrPoints(ctypes.Structure):
    # layout of zr_points in include/zippel.h
    _fields_ = [("nvars", ctypes.c_uint32), ("k", ctypes.c_uint32), ("i_first", ctypes.c_uint64),
                ("ni", ctypes.c_uint64), ("nj", ctypes.c_uint64), ("y", ctypes.POINTER(ctypes.c_uint64)),
                ("anchor", ctypes.POINTER(ctypes.c_uint64)), ("xk", ctypes.POINTER(ctypes.c_uint64)),
                ("p", ctypes.c_uint64), ("nexpr", ctypes.c_uint32)]


_BB_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(_ZrPoints), ctypes.c_void_p,
                          ctypes.c_void_p)
_DEV = None
_HIP = None


def dev_lib():
    global _DEV, _HIP
    if _DEV is None:
        import torch  # noqa: F401  (one HIP runtime per process: PyTorch's, loaded first)
        D = ctypes.CDLL(dev_lib_path())
        D.zsd_apply.restype = ctypes.c_int
        D.zsd_apply.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        D.zsd_divide.restype = ctypes.c_int
        D.zsd_divide.argtypes = [ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]
        D.zsd_apply_scratch_words.restype = ctypes.c_size_t
        D.zsd_apply_scratch_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
        _DEV = D
        H = ctypes.CDLL("libamdhip64.so")
        H.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
        H.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        _HIP = H
    return _DEV, _HIP


class DeviceBlackBox:
    """Black box for a hidden polynomial (or P/Q) usable by the GPU
    reconstruction: the library passes a zr_points descriptor and a device
    buffer.  Large stage requests are evaluated on the GPU (zsd_apply, and
    zsd_divide for P/Q); small ones on the host."""

    HOST_LIMIT = 1 << 14
    MAX_NJ = 48  # values of x_k per request handled on the device

    def __init__(self, poly: SparsePoly, den: Optional[SparsePoly] = None, nthreads: int = 0):
        self.host = BlackBox(poly, den, nthreads=nthreads)
        self.p = poly.p
        self.nvars = poly.nvars
        self.calls = 0
        self.error = None
        self._cb = _BB_FN(self._call)
        self._bufs = {}

    def _dev(self, name, n):
        import torch
        buf = self._bufs.get(name)
        if buf is None or buf.numel() < n:
            buf = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
            self._bufs[name] = buf
        return buf

    def _apply(self, den, k, i_first, ni, y, anchor, xk, d_out, stream):
        D, H = dev_lib()
        nj = len(xk)
        poly = self.host.den if den else self.host.num
        T = poly.nterms
        Y = np.zeros(max(T, 1), dtype=np.uint64)
        W = np.zeros(max(T * nj, 1), dtype=np.uint64)
        ng = lib().zs_group_stage(self.host.ctx(), 1 if den else 0, k, y.ctypes.data, anchor.ctypes.data, nj,
                                  xk.ctypes.data, Y.ctypes.data, W.ctypes.data)
        dY = self._dev("Y", ng)
        dW = self._dev("W", ng * nj)
        H.hipMemcpyAsync(dY.data_ptr(), Y.ctypes.data, ng * 8, 1, stream)
        H.hipMemcpyAsync(dW.data_ptr(), W.ctypes.data, ng * nj * 8, 1, stream)
        sw = D.zsd_apply_scratch_words(ng, nj, ni)
        dS = self._dev("S", sw) if sw else None
        st = D.zsd_apply(self.p, ng, dY.data_ptr(), dW.data_ptr(), nj, i_first, ni, d_out,
                         dS.data_ptr() if dS is not None else None, stream)
        if st != 0:
            raise RuntimeError(f"zsd_apply failed with {st}")
        # the host arrays must outlive the asynchronous copies
        H.hipStreamSynchronize(stream)

    def device_eval(self, k, i_first, ni, y, anchor, xk, d_out: int, stream: int = 0) -> None:
        """Values at the stage-k points, written [jj][ii] to device memory d_out
        (numerator / denominator for a rational box)."""
        D, H = dev_lib()
        y = _arr(y, np.uint64)
        anchor = _arr(anchor, np.uint64)
        xk = _arr(xk, np.uint64)
        if self.host.den is None:
            self._apply(False, k, i_first, ni, y, anchor, xk, d_out, stream)
            return
        n = ni * len(xk)
        dN = self._dev("N", n)
        dD = self._dev("D", n)
        flag = self._dev("F", 1)
        flag.zero_()
        import torch
        torch.cuda.synchronize()
        self._apply(False, k, i_first, ni, y, anchor, xk, dN.data_ptr(), stream)
        self._apply(True, k, i_first, ni, y, anchor, xk, dD.data_ptr(), stream)
        st = D.zsd_divide(self.p, n, dN.data_ptr(), dD.data_ptr(), d_out, flag.data_ptr(), stream)
        if st != 0:
            raise RuntimeError(f"zsd_divide failed with {st}")
        H.hipStreamSynchronize(stream)
        if int(flag[0].item()) != 0:
            raise ZeroDivisionError("black box: denominator vanishes at a requested point")

    def _call(self, ctx, pts_ptr, d_vals, stream):
        try:
            pts = pts_ptr.contents
            nv, k, ni, nj = pts.nvars, pts.k, pts.ni, pts.nj
            y = np.ctypeslib.as_array(pts.y, shape=(nv,)).copy()
            a = np.ctypeslib.as_array(pts.anchor, shape=(nv,)).copy()
            xk = np.ctypeslib.as_array(pts.xk, shape=(nj,)).copy()
            _, H = dev_lib()
            if ni * nj <= self.HOST_LIMIT or k == 1 or nj > self.MAX_NJ:
                vals = self.host.eval(k, pts.i_first, ni, y, a, xk)
                H.hipMemcpyAsync(d_vals, vals.ctypes.data, vals.nbytes, 1, stream)
                H.hipStreamSynchronize(stream)
            else:
                self.device_eval(k, pts.i_first, ni, y, a, xk, d_vals, stream)
            self.calls += 1
            return 0
        except BaseException as e:  # noqa: BLE001 - reported through the status code
            self.error = e
            return 23

    @property
    def fn_ptr(self):
        return ctypes.cast(self._cb, ctypes.c_void_p)

    ctx = None


class MultiDeviceBlackBox:
    """Several hidden polynomials sampled at the same points (zr_points.nexpr
    of them): expression e's values go to d_vals[e * nj * ni ...]."""

    def __init__(self, polys: Sequence[SparsePoly], nthreads: int = 0):
        self.boxes = [DeviceBlackBox(h, nthreads=nthreads) for h in polys]
        self.calls = 0
        self.error = None
        self._cb = _BB_FN(self._call)

    def _call(self, ctx, pts_ptr, d_vals, stream):
        try:
            pts = pts_ptr.contents
            if pts.nexpr != len(self.boxes):
                return 31
            n = pts.ni * pts.nj
            for e, b in enumerate(self.boxes):
                st = b._call(ctx, pts_ptr, (d_vals or 0) + 8 * n * e, stream)
                if st:
                    self.error = b.error
                    return st
            self.calls += 1
            return 0
        except BaseException as e:  # noqa: BLE001 - reported through the status code
            self.error = e
            return 32

    @property
    def fn_ptr(self):
        return ctypes.cast(self._cb, ctypes.c_void_p)

    ctx = None


class PrimeDeviceBlackBox:
    """A polynomial with rational coefficients, evaluated modulo whichever
    prime a call names (zr_points.p): one DeviceBlackBox per prime."""

    def __init__(self, q: QPoly, nthreads: int = 0):
        self.q = q
        self.nthreads = nthreads
        self.boxes = {}
        self.calls = 0
        self.error = None
        self._cb = _BB_FN(self._call)

    def _call(self, ctx, pts_ptr, d_vals, stream):
        try:
            p = int(pts_ptr.contents.p)
            b = self.boxes.get(p)
            if b is None:
                b = self.boxes[p] = DeviceBlackBox(self.q.mod(p), nthreads=self.nthreads)
            st = b._call(ctx, pts_ptr, d_vals, stream)
            if st:
                self.error = b.error
                return st
            self.calls += 1
            return 0
        except BaseException as e:  # noqa: BLE001 - reported through the status code
            self.error = e
            return 33

    @property
    def fn_ptr(self):
        return ctypes.cast(self._cb, ctypes.c_void_p)

    ctx = None
