"""ORACLE — test infrastructure only.

Rational coefficients from reconstructions modulo several primes: the step
that the paper performs last, after the modular reconstruction (§1: results
modulo large primes are combined and turned into rational numbers; §2.2 names
the multi-prime Zippel routine as one of the two that dominate the time).
Written with Python integers, each function the plain definition:

- ``crt``: the Chinese remainder theorem in its textbook form,
  X = sum_j r_j (P/p_j) ((P/p_j)^-1 mod p_j) mod P.
- ``rational_reconstruct``: Wang's method (P. S. Wang, "A p-adic algorithm for
  univariate partial fractions", SYMSAC 1981; the extended-Euclid form of
  von zur Gathen and Gerhard, "Modern Computer Algebra", §5.10): run the
  extended Euclidean algorithm on (P, u) until the remainder drops below the
  bound N, then accept r / t if |t| < N and gcd(r, t) = 1.  Bound (a reading,
  see ``bound_exponent``): N = 2^e, e = floor((bitlen(P) - 2) / 2), so that
  2 N^2 <= P and a fraction within the bound is unique.
- ``skeleton_solve``: with the term set known, the coefficients modulo a
  further prime come from one transposed Vandermonde system over all n
  variables (x_v = y_v^i, i = 1..t), solved by the oracle's own solve.
- ``multiprime_zippel``: Zippel modulo the first prime fixes the term set;
  each further prime j (bases from the seeded schedule with seed + j) gives
  one more residue per term; after each prime the reconstruction from the
  primes so far is checked against the next prime's residues, and accepted
  when every term agrees (a reading: the paper does not state its stopping
  rule; one confirming prime).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product library never imports it.
"""
from __future__ import annotations

import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import EPROBE, ESINGULAR, OracleError, vandermonde_solve, zippel


def crt(residues: Sequence[int], primes: Sequence[int]) -> Tuple[int, int]:
    """(X, P): 0 <= X < P = prod p_j with X = r_j mod p_j for every j."""
    P = 1
    for q in primes:
        P *= q
    X = 0
    for r, q in zip(residues, primes):
        Pq = P // q
        X += int(r) * Pq * pow(Pq % q, -1, q)
    return X % P, P


def bound_exponent(P: int) -> int:
    """e with N = 2^e the numerator and denominator bound: floor((bitlen(P) - 2) / 2)."""
    return max(0, (P.bit_length() - 2) // 2)


def rational_reconstruct(u: int, P: int) -> Optional[Tuple[int, int]]:
    """(a, b) with a = b u mod P, |a| < 2^e, 0 < b < 2^e, gcd(a, b) = 1, or None."""
    N = 1 << bound_exponent(P)
    r0, r1 = P, u % P
    t0, t1 = 0, 1
    while r1 >= N:
        q = r0 // r1
        r0, r1 = r1, r0 - q * r1
        t0, t1 = t1, t0 - q * t1
    if t1 == 0 or abs(t1) >= N or math.gcd(r1, abs(t1)) != 1:
        return None
    return (r1, t1) if t1 > 0 else (-r1, -t1)


def monomial_values(p: int, exps: np.ndarray, y: Sequence[int]) -> np.ndarray:
    """m_l = prod_v y_v^{e_{l,v}} mod p over all variables."""
    out = np.zeros(exps.shape[0], dtype=np.uint64)
    for l in range(exps.shape[0]):
        m = 1
        for v in range(exps.shape[1]):
            m = m * pow(int(y[v]), int(exps[l, v]), p) % p
        out[l] = m
    return out


def skeleton_solve(p: int, exps: np.ndarray, y: Sequence[int], samples: Sequence[int]) -> np.ndarray:
    """Coefficients a_l mod p of the terms exps from samples v_i = f(y^i),
    i = 1..t: the system sum_l a_l m_l^i = v_i."""
    m = monomial_values(p, exps, y)
    t = len(m)
    if t == 0:
        return np.zeros(0, dtype=np.uint64)
    return vandermonde_solve(p, m, np.asarray(samples, dtype=np.uint64).reshape(1, t))[0]


def further_bases(p: int, nvars: int, seed: int) -> np.ndarray:
    """Zippel bases y_1..y_n for a further prime: the first draws of the seeded schedule."""
    import synth
    return synth.make_schedule(p, nvars, [0] * nvars, seed).y


def agrees(rec: Sequence[Optional[Tuple[int, int]]], residues: Sequence[int], p: int) -> bool:
    """Every reconstructed a/b reduces to the given residue modulo p (b invertible)."""
    for r, c in zip(rec, residues):
        if r is None:
            return False
        a, b = r
        if b % p == 0 or (a - int(c) * b) % p != 0:
            return False
    return True


def multiprime_zippel(primes: Sequence[int], deg: Sequence[int], schedule, box_for_prime: Callable,
                      seed: int):
    """Rational coefficients of a black box over Q.

    primes[0]  the prime of the Zippel reconstruction (schedule drawn for it);
    primes[j]  further primes, used in order, bases from seed + j;
    box_for_prime(p) -> an object with eval(k, i_first, ni, y, anchor, xk)
               (synth.BlackBox) evaluating the black box modulo p.
    Returns (exps, [(num, den)], primes used, the confirming one included);
    raises OracleError(EPROBE) when the primes run out first."""
    p0 = primes[0]
    exps, c0 = zippel(p0, deg, schedule, box_for_prime(p0))
    t, n = exps.shape
    used = [p0]
    res = [[int(c)] for c in c0]
    rec = [rational_reconstruct(r[0], p0) for r in res]
    for j in range(1, len(primes)):
        q = primes[j]
        y = further_bases(q, n, seed + j)
        box = box_for_prime(q)
        samples = box.eval(n + 1, 1, t, y, np.zeros(n, dtype=np.uint64), np.zeros(1, dtype=np.uint64))
        m = monomial_values(q, exps, y)
        if len(set(int(x) for x in m)) != t or any(int(x) == 0 for x in m):
            raise OracleError(ESINGULAR, "monomial values collide")
        cj = skeleton_solve(q, exps, y, samples)
        if agrees(rec, cj, q):
            return exps, rec, len(used) + 1
        used.append(q)
        for l in range(t):
            res[l].append(int(cj[l]))
        rec = [rational_reconstruct(crt(res[l], used)[0], math.prod(used)) for l in range(t)]
    raise OracleError(EPROBE, "primes ran out before a confirmation")
