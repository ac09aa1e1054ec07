"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
library routines (sympy), closed forms, brute force, and independent methods.
None of these retype the oracle's own formulas."""
import json
import os
import random

import numpy as np
import pytest
import sympy
from sympy.functions.combinatorial.numbers import stirling

import oracle
import synth
from balanced_cases import LimitBox, fallback_case

P63 = (1 << 63) - 25          # largest prime below 2^63
P61 = (1 << 61) - 1           # Mersenne prime
PRIMES = [P63, P61, synth.make_prime(), 1000000007, 101]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- field (§2.1)

@pytest.mark.parametrize("p", PRIMES)
def test_field_ops_match_bigint(p):
    rng = random.Random(p)
    edge = [0, 1, 2, p - 1, p - 2, p // 2, (p + 1) // 2]
    vals = edge + [rng.randrange(p) for _ in range(300)]
    for a in vals:
        for b in edge + [rng.randrange(p) for _ in range(3)]:
            assert oracle.mul(a, b, p) == a * b % p
            assert oracle.add(a, b, p) == (a + b) % p
            assert oracle.sub(a, b, p) == (a - b) % p
    for a in vals[1:60]:
        if a % p == 0:
            continue
        ia = oracle.inv(a, p)
        assert a * ia % p == 1
        assert oracle.power(a, p - 1, p) == 1          # Fermat
        e = rng.randrange(1 << 64)
        assert oracle.power(a, e, p) == pow(a, e, p)
    assert oracle.inv(0, p) == 0


def test_known_primes():
    assert oracle.is_prime(P61) and synth.is_prime(P61)
    assert oracle.is_prime(P63) and synth.is_prime(P63)
    for c in range(P63 + 2, (1 << 63), 2):
        assert not oracle.is_prime(c)
    assert sympy.prevprime(1 << 63) == P63


def test_miller_rabin_agrees_with_sympy():
    rng = random.Random(7)
    xs = [rng.randrange(1 << 62, 1 << 63) | 1 for _ in range(3000)]
    # strong pseudoprimes to small bases and Carmichael numbers
    xs += [2047, 1373653, 25326001, 3215031751, 2152302898747, 3474749660383, 341550071728321,
           3825123056546413051, 561, 1105, 1729, 2465, 2821, 6601, 8911]
    xs += [sympy.prevprime(1 << 62), sympy.nextprime(1 << 62)]
    for x in xs:
        assert oracle.is_prime(x) == sympy.isprime(x), x
        assert synth.is_prime(x) == sympy.isprime(x), x


def test_seeded_prime_is_in_range():
    p = synth.make_prime()
    assert (1 << 62) < p < (1 << 63)
    assert sympy.isprime(p)


# ---------------------------------------------------------------- SplitMix64

def test_splitmix_block_equals_stream():
    g1 = synth.SplitMix64(12345)
    g2 = synth.SplitMix64(12345)
    a = [g1.next() for _ in range(100)]
    b = g2.block(100)
    assert [int(x) for x in b] == a
    # rejection-heavy range: n just above 2^63 rejects about half of all draws
    n_hi = (1 << 63) + 12345
    g1 = synth.SplitMix64(99)
    g2 = synth.SplitMix64(99)
    a = [g1.uniform(0, n_hi) for _ in range(500)]
    b = g2.uniform_block(0, n_hi, 500)
    assert [int(x) for x in b] == a
    assert g1.state == g2.state


def test_schedule_nodes_distinct():
    p = synth.make_prime()
    s = synth.make_schedule(p, 4, [30, 31, 5, 0], seed=3, nprobes=3)
    for k in range(4):
        allv = [int(s.anchor[k])] + [int(x) for x in s.nodes[k]]
        assert len(set(allv)) == len(allv)
        assert all(1 <= v < p for v in allv)
    assert all(2 <= int(v) < p - 1 for v in s.y)
    assert s.probes.shape == (3, 4)


# ---------------------------------------------------------------- Vandermonde (§1, §2.2)

def _rand_distinct(rng, p, t):
    s = set()
    while len(s) < t:
        s.add(rng.randrange(1, p))
    return list(s)


@pytest.mark.parametrize("p", [P63, 1000000007, 101])
@pytest.mark.parametrize("t", [1, 2, 7, 33])
def test_vandermonde_equals_gauss_jordan(p, t):
    rng = random.Random(t * 7 + p % 97)
    m = _rand_distinct(rng, p, t)
    R = 3
    rhs = np.array([[rng.randrange(p) for _ in range(t)] for _ in range(R)], dtype=np.uint64)
    a = oracle.vandermonde_solve(p, m, rhs)
    g = oracle.gauss_vandermonde(p, m, rhs)
    assert np.array_equal(a, g)
    # plug into the definition with big integers
    for j in range(R):
        for i in range(1, t + 1):
            assert sum(int(a[j, l]) * pow(m[l], i, p) for l in range(t)) % p == int(rhs[j, i - 1])


def test_vandermonde_multiply_back_large():
    p = P63
    rng = random.Random(5)
    t = 400
    m = _rand_distinct(rng, p, t)
    coef = [rng.randrange(p) for _ in range(t)]
    v = oracle.vandermonde_apply(p, m, coef, 1, t)
    # apply pinned by big integers at sampled powers
    for i in rng.sample(range(1, t + 1), 20):
        assert int(v[i - 1]) == sum(c * pow(x, i, p) for c, x in zip(coef, m)) % p
    a = oracle.vandermonde_solve(p, m, v[None, :])
    assert [int(x) for x in a[0]] == coef


def test_gauss_solve_random_system_bigint():
    p = 1000000007
    rng = random.Random(1)
    n = 9
    A = sympy.Matrix(n, n, lambda i, j: rng.randrange(p))
    b = sympy.Matrix(n, 1, lambda i, j: rng.randrange(p))
    x = oracle.gauss_solve(p, np.array(A.tolist(), dtype=np.uint64), np.array(b.tolist(), dtype=np.uint64))
    xs = (A.inv_mod(p) * b).applyfunc(lambda z: z % p)
    assert [int(v) for v in x[:, 0]] == [int(v) for v in xs]


@pytest.mark.parametrize("t", [1, 5, 40, 120])
def test_master_polynomial_stirling(t):
    """m_l = 1..t: prod (z - l) = (z)_{t+1} / z, so M_r = s(t+1, r+1) (signed Stirling, first kind)."""
    p = P63
    M = oracle.master(p, list(range(1, t + 1)))
    for r in range(t + 1):
        assert int(M[r]) == int(stirling(t + 1, r + 1, kind=1, signed=True)) % p


@pytest.mark.parametrize("t", [1, 6, 50])
def test_master_polynomial_q_binomial(t):
    """m_l = g^l (l = 0..t-1): Cauchy's q-binomial theorem gives
    prod (z - g^l) = sum_k (-1)^(t-k) g^((t-k)(t-k-1)/2) [t choose k]_g z^k."""
    p = 1000000007
    g = 3
    M = oracle.master(p, [pow(g, l, p) for l in range(t)])

    def qbinom(n, k):
        num = 1
        den = 1
        for i in range(k):
            num = num * (1 - pow(g, n - i, p)) % p
            den = den * (1 - pow(g, i + 1, p)) % p
        return num * pow(den, p - 2, p) % p

    for k in range(t + 1):
        e = t - k
        want = (-1) ** e * pow(g, e * (e - 1) // 2, p) * qbinom(t, k) % p
        assert int(M[k]) == want


def test_vandermonde_singular_cases():
    p = 1000000007
    with pytest.raises(oracle.OracleError) as ei:
        oracle.vandermonde_solve(p, [5, 9, 5], np.ones((1, 3), dtype=np.uint64))
    assert ei.value.code == oracle.ESINGULAR
    with pytest.raises(oracle.OracleError) as ei:
        oracle.vandermonde_solve(p, [5, 0, 7], np.ones((1, 3), dtype=np.uint64))
    assert ei.value.code == oracle.ESINGULAR


def test_vandermonde_rows_subset_matches_full():
    p = P63
    rng = random.Random(11)
    t = 150
    m = _rand_distinct(rng, p, t)
    rhs = np.array([[rng.randrange(p) for _ in range(t)] for _ in range(4)], dtype=np.uint64)
    full = oracle.vandermonde_solve(p, m, rhs)
    rows = [0, 17, 149, 3]
    sub = oracle.vandermonde_solve_rows(p, m, rhs, rows)
    assert np.array_equal(sub, full[:, rows])


# ---------------------------------------------------------------- Newton (eq. 1)

@pytest.mark.parametrize("D", [0, 1, 5, 30, 40])
def test_newton_reproduces_polynomials(D):
    p = P63
    rng = random.Random(D)
    x = _rand_distinct(rng, p, D + 1)
    c = [rng.randrange(p) for _ in range(D + 1)]
    f = [sum(ci * pow(xi, i, p) for i, ci in enumerate(c)) % p for xi in x]
    assert [int(v) for v in oracle.newton(p, x, f)] == c
    # monomials x^d and the zero polynomial
    for d in range(D + 1):
        f = [pow(xi, d, p) for xi in x]
        want = [0] * (D + 1)
        want[d] = 1
        assert [int(v) for v in oracle.newton(p, x, f)] == want
    assert [int(v) for v in oracle.newton(p, x, [0] * (D + 1))] == [0] * (D + 1)


def test_newton_equals_lagrange_at_new_point():
    p = 1000000007
    rng = random.Random(3)
    x = _rand_distinct(rng, p, 12)
    f = [rng.randrange(p) for _ in range(12)]
    c = [int(v) for v in oracle.newton(p, x, f)]
    z = rng.randrange(p)
    lag = 0
    for i in range(12):
        num = den = 1
        for j in range(12):
            if j != i:
                num = num * (z - x[j]) % p
                den = den * (x[i] - x[j]) % p
        lag = (lag + f[i] * num * pow(den, p - 2, p)) % p
    assert sum(ci * pow(z, i, p) for i, ci in enumerate(c)) % p == lag


# ---------------------------------------------------------------- Thiele (eq. 2)

def _peval(c, x, p):
    return sum(ci * pow(x, i, p) for i, ci in enumerate(c)) % p


def test_thiele_moebius_closed_form():
    p = 1000000007
    al, be, ga = 17, 123456, 98765
    x = [3, 10, 77, 1234, 5555, 80808]
    f = [(al + be * xi) * pow(1 + ga * xi, p - 2, p) % p for xi in x]
    A, B = oracle.thiele(p, x, f)
    assert [int(v) for v in A] == [al, be]
    assert [int(v) for v in B] == [1, ga]


def test_thiele_golden_fixture():
    with open(os.path.join(GOLDEN, "thiele_small.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        A, B = oracle.thiele(case["p"], case["x"], case["f"])
        assert [int(v) for v in A] == case["A"], case["note"]
        assert [int(v) for v in B] == case["B"], case["note"]


@pytest.mark.parametrize("a,b", [(3, 0), (0, 3), (1, 2), (2, 1), (2, 2), (5, 1), (1, 5), (20, 5), (20, 20)])
def test_thiele_random_types(a, b):
    p = P63
    rng = random.Random(a * 31 + b)
    P = [rng.randrange(1, p) for _ in range(a + 1)]
    Q = [1] + [rng.randrange(1, p) for _ in range(b)]
    m = max(2 * a - 1, 2 * b, 0)
    n = m + 2
    x = _rand_distinct(rng, p, n + 3)
    f = [_peval(P, xi, p) * pow(_peval(Q, xi, p), p - 2, p) % p for xi in x]
    A, B = oracle.thiele(p, x, f)
    assert len(A) - 1 == a and len(B) - 1 == b       # exact minimal degrees
    # cross-multiplication A*Q == B*P as polynomials (big integers)
    A = [int(v) for v in A]
    B = [int(v) for v in B]
    AQ = [0] * (a + b + 1)
    BP = [0] * (a + b + 1)
    for i, u in enumerate(A):
        for j, v in enumerate(Q):
            AQ[i + j] = (AQ[i + j] + u * v) % p
    for i, u in enumerate(B):
        for j, v in enumerate(P):
            BP[i + j] = (BP[i + j] + u * v) % p
    assert AQ == BP
    assert B[0] == 1


def test_thiele_matches_linear_system_bruteforce():
    """Rational interpolation of type (2,1) as a linear system solved by sympy."""
    p = 1000000007
    rng = random.Random(9)
    P = [5, 7, 11]
    Q = [1, 13]
    x = _rand_distinct(rng, p, 6)
    f = [_peval(P, xi, p) * pow(_peval(Q, xi, p), p - 2, p) % p for xi in x]
    # unknowns a0 a1 a2 b1 (b0 = 1): a0 + a1 x + a2 x^2 - f b1 x = f
    rows = [[1, xi, xi * xi % p, (-fi * xi) % p] for xi, fi in zip(x[:4], f[:4])]
    sol = (sympy.Matrix(rows).inv_mod(p) * sympy.Matrix(f[:4])).applyfunc(lambda z: z % p)
    A, B = oracle.thiele(p, x, f)
    assert [int(v) for v in A] == [int(v) for v in sol[:3]]
    assert [int(v) for v in B] == [1, int(sol[3])]


def test_thiele_needs_confirmation_sample():
    p = 1000000007
    x = [1, 2, 3]
    f = [5, 9, 17]       # no degree-(1,1) fit confirmed within 3 samples of a generic function
    with pytest.raises(oracle.OracleError) as ei:
        oracle.thiele(p, x, [4, 1, 77])
    assert ei.value.code == oracle.EPROBE
    del f


# ---------------------------------------------------------------- Zippel (§1)

def _projection(poly, L, anchor, p):
    """coefficients of f(x_1..x_L, anchors) with exponents of x_{>L} set to 0, lex order."""
    acc = {}
    for e, c in zip(poly.exps, poly.coefs):
        key = tuple(int(v) for v in e[:L]) + (0,) * (poly.nvars - L)
        w = int(c)
        for v in range(L, poly.nvars):
            w = w * pow(int(anchor[v]), int(e[v]), p) % p
        acc[key] = (acc.get(key, 0) + w) % p
    items = sorted((k, v) for k, v in acc.items() if v)
    return items


def _as_items(e, c):
    return [(tuple(int(v) for v in row), int(x)) for row, x in zip(e, c)]


def test_zippel_config1_every_stage_and_bruteforce():
    w = synth.config_workload(1)
    box = synth.BlackBox(w.hidden)
    for L in range(1, w.hidden.nvars + 1):
        e, c = oracle.zippel(w.p, w.deg, w.schedule, box, last_stage=L)
        assert _as_items(e, c) == _projection(w.hidden, L, w.schedule.anchor, w.p)
    T = oracle.dense_newton(w.p, w.deg, w.schedule, box)
    nz = np.argwhere(T != 0)
    assert np.array_equal(nz.astype(np.uint16), w.hidden.exps)
    assert np.array_equal(T[tuple(nz.T)], w.hidden.coefs)


@pytest.mark.parametrize("nvars,deg,nterms,seed", [(1, 12, 5, 1), (2, 6, 49, 2), (2, 9, 20, 3), (4, 8, 300, 4),
                                                   (5, 3, 1, 5), (3, 0, 1, 6)])
def test_zippel_recovers_hidden(nvars, deg, nterms, seed):
    w = synth.poly_workload("t", nvars, deg, nterms, seed, 1000 + seed, nprobes=2)
    e, c = oracle.zippel(w.p, w.deg, w.schedule, synth.BlackBox(w.hidden))
    assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)


def test_zippel_dense_tiny_bruteforce_small_prime():
    p = 1000003
    hidden = synth.random_poly(p, 3, [3, 2, 4], 40, 77)
    sched = synth.make_schedule(p, 3, [3, 2, 4], 5, 2)
    box = synth.BlackBox(hidden)
    e, c = oracle.zippel(p, [3, 2, 4], sched, box)
    T = oracle.dense_newton(p, [3, 2, 4], sched, box)
    nz = np.argwhere(T != 0)
    assert np.array_equal(nz.astype(np.uint16), e)
    assert np.array_equal(T[tuple(nz.T)], c)


def test_zippel_medium_projections():
    w = synth.poly_workload("m", 4, 12, 2000, 21, 1021, nprobes=3)
    box = synth.BlackBox(w.hidden)
    e, c = oracle.zippel(w.p, w.deg, w.schedule, box, last_stage=3)
    assert _as_items(e, c) == _projection(w.hidden, 3, w.schedule.anchor, w.p)
    e, c = oracle.zippel(w.p, w.deg, w.schedule, box)
    assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)


# ---------------------------------------------------------------- failure injection

def test_zippel_collision_is_singular():
    p = synth.make_prime()
    exps = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 1]], dtype=np.uint16)
    hidden = synth.SparsePoly(p, 3, exps, np.array([3, 5, 7], dtype=np.uint64)).sorted()
    sched = synth.make_schedule(p, 3, [2, 2, 2], 1, 0)
    sched.y[1] = sched.y[0]                       # y_1 = y_2: x1 and x2 collide
    with pytest.raises(oracle.OracleError) as ei:
        oracle.zippel(p, [2, 2, 2], sched, synth.BlackBox(hidden))
    assert ei.value.code == oracle.ESINGULAR


def test_zippel_low_degree_bound_fails_probe():
    w = synth.poly_workload("lo", 3, 6, 30, 8, 1008, nprobes=3)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.zippel(w.p, [6, 6, 3], w.schedule, synth.BlackBox(w.hidden))
    assert ei.value.code == oracle.EPROBE


def test_zippel_blackbox_error_and_bad_prime():
    w = synth.config_workload(1)

    def broken(*args):
        raise RuntimeError("black box down")

    with pytest.raises(oracle.OracleError) as ei:
        oracle.zippel(w.p, w.deg, w.schedule, broken)
    assert ei.value.code == oracle.EBLACKBOX
    with pytest.raises(oracle.OracleError) as ei:
        oracle.zippel(w.p + 2 if not synth.is_prime(w.p + 2) else w.p + 4, w.deg, w.schedule,
                      synth.BlackBox(w.hidden))
    assert ei.value.code == oracle.ENOTPRIME


# ---------------------------------------------------------------- balanced Zippel (§2.2)

@pytest.mark.parametrize("nvars,total,tn,td,seed", [(2, 5, 6, 4, 1), (3, 6, 12, 9, 7), (4, 8, 40, 25, 3),
                                                   (3, 4, 1, 1, 5), (5, 20, 60, 30, 11)])
def test_balanced_recovers_hidden(nvars, total, tn, td, seed):
    rw = synth.rational_workload(nvars, total, tn, td, seed)
    (en, cn), (ed, cd) = oracle.balanced_zippel(rw.p, rw.deg_num, rw.deg_den, rw.schedule,
                                               synth.BlackBox(rw.num, rw.den))
    assert np.array_equal(en, rw.num.exps) and np.array_equal(cn, rw.num.coefs)
    assert np.array_equal(ed, rw.den.exps) and np.array_equal(cd, rw.den.coefs)


def test_balanced_common_factor_every_stage():
    """After stage L the pair is C*P(x_1..x_L, anchors), C*Q(...) with a single C."""
    rw = synth.rational_workload(4, 8, 30, 20, 13)
    box = synth.BlackBox(rw.num, rw.den)
    p = rw.p
    for L in range(1, 4):
        (en, cn), (ed, cd) = oracle.balanced_zippel(p, rw.deg_num, rw.deg_den, rw.schedule, box, last_stage=L)
        pn = _projection(rw.num, L, rw.schedule.anchor, p)
        pd = _projection(rw.den, L, rw.schedule.anchor, p)
        got_n = _as_items(en, cn)
        got_d = _as_items(ed, cd)
        assert [k for k, _ in got_n] == [k for k, _ in pn]
        assert [k for k, _ in got_d] == [k for k, _ in pd]
        C = got_n[0][1] * pow(pn[0][1], p - 2, p) % p
        for (_, g), (_, h) in zip(got_n + got_d, pn + pd):
            assert g == C * h % p


def test_balanced_zero_constant_denominator_is_enorm():
    p = synth.make_prime()
    num = synth.SparsePoly(p, 2, np.array([[0, 0], [1, 1]], dtype=np.uint16), np.array([4, 9], dtype=np.uint64))
    den = synth.SparsePoly(p, 2, np.array([[1, 0], [0, 2]], dtype=np.uint16), np.array([1, 3], dtype=np.uint64))
    dn, dd = [2, 2], [2, 2]
    J = [synth.thiele_nodes_needed(a, b) for a, b in zip(dn, dd)]
    sched = synth.make_schedule(p, 2, J, 4, 1)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.balanced_zippel(p, dn, dd, sched, synth.BlackBox(num.sorted(), den.sorted()))
    assert ei.value.code == oracle.ENORM


# ---------------------------------------------------------------- black box

def test_blackbox_matches_bigint_evaluation():
    w = synth.poly_workload("bb", 4, 7, 60, 3, 1003)
    box = synth.BlackBox(w.hidden)
    p = w.p
    y, anc = w.schedule.y, w.schedule.anchor
    xk = [11, 222, 3333]
    for k in (1, 2, 4):
        vals = box.eval(k, 3, 5, y, anc, xk)
        for jj in range(3):
            for ii in range(5):
                pt = [pow(int(y[v]), 3 + ii, p) for v in range(k - 1)] + [xk[jj]] + \
                     [int(a) for a in anc[k:]]
                want = 0
                for e, c in zip(w.hidden.exps, w.hidden.coefs):
                    term = int(c)
                    for v in range(4):
                        term = term * pow(pt[v], int(e[v]), p) % p
                    want = (want + term) % p
                assert int(vals[jj * 5 + ii]) == want
                assert oracle.poly_eval(p, w.hidden.exps, w.hidden.coefs, pt) == want


# ---------------------------------------------------------------- balancing-factor fallback (§2.2)
#
# The balancing factor of slice i is beta_i = N_{k-1}(y^i) / A_i(c_k), and
# D_{k-1}(y^i) / B_i(c_k) when the numerator side vanishes.  These cases are
# built from the schedule so that the numerator side vanishes exactly, which a
# random input does with probability about deg/p.

@pytest.mark.parametrize("seed", [4, 5, 6])
def test_balanced_beta_fallback_slice(seed):
    """Slice 1 takes the denominator-side factor; the result is still P/Q."""
    p, dn, dd, sched, num, den = fallback_case(seed)
    (en, cn), (ed, cd) = oracle.balanced_zippel(p, dn, dd, sched, synth.BlackBox(num, den))
    assert np.array_equal(en, num.exps) and np.array_equal(cn, num.coefs)
    assert np.array_equal(ed, den.exps) and np.array_equal(cd, den.coefs)


def test_balanced_beta_fallback_every_slice():
    """A zero numerator: N_{k-1} = 0 and A_i = 0 on every slice, so every
    factor comes from the denominator side; 0/Q in lowest terms is 0/1."""
    p = synth.make_prime()
    rw = synth.rational_workload(3, 6, 5, 6, 17)
    zero = synth.SparsePoly(p, 3, np.zeros((0, 3), dtype=np.uint16), np.zeros(0, dtype=np.uint64))
    (en, cn), (ed, cd) = oracle.balanced_zippel(p, rw.deg_num, rw.deg_den, rw.schedule,
                                               synth.BlackBox(zero, rw.den))
    assert len(cn) == 0 and en.shape == (0, 3)
    assert np.array_equal(ed, np.zeros((1, 3), dtype=np.uint16)) and list(cd) == [1]


def test_balanced_both_sides_vanish_is_edegen():
    """P and Q vanish together at (y1, c2), the anchor node of slice 1 at stage 2:
    both balancing factors of that slice vanish.  Slice 1 has lost the common
    factor x2 - c2 (its reduced fraction is the constant -y1 c2), so its
    degrees differ from the other slices' and the stage reports EDEGEN; a
    black box that evaluates P/Q without reducing fails there instead."""
    p, dn, dd, sched, num, den = fallback_case(4, both_vanish=True)
    y1, c2 = int(sched.y[0]), int(sched.anchor[1])
    box = LimitBox(num, den, (-y1 * c2) % p)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.balanced_zippel(p, dn, dd, sched, box.eval)
    assert ei.value.code == oracle.EDEGEN
    with pytest.raises(oracle.OracleError) as ei:
        oracle.balanced_zippel(p, dn, dd, sched, synth.BlackBox(num, den))
    assert ei.value.code == oracle.EBLACKBOX
    # stage 1 alone (x2 at its anchor) is a regular fraction
    (en, cn), (ed, cd) = oracle.balanced_zippel(p, dn, dd, sched, box.eval, last_stage=1)
    assert len(cn) > 0 and len(cd) > 0
