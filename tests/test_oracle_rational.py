"""Pins of the oracle's multi-prime step (rational coefficients from residues
modulo several primes) against what mathematics fixes: the Chinese remainder
theorem by brute force on small moduli, rational reconstruction by an
exhaustive search over every fraction within the bound, round trips of random
fractions, the known-skeleton solve against the hidden polynomial, and a full
multi-prime reconstruction of a polynomial with rational coefficients.  No GPU."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import rational as orat


def test_crt_brute_force_small_moduli():
    primes = [3, 5, 7, 11]
    P = math.prod(primes)
    for rs in itertools.product(*[range(q) for q in primes]):
        X, PP = orat.crt(rs, primes)
        assert PP == P and 0 <= X < P
        # the unique X in [0, P) with these residues
        assert all(X % q == r for q, r in zip(primes, rs))
    # every X in [0, P) is hit exactly once
    seen = {orat.crt([x % q for q in primes], primes)[0] for x in range(P)}
    assert seen == set(range(P))


def test_crt_large_primes():
    primes = synth.prime_list(5)
    g = synth.SplitMix64(3)
    for _ in range(50):
        rs = [g.uniform(0, q) for q in primes]
        X, P = orat.crt(rs, primes)
        assert 0 <= X < P == math.prod(primes)
        assert [X % q for q in primes] == rs


def _brute_fractions(u, P):
    N = 1 << orat.bound_exponent(P)
    out = []
    for b in range(1, N):
        if math.gcd(b, P) != 1:
            continue
        for a in range(-N + 1, N):
            if math.gcd(a, b) == 1 and (a - b * u) % P == 0:
                out.append((a, b))
    return out


@pytest.mark.parametrize("P", [7 * 11 * 13, 2 * 3 * 5 * 7 * 11, 101 * 103])
def test_rational_reconstruction_exhaustive(P):
    N = 1 << orat.bound_exponent(P)
    assert 2 * N * N <= P
    for u in range(P):
        want = _brute_fractions(u, P)
        assert len(want) <= 1  # unique within the bound
        got = orat.rational_reconstruct(u, P)
        assert got == (want[0] if want else None), (u, got, want)


def test_rational_reconstruction_round_trip():
    g = synth.SplitMix64(11)
    for k in range(1, 7):
        primes = synth.prime_list(k, seed=500)
        P = math.prod(primes)
        e = orat.bound_exponent(P)
        for _ in range(40):
            a = g.next() % (1 << (e - 1)) if e > 1 else 0
            if g.next() & 1:
                a = -a
            b = 1 + g.next() % ((1 << (e - 1)) - 1) if e > 1 else 1
            d = math.gcd(a, b)
            a, b = a // d, b // d
            u = a * pow(b, -1, P) % P
            assert orat.rational_reconstruct(u, P) == (a, b)
    # integers and zero
    P = math.prod(synth.prime_list(2))
    assert orat.rational_reconstruct(0, P) == (0, 1)
    assert orat.rational_reconstruct(P - 5, P) == (-5, 1)
    assert orat.rational_reconstruct(pow(3, -1, P), P) == (1, 3)


def test_skeleton_solve_recovers_hidden_coefficients():
    p = synth.make_prime()
    h = synth.random_poly(p, 4, 7, 120, 31)
    y = orat.further_bases(p, 4, 99)
    box = synth.BlackBox(h)
    samples = box.eval(5, 1, h.nterms, y, np.zeros(4, np.uint64), np.zeros(1, np.uint64))
    got = orat.skeleton_solve(p, h.exps, y, samples)
    assert np.array_equal(got, h.coefs)
    # the samples are the values at x_v = y_v^i: one point checked directly
    i = 17
    assert int(samples[i - 1]) == box.at([pow(int(v), i, p) for v in y])


def _qbox_factory(q):
    cache = {}

    def box_for(p):
        if p not in cache:
            cache[p] = synth.BlackBox(q.mod(p))
        return cache[p]
    return box_for


def test_multiprime_zippel_recovers_rational_coefficients():
    q = synth.random_qpoly(3, 6, 40, 100, 21)
    primes = synth.prime_list(6)
    sched = synth.make_schedule(primes[0], 3, [6, 6, 6], 1021)
    exps, rec, used = orat.multiprime_zippel(primes, [6, 6, 6], sched, _qbox_factory(q), 1021)
    assert np.array_equal(exps, q.exps)
    assert rec == list(zip(q.num, q.den))
    # 100-bit numerators and denominators need e >= 100: four 63-bit primes
    # (e = 125; three give e = 93), plus one confirming prime
    assert used == 5


def test_multiprime_zippel_small_coefficients_use_two_primes():
    q = synth.random_qpoly(2, 5, 12, 20, 22)
    primes = synth.prime_list(4)
    sched = synth.make_schedule(primes[0], 2, [5, 5], 77)
    exps, rec, used = orat.multiprime_zippel(primes, [5, 5], sched, _qbox_factory(q), 77)
    assert rec == list(zip(q.num, q.den)) and used == 2


def test_multiprime_zippel_runs_out_of_primes():
    q = synth.random_qpoly(2, 4, 10, 100, 23)
    primes = synth.prime_list(3)
    sched = synth.make_schedule(primes[0], 2, [4, 4], 78)
    with pytest.raises(oracle.OracleError) as ei:
        orat.multiprime_zippel(primes, [4, 4], sched, _qbox_factory(q), 78)
    assert ei.value.code == oracle.EPROBE
