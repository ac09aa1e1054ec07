"""Multi-prime reconstruction on the GPU against the oracle: the known-term-set
solve modulo a further prime (zr_skeleton_solve) element by element, and
polynomials with rational coefficients (zippel_reconstruct_rational): the
same fractions and the same number of primes as the oracle's multi-prime
reconstruction, which equal the hidden ones."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import rational as orat

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def zr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_24256_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("nvars,deg,t", [(2, 3, 1), (3, 4, 7), (4, 9, 700), (5, 12, 3000), (6, 20, 20000)])
def test_skeleton_solve_matches_oracle(zr, nvars, deg, t):
    p = synth.prime_list(3)[2]
    h = synth.random_poly(p, nvars, deg, t, 40 + t)
    y = orat.further_bases(p, nvars, 7 + t)
    samples = synth.BlackBox(h).eval(nvars + 1, 1, t, y, np.zeros(nvars, np.uint64), np.zeros(1, np.uint64))
    _note(f"skeleton solve n={nvars} D={deg} t={t}")
    got, st = zr.skeleton_solve(p, h.exps, y, samples)
    assert st == 0
    assert np.array_equal(got, h.coefs)
    if t <= 3000:
        assert np.array_equal(got, orat.skeleton_solve(p, h.exps, y, samples))


def test_skeleton_solve_singular(zr):
    p = synth.make_prime()
    exps = np.array([[0, 1], [2, 0], [1, 1]], dtype=np.uint16)
    y = np.array([2, 4], dtype=np.uint64)  # y_1^2 = y_2: two equal monomial values
    _, st = zr.skeleton_solve(p, exps, y, np.array([1, 2, 3], dtype=np.uint64))
    assert st == zr.ZR_ESINGULAR


def _box(zr, q):
    cache = {}

    def box_for(p):
        if p not in cache:
            cache[p] = synth.BlackBox(q.mod(p))
        return cache[p]

    def fn(p, k, i_first, ni, y, a, xk):
        return box_for(p).eval(k, i_first, ni, y, a, xk)
    return zr.HostBlackBox(fn, q.nvars, with_prime=True), box_for


@pytest.mark.parametrize("nvars,deg,t,bits,used", [(3, 6, 40, 100, 5), (2, 5, 12, 20, 2), (4, 10, 2000, 150, 6)])
def test_rational_coefficients_match_oracle(zr, nvars, deg, t, bits, used):
    q = synth.random_qpoly(nvars, deg, t, bits, 100 + t)
    primes = synth.prime_list(8)
    seed = 3000 + t
    sched = synth.make_schedule(primes[0], nvars, [deg] * nvars, seed, 2)
    box, box_for = _box(zr, q)
    _note(f"rational n={nvars} D={deg} t={t} bits={bits}")
    e, fr, nused = zr.reconstruct_rational(primes[0], [deg] * nvars, box, primes[1:], sched=sched, seed=seed)
    oe, ofr, oused = orat.multiprime_zippel(primes, [deg] * nvars, sched, box_for, seed)
    assert np.array_equal(e, oe) and fr == ofr and nused == oused == used
    assert np.array_equal(e, q.exps) and fr == list(zip(q.num, q.den))


def test_rational_runs_out_of_primes(zr):
    q = synth.random_qpoly(2, 4, 10, 100, 23)
    primes = synth.prime_list(3)
    sched = synth.make_schedule(primes[0], 2, [4, 4], 78)
    box, _ = _box(zr, q)
    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct_rational(primes[0], [4, 4], box, primes[1:], sched=sched, seed=78)
    assert ei.value.code == zr.ZR_EPROBE


def test_rational_rejects_bad_primes(zr):
    q = synth.random_qpoly(2, 3, 5, 30, 24)
    primes = synth.prime_list(2)
    sched = synth.make_schedule(primes[0], 2, [3, 3], 79)
    box, _ = _box(zr, q)
    for bad in ([primes[0]], [(1 << 61) - 1], [primes[1] + 2 if not synth.is_prime(primes[1] + 2) else 9]):
        with pytest.raises(zr.ZippelError) as ei:
            zr.reconstruct_rational(primes[0], [3, 3], box, bad, sched=sched, seed=79)
        assert ei.value.code in (zr.ZR_EINVAL, zr.ZR_ENOTPRIME)
