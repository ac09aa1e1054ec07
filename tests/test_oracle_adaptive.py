"""Pins of the oracle's reconstruction without degree bounds: divided
differences against their closed forms (leading coefficient of a polynomial
of the order's degree, zero beyond it, the complete symmetric sum for x^m),
and the early-terminating reconstruction against the hidden polynomial, the
fixed-bound oracle and the true per-variable degrees.  No GPU."""
import numpy as np
import pytest

import oracle
import synth
from oracle import adaptive as oad


def test_divided_differences_closed_forms():
    p = synth.make_prime()
    g = synth.SplitMix64(12)
    x = [g.uniform(1, p) for _ in range(9)]
    c = [g.uniform(0, p) for _ in range(6)]  # degree 5

    def f(v):
        return sum(ci * pow(v, i, p) for i, ci in enumerate(c)) % p
    fx = [f(v) for v in x]
    assert oad.divided_difference(p, x[:6], fx[:6]) == c[5]
    for m in (7, 8, 9):
        assert oad.divided_difference(p, x[:m], fx[:m]) == 0
    # f = z^m: the order m-1 difference is the sum of the nodes, order m is 1
    for m in (2, 3, 5):
        xm = [pow(v, m, p) for v in x]
        assert oad.divided_difference(p, x[:m], xm[:m]) == sum(x[:m]) % p
        assert oad.divided_difference(p, x[:m + 1], xm[:m + 1]) == 1
    # the recursive table gives the same numbers
    for m in range(1, 8):
        tab = list(fx[:m + 1])
        for order in range(1, m + 1):
            tab = [(tab[i + 1] - tab[i]) * pow(x[i + order] - x[i], -1, p) % p for i in range(len(tab) - 1)]
        assert tab[0] == oad.divided_difference(p, x[:m + 1], fx[:m + 1])


@pytest.mark.parametrize("confirm", [1, 2])
def test_adaptive_recovers_hidden_and_degrees(confirm):
    p = synth.make_prime()
    h = synth.random_poly(p, 3, [5, 8, 3], 60, 44)
    true = [int(h.exps[:, v].max()) for v in range(3)]
    caps = [12, 12, 12]
    sched = synth.make_schedule(p, 3, [c + confirm for c in caps], 1044, 2)
    e, c, found = oad.adaptive_zippel(p, caps, sched, synth.BlackBox(h), confirm=confirm)
    assert np.array_equal(e, h.exps) and np.array_equal(c, h.coefs)
    assert found == true
    oe, oc = oracle.zippel(p, true, sched, synth.BlackBox(h))
    assert np.array_equal(e, oe) and np.array_equal(c, oc)


def test_adaptive_cap_below_degree_fails():
    p = synth.make_prime()
    h = synth.random_poly(p, 2, [6, 4], 20, 45)
    true = [int(h.exps[:, v].max()) for v in range(2)]
    caps = [true[0] - 1, 10]
    sched = synth.make_schedule(p, 2, [c + 1 for c in caps], 1045, 0)
    with pytest.raises(oracle.OracleError) as ei:
        oad.adaptive_zippel(p, caps, sched, synth.BlackBox(h), confirm=1)
    assert ei.value.code == oracle.EPROBE


def test_adaptive_univariate_gap():
    """x^5 + 1: the lower orders do not vanish, so the stop comes at order 6."""
    p = synth.make_prime()
    h = synth.SparsePoly(p, 1, np.array([[0], [5]], dtype=np.uint16), np.array([1, 1], dtype=np.uint64))
    sched = synth.make_schedule(p, 1, [11], 46, 1)
    e, c, found = oad.adaptive_zippel(p, [10], sched, synth.BlackBox(h), confirm=1)
    assert found == [5] and np.array_equal(e, h.exps) and np.array_equal(c, h.coefs)
