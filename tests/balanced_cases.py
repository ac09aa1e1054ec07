"""Rational black boxes built so that the balancing factor of one slice must
come from the denominator side (§2.2, the balancing equation): the previous
stage's numerator vanishes at that slice's Zippel point, which a random input
does with probability about deg/p.  Shared by the oracle pins and the GPU
parity tests."""
import numpy as np

import oracle
import synth


def fallback_case(seed, both_vanish=False):
    """n = 2, P(x1, x2) = x1 x2 + 3 x1^2 + kappa with kappa chosen so that
    P(y1, c2) = 0: at stage 2 slice i = 1 (x1 = y1) the previous numerator
    N_1(y1) = C P(y1, c2) is zero while the slice is a generic (1, 1) fraction.
    With both_vanish the denominator is chosen to vanish at (y1, c2) too."""
    p = synth.make_prime()
    dn, dd = [2, 1], [1, 1]
    J = [synth.thiele_nodes_needed(a, b) for a, b in zip(dn, dd)]
    sched = synth.make_schedule(p, 2, J, seed, 2)
    y1, c2 = int(sched.y[0]), int(sched.anchor[1])
    kappa = (-(y1 * c2 + 3 * y1 * y1)) % p
    num = synth.SparsePoly(p, 2, np.array([[0, 0], [1, 1], [2, 0]], dtype=np.uint16),
                           np.array([kappa, 1, 3], dtype=np.uint64)).sorted()
    if both_vanish:
        # Q = 1 + 2 x2 + beta x1 x2 with Q(y1, c2) = 0
        beta = (-(1 + 2 * c2) * pow(y1 * c2 % p, p - 2, p)) % p
        den = synth.SparsePoly(p, 2, np.array([[0, 0], [0, 1], [1, 1]], dtype=np.uint16),
                               np.array([1, 2, beta], dtype=np.uint64)).sorted()
        assert (1 + 2 * c2 + beta * y1 * c2) % p == 0
    else:
        den = synth.SparsePoly(p, 2, np.array([[0, 0], [0, 1], [1, 0], [1, 1]], dtype=np.uint16),
                               np.array([1, 7, 2, 1], dtype=np.uint64)).sorted()
        assert (1 + 7 * c2 + 2 * y1 + y1 * c2) % p != 0
    assert oracle.poly_eval(p, num.exps, num.coefs, [y1, c2]) == 0
    return p, dn, dd, sched, num, den


class LimitBox:
    """P/Q for the tiny two-variable case of _fallback_case(both_vanish=True),
    returning at a point where P and Q both vanish the value of the slice's
    reduced fraction there (what a black box that reduces P/Q before
    evaluating would return), instead of failing on 0/0."""

    def __init__(self, num, den, limit):
        self.num, self.den, self.limit, self.p = num, den, limit, num.p

    def at(self, pt):
        p = self.p
        a = oracle.poly_eval(p, self.num.exps, self.num.coefs, pt)
        b = oracle.poly_eval(p, self.den.exps, self.den.coefs, pt)
        if b == 0:
            assert a == 0, "pole of P/Q"
            return self.limit
        return a * pow(b, p - 2, p) % p

    def eval(self, k, i_first, ni, y, anchor, xk):
        p = self.p
        out = []
        for x in xk:
            for i in range(int(i_first), int(i_first) + int(ni)):
                pt = [pow(int(y[v]), i, p) for v in range(int(k) - 1)] + [int(x)] + [int(a) for a in anchor[int(k):]]
                out.append(self.at(pt))
        return np.array(out, dtype=np.uint64)
