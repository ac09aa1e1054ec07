"""Several expressions over one skeleton (zippel_reconstruct_multi) on the GPU:
every expression equals the oracle's reconstruction of that expression alone
on the same schedule (its own degree bounds, the first nodes of the shared
node lists) and the hidden polynomial, whether the expressions' term sets
overlap, nest or are disjoint; right-hand-side counts beyond one
producer/consumer workgroup are split into groups."""
import sys

import numpy as np
import pytest

import oracle
import synth

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


def _multi_box(zr, polys):
    boxes = [synth.BlackBox(h) for h in polys]

    def fn(k, i_first, ni, y, a, xk):
        return np.concatenate([b.eval(k, i_first, ni, y, a, xk) for b in boxes])
    return zr.HostBlackBox(fn, polys[0].nvars)


def _check(zr, polys, degs, seed, nprobes=2):
    p = polys[0].p
    n = polys[0].nvars
    dmax = np.max(np.asarray(degs), axis=0)
    sched = synth.make_schedule(p, n, [int(d) for d in dmax], seed, nprobes)
    res = zr.reconstruct_multi(p, degs, _multi_box(zr, polys), sched=sched)
    for e, (h, d) in enumerate(zip(polys, degs)):
        oe, oc = oracle.zippel(p, list(d), sched, synth.BlackBox(h))
        assert np.array_equal(res[e][0], oe) and np.array_equal(res[e][1], oc), e
        assert np.array_equal(res[e][0], h.exps) and np.array_equal(res[e][1], h.coefs), e
    return zr.last_counters()


def test_multi_various_degrees(zr):
    p = synth.make_prime()
    degs = [[6, 6, 6], [3, 8, 2], [10, 1, 5]]
    polys = [synth.random_poly(p, 3, d, t, 70 + e) for e, (d, t) in enumerate(zip(degs, (60, 25, 40)))]
    _note("3 expressions, n=3")
    _check(zr, polys, degs, 1070)


def test_multi_shared_and_disjoint_terms(zr):
    p = synth.make_prime()
    base = synth.random_poly(p, 4, 7, 300, 81)
    # same terms, other coefficients; a subset; a polynomial with its own terms
    other = synth.SparsePoly(p, 4, base.exps.copy(), synth.SplitMix64(5).uniform_block(1, p, 300)).sorted()
    sub = synth.SparsePoly(p, 4, base.exps[::3].copy(), base.coefs[::3].copy()).sorted()
    own = synth.random_poly(p, 4, 7, 200, 82)
    polys = [base, other, sub, own]
    _note("4 expressions, n=4, overlapping term sets")
    _check(zr, polys, [[7] * 4] * 4, 1081)


def test_multi_many_right_hand_sides(zr):
    """Five expressions of degree 20 in x_k: 100 right-hand sides per solve,
    two groups of the producer/consumer pass."""
    p = synth.make_prime()
    degs = [[20] * 3] * 5
    polys = [synth.random_poly(p, 3, 20, 1500, 90 + e) for e in range(5)]
    _note("5 expressions, R = 100")
    cnt = _check(zr, polys, degs, 1090)
    assert cnt["max_t"] >= 400


def test_multi_one_expression_equals_plain(zr):
    p = synth.make_prime()
    h = synth.random_poly(p, 4, 9, 500, 91)
    sched = synth.make_schedule(p, 4, [9] * 4, 1091, 2)
    (e, c), = zr.reconstruct_multi(p, [[9] * 4], _multi_box(zr, [h]), sched=sched)
    pe, pc = zr.reconstruct(p, [9] * 4, zr.HostBlackBox(synth.BlackBox(h).eval, 4), sched=sched)
    assert np.array_equal(e, pe) and np.array_equal(c, pc)
