"""GPU parity of the balancing factor's fallback (§2.2, the balancing
equation): slices whose previous-stage numerator vanishes at their Zippel
point take the factor from the denominator side.  The GPU result of the
one-reconstruction path and of the served path must equal the oracle's on
the same inputs, and the degenerate case must fail the same way."""
import sys

import numpy as np
import pytest

import oracle
import synth
from balanced_cases import LimitBox, fallback_case

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


def _zero_numerator():
    p = synth.make_prime()
    rw = synth.rational_workload(3, 6, 5, 6, 17)
    zero = synth.SparsePoly(p, 3, np.zeros((0, 3), dtype=np.uint16), np.zeros(0, dtype=np.uint64))
    return p, rw.deg_num, rw.deg_den, rw.schedule, zero, rw.den


def _cases():
    return [fallback_case(s) for s in (4, 5, 6)] + [_zero_numerator()]


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_fallback_matches_oracle(zr):
    for i, (p, dn, dd, sched, num, den) in enumerate(_cases()):
        _note(f"balanced fallback case {i}")
        n, d = zr.balanced_reconstruct(p, dn, dd, zr.HostBlackBox(synth.BlackBox(num, den).eval, len(dn)),
                                       sched=sched)
        on, od = oracle.balanced_zippel(p, dn, dd, sched, synth.BlackBox(num, den))
        assert _same(n, on) and _same(d, od)


def test_fallback_served_matches_oracle(zr):
    cases = _cases()
    srv = zr.Server(cases[0][0], max_active=8)
    try:
        ids = [srv.submit(dn, zr.HostBlackBox(synth.BlackBox(num, den).eval, len(dn)), sched=sched, deg_den=dd)
               for (p, dn, dd, sched, num, den) in cases]
        res = {}
        for _ in range(64):
            srv.step()
            for i, rid in enumerate(ids):
                if i not in res:
                    r = srv.poll(rid)
                    if r is not None:
                        res[i] = r
            if len(res) == len(ids):
                break
        assert len(res) == len(ids)
        for i, (p, dn, dd, sched, num, den) in enumerate(cases):
            st, n, d = res[i]
            on, od = oracle.balanced_zippel(p, dn, dd, sched, synth.BlackBox(num, den))
            assert st == zr.ZR_OK and _same(n, on) and _same(d, od)
    finally:
        srv.close()


def test_both_sides_vanish(zr):
    p, dn, dd, sched, num, den = fallback_case(4, both_vanish=True)
    y1, c2 = int(sched.y[0]), int(sched.anchor[1])
    box = LimitBox(num, den, (-y1 * c2) % p)
    with pytest.raises(oracle.OracleError) as eo:
        oracle.balanced_zippel(p, dn, dd, sched, box.eval)
    with pytest.raises(zr.ZippelError) as eg:
        zr.balanced_reconstruct(p, dn, dd, zr.HostBlackBox(box.eval, 2), sched=sched)
    assert eg.value.code == eo.value.code == zr.ZR_EDEGEN
