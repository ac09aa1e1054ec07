"""Served form on the GPU: requests admitted by footprint and advanced in
continuous batches give exactly the result of the same request run alone."""
import sys

import numpy as np
import pytest

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


def _box(zr, num, den=None):
    return zr.HostBlackBox(synth.BlackBox(num, den).eval, num.nvars)


def _rational_mix(count, seed):
    """Rational requests of uneven sizes (n 2..5, total degree 3..12, t_N, t_D log-uniform)."""
    g = synth.SplitMix64(seed)
    out = []
    for i in range(count):
        n = 2 + int(g.uniform(0, 4))
        tot = 3 + int(g.uniform(0, 10))
        tn = max(1, int(np.exp(g.uniform(0, 1000) / 1000.0 * np.log(120))))
        td = max(1, int(np.exp(g.uniform(0, 1000) / 1000.0 * np.log(120))))
        from math import comb
        cap = comb(tot + n, n)
        out.append(synth.rational_workload(n, tot, min(tn, cap), min(td, cap - 1) + 1 if cap > 1 else 1,
                                           9000 + seed * 100 + i))
    return out


def _alone(zr, w):
    """(status, num, den) of the request run alone through the one-request entry point."""
    try:
        if hasattr(w, "num"):
            n, d = zr.balanced_reconstruct(w.p, w.deg_num, w.deg_den, _box(zr, w.num, w.den), sched=w.schedule)
            return zr.ZR_OK, n, d
        return zr.ZR_OK, zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule), None
    except zr.ZippelError as e:
        return e.code, None, None


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _run(srv, ids):
    results = {}
    while len(results) < len(ids):
        srv.step()
        for i in ids:
            if i not in results:
                r = srv.poll(i)
                if r is not None:
                    results[i] = r
    return results


def test_served_equals_alone_balanced(zr):
    ws = _rational_mix(16, 1)
    srv = zr.Server(ws[0].p, hbm_budget=1 << 30, max_active=5)
    ids = [srv.submit(w.deg_num, _box(zr, w.num, w.den), sched=w.schedule, deg_den=w.deg_den) for w in ws]
    res = _run(srv, ids)
    st = srv.stats()
    _note(f"stats {st}")
    assert st["peak_active"] <= 5 and st["completed"] == len(ws) and st["failed"] == 0
    for w, i in zip(ws, ids):
        status, num, den = res[i]
        ast, an, ad = _alone(zr, w)
        assert status == ast == zr.ZR_OK
        assert _same(num, an) and _same(den, ad)
        assert np.array_equal(num[0], w.num.exps) and np.array_equal(num[1], w.num.coefs)
        assert np.array_equal(den[0], w.den.exps) and np.array_equal(den[1], w.den.coefs)
    srv.close()


def test_served_arrivals_mixed_kinds_and_failures(zr):
    """Requests arrive between steps; polynomial and rational requests share
    steps; a failing black box only fails its own request."""
    rs = _rational_mix(8, 2)
    ps = [synth.poly_workload(f"s{i}", 3 + i % 3, 8, 40 + 30 * i, 300 + i, 1300 + i, p=rs[0].p) for i in range(6)]
    srv = zr.Server(rs[0].p, hbm_budget=4 << 30, max_active=64)

    def broken(*a):
        raise RuntimeError("down")

    queue = []
    for i in range(max(len(rs), len(ps))):
        if i < len(rs):
            queue.append(("r", rs[i]))
        if i < len(ps):
            queue.append(("p", ps[i]))
    ids = {}
    bad = None
    step = 0
    results = {}
    while queue or len(results) < len(ids):
        # two arrivals per step
        for _ in range(2):
            if queue:
                kind, w = queue.pop(0)
                if kind == "r":
                    i = srv.submit(w.deg_num, _box(zr, w.num, w.den), sched=w.schedule, deg_den=w.deg_den)
                else:
                    i = srv.submit(w.deg, _box(zr, w.hidden), sched=w.schedule)
                ids[i] = (kind, w)
                if bad is None and step == 1:
                    bad = srv.submit(ps[0].deg, zr.HostBlackBox(broken, ps[0].hidden.nvars), sched=ps[0].schedule)
                    ids[bad] = ("bad", None)
        srv.step()
        step += 1
        for i in ids:
            if i not in results:
                r = srv.poll(i)
                if r is not None:
                    results[i] = r
        assert step < 200
    for i, (kind, w) in ids.items():
        status, num, den = results[i]
        if kind == "bad":
            assert status == zr.ZR_EBLACKBOX
            continue
        ast, an, ad = _alone(zr, w)
        assert status == ast == zr.ZR_OK
        if kind == "r":
            assert _same(num, an) and _same(den, ad)
        else:
            assert _same(num, an)
            assert np.array_equal(num[0], w.hidden.exps) and np.array_equal(num[1], w.hidden.coefs)
            assert den is None
    srv.close()


def _lying_at_probes(base, sched):
    """A black box that is right everywhere except at the schedule's probe
    points (a single point whose last coordinate is a probe's), where it adds 1."""
    last = {int(v) for v in sched.probes[:, -1]}

    def f(k, i_first, ni, y, anchor, xk):
        v = np.asarray(base(k, i_first, ni, y, anchor, xk), dtype=np.uint64).copy()
        if ni == 1 and len(xk) == 1 and int(xk[0]) in last:
            v[0] = np.uint64((int(v[0]) + 1) % sched.p)
        return v
    return f


def test_served_finish_failures(zr):
    """Requests that fail while their results are finished (a probe that
    disagrees, a denominator without a constant term) fail alone, with the
    status the one-request path gives; the others in the same steps equal
    their runs alone."""
    ws = _rational_mix(6, 3)
    p = ws[0].p
    pw = synth.poly_workload("probe", 3, 6, 60, 77, 1777, p=p)
    num = synth.SparsePoly(p, 2, np.array([[0, 0], [1, 1]], dtype=np.uint16), np.array([4, 9], dtype=np.uint64))
    den = synth.SparsePoly(p, 2, np.array([[1, 0], [0, 2]], dtype=np.uint16), np.array([1, 3], dtype=np.uint64))
    dn, dd = [2, 2], [2, 2]
    sn = synth.make_schedule(p, 2, [synth.thiele_nodes_needed(a, b) for a, b in zip(dn, dd)], 4, 1)
    srv = zr.Server(p, hbm_budget=1 << 30, max_active=16)
    ids = {}
    for w in ws:
        ids[srv.submit(w.deg_num, _box(zr, w.num, w.den), sched=w.schedule, deg_den=w.deg_den)] = ("ok", w)
    ids[srv.submit(dn, _box(zr, num.sorted(), den.sorted()), sched=sn, deg_den=dd)] = ("norm", None)
    rw = ws[1]
    lie_r = zr.HostBlackBox(_lying_at_probes(synth.BlackBox(rw.num, rw.den).eval, rw.schedule), rw.num.nvars)
    ids[srv.submit(rw.deg_num, lie_r, sched=rw.schedule, deg_den=rw.deg_den)] = ("probe", None)
    lie_p = zr.HostBlackBox(_lying_at_probes(synth.BlackBox(pw.hidden).eval, pw.schedule), pw.hidden.nvars)
    ids[srv.submit(pw.deg, lie_p, sched=pw.schedule)] = ("probe", None)
    # results collected through the finished-ids query: every id exactly once
    res = {}
    steps = 0
    while len(res) < len(ids):
        srv.step()
        steps += 1
        assert steps < 100
        for rid in srv.finished():
            assert rid in ids and rid not in res
            res[rid] = srv.poll(rid)
            assert res[rid] is not None
    assert srv.finished() == []
    st = srv.stats()
    _note(f"stats {st}")
    assert st["completed"] == len(ids) and st["failed"] == 3
    # the one-request paths give the same statuses
    with pytest.raises(zr.ZippelError) as ei:
        zr.balanced_reconstruct(p, dn, dd, _box(zr, num.sorted(), den.sorted()), sched=sn)
    assert ei.value.code == zr.ZR_ENORM
    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct(p, pw.deg, zr.HostBlackBox(_lying_at_probes(synth.BlackBox(pw.hidden).eval, pw.schedule),
                                                  pw.hidden.nvars), sched=pw.schedule)
    assert ei.value.code == zr.ZR_EPROBE
    for i, (kind, w) in ids.items():
        status, n_, d_ = res[i]
        if kind == "norm":
            assert status == zr.ZR_ENORM
        elif kind == "probe":
            assert status == zr.ZR_EPROBE
        else:
            ast, an, ad = _alone(zr, w)
            assert status == ast == zr.ZR_OK
            assert _same(n_, an) and _same(d_, ad)
    srv.close()


def test_served_admission_by_footprint(zr):
    """A budget below every request's footprint: requests run one at a time
    (a request that does not fit still runs when nothing else is active), and
    every one completes with the result it has alone."""
    ws = _rational_mix(6, 3)
    srv = zr.Server(ws[0].p, hbm_budget=1, max_active=64)  # every request exceeds it: one at a time
    ids = [srv.submit(w.deg_num, _box(zr, w.num, w.den), sched=w.schedule, deg_den=w.deg_den) for w in ws]
    res = _run(srv, ids)
    st = srv.stats()
    assert st["peak_active"] == 1 and st["completed"] == len(ws)
    for w, i in zip(ws, ids):
        status, num, den = res[i]
        ast, an, ad = _alone(zr, w)
        assert status == ast == zr.ZR_OK and _same(num, an) and _same(den, ad)
    srv.close()


def test_served_finished_skips_polled(zr):
    """zr_server_finished lists each finished request once and leaves out the
    ones already collected with zr_server_poll."""
    p = synth.make_prime()
    ps = [synth.poly_workload(f"f{i}", 3, 6, 30 + 10 * i, 500 + i, 1500 + i, p=p) for i in range(5)]
    srv = zr.Server(p, hbm_budget=1 << 30, max_active=8)
    ids = [srv.submit(w.deg, _box(zr, w.hidden), sched=w.schedule) for w in ps]
    while srv.stats()["completed"] < len(ids):
        srv.step()
    early = {ids[1]: srv.poll(ids[1]), ids[3]: srv.poll(ids[3])}
    rest = srv.finished()
    assert sorted(rest) == sorted(set(ids) - set(early))
    assert srv.finished() == []
    for i, w in zip(ids, ps):
        r = early[i] if i in early else srv.poll(i)
        assert r[0] == zr.ZR_OK
        assert np.array_equal(r[1][0], w.hidden.exps) and np.array_equal(r[1][1], w.hidden.coefs)
    srv.close()
