"""Batched forms on the GPU: zippel_reconstruct_batch against the hidden
polynomials, the oracle and the one-at-a-time path; every band choice of the
batched solve gives the same exact result."""
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


def _box(zr, hidden):
    return zr.HostBlackBox(synth.BlackBox(hidden).eval, hidden.nvars)


def _mixed(count, seed):
    """Instances of uneven sizes: n in 1..5, per-variable degree 0..12, t log-uniform."""
    g = synth.SplitMix64(seed)
    out = []
    for i in range(count):
        n = 1 + int(g.uniform(0, 5))
        d = int(g.uniform(0, 13))
        space = (d + 1) ** n
        t = int(round(np.exp(g.uniform(0, 1000) / 1000.0 * np.log(min(space, 600)))))
        t = max(1, min(t, space))
        out.append(synth.poly_workload(f"b{i}", n, d, t, 5000 + seed * 100 + i, 7000 + seed * 100 + i, nprobes=2))
    return out


def _items(zr, ws):
    return [{"deg": w.deg, "box": _box(zr, w.hidden), "sched": w.schedule} for w in ws]


def test_batch_matches_hidden_and_plain(zr):
    ws = _mixed(40, 1)
    _note(f"batch of {len(ws)}: t = {[w.hidden.nterms for w in ws]}")
    res = zr.reconstruct_batch(ws[0].p, _items(zr, ws))
    for w, r in zip(ws, res):
        assert not isinstance(r, Exception), r
        e, c = r
        assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)
    for w in ws[:6]:
        e, c = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule)
        oe, oc = oracle.zippel(w.p, w.deg, w.schedule, synth.BlackBox(w.hidden))
        assert np.array_equal(e, oe) and np.array_equal(c, oc)


def test_batch_band_choices_agree(zr):
    ws = _mixed(24, 2)
    base = None
    for packed in (0, 1):
        for min_chunk in (16, 128, 1 << 30):
            zr.tuning_set([(packed, min_chunk)] + [(0, min_chunk)] * 4)
            _note(f"tuning packed={packed} min_chunk={min_chunk}")
            res = zr.reconstruct_batch(ws[0].p, _items(zr, ws))
            flat = [(r[0].tobytes(), r[1].tobytes()) for r in res]
            if base is None:
                base = flat
            assert flat == base
    for w, r in zip(ws, res):
        assert np.array_equal(r[0], w.hidden.exps) and np.array_equal(r[1], w.hidden.coefs)


def test_batch_uneven_stages_and_failures(zr):
    """Instances stopping at different stages, a failing black box and a
    singular schedule in the same batch: each gets its own status, the others
    are unaffected."""
    ws = _mixed(6, 3)
    items = _items(zr, ws)
    # partial reconstruction
    w0 = synth.poly_workload("s", 4, 6, 150, 41, 1041, nprobes=0)
    items.append({"deg": w0.deg, "box": _box(zr, w0.hidden), "sched": w0.schedule, "last_stage": 2})

    def broken(*a):
        raise RuntimeError("down")

    items.append({"deg": ws[0].deg, "box": zr.HostBlackBox(broken, ws[0].hidden.nvars), "sched": ws[0].schedule})
    p = ws[0].p
    exps = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 1]], dtype=np.uint16)
    hidden = synth.SparsePoly(p, 3, exps, np.array([3, 5, 7], dtype=np.uint64)).sorted()
    sched = synth.make_schedule(p, 3, [2, 2, 2], 1, 0)
    sched.y[1] = sched.y[0]
    items.append({"deg": [2, 2, 2], "box": _box(zr, hidden), "sched": sched})
    res = zr.reconstruct_batch(p, items)
    for w, r in zip(ws, res[:6]):
        assert np.array_equal(r[0], w.hidden.exps) and np.array_equal(r[1], w.hidden.coefs)
    oe, oc = oracle.zippel(w0.p, w0.deg, w0.schedule, synth.BlackBox(w0.hidden), last_stage=2)
    assert np.array_equal(res[6][0], oe) and np.array_equal(res[6][1], oc)
    assert isinstance(res[7], zr.ZippelError) and res[7].code == zr.ZR_EBLACKBOX
    assert isinstance(res[8], zr.ZippelError) and res[8].code == zr.ZR_ESINGULAR


def test_batch_recorded_replay_and_autotune(zr):
    ws = _mixed(16, 4)
    recs = [zr.Recorder(_box(zr, w.hidden)) for w in ws]
    items = [{"deg": w.deg, "box": r, "sched": w.schedule} for w, r in zip(ws, recs)]
    first = zr.reconstruct_batch(ws[0].p, items)
    for r in recs:
        r.replay(True)
    choices = zr.autotune(ws[0].p)
    _note(f"autotune: {choices}")
    assert zr.tuning_get()[0]
    assert len(choices) == zr.NBANDS and all(c[1] > 0 for c in choices)
    again = zr.reconstruct_batch(ws[0].p, items)
    for w, a, b in zip(ws, first, again):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.array_equal(a[0], w.hidden.exps) and np.array_equal(a[1], w.hidden.coefs)


def test_batch_graphs_identical(zr):
    """Graph mode (each stage's solve captured and launched as one hipGraph)
    gives the same results as direct launches, on repeated runs."""
    ws = _mixed(20, 5)
    zr.batch_graphs(False)
    base = zr.reconstruct_batch(ws[0].p, _items(zr, ws))
    try:
        zr.batch_graphs(True)
        for rep in range(3):
            again = zr.reconstruct_batch(ws[0].p, _items(zr, ws))
            for w, a, b in zip(ws, base, again):
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
                assert np.array_equal(b[0], w.hidden.exps) and np.array_equal(b[1], w.hidden.coefs)
    finally:
        zr.batch_graphs(False)


def test_long_unsplit_chain_is_exact(zr):
    """One system of 20000 rows solved without chunking (every row's sum runs
    over all 20000 steps) and right-hand sides just below p, so that the
    accumulator columns would wrap without their periodic reduction; rows
    sampled against the oracle."""
    import random
    p = synth.make_prime()
    t, R = 20_000, 16
    g = synth.SplitMix64(2024)
    m = g.uniform_block(1, p, t)
    assert len(set(int(x) for x in m)) == t
    rhs = (np.uint64(p - 1) - g.uniform_block(0, 1 << 20, t * R)).reshape(R, t)
    saved = zr.tuning_get()[1]
    try:
        zr.tuning_set([(0, 1 << 30)] * zr.NBANDS)  # never split a system
        got, status = zr.vandermonde_solve_batch(p, [(m, rhs)])
    finally:
        zr.tuning_set(saved)
    assert status[0] == 0
    rows = sorted(random.Random(5).sample(range(t), 24) + [0, t - 1])
    want = oracle.vandermonde_solve_rows(p, m, rhs, rows)
    assert np.array_equal(got[0][:, rows], want)
