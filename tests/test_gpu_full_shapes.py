"""Parity at the full shapes of the batched and served workloads.

Batched: a stratified subset of the 4096-instance workload (n uniform in 3..8,
per-variable degree 30, t log-uniform in 10..2*10^4, one shared prime), drawn
from every size band, the largest instance of the whole workload included,
reconstructed together in one zippel_reconstruct_batch call; every instance
equals the oracle's reconstruction and the hidden polynomial.

Served: requests shaped like the served rational workload (n = 5, total
degree 20, t_N and t_D log-uniform, Q(0) = 1) submitted two per step while
earlier ones are on the device; every result equals the oracle's balanced
reconstruction and the hidden P, Q."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

BANDS = [(1, 64), (64, 256), (256, 1024), (1024, 4096), (4096, 1 << 30)]


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


def stratified_batch_indices(per_band=8, top_band=4):
    """Indices into the 4096-instance workload: the first per_band instances
    of each of the four lower size bands in index order; in the top band
    (t >= 4096) the largest instance of the workload and the smallest ones."""
    shapes = synth.batch_shapes(4096)
    out = []
    for lo, hi in BANDS:
        idx = [i for i, (n, t) in enumerate(shapes) if lo <= t < hi]
        if hi > 1 << 20:
            big = max(idx, key=lambda i: shapes[i][1])
            pick = [big] + sorted((i for i in idx if i != big), key=lambda i: shapes[i][1])[:top_band - 1]
        else:
            pick = idx[:per_band]
        out.extend(pick)
    return shapes, out


def test_batched_full_shape_subset_matches_oracle(zr):
    shapes, idx = stratified_batch_indices()
    ws = [synth.batch_instance(i, *shapes[i]) for i in idx]
    _note("instances (n, t): " + ", ".join(f"{i}:{shapes[i]}" for i in idx))
    assert max(w.hidden.nvars for w in ws) == 8 and max(w.hidden.nterms for w in ws) > 19_000
    items = [{"deg": w.deg, "box": zr.HostBlackBox(synth.BlackBox(w.hidden).eval, w.hidden.nvars),
              "sched": w.schedule} for w in ws]
    res = zr.reconstruct_batch(ws[0].p, items)
    _note("batched call done; oracle per instance")
    for i, w, r in zip(idx, ws, res):
        assert not isinstance(r, Exception), (i, r)
        e, c = r
        oe, oc = oracle.zippel(w.p, w.deg, w.schedule, synth.BlackBox(w.hidden))
        assert np.array_equal(e, oe) and np.array_equal(c, oc), i
        assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs), i


def served_full_shape_requests(count=12, seed=5005, tmax=2000):
    """Rational requests of the served workload's shape: n = 5, total degree
    20, t_N and t_D log-uniform in [10, tmax]."""
    g = synth.SplitMix64(seed)
    out = []
    for i in range(count):
        tn = synth.loguniform_int(g, 10, tmax)
        td = synth.loguniform_int(g, 10, tmax)
        out.append(synth.rational_workload(5, 20, tn, td, 60_000 + i))
    return out


def test_served_full_shape_mix_matches_oracle(zr):
    ws = served_full_shape_requests()
    _note("requests (t_N, t_D): " + ", ".join(f"({w.num.nterms}, {w.den.nterms})" for w in ws))
    srv = zr.Server(ws[0].p, hbm_budget=16 << 30, max_active=256)
    queue = list(range(len(ws)))
    ids, results, steps = {}, {}, 0
    while queue or len(results) < len(ids):
        for _ in range(2):  # two arrivals per step, while earlier requests are mid-way
            if queue:
                k = queue.pop(0)
                w = ws[k]
                rid = srv.submit(w.deg_num, zr.HostBlackBox(synth.BlackBox(w.num, w.den).eval, 5),
                                 sched=w.schedule, deg_den=w.deg_den)
                ids[rid] = k
        srv.step()
        steps += 1
        for rid in ids:
            if rid not in results:
                r = srv.poll(rid)
                if r is not None:
                    results[rid] = r
        assert steps < 400
    st = srv.stats()
    srv.close()
    _note(f"served in {steps} steps, stats {st}")
    assert st["peak_active"] > 1
    for rid, k in ids.items():
        w = ws[k]
        status, num, den = results[rid]
        assert status == zr.ZR_OK, (k, status)
        (on, ocn), (od, ocd) = oracle.balanced_zippel(w.p, w.deg_num, w.deg_den, w.schedule,
                                                      synth.BlackBox(w.num, w.den))
        assert np.array_equal(num[0], on) and np.array_equal(num[1], ocn), k
        assert np.array_equal(den[0], od) and np.array_equal(den[1], ocd), k
        assert np.array_equal(num[0], w.num.exps) and np.array_equal(num[1], w.num.coefs), k
        assert np.array_equal(den[0], w.den.exps) and np.array_equal(den[1], w.den.coefs), k
