#!/usr/bin/env python
"""Benchmark of the Zippel reconstruction's hot path on one MI355X.

Headline workload: the final stage of a large plain polynomial Zippel
reconstruction, the quantity the paper times (§3.1, Table 3: the
reconstruction over the last variable, 125k-4.8m skeleton terms).  Hidden
sparse polynomial in n = 8 variables, per-variable degree <= 40, t = 5*10^5
terms with uniform distinct exponents, coefficients uniform mod a seeded
63-bit prime (hidden-polynomial seed 3, schedule seed 1003).  One step =
stage 8 from the stage-7 result f(x_1..x_7, c_8): one transposed Vandermonde
system of 5*10^5 unknowns with 40 right-hand sides (master polynomial,
synthetic-division dot products, inverse and scaling), the Newton lift of
every term over 41 nodes, the expansion into the final skeleton, and the two
probe checks.  The black box's samples are computed once on the device,
recorded and replayed (a device-to-device copy per call) inside the timed
region.

Further legs, reported under their own keys: the n = 6, t = 10^4 whole
reconstruction; 4096 batched reconstructions against one at a time; served
rational requests with Poisson arrivals.

Prints one JSON line.  ``--microbench`` instead prints the throughput probes
used for the roofline (see include/zippel_microbench.h).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  The derived ceiling is one
# 32x32-bit multiply per lane per clock; a 64x64-bit product needs four.  The
# v_mad_u64_u32 throughput probe (include/zippel_microbench.h) measures what the
# chip sustains for that multiply (about three quarters of the derived figure);
# it runs inside every bench and both fractions are reported.
CU, SIMD, LANES, CLOCK_GHZ = 256, 4, 16, 2.4
MUL32_PEAK_TOPS = CU * SIMD * LANES * CLOCK_GHZ * 1e9 / 1e12
MUL32_PER_MULMOD = 4

# HBM bytes per launch of the dominant solve kernel on the headline workload,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by the copy-probe calibration
# (profiles/k_vs_dots_pc_n8_d40_t5e5_hbm_counters.md).  Valid only for the
# kernel sources the counters were taken on (None: not measured for them).
DOTS_TRAFFIC = {"sources_sha16": "e1ba96d12974ac06", "bytes_per_launch": 7713177498}

HEADLINE_STAGE = 8  # the last variable of the n = 8 workload


def _system_sizes(w):
    """Sizes t of the Vandermonde systems of a reconstruction: the number of
    distinct exponent prefixes of the hidden polynomial before each added
    variable (stages 2..n)."""
    e = np.asarray(w.hidden.exps)
    return [int(len(np.unique(e[:, :k], axis=0))) for k in range(1, e.shape[1])]


def _dots_work(c) -> int:
    """Algorithmic modular products of the solves' dot-product passes: the R t^2
    products and the t(t-1) chain steps per system (the denominators m_l M'(m_l)
    come from the chain pass, not from this one)."""
    return c["dot_products"] + c["chain_steps"]


def _dots_sources_sha16() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("field.hpp", "kernels_dev.hpp", "kernels.hip"):
        with open(os.path.join(ROOT, "paper_2505_24256_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


class CachingBox:
    """Host black box (synth) whose answers are kept for re-use."""

    def __init__(self, inner):
        self.inner = inner
        self.cache = {}

    def eval(self, k, i_first, ni, y, anchor, xk):
        key = (int(k), int(i_first), int(ni), tuple(int(v) for v in y[:max(int(k) - 1, 0)]),
               tuple(int(v) for v in anchor[int(k):]), tuple(int(v) for v in xk))
        v = self.cache.get(key)
        if v is None:
            v = self.inner.eval(k, i_first, ni, y, anchor, xk)
            self.cache[key] = v
        return v


def microbench(zr):
    out = {}
    for kind in ("add_u32", "mul_lo_u32", "mul_hi_u32", "mad_u64_u32", "mac192", "shoup"):
        ms, ops = zr.microbench(kind, blocks=2048, iters=4096)
        out[kind] = {"ms": round(ms, 4), "Gops_per_s": round(ops / ms / 1e6, 1)}
    ms, nbytes = zr.microbench("copy", blocks=8192, nbytes=2 << 30)
    out["copy"] = {"ms": round(ms, 4), "GB_per_s": round(nbytes / ms / 1e6, 1), "bytes": nbytes}
    for kind in ("lds_read", "lds_bcast"):  # bytes delivered to lanes
        ms, nbytes = zr.microbench(kind, blocks=2048, iters=4096)
        out[kind] = {"ms": round(ms, 4), "GB_per_s": round(nbytes / ms / 1e6, 1)}
    return out


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched_vs_plain(zr, synth, args, stream):
    """Batched workload: independent instances sharing p, n uniform in 3..8,
    t log-uniform in 10..2*10^4, per-variable degree <= 30.  Samples come from
    the device black box, recorded once per instance and replayed; the same
    recordings serve the batched call and the one-at-a-time plain calls."""
    import torch
    t0 = time.perf_counter()
    ws = synth.batch_workload(args.batch_instances)
    t_gen = time.perf_counter() - t0
    _progress(f"batch workload generated ({len(ws)} instances, {t_gen:.1f} s); recording")
    recs = [zr.Recorder(synth.DeviceBlackBox(w.hidden, nthreads=args.cpu_threads)) for w in ws]
    items = [{"deg": w.deg, "box": r, "sched": w.schedule} for w, r in zip(ws, recs)]
    p = ws[0].p
    t0 = time.perf_counter()
    res = zr.reconstruct_batch(p, items, stream=stream)
    t_rec = time.perf_counter() - t0
    exact = all(not isinstance(r, Exception) and np.array_equal(r[0], w.hidden.exps) and
                np.array_equal(r[1], w.hidden.coefs) for w, r in zip(ws, res))
    for r in recs:
        r.replay(True)
    _progress(f"recorded in {t_rec:.1f} s; autotune")
    tuned = zr.autotune(p, stream=stream)
    _progress(f"band choices {tuned}; batched runs")
    # batched
    times = []
    cnt = None
    for _ in range(max(1, args.batch_steps)):
        for r in recs:
            zr.lib().zr_recorder_rewind(r.handle)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        res = zr.reconstruct_batch(p, items, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        cnt = zr.last_counters()
        exact = exact and all(not isinstance(r, Exception) and np.array_equal(r[0], w.hidden.exps) and
                              np.array_equal(r[1], w.hidden.coefs) for w, r in zip(ws, res))
    tb = statistics.median(times)
    # the same with each stage's solve captured into a hipGraph
    zr.batch_graphs(True)
    try:
        for r in recs:
            zr.lib().zr_recorder_rewind(r.handle)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        res = zr.reconstruct_batch(p, items, stream=stream)
        torch.cuda.synchronize()
        tg = time.perf_counter() - ts
    finally:
        zr.batch_graphs(False)
    exact = exact and all(not isinstance(r, Exception) and np.array_equal(r[0], w.hidden.exps) and
                          np.array_equal(r[1], w.hidden.coefs) for w, r in zip(ws, res))
    # one more batched run with every named launch timed: where the batch's time goes
    for r in recs:
        zr.lib().zr_recorder_rewind(r.handle)
    zr.timing(True)
    zr.timing_reset()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    zr.reconstruct_batch(p, items, stream=stream)
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - ts
    zr.timing(False)
    breakdown = {}
    for name in ("batch_master", "batch_pack", "batch_chain", "batch_dots", "batch_finish", "batch_newton",
                 "batch_expand", "master", "vs_pack", "vs_chain", "vs_scan", "vs_dots", "vs_finish"):
        k, ms = zr.timing_get(name)
        if k:
            breakdown[name] = {"launches": k, "ms_total": round(ms, 2)}
    # the persistent dot-product passes of the timed run against their work
    # (dot products and chains of q of every system, 4 32-bit multiplies each)
    solve_kernel = None
    if "batch_dots" in breakdown and breakdown["batch_dots"]["ms_total"] > 0:
        tops = 4.0 * _dots_work(cnt) / (breakdown["batch_dots"]["ms_total"] * 1e-3) / 1e12
        solve_kernel = {"kernel": "k_b_dots_pc", "achieved_TOPs": round(tops, 3),
                        "frac_of_derived_peak": round(tops / MUL32_PEAK_TOPS, 4)}
    _progress(f"batched {times}, with graphs {tg:.3f}; plain one at a time")
    # plain, one at a time, same recordings
    for r in recs:
        zr.lib().zr_recorder_rewind(r.handle)
    lat = []
    mul_plain = 0
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for w, r in zip(ws, recs):
        t1 = time.perf_counter()
        e, c = zr.reconstruct(p, w.deg, r, sched=w.schedule, stream=stream)
        lat.append(time.perf_counter() - t1)
        mul_plain += zr.last_counters()["mulmods"]
        exact = exact and bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    torch.cuda.synchronize()
    tp = time.perf_counter() - ts
    n = len(ws)
    return {
        "workload": f"{n} independent polynomial reconstructions, n uniform in 3..8, t log-uniform in 10..2*10^4, "
                    "per-variable degree<=30, shared 63-bit prime",
        "instances": n, "terms_total": int(sum(w.hidden.nterms for w in ws)),
        "batched": {"reconstructions_per_s": round(n / tb, 2), "mulmod_per_s": round(cnt["mulmods"] / tb, 1),
                    "seconds": round(tb, 3), "runs": len(times), "seconds_with_graphs": round(tg, 3)},
        "plain": {"reconstructions_per_s": round(n / tp, 2), "mulmod_per_s": round(mul_plain / tp, 1),
                  "seconds": round(tp, 3), "latency_ms": {"p50": round(statistics.median(lat) * 1e3, 3),
                                                         "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)}},
        "speedup": round(tp / tb, 3), "mulmods": cnt["mulmods"], "bit_exact": bool(exact),
        "band_choices": tuned, "setup_seconds": {"generate": round(t_gen, 1), "record": round(t_rec, 1)},
        "timed_run": {"seconds": round(t_timed, 3), "per_kernel": breakdown},
        "solve_kernel": solve_kernel,
    }


def served(zr, synth, args, stream):
    """Served balanced Zippel: rational requests P/Q, n = 5, total degree <= 20,
    t_N and t_D log-uniform in 10..5*10^3, Q(0) = 1.  Each request's samples are
    recorded once (its run alone, device black box), then replayed for every
    timed pass: one at a time; all submitted at once (saturated throughput);
    and Poisson arrivals at 0.7 x the saturated rate and at a fixed rate,
    admitted by device footprint and advanced in continuous batches (latency
    p50/p99)."""
    import math
    import torch
    g = synth.SplitMix64(5005)
    ws = []
    for i in range(args.serve_requests):
        def logu():
            u = g.next() / 2.0 ** 64
            return int(round(math.exp(math.log(10) + u * (math.log(5000) - math.log(10)))))
        ws.append(synth.rational_workload(5, 20, logu(), logu(), 50_000 + i))
    recs = [zr.Recorder(synth.DeviceBlackBox(w.num, w.den, nthreads=args.cpu_threads)) for w in ws]
    alone = []
    t0 = time.perf_counter()
    for w, r in zip(ws, recs):
        alone.append(zr.balanced_reconstruct(w.p, w.deg_num, w.deg_den, r, sched=w.schedule, stream=stream))
        r.replay(True)
    _progress(f"served: {len(ws)} requests recorded in {time.perf_counter() - t0:.1f} s")

    def rewind():
        for r in recs:
            zr.lib().zr_recorder_rewind(r.handle)

    # one at a time
    rewind()
    lat1 = []
    for w, r in zip(ws, recs):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        zr.balanced_reconstruct(w.p, w.deg_num, w.deg_den, r, sched=w.schedule, stream=stream)
        lat1.append(time.perf_counter() - t1)

    def serve(arrivals):
        rewind()
        srv = zr.Server(ws[0].p, hbm_budget=args.serve_budget_gib << 30, max_active=args.serve_slots, stream=stream)
        ids, sub, fin, res = {}, 0, {}, {}
        t0 = time.perf_counter()
        while len(fin) < len(ws):
            now = time.perf_counter() - t0
            while sub < len(ws) and arrivals[sub] <= now:
                w = ws[sub]
                # no size hint: the server sizes each request from the skeletons it has reached
                rid = srv.submit(w.deg_num, recs[sub], sched=w.schedule, deg_den=w.deg_den)
                ids[rid] = sub
                sub += 1
            st = srv.stats()
            if st["active"] == 0 and st["pending"] == 0:
                if sub < len(ws):
                    time.sleep(max(0.0, arrivals[sub] - (time.perf_counter() - t0)))
                continue
            srv.step()
            tn = time.perf_counter() - t0
            for rid in srv.finished():
                i = ids[rid]
                fin[i] = tn
                res[i] = srv.poll(rid)
        stats = srv.stats()
        srv.close()
        lat = [fin[i] - arrivals[i] for i in range(len(ws))]
        span = max(fin.values()) - min(arrivals)
        same = all(res[i][0] == zr.ZR_OK and np.array_equal(res[i][1][0], alone[i][0][0]) and
                   np.array_equal(res[i][1][1], alone[i][0][1]) and np.array_equal(res[i][2][0], alone[i][1][0]) and
                   np.array_equal(res[i][2][1], alone[i][1][1]) for i in range(len(ws)))
        return span, lat, stats, same

    span_sat, _, st_sat, same_sat = serve([0.0] * len(ws))
    sat = len(ws) / span_sat
    rate = 0.7 * sat
    arr, t = [], 0.0
    for _ in ws:
        t += -math.log(1.0 - g.next() / 2.0 ** 64) / rate
        arr.append(t)
    span, lat, st, same = serve(arr)
    # Poisson arrivals at a fixed rate as well, so that latencies compare
    # across builds whose saturated rates differ
    arr_f, t = [], 0.0
    for _ in ws:
        t += -math.log(1.0 - g.next() / 2.0 ** 64) / args.serve_fixed_rate
        arr_f.append(t)
    span_f, lat_f, st_f, same_f = serve(arr_f)
    _progress(f"served: saturated {sat:.1f} req/s, Poisson at {rate:.1f} and {args.serve_fixed_rate:.0f} req/s")
    return {
        "workload": f"{len(ws)} rational requests P/Q, n=5, total degree<=20, t_N and t_D log-uniform in 10..5*10^3, "
                    "Q(0)=1; Poisson arrivals at 0.7 x the saturated throughput",
        "saturated": {"requests_per_s": round(sat, 2), "steps": st_sat["steps"], "peak_active": st_sat["peak_active"]},
        "poisson": {"rate_per_s": round(rate, 2), "requests_per_s": round(len(ws) / span, 2),
                    "latency_ms": {"p50": round(statistics.median(lat) * 1e3, 2),
                                   "p99": round(float(np.percentile(lat, 99)) * 1e3, 2)},
                    "steps": st["steps"], "peak_active": st["peak_active"],
                    "peak_footprint_bytes": st["peak_footprint"]},
        "poisson_fixed_rate": {"rate_per_s": args.serve_fixed_rate, "requests_per_s": round(len(ws) / span_f, 2),
                               "latency_ms": {"p50": round(statistics.median(lat_f) * 1e3, 2),
                                              "p99": round(float(np.percentile(lat_f, 99)) * 1e3, 2)},
                               "steps": st_f["steps"], "peak_active": st_f["peak_active"]},
        "one_at_a_time": {"requests_per_s": round(len(ws) / sum(lat1), 2), "latency_ms": {
            "p50": round(statistics.median(lat1) * 1e3, 2), "p99": round(float(np.percentile(lat1, 99)) * 1e3, 2)}},
        "identical_to_alone": bool(same and same_sat and same_f),
        "slots": args.serve_slots, "budget_gib": args.serve_budget_gib,
    }


def headline(zr, synth, args, stream):
    """The final stage of the n = 8, t = 5*10^5 reconstruction (see the module
    docstring): recording run, warm-up steps with every named launch timed,
    then the timed steps with HIP events around the dot-product launches."""
    import torch
    t0 = time.perf_counter()
    w = synth.config_workload(3)
    k = HEADLINE_STAGE
    start = synth.stage_result(w.hidden, w.schedule.anchor, k - 1)
    _progress(f"headline workload generated in {time.perf_counter() - t0:.1f} s: stage {k} from a "
              f"{len(start[1])}-term skeleton")
    rec = zr.Recorder(synth.DeviceBlackBox(w.hidden, nthreads=args.cpu_threads))

    def step():
        zr.lib().zr_recorder_rewind(rec.handle)
        return zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream, first_stage=k, start=start)

    # recording run (device black box): also checks the result
    t0 = time.perf_counter()
    e, c = zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream, first_stage=k, start=start)
    exact = bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    _progress(f"recorded in {time.perf_counter() - t0:.1f} s; bit exact {exact}")
    if not exact:
        print("bench.py: the final stage does not reproduce the hidden polynomial", file=sys.stderr)
        sys.exit(3)
    rec.replay(True)
    zr.timing(True)
    zr.timing_reset()
    for i in range(args.warmup):
        step()
        _progress(f"warm-up step {i + 1}/{args.warmup}")
    cnt = zr.last_counters()
    torch.cuda.synchronize()
    zr.timing(False)
    kernels = {}
    for name in ("mono", "master", "vs_pack", "vs_chain", "vs_scan", "vs_dots", "vs_finish", "newton", "scan",
                 "expand"):
        n, ms = zr.timing_get(name)
        if n:
            kernels[name] = {"launches": n, "ms_total": round(ms, 3)}
    zr.timing(True, dots_only=True)
    zr.timing_reset()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        e, c = step()
        lat.append(time.perf_counter() - ts)
        _progress(f"step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    zr.timing(False)
    exact = exact and bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    n_dots, ms_dots = zr.timing_get("vs_dots")
    return {"w": w, "start": start, "cnt": cnt, "elapsed": elapsed, "lat": lat, "exact": exact,
            "n_dots": n_dots, "ms_dots": ms_dots, "kernels": kernels}


def config2_leg(zr, synth, args, stream):
    """Whole reconstruction of the n = 6, per-variable degree 30, t = 10^4
    polynomial (six stages, systems up to 10^4 unknowns with 30 right-hand
    sides), samples recorded once and replayed."""
    import torch
    w = synth.config_workload(2)
    rec = zr.Recorder(synth.DeviceBlackBox(w.hidden, nthreads=args.cpu_threads))
    e, c = zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream)
    exact = bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    rec.replay(True)
    for _ in range(2):
        zr.lib().zr_recorder_rewind(rec.handle)
        zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream)
    cnt = zr.last_counters()
    zr.timing(True, dots_only=True)
    zr.timing_reset()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.config2_steps):
        ts = time.perf_counter()
        zr.lib().zr_recorder_rewind(rec.handle)
        e, c = zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    zr.timing(False)
    exact = exact and bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    n_dots, ms_dots = zr.timing_get("vs_dots")
    steps = args.config2_steps
    alu = _dots_work(cnt) * steps * MUL32_PER_MULMOD / (ms_dots / 1e3) / 1e12 if ms_dots else 0.0
    return {"workload": "plain polynomial Zippel, whole reconstruction, n=6, per-variable degree<=30, t=10^4",
            "system_sizes": _system_sizes(w), "right_hand_sides": int(w.deg[0]),
            "mulmod_per_s": round(cnt["mulmods"] * steps / el, 1), "ms_per_reconstruction": round(el / steps * 1e3, 3),
            "reconstructions_per_s": round(steps / el, 3),
            "latency_ms": {"p50": round(statistics.median(lat) * 1e3, 3),
                           "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
            "solve_kernel": {"kernel": "k_vs_dots_pc", "achieved_TOPs": round(alu, 3),
                             "frac_of_derived_peak": round(alu / MUL32_PEAK_TOPS, 4),
                             "avg_launch_ms": round(ms_dots / n_dots, 4) if n_dots else None},
            "mulmods_per_reconstruction": cnt["mulmods"], "steps": steps, "bit_exact": exact}


def _replayed(zr, rec, run, steps):
    """Median wall time of `steps` replays of a recorded call sequence."""
    import torch
    times = []
    out = None
    for _ in range(max(1, steps)):
        zr.lib().zr_recorder_rewind(rec.handle)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        out = run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
    return statistics.median(times), out


def multi_expression_leg(zr, synth, args, stream):
    """Eight expressions sampled at the same points, each of few nodes per
    variable: n = 6, about 10^4 terms each, each keeping a random 99% of a
    common term set plus 0.5% terms of its own; degree bounds 8 in x_1..x_5
    and 8, 8, 7, 7, 6, 6, 5, 5 in x_6 (terms beyond an expression's bound left
    out).  One reconstruction of all eight over the union skeleton (one solve
    per stage with about 64 right-hand sides) against eight separate
    reconstructions (8 or fewer right-hand sides each), samples recorded once
    and replayed."""
    n, t = 6, args.multi_terms
    last = [8, 8, 7, 7, 6, 6, 5, 5]
    p = synth.make_prime()
    base = synth.random_poly(p, n, 8, t, 4001)
    g = synth.SplitMix64(4002)
    polys = []
    for e, d in enumerate(last):
        bound = [8] * (n - 1) + [d]
        ok = np.flatnonzero(base.exps[:, n - 1] <= d)
        u = g.uniform_block(0, 1000, len(ok))
        own = synth.random_poly(p, n, bound, max(1, t // 200), 4010 + e)
        ex = np.concatenate([base.exps[ok[u < 990]], own.exps])
        _, first = np.unique(ex, axis=0, return_index=True)
        ex = ex[np.sort(first)]
        polys.append(synth.SparsePoly(p, n, ex, g.uniform_block(1, p, len(ex))).sorted())
    sched = synth.make_schedule(p, n, [8] * n, 4003, 2)
    dg = [[8] * (n - 1) + [d] for d in last]
    rec = zr.Recorder(synth.MultiDeviceBlackBox(polys, nthreads=args.cpu_threads))
    res = zr.reconstruct_multi(p, dg, rec, sched=sched, stream=stream)
    exact = all(np.array_equal(r[0], h.exps) and np.array_equal(r[1], h.coefs) for r, h in zip(res, polys))
    rec.replay(True)
    zr.timing(True, dots_only=True)
    zr.timing_reset()
    tm, res = _replayed(zr, rec, lambda: zr.reconstruct_multi(p, dg, rec, sched=sched, stream=stream),
                        args.multi_steps)
    zr.timing(False)
    n_dots, ms_dots = zr.timing_get("vs_dots")
    cm = zr.last_counters()
    exact = exact and all(np.array_equal(r[0], h.exps) and np.array_equal(r[1], h.coefs) for r, h in zip(res, polys))
    steps = max(1, args.multi_steps)
    alu_m = _dots_work(cm) * steps * MUL32_PER_MULMOD / (ms_dots / 1e3) / 1e12 if ms_dots else 0.0
    # the same expressions one at a time
    sep_s, sep_mul, sep_solve, sep_ms = 0.0, 0, 0, 0.0
    for h, d in zip(polys, dg):
        r1 = zr.Recorder(synth.DeviceBlackBox(h, nthreads=args.cpu_threads))
        e1, c1 = zr.reconstruct(p, d, r1, sched=sched, stream=stream)
        exact = exact and bool(np.array_equal(e1, h.exps) and np.array_equal(c1, h.coefs))
        r1.replay(True)
        zr.timing(True, dots_only=True)
        zr.timing_reset()
        t1, _ = _replayed(zr, r1, lambda: zr.reconstruct(p, d, r1, sched=sched, stream=stream), args.multi_steps)
        zr.timing(False)
        sep_ms += zr.timing_get("vs_dots")[1] / steps
        c = zr.last_counters()
        sep_s += t1
        sep_mul += c["mulmods"]
        sep_solve += _dots_work(c)
        r1.close()
    alu_s = sep_solve * MUL32_PER_MULMOD / (sep_ms / 1e3) / 1e12 if sep_ms else 0.0
    rec.close()
    return {"workload": "8 expressions sampled together, n=6, degree bounds 8 in x_1..x_5 and 8/8/7/7/6/6/5/5 in x_6, "
                        f"each 99% of a common {t}-term set within its bounds plus 0.5% own terms",
            "terms": [int(h.nterms) for h in polys],
            "together": {"seconds": round(tm, 4), "mulmods": cm["mulmods"], "max_system": cm["max_t"],
                         "solve_kernel_TOPs": round(alu_m, 3), "frac_of_derived_peak": round(alu_m / MUL32_PEAK_TOPS, 4)},
            "separately": {"seconds": round(sep_s, 4), "mulmods": sep_mul, "solve_kernel_TOPs": round(alu_s, 3),
                           "frac_of_derived_peak": round(alu_s / MUL32_PEAK_TOPS, 4)},
            "speedup": round(sep_s / tm, 3) if tm else None, "bit_exact": bool(exact)}


def multiprime_leg(zr, synth, args, stream):
    """Polynomial with rational coefficients (n = 6, per-variable degree 30,
    10^4 terms, numerators and denominators of 100 bits): Zippel modulo the
    first prime, then one single-right-hand-side solve per further prime until
    a prime confirms the reconstructed fractions."""
    n, D, t = 6, 30, args.multi_terms
    q = synth.random_qpoly(n, D, t, 100, 4101)
    primes = synth.prime_list(8, seed=4100)
    sched = synth.make_schedule(primes[0], n, [D] * n, 4102, 2)
    rec = zr.Recorder(synth.PrimeDeviceBlackBox(q, nthreads=args.cpu_threads))
    e, fr, used = zr.reconstruct_rational(primes[0], [D] * n, rec, primes[1:], sched=sched, seed=4102,
                                          stream=stream)
    exact = bool(np.array_equal(e, q.exps) and fr == list(zip(q.num, q.den)))
    rec.replay(True)

    def run():
        return zr.reconstruct_rational(primes[0], [D] * n, rec, primes[1:], sched=sched, seed=4102, stream=stream,
                                       raw=True)
    tm, out = _replayed(zr, rec, run, args.multi_steps)
    e, fr, used = zr.rational_from_words(out)
    # one more run with every named launch timed: where the time goes
    zr.timing(True)
    zr.timing_reset()
    _replayed(zr, rec, run, 1)
    zr.timing(False)
    per = {k: round(zr.timing_get(k)[1], 3) for k in ("mp_corr", "mp_eval", "mp_crt_rr", "vs_dots", "master")}
    exact = exact and bool(np.array_equal(e, q.exps) and fr == list(zip(q.num, q.den)))
    # the first prime alone
    r0 = zr.Recorder(synth.DeviceBlackBox(q.mod(primes[0]), nthreads=args.cpu_threads))
    zr.reconstruct(primes[0], [D] * n, r0, sched=sched, stream=stream)
    r0.replay(True)
    t0, _ = _replayed(zr, r0, lambda: zr.reconstruct(primes[0], [D] * n, r0, sched=sched, stream=stream),
                      args.multi_steps)
    r0.close()
    rec.close()
    W1 = t * t + 2 * t * (t - 1) + t * (t - 1) // 2 + 4 * t  # one further prime's solve
    further = used - 1
    return {"workload": f"polynomial with rational coefficients, n={n}, per-variable degree<={D}, {t} terms, "
                        "100-bit numerators and denominators",
            "primes_used": used, "seconds": round(tm, 4), "first_prime_seconds": round(t0, 4),
            "further_primes_seconds": round(tm - t0, 4),
            "further_prime_solve_mulmod_per_s": round(further * W1 / max(tm - t0, 1e-9), 1),
            "per_kernel_ms": per, "bit_exact": exact}


def adaptive_leg(zr, synth, args, stream):
    """The n = 6, t = 10^4 polynomial without its degree bounds: caps of 40
    per variable (true bound 30), one confirming order, against the
    fixed-bound reconstruction with the degrees found, same schedule."""
    w = synth.config_workload(2)
    caps = [40] * 6
    sched = synth.make_schedule(w.p, 6, [41] * 6, 1002, 2)
    rec = zr.Recorder(synth.DeviceBlackBox(w.hidden, nthreads=args.cpu_threads))
    e, c, found = zr.reconstruct_adaptive(w.p, caps, rec, sched=sched, stream=stream)
    exact = bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    rec.replay(True)
    ta, (e, c, found) = _replayed(zr, rec, lambda: zr.reconstruct_adaptive(w.p, caps, rec, sched=sched,
                                                                             stream=stream), args.multi_steps)
    ca = zr.last_counters()
    exact = exact and bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    rf = zr.Recorder(synth.DeviceBlackBox(w.hidden, nthreads=args.cpu_threads))
    zr.reconstruct(w.p, found, rf, sched=sched, stream=stream)
    rf.replay(True)
    tf, _ = _replayed(zr, rf, lambda: zr.reconstruct(w.p, found, rf, sched=sched, stream=stream), args.multi_steps)
    cf = zr.last_counters()
    rec.close()
    rf.close()
    return {"workload": "n=6, t=10^4 polynomial (true per-variable degree 30) with caps of 40, one confirming order",
            "degrees_found": found, "seconds": round(ta, 4), "fixed_bound_seconds": round(tf, 4),
            "ratio": round(ta / tf, 3) if tf else None, "mulmods": ca["mulmods"], "fixed_bound_mulmods": cf["mulmods"],
            "bit_exact": exact}


def cpu_baseline(zr, synth, args, stream, W_step):
    """The oracle's transposed Vandermonde solve (master polynomial, synthetic
    division and dot products, inverse and scaling; unsigned __int128 products
    reduced with %) on a bounded sample of the headline's operation mix: one
    system of t = 2*10^4 random distinct monomial values with 40 right-hand
    sides.  Its cost grows as t^2 like the headline's, so its mulmod/s is
    the comparable rate; the full step's oracle time is extrapolated from it."""
    import oracle
    nthr = max(1, min(args.cpu_threads, os.cpu_count() or 1))
    t, R = args.cpu_sample_t, 40
    p = synth.make_prime()
    g = synth.SplitMix64(77)
    m = g.uniform_block(1, p, t)
    assert len(set(int(x) for x in m)) == t
    rhs = g.uniform_block(0, p, t * R).reshape(R, t)
    tc = time.perf_counter()
    want = oracle.vandermonde_solve(p, m, rhs, nthreads=nthr)
    tcpu = time.perf_counter() - tc
    got, st = zr.vandermonde_solve(p, m, rhs, stream=stream)
    W = R * t * t + 2 * t * (t - 1) + t * (t - 1) // 2 + t * (R + 3)
    rate = W / tcpu
    return {"value": round(rate, 1), "unit": "mulmod/s", "cores": nthr, "kind": "oracle",
            "sample": f"the oracle's transposed Vandermonde solve of one t={t}, R={R} system with random distinct "
                      "monomial values (the headline step's operation mix at a size the oracle finishes in seconds; "
                      "cost grows as t^2 in both); unsigned __int128 products reduced with %, OpenMP over rows",
            "seconds": round(tcpu, 2), "matches_gpu": bool(st == 0 and np.array_equal(got, want)),
            "extrapolated_step_seconds": round(W_step / rate, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--microbench", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--cpu-sample-t", type=int, default=20_000)
    ap.add_argument("--no-config2", action="store_true", help="skip the n = 6, t = 10^4 whole reconstruction")
    ap.add_argument("--config2-steps", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-instances", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the multi-expression, multi-prime and unknown-degree legs")
    ap.add_argument("--multi-terms", type=int, default=10_000)
    ap.add_argument("--multi-steps", type=int, default=2)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-budget-gib", type=int, default=16)
    ap.add_argument("--serve-fixed-rate", type=float, default=1000.0,
                    help="arrival rate (requests/s) of the served leg's fixed-rate Poisson pass")
    ap.add_argument("--solve-variant", default="producer_consumer", choices=["waves", "producer_consumer"],
                    help="dot-product pass of the one-system solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; the reconstruction of independent instances would "
              "shard across GPUs with no communication, but no multi-GPU run is part of it.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2505_24256_amd as zr
    import synth
    zr.lib()  # raises if the HIP library is missing
    zr.solve_variant(args.solve_variant)

    if args.microbench:
        print(json.dumps({"microbench": microbench(zr)}), flush=True)
        return

    stream = torch.cuda.current_stream()
    H = headline(zr, synth, args, stream)
    w, cnt, steps, elapsed = H["w"], H["cnt"], args.steps, H["elapsed"]
    t_sys = len(H["start"][1])
    R = int(w.deg[HEADLINE_STAGE - 1])
    mulmods = cnt["mulmods"] * steps
    value = mulmods / elapsed
    n_dots, ms_dots = H["n_dots"], H["ms_dots"]
    solve_alg = _dots_work(cnt) * steps               # R t^2 + t (t-1): what the dot-product pass computes
    achieved_mulmod_s = solve_alg / (ms_dots / 1e3) if ms_dots else 0.0
    alu = achieved_mulmod_s * MUL32_PER_MULMOD / 1e12
    traffic = (DOTS_TRAFFIC["bytes_per_launch"]
               if DOTS_TRAFFIC["sources_sha16"] == _dots_sources_sha16() and args.solve_variant == "producer_consumer"
               else None)
    # measured ceiling of the 32x32->64-bit multiply: the v_mad_u64_u32 probe
    # (independent streams at full occupancy), run here on the same GPU
    mad_ms, mad_ops = zr.microbench("mad_u64_u32", blocks=2048, iters=131072)
    mad_peak = mad_ops / mad_ms / 1e9 if mad_ms > 0 else None
    roofline = {"bound": "alu", "achieved": round(alu, 3), "peak": round(MUL32_PEAK_TOPS, 3),
                "unit": "TOP/s (32x32-bit multiplies; one 64x64-bit modular product or multiply-accumulate = 4)",
                "frac": round(alu / MUL32_PEAK_TOPS, 4), "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM, rocprofv3 counters, calibrated)",
                "kernel": "k_vs_dots_pc" if args.solve_variant == "producer_consumer" else "k_vs_dots",
                "launches_per_step": n_dots // steps if steps else 0,
                "avg_launch_ms": round(ms_dots / n_dots, 3) if n_dots else None,
                "work_per_step": "4 (R t^2 + t (t-1)) 32x32-bit multiplies (the dot products and the chain of "
                                 "q), t = %d, R = %d, over the step's launches (chunk groups of equal size)" % (t_sys, R),
                "measured_mul32_peak": {
                    "value": round(mad_peak, 3) if mad_peak else None, "unit": "TOP/s",
                    "probe": "v_mad_u64_u32, 8 independent chains per lane, 2048 x 256 threads, 131072 iterations "
                             "(about 17 ms, so that the clock settles as in the solve), this GPU, this run",
                    "frac": round(alu / mad_peak, 4) if mad_peak else None}}
    _progress("headline measured")

    cpu = None if args.no_cpu_baseline else cpu_baseline(zr, synth, args, stream, cnt["mulmods"])
    _progress("cpu baseline done")
    c2 = None if args.no_config2 else config2_leg(zr, synth, args, stream)
    _progress("n=6 leg done")
    multi = mprime = adapt = None
    if not args.no_extras:
        multi = multi_expression_leg(zr, synth, args, stream)
        _progress("multi-expression leg done")
        mprime = multiprime_leg(zr, synth, args, stream)
        _progress("multi-prime leg done")
        adapt = adaptive_leg(zr, synth, args, stream)
        _progress("unknown-degree leg done")
    batch = None if args.no_batch else batched_vs_plain(zr, synth, args, stream)
    serve = None if args.no_serve else served(zr, synth, args, stream)

    out = {
        "metric": "mulmod/s (algorithmic modular products per second, final Zippel stage of a 5*10^5-term "
                  "reconstruction, bit-exact)",
        "value": round(value, 1),
        "unit": "mulmod/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "arithmetic": "residues mod a 63-bit prime in u64, exact 128/192-bit integer intermediates",
        "data": "synthetic",
        "config": {"workload": "plain polynomial Zippel, n=8, per-variable degree<=40, t=5*10^5 terms, uniform "
                               "distinct exponents, coefficients uniform mod a seeded 63-bit prime; step = the final "
                               "stage (x_8) from the stage-7 result",
                   "p": w.p, "system_size": t_sys, "right_hand_sides": R, "final_terms": int(w.hidden.nterms),
                   "parallelism": "single GPU"},
        "stages_per_s": round(steps / elapsed, 4),
        "vandermonde_terms_per_s": round(cnt["vsolve_terms"] * steps / elapsed, 1),
        "latency_ms": {"p50": round(statistics.median(H["lat"]) * 1e3, 3),
                       "p99": round(float(np.percentile(H["lat"], 99)) * 1e3, 3)},
        "bit_exact": H["exact"],
        "mulmods_per_step": cnt["mulmods"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_warmup": {"steps": args.warmup, "per_kernel": H["kernels"]},
        "config2": c2,
        "multi_expression": multi,
        "multiprime": mprime,
        "unknown_degrees": adapt,
        "batch": batch,
        "serve": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
