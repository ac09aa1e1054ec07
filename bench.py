#!/usr/bin/env python
"""Benchmark of the plain polynomial Zippel reconstruction on one MI355X.

Workload: synthetic sparse polynomial, n = 6 variables, per-variable degree
<= 30, t = 10^4 terms with uniform distinct exponents, coefficients uniform
mod a seeded 63-bit prime (hidden-polynomial seed 2, schedule seed 1002).
One step = one full reconstruction (6 stages; Vandermonde systems of size up
to 10^4 with 30 right-hand sides each, Newton lifts, expansions, 2 probes).
The black box's samples are computed once on the host, recorded on the device
and replayed (a device-to-device copy per stage) inside the timed region.

Prints one JSON line.  ``--microbench`` instead prints the throughput probes
used for the roofline (see include/zippel_microbench.h).
"""
from __future__ import annotations

import argparse
import json
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
# MI355X dense int8 matrix-core peak (no sparsity)
INT8_PEAK_TOPS = 5000.0
INT8_OPS_PER_PRODUCT = 2 * 64

# HBM bytes per launch of the dominant solve kernel on this workload, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by the copy-probe calibration (0.5x
# read, 1.0x write); see profiles/k_vs_dots_pc_n6_d30_t1e4_hbm_counters.md.
# Valid only for the kernel sources and solve variant those counters were taken on.
DOTS_TRAFFIC = {"sources_sha16": "9c07805449d74c8d", "variant": "producer_consumer", "bytes_per_launch": 74.80e6}


def _system_sizes(w):
    """Sizes t of the Vandermonde systems of a reconstruction: the number of
    distinct exponent prefixes of the hidden polynomial before each added
    variable (stages 2..n)."""
    e = np.asarray(w.hidden.exps)
    return [int(len(np.unique(e[:, :k], axis=0))) for k in range(1, e.shape[1])]


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
    }


def served(zr, synth, args, stream):
    """Served balanced Zippel: rational requests P/Q, n = 5, total degree <= 20,
    t_N and t_D log-uniform in 10..5*10^3, Q(0) = 1.  Each request's samples are
    recorded once (its run alone, device black box), then replayed for every
    timed pass: one at a time; all submitted at once (saturated throughput);
    and Poisson arrivals at 0.7 x the saturated rate, admitted by device
    footprint and advanced in continuous batches (latency p50/p99)."""
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
                rid = srv.submit(w.deg_num, recs[sub], sched=w.schedule, deg_den=w.deg_den,
                                 expected_terms=max(w.num.nterms, w.den.nterms))
                ids[rid] = sub
                sub += 1
            st = srv.stats()
            if st["active"] == 0 and st["pending"] == 0:
                if sub < len(ws):
                    time.sleep(max(0.0, arrivals[sub] - (time.perf_counter() - t0)))
                continue
            srv.step()
            tn = time.perf_counter() - t0
            for rid, i in list(ids.items()):
                if i in fin:
                    continue
                r = srv.poll(rid)
                if r is not None:
                    fin[i] = tn
                    res[i] = r
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
    _progress(f"served: saturated {sat:.1f} req/s, Poisson at {rate:.1f} req/s")
    return {
        "workload": f"{len(ws)} rational requests P/Q, n=5, total degree<=20, t_N and t_D log-uniform in 10..5*10^3, "
                    "Q(0)=1; Poisson arrivals at 0.7 x the saturated throughput",
        "saturated": {"requests_per_s": round(sat, 2), "steps": st_sat["steps"], "peak_active": st_sat["peak_active"]},
        "poisson": {"rate_per_s": round(rate, 2), "requests_per_s": round(len(ws) / span, 2),
                    "latency_ms": {"p50": round(statistics.median(lat) * 1e3, 2),
                                   "p99": round(float(np.percentile(lat, 99)) * 1e3, 2)},
                    "steps": st["steps"], "peak_active": st["peak_active"],
                    "peak_footprint_bytes": st["peak_footprint"]},
        "one_at_a_time": {"requests_per_s": round(len(ws) / sum(lat1), 2), "latency_ms": {
            "p50": round(statistics.median(lat1) * 1e3, 2), "p99": round(float(np.percentile(lat1, 99)) * 1e3, 2)}},
        "identical_to_alone": bool(same and same_sat),
        "slots": args.serve_slots, "budget_gib": args.serve_budget_gib,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--microbench", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-instances", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-budget-gib", type=int, default=16)
    ap.add_argument("--time-all-kernels", action="store_true",
                    help="bracket every named launch of the timed steps with HIP events (default: the dot-product pass only)")
    ap.add_argument("--solve-variant", default="producer_consumer", choices=["waves", "producer_consumer", "mfma"],
                    help="dot-product pass of the one-system solve (mfma: the opt-in int8 matrix-core pass)")
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

    w = synth.config_workload(2)
    cache = CachingBox(synth.BlackBox(w.hidden, nthreads=args.cpu_threads))
    rec = zr.Recorder(zr.HostBlackBox(cache.eval, w.hidden.nvars))
    stream = torch.cuda.current_stream()

    # recording run: also checks the result against the hidden polynomial
    e, c = zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream)
    exact = bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))
    if not exact:
        print("bench.py: reconstruction does not match the hidden polynomial", file=sys.stderr)
        sys.exit(3)
    rec.replay(True)
    # warm-up steps: every named launch timed, for the per-kernel breakdown
    zr.timing(True)
    zr.timing_reset()
    for _ in range(args.warmup):
        zr.lib().zr_recorder_rewind(rec.handle)
        zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream)
    cnt = zr.last_counters()
    torch.cuda.synchronize()
    zr.timing(False)
    kernels = {}
    for name in ("master", "vs_pack", "vs_chain", "vs_scan", "vs_dots", "vs_finish", "newton", "scan", "expand"):
        n, ms = zr.timing_get(name)
        if n:
            kernels[name] = {"launches": n, "ms_total": round(ms, 3)}

    # timed steps: HIP events around the dot-product launches only (events
    # around every launch add host work between launches), unless asked
    zr.timing(True, dots_only=not args.time_all_kernels)
    zr.timing_reset()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        zr.lib().zr_recorder_rewind(rec.handle)
        e, c = zr.reconstruct(w.p, w.deg, rec, sched=w.schedule, stream=stream)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    zr.timing(False)
    exact = exact and bool(np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs))

    n_dots, ms_dots = zr.timing_get("vs_dots")
    steps = args.steps
    mulmods = cnt["mulmods"] * steps
    value = mulmods / elapsed
    solve_alg = cnt["solve_mulmods"] * steps          # R t^2 + 2 t (t-1) per system: what vs_dots computes
    achieved_mulmod_s = solve_alg / (ms_dots / 1e3) if ms_dots else 0.0
    alu = achieved_mulmod_s * MUL32_PER_MULMOD / 1e12
    traffic = (DOTS_TRAFFIC["bytes_per_launch"]
               if _dots_sources_sha16() == DOTS_TRAFFIC["sources_sha16"] and DOTS_TRAFFIC["variant"] == args.solve_variant
               else None)
    common = {"traffic": traffic, "traffic_unit": "bytes per launch (HBM, rocprofv3 counters, calibrated)",
              "launches_per_step": n_dots // steps if steps else 0,
              "avg_launch_ms": round(ms_dots / n_dots, 4) if n_dots else None}
    # measured ceiling of the 32x32->64-bit multiply: the v_mad_u64_u32 probe
    # (independent streams at full occupancy), run here on the same GPU
    mad_ms, mad_ops = zr.microbench("mad_u64_u32", blocks=2048, iters=4096)
    mad_peak = mad_ops / mad_ms / 1e9 if mad_ms > 0 else None
    if args.solve_variant == "mfma":
        # the R t^2 dot products run on the int8 matrix cores: one 63x63-bit
        # product is 64 digit products (8 x 8 signed base-256 digits), two ops each
        dots = cnt["dot_products"] * steps
        achieved = dots * INT8_OPS_PER_PRODUCT / (ms_dots / 1e3) / 1e12 if ms_dots else 0.0
        roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": INT8_PEAK_TOPS,
                    "unit": "TOP/s (int8 MFMA ops; one 64x64-bit product = 64 digit products = 128 ops)",
                    "frac": round(achieved / INT8_PEAK_TOPS, 4), **common, "kernel": "k_vs_mfma",
                    "alu_equivalent": {"achieved": round(alu, 3), "peak": round(MUL32_PEAK_TOPS, 3),
                                       "frac": round(alu / MUL32_PEAK_TOPS, 4),
                                       "unit": "TOP/s of 32x32-bit multiplies at 4 per modular product (whole solve work)"}}
    else:
        roofline = {"bound": "alu", "achieved": round(alu, 3), "peak": round(MUL32_PEAK_TOPS, 3),
                    "unit": "TOP/s (32x32-bit multiplies; one 64x64-bit modular product or multiply-accumulate = 4)",
                    "frac": round(alu / MUL32_PEAK_TOPS, 4), **common,
                    "kernel": "k_vs_dots_pc" if args.solve_variant == "producer_consumer" else "k_vs_dots"}
    roofline["measured_mul32_peak"] = {
        "value": round(mad_peak, 3) if mad_peak else None, "unit": "TOP/s",
        "probe": "v_mad_u64_u32, 8 independent chains per lane, 2048 x 256 threads, this GPU, this run",
        "frac": round(alu / mad_peak, 4) if mad_peak else None}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthr = max(1, min(args.cpu_threads, os.cpu_count() or 1))
        tc = time.perf_counter()
        oe, oc = oracle.zippel(w.p, w.deg, w.schedule, cache.eval, nthreads=nthr)
        tcpu = time.perf_counter() - tc
        same = bool(np.array_equal(oe, e) and np.array_equal(oc, c))
        cpu = {"value": round(cnt["mulmods"] / tcpu, 1), "unit": "mulmod/s", "cores": nthr, "kind": "oracle",
               "sample": "one full reconstruction of the same workload (all 6 stages) with the black box's "
                         "samples served from the host cache; unsigned __int128 products reduced with %",
               "seconds": round(tcpu, 2), "matches_gpu": same}

    batch = None
    _progress("plain configuration measured")
    if not args.no_batch:
        batch = batched_vs_plain(zr, synth, args, stream)
    serve = None
    if not args.no_serve:
        serve = served(zr, synth, args, stream)

    out = {
        "metric": "mulmod/s (algorithmic modular products per second, whole reconstruction)",
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
        "config": {"workload": "plain polynomial Zippel, n=6, per-variable degree<=30, t=10^4 terms, uniform "
                               "distinct exponents, coefficients uniform mod a seeded 63-bit prime",
                   "p": w.p, "system_sizes": _system_sizes(w), "right_hand_sides": int(w.deg[0]),
                   "parallelism": "single GPU"},
        "reconstructions_per_s": round(steps / elapsed, 3),
        "vandermonde_terms_per_s": round(cnt["vsolve_terms"] * steps / elapsed, 1),
        "latency_ms": {"p50": round(statistics.median(lat) * 1e3, 3),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "bit_exact": exact,
        "mulmods_per_step": cnt["mulmods"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_warmup": {"steps": args.warmup, "per_kernel": kernels},
        "batch": batch,
        "serve": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
