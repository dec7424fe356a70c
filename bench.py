#!/usr/bin/env python3
"""Benchmark of the butterfly-filtering hot path on one MI355X.

Workload (the strain-like configuration): 32 s at 4096 Hz of seeded white Gaussian noise
(float32) with an SNR-8 ascending chirp, plus its time-randomised control, searched in one
batch against a bank of 65,536 one-second templates (L = 4096; f0 in [50, 2000] Hz x fdot in
[-2000, 2000] Hz/s, 256 x 256).  One step = one pass of the whole search on device-resident
inputs: window norms, the template x window contraction with its fused reductions
(butterfly output, spectrogram, spectrum), the histogram of maxima, for both series.
Bank construction is done once, outside the timed region.

value = template x offset correlations per second of the chosen precision form (the BF16
hi/lo split by default); the plain FP32 path is timed beside it.  The JSON line carries the
roofline of the contraction kernel (its HIP-event duration inside the timed region), the
measured error against the FP64 oracle on sampled offsets, and the oracle's own rate on the
host cores (cpu_baseline).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "template×offset correlations/s vs plain FP32 at stated error; p50/p99 latency"
# MI355X dense MFMA peaks; F16F8 is priced at the fp16 peak of its main product
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "f16x2": 2500.0, "f16f8": 2500.0,
               "f16f6": 2500.0}
# MFMA products per tap, in units of one product at the priced peak (F16F8: one fp16
# product plus two e4m3 products at twice the rate; F16F6: two e2m3 products at four times)
MFMA_TERMS = {"fp32": 1, "bf16x3": 3, "f16x2": 2, "f16f8": 2, "f16f6": 1.5}
TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "f16x2": 1e-3, "fft": 1e-5, "f16f8": 1e-4, "f16f6": 1e-4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_form(bf, torch, p, xs, prec, steps, warmup):
    """Times `steps` batched searches of the series `xs` (device tensors) with the bank in
    precision `prec`; returns timing, kernel times and the outputs of the last step."""
    bank = bf.bank_create(p, prec)
    prm = bf.make_params()
    outs = [bf.alloc_outputs(bank, int(x.shape[0]), prm, x.device) for x in xs]
    ws = bf.alloc_workspace(bank, [int(x.shape[0]) for x in xs], prm, xs[0].device)
    n_ranges, n_items = bf.plan(bank, [int(x.shape[0]) for x in xs])
    for _ in range(warmup):
        bf.search_batch(bank, xs, prm, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    bf.set_timing(True)
    try:
        bf.kernel_times()          # forget records from before the timed region
    except bf.BflyError:
        pass
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        bf.search_batch(bank, xs, prm, outs=outs, workspace=ws)
        e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bf.set_timing(False)
    kt, n_timed = bf.kernel_times()
    step_ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    K = bank.K
    W = [int(x.shape[0]) - p.L + 1 for x in xs]
    corr = K * sum(W)
    res = {
        "prec": prec, "wall_s": wall, "step_ms": step_ms,
        "ms_per_step": wall / steps * 1e3,
        "corr_per_step": corr,
        "value": corr * steps / wall,
        "kernel_ms": {k: v / n_timed for k, v in kt.items()},
        "K": K, "W": W,
        "n_ranges": n_ranges, "n_items": n_items,
        "outs": [{k: v.cpu().numpy() for k, v in o.items()} for o in outs],
    }
    del bank, outs, ws
    torch.cuda.empty_cache()
    return res


def fft_roofline(res, p, bf):
    """The FFT form's fused kernel against the float32 vector peak: per (template, block) a
    complex inverse FFT of M = N/2 points (5 M log2 M flop) plus the spectrum product and
    real-FFT post-processing (~16 M flop)."""
    import math
    ms = res["kernel_ms"]["main"]
    m, best = 512, 1e300
    for mm, lg in ((512, 9), (1024, 10), (2048, 11), (4096, 12)):   # as the library picks N
        v = 2 * mm - p.L + 1
        if v >= 1 and mm * lg / v < best * 0.999:
            m, best = mm, mm * lg / v
    valid = 2 * m - p.L + 1
    blocks = sum(-(-w // valid) for w in res["W"])
    flops = res["K"] * blocks * (5.0 * m * math.log2(m) + 16.0 * m)
    achieved = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": 157.3, "unit": "TFLOP/s",
            "frac": round(achieved / 157.3, 4), "traffic": recorded_traffic("fft", "fft"),
            "kernel": "k_fft_data+k_fft_main",
            "kernel_ms": round(ms, 3), "fft_points": 2 * m, "valid_per_block": valid}


def roofline(res, p, prec, tile, with_traffic=True):
    """k_main against its MFMA peak.  `traffic` comes from the committed counter summary of
    the strain workload, so other workloads pass with_traffic=False."""
    if prec == "fft":
        return fft_roofline(res, p, None)
    ms = res["kernel_ms"]["main"]
    flops = 2.0 * p.L * res["corr_per_step"]           # algorithmic: one multiply-add per tap
    achieved = flops / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": recorded_traffic(prec, tile) if with_traffic else None,
            "kernel": "k_main", "kernel_ms": round(ms, 3),
            "mfma_terms": MFMA_TERMS[prec],
            "executed_frac": round(achieved * MFMA_TERMS[prec] / peak, 4),
            # correlations/s x 2L against the FP32 MFMA peak: the like-for-like speed-up
            "effective_vs_fp32_peak": round(achieved / PEAK_TFLOPS["fp32"], 3)}


def lightcurve_leg(bf, torch, forms, steps):
    """One GPU's share of the 8.64M-template light-curve bank: 720,000 templates of L = 2000
    against the 64 s Kolmogorov-envelope photon-count series and its time-randomised control
    (2 x 126,001 offsets), one batch per step.  Timing only; parity on this workload is a
    GPU test."""
    from synth import bank_params, light_curve_series
    p3 = bank_params("light_curve_share")
    xs = [torch.from_numpy(light_curve_series()).cuda(), torch.from_numpy(light_curve_series(control=True)).cuda()]
    out = {}
    for form, n in forms:
        log(f"light-curve share: {form}, 1 warmup + {n} steps")
        r = time_form(bf, torch, p3, xs, form, n, 1)
        out[form] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "steps": n,
                     "roofline": roofline(r, p3, form, kernel_tile(form), with_traffic=False)}
        log(f"  {r['value']:.4g} corr/s, {r['ms_per_step']:.1f} ms/step")
        del r
        torch.cuda.synchronize()
    return {"workload": "light-curve bank share: 64 s photon counts (0.5 ms bins, 2000/s, "
                        "Kolmogorov envelope) + time-randomised control; shard 0/12 of "
                        "2880 f0 x 3000 fdot = 720,000 templates, L = 2000",
            "correlations_per_step": 2 * 126001 * p3.K, "forms": out}


def cpu_baseline(p, x64, xc64, n_off):
    """The FP64 oracle on a bounded sample: n_off offsets of the data series (a contiguous
    block around the injection plus seeded random picks) against the full bank."""
    import numpy as np
    from oracle import bfly_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    W = x64.shape[0] - p.L + 1
    rng = np.random.default_rng(22)
    blk = np.arange(49152 - n_off // 4, 49152 + n_off // 4)
    offs = np.unique(np.concatenate([blk, rng.choice(W, n_off - blk.shape[0], replace=False)]))
    t0 = time.perf_counter()
    orc = O.search(x64, p, offsets=offs)
    dt = time.perf_counter() - t0
    K = p.n_f0 * p.n_fdot
    return orc, {"value": offs.shape[0] * K / dt, "unit": "correlations/s", "cores": cores,
                 "kind": "oracle",
                 "sample": f"{offs.shape[0]} offsets of the 32 s data series (a block around "
                           f"the injection + seeded random picks) x all {K} templates, "
                           f"float64 NumPy/BLAS, {dt:.1f} s"}


def tails_leg(bf, torch, p, xs, prec, kappa, steps):
    """Times the search with kappa-sigma tails (two contraction passes) on the same series:
    one untimed run, then `steps` timed runs."""
    import numpy as np
    bank = bf.bank_create(p, prec)
    prm = bf.make_params()
    ns = [int(x.shape[0]) for x in xs]
    outs = [bf.alloc_outputs(bank, n, prm, x.device) for n, x in zip(ns, xs)]
    tails = [bf.alloc_tails(bank, 1 << 22, x.device) for x in xs]
    ws = torch.empty(bf.tails_workspace_bytes(bank, ns, prm), dtype=torch.uint8,
                     device=xs[0].device)
    bf.search_tails(bank, xs, kappa, 0, prm, outs=outs, tails=tails, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bf.search_tails(bank, xs, kappa, 0, prm, outs=outs, tails=tails, workspace=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    corr = bank.K * sum(n - p.L + 1 for n in ns)
    n_tails = [int(t["n_tails"][0]) for t in tails]
    counts = [t["bin_counts"].cpu().numpy().view("uint32").astype("int64") for t in tails]
    sig = tails[0]["sigma"].cpu().numpy()
    res = {"kappa": kappa, "precision_form": prec, "ms_per_step": wall / steps * 1e3,
           "correlations_per_s": corr * steps / wall, "passes": 3 if prec == "fft" else 2,
           "n_tails": n_tails, "tail_counts_total": [int(c.sum()) for c in counts],
           "sigma_median_x_sqrtL": float(np.median(sig) * np.sqrt(p.L)),
           "series": ["data", "control"][:len(xs)]}
    del bank, outs, tails, ws
    torch.cuda.empty_cache()
    return res


def serving_leg(bf, prec, n_segments, budget_gib, slots):
    """Serving workload: a device-resident bank of 512 x 512 = 262,144 templates (L = 4096,
    f0 in [50, 2000] Hz, fdot in [-2000, 2000] Hz/s) and a seeded trace of two-channel
    4096 Hz segments of 1-64 s (30% with chirps, SNR 6-12), submitted at their arrival times.
    Two points: the literal 50 segments/s (more than one GPU can serve, so queueing
    dominates latency), and the same trace with arrivals scaled to ~70% of the capacity
    measured on the first point.  Latency = submit to done, from the server's own clock."""
    import numpy as np
    from synth import bank_params, serving_trace, serving_segment
    p5 = bank_params("serving")
    bank = bf.bank_create(p5, prec)
    prm = bf.make_params(t_block=256)
    srv = bf.server_create(bank, budget_gib << 30, max_slots=slots, ticks_in_flight=2, params=prm)

    def run(trace):
        xs = [serving_segment(e) for e in trace]
        t0 = time.perf_counter()
        a0 = trace[0]["t_arrival"]
        tickets = []
        for e, x in zip(trace, xs):
            delay = (e["t_arrival"] - a0) - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append((bf.submit(srv, x), x.shape[0]))
        lat, starts, dones = [], [], []
        for t, n in tickets:
            while True:
                st, ts, tb, td = bf.poll(srv, t)
                if st in ("done", "failed", "cancelled"):
                    break
                time.sleep(0.0005)
            assert st == "done", st
            lat.append((td - ts) * 1e3)
            starts.append(tb)
            dones.append(td)
            bf.fetch(srv, t, n)
        corr = sum(bank.K * (n - p5.L + 1) for _, n in tickets)
        busy = max(dones) - min(starts)
        return {"segments": len(trace), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(max(lat)),
                "correlations_per_s": corr / busy, "busy_s": busy,
                "offered_segments_per_s": (len(trace) - 1) / max(trace[-1]["t_arrival"] - a0, 1e-9)}

    literal = run(serving_trace(n_segments))
    mean_corr = np.mean([bank.K * (e["n"] - p5.L + 1) for e in serving_trace(n_segments)])
    capacity = literal["correlations_per_s"] / mean_corr          # segments/s
    scale = 0.7 * capacity / 50.0
    scaled = run(serving_trace(n_segments, rate_scale=scale))
    scaled["rate_scale"] = scale
    stats = bf.server_stats(srv)
    bf.server_destroy(srv)
    del bank
    return {"precision_form": prec,
            "workload": "serving: 512 x 512 bank (262,144 templates), L = 4096, 1-64 s "
                        "two-channel segments, HBM budget %d GiB, %d slots, 2 ticks in flight"
                        % (budget_gib, slots),
            "literal_50_per_s": literal, "at_70pct_capacity": scaled,
            "capacity_segments_per_s": capacity, "ticks": stats["ticks"]}


def kernel_tile(prec):
    """The tile shape bf_search uses (BF_TILE overrides the library default)."""
    env = os.environ.get("BF_TILE")
    if env:
        return env
    if prec == "fft":
        return "fft"
    if prec in ("f16f8", "f16f6"):
        return "2x8p"
    return "2x8i" if prec in ("bf16x3", "f16x2") else "2x4"


def recorded_traffic(prec, tile):
    """HBM bytes per launch of the contraction kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, scaled by the same counters on a copy of known
    size), if it was taken on exactly the current kernel source and tile; else None.  The
    hash covers the kernel file followed by the internal header it includes."""
    import glob
    import hashlib
    kernel_file = "bfly_fft.hip" if prec == "fft" else "bfly_kernels.hip"
    csrc = os.path.join(ROOT, "paper_1802_01685_amd", "csrc")
    h = hashlib.sha256()
    for name in (kernel_file, "bfly_internal.h"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    sha = h.hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic-record:"):
                continue
            try:
                rec = json.loads(line.split(":", 1)[1])
            except ValueError:
                continue
            if rec.get("kernel_sha256") == sha and rec.get("precision") == prec \
                    and rec.get("tile") == tile:
                return rec["fetch_bytes"] + rec["write_bytes"]
    return None


def errors(orc, out, tol):
    import numpy as np
    offs = orc["offsets"]
    ok = ~orc["degen"]
    m_g = out["max_abs"][offs].astype(np.float64)[ok]
    a_g = out["argmax"][offs][ok]
    rel = np.abs(m_g - orc["m"][ok]) / orc["m"][ok]
    return {"max_rel_err": float(rel.max()), "tol": tol,
            "argmax_agreement": float(np.mean(a_g == orc["a"][ok])), "n_offsets": int(ok.sum())}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f16f6",
                    choices=["bf16x3", "f16x2", "fp32", "fft", "f16f8", "f16f6"])
    ap.add_argument("--fp32-steps", type=int, default=3, help="steps of the FP32 comparison")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison leg")
    ap.add_argument("--tails-kappa", type=float, default=5.0,
                    help="search depth of the kappa-sigma tail leg (0 skips it)")
    ap.add_argument("--extra-forms", default="bf16x3,f16f8,f16x2,fft",
                    help="comma-separated further precision forms to time and check ('' skips)")
    ap.add_argument("--cpu-offsets", type=int, default=16384, help="0 skips the oracle leg")
    ap.add_argument("--lightcurve", type=int, default=1,
                    help="time the light-curve bank share too (0 skips it)")
    ap.add_argument("--serve-segments", type=int, default=16,
                    help="segments per point of the serving leg (0 skips it)")
    ap.add_argument("--serve-precision", default="bf16x3",
                    choices=["bf16x3", "f16x2", "fp32", "fft", "f16f8", "f16f6"],
                    help="form of the serving leg's device-resident bank (the chosen form and "
                         "the FFT form are served beside it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a known-size reference "
                         "for hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the multi-GPU bank-sharded search is a design "
              "(max-loc all-reduce over the f0 shards), not implemented here.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1802_01685_amd import bfly as bf
    from synth import bank_params, strain_series, time_randomised

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    bf.lib()
    p = bank_params("strain")
    x = strain_series()
    xc = time_randomised(x, seed=102)
    xs = [torch.from_numpy(x).cuda(), torch.from_numpy(xc).cuda()]
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + written")
        del src, dst
    torch.cuda.synchronize()

    log(f"timing {args.precision}: {args.warmup} warmup + {args.steps} steps")
    main_res = time_form(bf, torch, p, xs, args.precision, args.steps, args.warmup)
    log(f"  {main_res['value']:.4g} corr/s, {main_res['ms_per_step']:.1f} ms/step, "
        f"kernels {main_res['kernel_ms']}")
    fp32_res = None
    if not args.no_fp32 and args.precision != "fp32":
        log(f"timing fp32: 1 warmup + {args.fp32_steps} steps")
        fp32_res = time_form(bf, torch, p, xs, "fp32", args.fp32_steps, 1)
        log(f"  {fp32_res['value']:.4g} corr/s, {fp32_res['ms_per_step']:.1f} ms/step")
    extra = {}
    for form in [f for f in args.extra_forms.split(",") if f and f != args.precision]:
        log(f"timing {form}: 1 warmup + {args.fp32_steps} steps")
        extra[form] = time_form(bf, torch, p, xs, form, args.fp32_steps, 1)
        log(f"  {extra[form]['value']:.4g} corr/s, {extra[form]['ms_per_step']:.1f} ms/step")

    lightcurve = None
    if args.lightcurve:
        lightcurve = lightcurve_leg(bf, torch, [(args.precision, 2), ("bf16x3", 2), ("fp32", 1)]
                                    if args.precision not in ("bf16x3", "fp32")
                                    else [(args.precision, 2), ("fp32", 1)], 2)
        if "fp32" in lightcurve["forms"] and args.precision in lightcurve["forms"]:
            lightcurve["speedup_of_chosen_form"] = (lightcurve["forms"][args.precision]["value"] /
                                                    lightcurve["forms"]["fp32"]["value"])

    tails = None
    if args.tails_kappa > 0:
        tails = {}
        for form in dict.fromkeys([args.precision, "fft"]):
            log(f"tails leg: kappa = {args.tails_kappa}, {form}, 1 + 2 runs")
            tails[form] = tails_leg(bf, torch, p, xs, form, args.tails_kappa, 2)
            log(f"  {tails[form]}")

    cpu = None
    err = {}
    if args.cpu_offsets > 0:
        log(f"oracle leg: {args.cpu_offsets} offsets x {p.n_f0 * p.n_fdot} templates")
        orc, cpu = cpu_baseline(p, x.astype(np.float64), xc.astype(np.float64), args.cpu_offsets)
        err[args.precision] = errors(orc, main_res["outs"][0], TOL[args.precision])
        if fp32_res:
            err["fp32"] = errors(orc, fp32_res["outs"][0], TOL["fp32"])
        for form, r in extra.items():
            err[form] = errors(orc, r["outs"][0], TOL[form])
        log(f"  oracle {cpu['value']:.4g} corr/s on {cpu['cores']} threads; errors {err}")

    serving = None
    serving_other = {}
    if args.serve_segments > 0:
        log(f"serving leg: {args.serve_segments} segments per point")
        serving = serving_leg(bf, args.serve_precision, args.serve_segments, 32, 16)
        log(f"  {serving}")
        for form in dict.fromkeys([args.precision, "fft"]):
            if form == args.serve_precision or (form == "fft" and
                                                "fft" not in args.extra_forms.split(",")):
                continue
            log(f"serving leg on the {form} form")
            serving_other[form] = serving_leg(bf, form, args.serve_segments, 32, 16)
            log(f"  {serving_other[form]}")

    steps_ms = main_res["step_ms"]
    lat = serving["at_70pct_capacity"] if serving else None
    rec = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "correlations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "f16x2": "f16", "f16f8": "f16+fp8",
                  "f16f6": "f16+fp6"}.get(args.precision, "f32"),
        "data": "synthetic",
        "config": {"workload": "strain-like 32 s at 4096 Hz (131,072 samples, SNR-8 chirp) + "
                               "time-randomised control; bank 256 f0 x 256 fdot = 65,536 "
                               "templates, L = 4096",
                   "precision_form": args.precision,
                   "series": 2, "samples_per_series": int(x.shape[0]),
                   "templates": main_res["corr_per_step"] // (2 * (x.shape[0] - p.L + 1)),
                   "L": p.L, "work_items": main_res["n_items"], "bin_ranges": main_res["n_ranges"],
                   "tile": kernel_tile(args.precision)},
        "latency_ms": ({"p50": lat["p50_ms"], "p99": lat["p99_ms"],
                        "of": "serving requests, submit to done, arrivals at 70% of capacity"}
                       if lat else None),
        "step_latency_ms": {"p50": float(np.percentile(steps_ms, 50)),
                            "p99": float(np.percentile(steps_ms, 99))},
        "kernel_ms": {k: round(v, 4) for k, v in main_res["kernel_ms"].items()},
        "roofline": roofline(main_res, p, args.precision, kernel_tile(args.precision)),
        "fp32": None if fp32_res is None else {
            "value": fp32_res["value"], "ms_per_step": fp32_res["ms_per_step"],
            "roofline": roofline(fp32_res, p, "fp32", kernel_tile("fp32")),
            "speedup_of_chosen_form": main_res["value"] / fp32_res["value"]},
        "other_forms": {form: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                               "tile": kernel_tile(form),
                               "roofline": roofline(r, p, form, kernel_tile(form))}
                        for form, r in extra.items()} or None,
        "tails": tails,
        "error_vs_fp64": err or None,
        "cpu_baseline": cpu,
        "lightcurve_share": lightcurve,
        "serving": serving,
        "serving_other_forms": serving_other or None,
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
