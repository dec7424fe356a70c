#!/usr/bin/env python3
"""Benchmark of the butterfly-filtering hot path on one MI355X.

Headline workload (the light-curve bank share, one GPU's share of the 8.64M-template bank):
a 64 s photon-count series in 0.5 ms bins (128,000 samples; Poisson, 2000 counts/s, with a
Kolmogorov-envelope rate) and its time-randomised control, searched in one batch against
720,000 one-second templates (L = 2000; shard 0 of 12 of 2880 f0 x 3000 fdot, f0 in
[10, 1000] Hz, fdot in [-1000, 1000] Hz/s).  One step = one pass of the whole search on
device-resident inputs (window norms, the template x window correlation with its fused
reductions: butterfly output, spectrogram, spectrum, histogram of maxima) for both series:
2 x 126,001 offsets x 720,000 templates = 1.81e11 correlations.  Bank construction is done
once, outside the timed region.

value = template x offset correlations per second of the headline form, the FFT form by
default: float32 arithmetic, held to the FP32 bound (1e-5).  Every other form (plain FP32 on
MFMA, the BF16 split, FP16 split, F16F8, F16F6, FP8) is timed on the same batch beside it, and
every form's error against the FP64 oracle (max relative error of m and S, argmax agreement
overall and where the FP64 top-2 margin exceeds twice the bound) comes from a seeded sample of
1,024 offsets of the series and 1,024 of the control.  The oracle runs on the host cores in a
child process started before the GPU is touched, concurrently with the GPU legs, and is timed
for the cpu_baseline.  Further legs: the 42-light-curve batch (84 series in one launch), the
kappa-sigma tail search, and the serving loop (latency p50/p99).
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "template×offset correlations/s vs plain FP32 at stated error; p50/p99 latency"
FORMS = ["fft", "fp32", "bf16x3", "f16f6", "f16f8", "f16x2", "fp8"]
# MI355X dense MFMA peaks (TFLOP/s) of each form's main product; the FFT form is priced
# against the float32 vector peak
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "f16x2": 2500.0, "f16f8": 2500.0,
               "f16f6": 2500.0, "fp8": 5000.0, "fft": 157.3}
# MFMA products per tap, in units of one product at the priced peak (F16F8: one fp16
# product plus two e4m3 products at twice the rate; F16F6: two e2m3 products at four times)
MFMA_TERMS = {"fp32": 1, "bf16x3": 3, "f16x2": 2, "f16f8": 2, "f16f6": 1.5, "fp8": 1}
DTYPE = {"fp32": "f32", "fft": "f32", "bf16x3": "bf16", "f16x2": "f16", "f16f8": "f16+fp8",
         "f16f6": "f16+fp6", "fp8": "fp8"}
LC_WORKLOAD = ("light-curve bank share: 64 s photon counts in 0.5 ms bins (128,000 samples, "
               "2000 counts/s, Kolmogorov envelope) + time-randomised control; shard 0/12 of "
               "2880 f0 x 3000 fdot = 720,000 templates, L = 2000")
SAMPLE_SEEDS = (71, 72)        # oracle offset picks of the series and of the control


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------------------
# the FP64 oracle on a sample (child process: it never touches the GPU)
# ---------------------------------------------------------------------------------------
def sample_offsets(W: int, n: int):
    """Seeded oracle sample of each series: a contiguous block of n/4 offsets plus random
    picks, n in total per series (data block in the middle, control block at a third)."""
    import numpy as np
    out = []
    for centre, seed in ((W // 2, SAMPLE_SEEDS[0]), (W // 3, SAMPLE_SEEDS[1])):
        blk = np.arange(centre - n // 8, centre + n // 8)
        rng = np.random.default_rng(seed)
        rest = np.setdiff1d(np.arange(W), blk)
        pick = rng.choice(rest, n - blk.shape[0], replace=False)
        out.append(np.sort(np.concatenate([blk, pick])))
    return out


def oracle_worker(n_per_series: int, out_path: str) -> int:
    """Runs the oracle on the light-curve sample and writes its outputs and timing."""
    import numpy as np
    from oracle import bfly_oracle as O
    from synth import bank_params, light_curve_series
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    p = bank_params("light_curve_share")
    xs = [light_curve_series().astype(np.float64),
          light_curve_series(control=True).astype(np.float64)]
    offs = sample_offsets(xs[0].shape[0] - p.L + 1, n_per_series)
    t0 = time.perf_counter()
    res = O.search_many(xs, p, offs)
    dt = time.perf_counter() - t0
    np.savez(out_path, seconds=dt, cores=cores,
             **{f"{k}{i}": r[k] for i, r in enumerate(res)
                for k in ("offsets", "m", "a", "second", "S", "degen")})
    return 0


def start_oracle(n_per_series: int):
    """Starts the oracle child before this process touches the GPU."""
    fd, path = tempfile.mkstemp(prefix="bfly_oracle_", suffix=".npz")
    os.close(fd)
    proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                             str(n_per_series), path], cwd=ROOT)
    return proc, path


def finish_oracle(proc, path, n_per_series, K):
    import numpy as np
    rc = proc.wait()
    if rc != 0:
        raise RuntimeError(f"oracle worker failed with {rc}")
    z = np.load(path)
    orcs = [{k: z[f"{k}{i}"] for k in ("offsets", "m", "a", "second", "S", "degen")}
            for i in range(2)]
    os.unlink(path)
    dt, cores = float(z["seconds"]), int(z["cores"])
    n = sum(o["offsets"].shape[0] for o in orcs)
    cpu = {"value": n * K / dt, "unit": "correlations/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_per_series} offsets of the light curve and {n_per_series} of its "
                     f"control (a block of {n_per_series // 4} + seeded random picks each) x "
                     f"all {K} templates, float64 NumPy/BLAS (templates generated once for "
                     f"both), {dt:.1f} s, run beside the GPU legs"}
    return orcs, cpu


# ---------------------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------------------
def time_form(bf, torch, p, xs, prec, steps, warmup, keep_offsets=None, t_block=1):
    """Times `steps` batched searches of the device series `xs` with a bank in precision
    `prec` (bank built outside the timed region).  Returns timing, per-kernel times and,
    for keep_offsets (one array per series), the outputs at those offsets."""
    import numpy as np
    t_b = time.perf_counter()
    bank = bf.bank_create(p, prec)
    torch.cuda.synchronize()
    bank_s = time.perf_counter() - t_b
    prm = bf.make_params(t_block=t_block)
    ns = [int(x.shape[0]) for x in xs]
    outs = [bf.alloc_outputs(bank, n, prm, x.device) for n, x in zip(ns, xs)]
    ws = bf.alloc_workspace(bank, ns, prm, xs[0].device)
    n_ranges, n_items = bf.plan(bank, ns)
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
    corr = bank.K * sum(n - p.L + 1 for n in ns)
    res = {"prec": prec, "wall_s": wall, "step_ms": step_ms, "steps": steps,
           "warmup": warmup, "ms_per_step": wall / steps * 1e3, "corr_per_step": corr,
           "value": corr * steps / wall, "bank_build_s": bank_s,
           "kernel_ms": {k: v / n_timed for k, v in kt.items()},
           "K": bank.K, "W": [n - p.L + 1 for n in ns], "n_ranges": n_ranges,
           "n_items": n_items}
    if keep_offsets is not None:
        res["kept"] = []
        for o, offs in zip(outs, keep_offsets):
            idx = torch.from_numpy(np.asarray(offs)).to(o["max_abs"].device)
            res["kept"].append({"max_abs": o["max_abs"][idx].cpu().numpy(),
                                "argmax": o["argmax"][idx].cpu().numpy(),
                                "spec": o["spec"][:, idx].cpu().numpy().T})
    del bank, outs, ws
    torch.cuda.empty_cache()
    return res


def fft_points(L):
    """The complex transform length M (real FFT length N = 2M) the library uses: 4096 for
    every template length (BF_FFT_POINTS = N picks a shorter one)."""
    v = os.environ.get("BF_FFT_POINTS")
    if v in ("1024", "2048", "4096") and int(v) - L + 1 >= 1:
        return int(v) // 2
    return 4096


def roofline(res, p, prec, tile):
    """The dominant kernel of a form against its roofline.  Direct forms: k_main, 2L flop per
    correlation (one multiply-add per tap) against the dense MFMA peak of the form's main
    product.  FFT form: k_fft_data + k_fft_main, per (template, block) one complex inverse
    FFT of M = N/2 points (5 M log2 M flop) plus the spectrum product and the real-FFT
    post-processing (16 M flop), against the float32 vector peak.  `traffic` comes from the
    committed counter record of this workload, if it was taken on the current kernel
    source and tile."""
    import math
    ms = res["kernel_ms"]["main"]
    traffic = recorded_traffic(prec, tile, "light_curve_share")
    counters = recorded_counters(prec, tile, "light_curve_share")
    if prec == "fft":
        m = fft_points(p.L)
        valid = 2 * m - p.L + 1
        blocks = sum(-(-w // valid) for w in res["W"])
        flops = res["K"] * blocks * (5.0 * m * math.log2(m) + 16.0 * m)
        achieved = flops / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_TFLOPS["fft"],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["fft"], 4),
                "traffic": traffic, "counters": counters, "kernel": "k_fft_data+k_fft4k",
                "kernel_ms": round(ms, 3), "fft_points": 2 * m, "valid_per_block": valid,
                "flop_per_launch": flops,
                "effective_vs_fp32_peak": round(2.0 * p.L * res["corr_per_step"] /
                                                (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"], 3)}
    flops = 2.0 * p.L * res["corr_per_step"]
    achieved = flops / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic, "counters": counters,
            "kernel": "k_main",
            "kernel_ms": round(ms, 3), "mfma_terms": MFMA_TERMS[prec],
            "executed_frac": round(achieved * MFMA_TERMS[prec] / peak, 4),
            "flop_per_launch": flops,
            "effective_vs_fp32_peak": round(achieved / PEAK_TFLOPS["fp32"], 3)}


def kernel_tile(prec):
    """The tile shape the search uses (BF_TILE overrides the library default)."""
    env = os.environ.get("BF_TILE")
    if env:
        return env
    if prec == "fft":
        return "fft"
    if prec in ("f16f8", "f16f6"):
        return "2x8p"
    return "2x8i" if prec in ("bf16x3", "f16x2") else "2x4"


def _record(kind, prec, tile, workload):
    """The committed `kind` record (a line "<kind>: {json}" in a profiles/ summary) of the
    form's dominant kernel, if it was taken on this workload and on exactly the current
    kernel source and tile; else None.  The hash covers the kernel file followed by the
    internal header it includes."""
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
            if not line.startswith(kind + ":"):
                continue
            try:
                rec = json.loads(line.split(":", 1)[1])
            except ValueError:
                continue
            if rec.get("kernel_sha256") == sha and rec.get("precision") == prec \
                    and rec.get("tile") == tile and rec.get("workload") == workload:
                return rec
    return None


def recorded_traffic(prec, tile, workload):
    """HBM bytes per launch from the committed counter record (FETCH_SIZE and WRITE_SIZE
    passes, scaled by the same counters on a copy of known size), or None."""
    rec = _record("traffic-record", prec, tile, workload)
    return None if rec is None else rec["fetch_bytes"] + rec["write_bytes"]


def recorded_counters(prec, tile, workload):
    """MFMA busy fraction, shader clock and VALU issue fraction of the same launches from the
    committed counter record, or None."""
    rec = _record("counter-record", prec, tile, workload)
    if rec is None:
        return None
    return {k: rec[k] for k in ("mfma_busy", "clock_mhz", "valu_issue") if k in rec}


def errors(orcs, kept, p, prec):
    """Error of a form against the oracle sample (both series together): max relative error
    of m and of S against max(value, 1/sqrt(L)), argmax agreement overall and where the FP64
    top-2 margin exceeds twice the form's bound."""
    import numpy as np
    from tests.parity_util import TOL, tolerance
    from synth import light_curve_series
    floor = 1.0 / np.sqrt(p.L)
    rel_m, rel_s, agree, dec_ok, dec_n, n = 0.0, 0.0, 0, 0, 0, 0
    over = 0
    for orc, g, x in zip(orcs, kept, (light_curve_series(), light_curve_series(control=True))):
        ok = ~orc["degen"]
        mo = orc["m"][ok]
        den = np.maximum(mo, floor)
        tol = tolerance(prec, x.astype(np.float64), p.L, orc["offsets"])[ok]
        r = np.abs(g["max_abs"][ok].astype(np.float64) - mo) / den
        rs = np.abs(g["spec"][ok].astype(np.float64) - orc["S"][ok]) / \
            np.maximum(orc["S"][ok], floor)
        over += int(np.sum(r > tol)) + int(np.sum(rs > tol[:, None]))
        rel_m, rel_s = max(rel_m, float(r.max())), max(rel_s, float(rs.max()))
        a = g["argmax"][ok] == orc["a"][ok]
        dec = (mo - orc["second"][ok]) > 2.0 * tol * den
        agree += int(a.sum())
        dec_n += int(dec.sum())
        dec_ok += int(a[dec].sum())
        n += int(ok.sum())
    return {"max_rel_err_m": rel_m, "max_rel_err_S": rel_s, "tol": TOL[prec],
            "within_bound": over == 0, "argmax_agreement": agree / max(n, 1),
            "argmax_agreement_where_margin_exceeds_2tol": dec_ok / max(dec_n, 1),
            "offsets_with_margin_above_2tol": dec_n, "n_offsets": n}


def batch_leg(bf, torch, forms):
    """The 42-light-curve batch: 42 series of 20-200 s at 500-5000 counts/s and their
    time-randomised controls, 84 series in one launch against the 512 x 512 bank (L = 2000),
    spectrogram rows decimated by 256.  One step per form."""
    import numpy as np
    from synth import bank_params, light_curve_batch
    p4 = bank_params("light_curve_batch")
    batch = light_curve_batch()
    xs = [torch.from_numpy(e["x"]).cuda() for e in batch]
    out = {}
    for form in forms:
        log(f"batch leg: {form}, 84 series, 1 step")
        r = time_form(bf, torch, p4, xs, form, 1, 0, t_block=256)
        out[form] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                     "kernel_ms": {k: round(v, 3) for k, v in r["kernel_ms"].items()}}
        log(f"  {r['value']:.4g} corr/s, {r['ms_per_step'] / 1e3:.1f} s")
    corr = p4.K * sum(e["x"].shape[0] - p4.L + 1 for e in batch)
    return {"workload": "42 light curves of 20-200 s (0.5 ms bins, 500-5000 counts/s, "
                        "Kolmogorov envelopes) + their time-randomised controls = 84 series "
                        "in one search; bank 512 x 512 = 262,144 templates, L = 2000, "
                        "t_block 256",
            "series": len(batch), "samples": int(sum(e["x"].shape[0] for e in batch)),
            "correlations_per_step": corr, "forms": out}


def tails_leg(bf, torch, p, xs, prec, kappa, steps):
    """The search with kappa-sigma tails on the headline batch: one untimed run, then
    `steps` timed runs."""
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
    sig = tails[0]["sigma"].cpu().numpy()
    res = {"kappa": kappa, "precision_form": prec, "ms_per_step": wall / steps * 1e3,
           "correlations_per_s": corr * steps / wall,
           "passes": ("1, then the listed (block, template) pairs transformed again"
                      if prec == "fft" else "1") +
                     " (a second full pass only for a series whose predicted threshold check "
                     "fails)" if prec != "fft" or fft_points(p.L) == 4096 else 3,
           "n_tails": n_tails, "sigma_median_x_sqrtL": float(np.median(sig) * np.sqrt(p.L)),
           "series": ["data", "control"][:len(xs)]}
    del bank, outs, tails, ws
    torch.cuda.empty_cache()
    return res


def serving_leg(bf, prec, n_segments, budget_gib, slots):
    """Serving workload: a device-resident bank of 512 x 512 = 262,144 templates (L = 4096,
    f0 in [50, 2000] Hz, fdot in [-2000, 2000] Hz/s) and a seeded trace of two-channel
    4096 Hz segments of 1-64 s (30% with chirps, SNR 6-12), submitted at their arrival times.
    Two points: the literal 50 segments/s (more than one GPU serves, so queueing dominates
    latency), and the same trace with arrivals scaled to ~70% of the capacity measured on
    the first point.  Latency = submit to done, from the server's own clock."""
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


def length_sweep(bf, torch, lengths=(256, 512, 1024, 2048, 4096),
                 forms=("fft", "f16f6", "fp8", "fp32")):
    """Correlations/s by template length: 65,536 templates (256 f0 x 256 fdot, fs = L so the
    chirps stay 1 s long) against 131,072 samples of seeded white noise, 1 untimed and 3 timed
    steps per (L, form)."""
    import numpy as np
    from synth import BankParams, white_noise
    x = torch.from_numpy(white_noise(131072, seed=7).astype(np.float32)).cuda()
    rows = []
    for L in lengths:
        fs = float(L)
        p = BankParams(fs=fs, L=L, n_f0=256, n_fdot=256, f0_min=fs / 50, f0_max=fs / 4,
                       fdot_min=-fs / 4, fdot_max=fs / 4)
        for prec in forms:
            r = time_form(bf, torch, p, [x], prec, steps=3, warmup=1)
            rows.append({"L": L, "form": prec, "ms_per_step": round(r["ms_per_step"], 3),
                         "correlations_per_s": r["value"], "correlations_per_step": r["corr_per_step"],
                         "fft_points": 2 * fft_points(L) if prec == "fft" else None})
            log(f"L = {L} {prec}: {r['value']:.3g} corr/s")
    return rows


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fft", choices=FORMS,
                    help="the headline form (value, roofline)")
    ap.add_argument("--form-steps", type=int, default=5,
                    help="timed steps of each other form on the headline batch")
    ap.add_argument("--forms", default=",".join(FORMS),
                    help="forms timed beside the headline ('' skips)")
    ap.add_argument("--cpu-offsets", type=int, default=1024,
                    help="oracle offsets per series of the sample (0 skips the oracle leg)")
    ap.add_argument("--batch-forms", default="fft,f16f6,bf16x3,fp32",
                    help="forms timed on the 84-series batch ('' skips the leg)")
    ap.add_argument("--tails-kappa", type=float, default=5.0,
                    help="search depth of the tail leg (0 skips it)")
    ap.add_argument("--serve-segments", type=int, default=256,
                    help="trace segments per point on the headline form's bank (0 skips)")
    ap.add_argument("--serve-bf16-segments", type=int, default=16,
                    help="trace segments per point on the BF16-split bank (0 skips)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a known-size reference "
                         "for hardware byte counters)")
    ap.add_argument("--length-sweep", action="store_true",
                    help="instead of the benchmark: the FFT form against the direct forms by "
                         "template length (one JSON line)")
    ap.add_argument("--oracle-worker", nargs=2, metavar=("N", "OUT"), help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.oracle_worker:
        return oracle_worker(int(args.oracle_worker[0]), args.oracle_worker[1])

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the multi-GPU bank-sharded search is a design "
              "(max-loc all-reduce over the f0 shards), not implemented here.", file=sys.stderr)
        return 2
    t_start = time.perf_counter()

    # the oracle child starts before this process touches the GPU
    oracle = (start_oracle(args.cpu_offsets)
              if args.cpu_offsets > 0 and not args.length_sweep else None)

    import numpy as np
    import torch
    from paper_1802_01685_amd import bfly as bf
    from synth import bank_params, light_curve_series

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    bf.lib()
    if args.length_sweep:
        print(json.dumps({"length_sweep": length_sweep(bf, torch)}), flush=True)
        return 0
    p = bank_params("light_curve_share")
    x = light_curve_series()
    xc = light_curve_series(control=True)
    xs = [torch.from_numpy(x).cuda(), torch.from_numpy(xc).cuda()]
    W = x.shape[0] - p.L + 1
    keep = sample_offsets(W, args.cpu_offsets) if args.cpu_offsets > 0 else None
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + written")
        del src, dst
    torch.cuda.synchronize()

    log(f"headline {args.precision}: {args.warmup} warmup + {args.steps} steps")
    main_res = time_form(bf, torch, p, xs, args.precision, args.steps, args.warmup, keep)
    log(f"  {main_res['value']:.4g} corr/s, {main_res['ms_per_step']:.1f} ms/step, "
        f"kernels {main_res['kernel_ms']}")
    forms = {}
    for form in [f for f in args.forms.split(",") if f and f != args.precision]:
        n = max(1, args.form_steps)
        log(f"{form}: 1 warmup + {n} steps")
        forms[form] = time_form(bf, torch, p, xs, form, n, 1, keep)
        log(f"  {forms[form]['value']:.4g} corr/s, {forms[form]['ms_per_step']:.1f} ms/step")

    batch = None
    if args.batch_forms:
        batch = batch_leg(bf, torch, [f for f in args.batch_forms.split(",") if f])

    tails = None
    if args.tails_kappa > 0:
        tails = {}
        for form in dict.fromkeys([args.precision, "f16f6"]):
            log(f"tails leg: kappa = {args.tails_kappa}, {form}, 1 + 2 runs")
            tails[form] = tails_leg(bf, torch, p, xs, form, args.tails_kappa, 2)
            plain = main_res if form == args.precision else forms.get(form)
            if plain is not None:
                tails[form]["vs_plain_search"] = tails[form]["ms_per_step"] / plain["ms_per_step"]
            log(f"  {tails[form]}")

    serving = {}
    if args.serve_segments > 0:
        log(f"serving leg ({args.precision}): {args.serve_segments} segments per point")
        serving[args.precision] = serving_leg(bf, args.precision, args.serve_segments, 32, 16)
        log(f"  {serving[args.precision]}")
    if args.serve_bf16_segments > 0 and args.precision != "bf16x3":
        log(f"serving leg (bf16x3): {args.serve_bf16_segments} segments per point")
        serving["bf16x3"] = serving_leg(bf, "bf16x3", args.serve_bf16_segments, 32, 16)
        log(f"  {serving['bf16x3']}")

    cpu, err = None, {}
    if oracle is not None:
        log("waiting for the oracle sample")
        orcs, cpu = finish_oracle(*oracle, args.cpu_offsets, p.K)
        for form, r in [(args.precision, main_res)] + list(forms.items()):
            err[form] = errors(orcs, r["kept"], p, form)
        log(f"  oracle {cpu['value']:.4g} corr/s on {cpu['cores']} threads; errors {err}")

    fp32 = forms.get("fp32")
    steps_ms = main_res["step_ms"]
    head_serv = serving.get(args.precision)
    lat = head_serv["at_70pct_capacity"] if head_serv else None
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
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": LC_WORKLOAD, "precision_form": args.precision,
                   "series": 2, "samples_per_series": int(x.shape[0]),
                   "templates": main_res["K"], "L": p.L,
                   "correlations_per_step": main_res["corr_per_step"],
                   "work_items": main_res["n_items"], "bin_ranges": main_res["n_ranges"],
                   "tile": kernel_tile(args.precision)},
        "vs_plain_fp32": (None if fp32 is None else main_res["value"] / fp32["value"]),
        "at_stated_error": (err[args.precision]["within_bound"]
                            if args.precision in err else None),
        "latency_ms": ({"p50": lat["p50_ms"], "p99": lat["p99_ms"],
                        "of": f"serving requests on the {args.precision} bank, submit to "
                              f"done, {lat['segments']} segments arriving at 70% of capacity"}
                       if lat else None),
        "step_latency_ms": {"p50": float(np.percentile(steps_ms, 50)),
                            "p99": float(np.percentile(steps_ms, 99))},
        "kernel_ms": {k: round(v, 4) for k, v in main_res["kernel_ms"].items()},
        "bank_build_s": round(main_res["bank_build_s"], 3),
        "roofline": roofline(main_res, p, args.precision, kernel_tile(args.precision)),
        "other_forms": {form: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                               "steps": r["steps"], "dtype": DTYPE[form],
                               "tile": kernel_tile(form),
                               "speedup_vs_fp32": (r["value"] / fp32["value"] if fp32 else None),
                               "roofline": roofline(r, p, form, kernel_tile(form))}
                        for form, r in forms.items()} or None,
        "error_vs_fp64": err or None,
        "cpu_baseline": cpu,
        "lightcurve_batch": batch,
        "tails": tails,
        "serving": serving or None,
        "bench_wall_s": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
