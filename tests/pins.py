"""Pins of the FP64 oracle: checks against closed forms, library routines, brute force and
invariants that do not come from the oracle itself.

Each ``pin_*`` takes the oracle module as its argument and raises AssertionError on a
mismatch.  The same pins run against the real oracle (test_oracle_pins.py) and against
copies of it with planted mistakes (test_oracle_mutants.py), where at least one must fail.
"""

from __future__ import annotations

import json
import math
import os

import numpy as np
import scipy.signal

from synth import BankParams, time_randomised

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _small_bank(L=32, n_f0=3, n_fdot=4, fs=64.0):
    return BankParams(fs=fs, L=L, n_f0=n_f0, n_fdot=n_fdot, f0_min=5.0, f0_max=20.0,
                      fdot_min=-12.0, fdot_max=12.0)


# ---------------------------------------------------------------------------------------
def pin_template_closed_forms(o):
    """Hand-derived template values (golden file) for ascending, descending and constant-
    frequency cases whose phases are exact multiples of 1/8."""
    with open(os.path.join(GOLDEN, "templates_closed_form.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        h = o.templates(c["fs"], c["L"], np.array([c["f0"]]), np.array([c["fdot"]]))[0]
        if "h" in c:
            want = np.array(c["h"])
        elif "h_times_sqrt102" in c:
            want = np.array(c["h_times_sqrt102"]) / math.sqrt(102.0)
        else:
            r = 1.0 / math.sqrt(2.0)
            want = np.array([1 - r / 2, r / 2, -1 - r / 2, r / 2] * 2) / math.sqrt(5.0)
        assert np.allclose(h, want, rtol=0, atol=1e-13), (c, h, want)


def pin_template_norms(o):
    """Every template of a random grid has mean 0 and L2 norm 1 (closed forms)."""
    rng = np.random.default_rng(11)
    f0 = rng.uniform(1, 200, 50)
    fd = rng.uniform(-300, 300, 50)
    H = o.templates(512.0, 300, f0, fd)
    assert np.abs(H.mean(axis=1)).max() < 1e-15
    assert np.abs(np.linalg.norm(H, axis=1) - 1).max() < 1e-14


def pin_grid(o):
    """Grid: inclusive linspace endpoints and steps, f0-major order, bins, shard ranges and
    the paper's 8.64M bank total (golden file) split into 12 shares of 720,000."""
    p = BankParams(fs=512.0, L=512, n_f0=16, n_fdot=16, f0_min=20.0, f0_max=200.0,
                   fdot_min=-100.0, fdot_max=100.0)
    g = o.grid(p)
    assert g.f0.shape[0] == 256
    assert g.f0[0] == 20.0 and g.f0[-1] == 200.0
    assert g.fdot[0] == -100.0 and g.fdot[15] == 100.0
    assert abs(g.f0[16] - 32.0) < 1e-12           # f0 step (200-20)/15 = 12, f0-major
    assert abs(g.fdot[1] - (-100.0 + 200.0 / 15.0)) < 1e-12
    assert np.all(g.f0[:16] == 20.0)
    assert list(g.bin[:33:16]) == [0, 1, 2]
    with open(os.path.join(GOLDEN, "bank_sizes.json")) as f:
        gold = json.load(f)
    total = 0
    for s in range(gold["n_gpus"]):
        q = BankParams(fs=2000.0, L=16, n_f0=gold["n_f0"], n_fdot=gold["n_fdot"],
                       f0_min=10.0, f0_max=1000.0, fdot_min=-1000.0, fdot_max=1000.0,
                       shard_index=s, shard_count=gold["n_gpus"])
        gq = o.grid(q)
        if s == 0:
            assert gq.f0.shape[0] == gold["share_templates"]
            assert gq.n_bins == gold["share_bins"]
            assert gq.k_global[0] == 0
        if s == 1:
            assert gq.k_global[0] == gold["share_templates"]
            assert gq.f0[0] == np.linspace(10.0, 1000.0, 2880)[240]
        total += gq.f0.shape[0]
    assert total == gold["total_templates"]


def _brute_search(x, p, norm="centred", hist_bins=8):
    """Pure-Python loops: templates, correlation, window energy, rho and all reductions."""
    L = p.L
    f0s = [p.f0_min + i * (p.f0_max - p.f0_min) / (p.n_f0 - 1) for i in range(p.n_f0)]
    f0s[-1] = p.f0_max
    fds = [p.fdot_min + j * (p.fdot_max - p.fdot_min) / (p.n_fdot - 1) for j in range(p.n_fdot)]
    fds[-1] = p.fdot_max
    H = []
    for i in range(p.n_f0):
        for j in range(p.n_fdot):
            c = []
            for n in range(L):
                t = n / p.fs
                c.append(math.cos(2 * math.pi * (f0s[i] * t + 0.5 * fds[j] * t * t)))
            mu = sum(c) / L
            c = [v - mu for v in c]
            nr = math.sqrt(sum(v * v for v in c))
            H.append([v / nr for v in c])
    W = len(x) - L + 1
    out_m, out_a, out_S, out_deg = [], [], [], []
    for tau in range(W):
        win = [float(x[tau + n]) for n in range(L)]
        bad = any(not math.isfinite(v) for v in win)
        win = [v if math.isfinite(v) else 0.0 for v in win]
        R = sum(v * v for v in win)
        if norm == "centred":
            mu = sum(win) / L
            E = sum((v - mu) ** 2 for v in win)
        else:
            E = R
        deg = bad or R == 0.0 or E <= 1e-12 * R
        out_deg.append(deg)
        if deg:
            out_m.append(0.0)
            out_a.append(-1)
            out_S.append([0.0] * p.n_f0)
            continue
        best, arg = -1.0, -1
        S = [0.0] * p.n_f0
        for k in range(len(H)):
            d = 0.0
            for n in range(L):
                d += H[k][n] * win[n]
            r = abs(d) / math.sqrt(E)
            if r > best:
                best, arg = r, k
            b = k // p.n_fdot
            S[b] = max(S[b], r)
        out_m.append(best)
        out_a.append(arg)
        out_S.append(S)
    hist = [0] * hist_bins
    for m, deg in zip(out_m, out_deg):
        if not deg:
            b = int(math.floor(m * hist_bins))
            hist[min(hist_bins - 1, max(0, b))] += 1
    return (np.array(out_m), np.array(out_a), np.array(out_S), np.array(out_deg),
            np.array(hist))


def pin_brute_force(o):
    """Tiny inputs (N <= 64, L <= 8, K <= 6) against pure-Python loops, including a constant
    (degenerate) window, a NaN, and the raw norm."""
    p = BankParams(fs=16.0, L=7, n_f0=2, n_fdot=3, f0_min=1.5, f0_max=4.0,
                   fdot_min=-3.0, fdot_max=5.0)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(40)
    x[20:28] = 0.7            # constant run: windows 20, 21 are degenerate
    x[33] = np.nan            # windows 27..33 hold a NaN
    for norm in ("centred", "raw"):
        m, a, S, deg, hist = _brute_search(x, p, norm, hist_bins=8)
        r = o.search(x, p, norm=norm, hist_bins=8)
        assert np.array_equal(r["degen"], deg)
        assert np.allclose(r["m"], m, rtol=0, atol=1e-13)
        assert np.array_equal(r["a"], a)
        assert np.allclose(r["S"], S, rtol=0, atol=1e-13)
        assert np.array_equal(r["hist"], hist)
        assert r["n_degenerate"] == int(deg.sum())


def pin_np_correlate(o):
    """The numerator equals numpy.correlate(x, h, 'valid') for each template."""
    p = _small_bank()
    H = o.bank_templates(p)
    x = np.random.default_rng(6).standard_normal(300)
    d = o.numerator(x, H)
    for k in range(H.shape[0]):
        ref = np.correlate(x, H[k], mode="valid")
        assert np.allclose(d[:, k], ref, rtol=0, atol=1e-12)


def pin_fft_agreement(o):
    """Direct correlation equals FFT correlation (scipy, an independent library) to 1e-12
    of the window norm; the oracle's own FFT path agrees too."""
    p = _small_bank(L=64)
    H = o.bank_templates(p)
    x = np.random.default_rng(7).standard_normal(1000) * 3.0 + 1.0
    d = o.numerator(x, H)
    _, R, _ = o.window_energy(x, p.L)
    for k in range(H.shape[0]):
        ref = scipy.signal.correlate(x, H[k], mode="valid", method="fft")
        assert np.all(np.abs(d[:, k] - ref) <= 1e-12 * np.sqrt(R) + 1e-13)
        own = o.numerator_fft(x, H[k])
        assert np.all(np.abs(d[:, k] - own) <= 1e-12 * np.sqrt(R) + 1e-13)


def pin_self_correlation(o):
    """A series holding template k at offset s (zeros elsewhere) gives rho(s, k) = 1, the
    butterfly output 1 at (s, k), and all-zero windows are degenerate."""
    p = _small_bank(L=40)
    H = o.bank_templates(p)
    for k in (0, 5, H.shape[0] - 1):
        s = 97
        x = np.zeros(300)
        x[s:s + p.L] = H[k]
        r = o.search(x, p)
        i = s
        assert abs(r["m"][i] - 1.0) < 1e-14
        assert r["a"][i] == k
        assert r["degen"][s + p.L:].all() and r["degen"][: s - p.L + 1].all()
        assert not r["degen"][s]


def pin_cauchy_schwarz(o):
    """|rho| <= 1 on arbitrary data (Cauchy-Schwarz with a zero-mean unit-norm template)."""
    p = _small_bank(L=24)
    x = np.random.default_rng(8).standard_cauchy(500)
    r = o.search(x, p)
    assert np.all(r["m"] <= 1.0 + 1e-12)
    assert np.all(r["S"] <= 1.0 + 1e-12)


def pin_invariants(o):
    """Centred rho is invariant to affine maps of x up to sign; rho(-x) = -rho(x); a shift
    of x shifts every output."""
    p = _small_bank(L=32)
    H = o.bank_templates(p)
    x = np.random.default_rng(9).standard_normal(400)
    r1, _ = o.rho(x, H)
    r2, _ = o.rho(3.5 * x - 7.25, H)
    r3, _ = o.rho(-x, H)
    assert np.allclose(r2, r1, rtol=0, atol=1e-12)
    assert np.allclose(r3, -r1, rtol=0, atol=1e-12)
    a = o.search(x, p)
    b = o.search(x[13:], p)
    assert np.allclose(b["m"], a["m"][13:], rtol=0, atol=1e-13)
    assert np.array_equal(b["a"], a["a"][13:])


def pin_noise_statistic(o):
    """For iid Gaussian data, E[rho^2] = 1/(L-1) for the centred norm (x - mean is uniform
    on the sphere of the complement of the constant vector, which holds h) and 1/L for the
    raw norm.  Checked on 6000 independent windows (statistical error about 2%)."""
    L = 48
    p = BankParams(fs=64.0, L=L, n_f0=1, n_fdot=2, f0_min=9.0, f0_max=9.0,
                   fdot_min=-20.0, fdot_max=20.0)
    H = o.bank_templates(p)
    x = np.random.default_rng(10).standard_normal(6000 * L)
    offs = np.arange(0, 6000 * L - L + 1, L)
    for norm, want in (("centred", 1.0 / (L - 1)), ("raw", 1.0 / L)):
        r, _ = o.rho(x, H, offs, norm)
        est = float((r[:, 0] ** 2).mean())
        assert abs(est / want - 1.0) < 0.08, (norm, est, want)


def pin_recovery(o):
    """An on-grid chirp (a bank template's waveform, amplitude 0.5) injected at an integer
    start into unit noise is recovered at exactly that offset and template."""
    p = BankParams(fs=512.0, L=512, n_f0=16, n_fdot=16, f0_min=20.0, f0_max=200.0,
                   fdot_min=-100.0, fdot_max=100.0)
    g = o.grid(p)
    k = 3 * 16 + 11                       # f0 = 56 Hz, fdot = +46.67 Hz/s
    t = np.arange(512) / 512.0
    chirp = np.cos(2 * np.pi * (g.f0[k] * t + 0.5 * g.fdot[k] * t * t))
    for seed in (1, 2, 3):
        x = np.random.default_rng(seed).standard_normal(2048)
        x[666:666 + 512] += 0.5 * chirp
        r = o.search(x, p, offsets=np.arange(500, 900))
        i = int(np.argmax(r["m"]))
        assert r["offsets"][i] == 666 and r["a"][i] == k, (seed, r["offsets"][i], r["a"][i])


def pin_spectrogram_histogram(o):
    """max_i S[tau, i] = m[tau]; decimated rows are row-block maxima; the histogram sums to
    W - n_degenerate; the spectrum is the time mean of S; bin edges follow the floor rule."""
    p = _small_bank(L=16)
    x = np.random.default_rng(12).standard_normal(300)
    x[100:130] = 2.0
    r = o.search(x, p, hist_bins=16)
    assert np.allclose(r["S"].max(axis=1), r["m"], rtol=0, atol=0)
    W = x.shape[0] - p.L + 1
    assert int(r["hist"].sum()) == W - r["n_degenerate"] and r["n_degenerate"] > 0
    Sd = o.decimate(r["S"], 7)
    assert Sd.shape == (-(-W // 7), p.n_f0)
    assert np.array_equal(Sd[3], r["S"][21:28].max(axis=0))
    assert np.allclose(r["spectrum"] * W, r["S"].sum(axis=0), rtol=1e-14, atol=0)
    b = o.hist_bin(np.array([-0.1, 0.0, 1 / 256, 0.5 - 1e-12, 0.5, 0.999, 1.0, 7.0]), 256, 0.0, 1.0)
    assert list(b) == [0, 0, 1, 127, 128, 255, 255, 255]
    # per-bin rows: bin i of the spectrogram only sees templates i*n_fdot .. i*n_fdot+n_fdot-1
    H = o.bank_templates(p)
    rr, _ = o.rho(x, H)
    want = np.abs(rr).reshape(W, p.n_f0, p.n_fdot).max(axis=2)
    assert np.allclose(r["S"], want, rtol=0, atol=1e-13)


def pin_average_spectrum(o):
    """The multi-series average is the mean of each series' own time mean of S (reading 10,
    Fig. 1 caption): pure-Python loops over series of uneven length, which differ from the
    mean pooled over all offsets."""
    p = _small_bank(L=16)
    rng = np.random.default_rng(24)
    xs = [rng.standard_normal(n) * s for n, s in ((90, 1.0), (400, 3.0), (150, 0.5))]
    rs = [o.search(x, p) for x in xs]
    got = o.average_spectrum([r["spectrum"] for r in rs])
    want = []
    for i in range(p.n_f0):
        per = []
        for r in rs:
            col = [float(row[i]) for row in r["S"]]
            per.append(sum(col) / len(col))
        want.append(sum(per) / len(per))
    assert np.allclose(got, want, rtol=1e-14, atol=0)
    pooled = np.concatenate([r["S"] for r in rs]).mean(axis=0)
    assert not np.allclose(got, pooled, rtol=1e-6, atol=0)


def pin_degenerate_rule(o):
    """Constant, all-zero and NaN windows are degenerate; a tiny non-constant one is not."""
    L = 8
    x = np.concatenate([np.full(8, 3.0), np.zeros(8), [1.0, np.nan] + [0.5] * 6,
                        1e-150 * np.arange(8.0)])
    E, R, deg = o.window_energy(x, L, np.array([0, 8, 16, 24]))
    assert list(deg) == [True, True, True, False]


def pin_ties(o):
    """Identical templates tie exactly: the smallest index wins, also across template chunks
    (a grid whose fdot axis collapses to one value repeats each f0 template n_fdot times)."""
    p = BankParams(fs=64.0, L=20, n_f0=3, n_fdot=3, f0_min=4.0, f0_max=9.0,
                   fdot_min=2.0, fdot_max=2.0)
    x = np.random.default_rng(14).standard_normal(200)
    for kc in (3, 9):
        r = o.search(x, p, k_chunk=kc)
        assert np.all(r["a"] % 3 == 0), r["a"][:20]
    q = BankParams(fs=64.0, L=20, n_f0=2, n_fdot=3, f0_min=6.0, f0_max=6.0,
                   fdot_min=1.0, fdot_max=1.0)
    for kc in (3, 6):
        r = o.search(x, q, k_chunk=kc)
        assert np.all(r["a"] == 0)


def pin_control(o):
    """Time randomisation keeps the value multiset (the histogram) and reorders samples."""
    x = np.random.default_rng(13).standard_normal(1000)
    xc = time_randomised(x, seed=103)
    assert np.array_equal(np.sort(xc), np.sort(x))
    assert not np.array_equal(xc, x)


# ---------------------------------------------------------------------------------------
# sigma of rho, the kappa-sigma tails and their pseudo-spectrum
# ---------------------------------------------------------------------------------------
def _brute_rho(x, p, norm="centred"):
    """Pure-Python loops over a possibly sharded bank: signed rho[tau][k_local] (0 on
    degenerate windows), the degenerate flags, and each local template's global index and
    f0 bin."""
    L = p.L
    f0s = [p.f0_min + i * (p.f0_max - p.f0_min) / (p.n_f0 - 1) for i in range(p.n_f0)]
    f0s[-1] = p.f0_max
    fds = [p.fdot_min + j * (p.fdot_max - p.fdot_min) / (p.n_fdot - 1) for j in range(p.n_fdot)]
    fds[-1] = p.fdot_max
    lo = p.shard_index * p.n_f0 // p.shard_count
    hi = (p.shard_index + 1) * p.n_f0 // p.shard_count
    H, kg, bins = [], [], []
    for i in range(lo, hi):
        for j in range(p.n_fdot):
            c = [math.cos(2 * math.pi * (f0s[i] * (n / p.fs) + 0.5 * fds[j] * (n / p.fs) ** 2))
                 for n in range(L)]
            mu = sum(c) / L
            c = [v - mu for v in c]
            nr = math.sqrt(sum(v * v for v in c))
            H.append([v / nr for v in c])
            kg.append(i * p.n_fdot + j)
            bins.append(i - lo)
    rho, deg = [], []
    for tau in range(len(x) - L + 1):
        win = [float(x[tau + n]) for n in range(L)]
        bad = any(not math.isfinite(v) for v in win)
        win = [v if math.isfinite(v) else 0.0 for v in win]
        R = sum(v * v for v in win)
        if norm == "centred":
            mu = sum(win) / L
            E = sum((v - mu) ** 2 for v in win)
        else:
            E = R
        d_ = bad or R == 0.0 or E <= 1e-12 * R
        deg.append(d_)
        row = []
        for k in range(len(H)):
            d = sum(H[k][n] * win[n] for n in range(L))
            row.append(0.0 if d_ else d / math.sqrt(E))
        rho.append(row)
    return rho, deg, kg, bins


def pin_tails_brute_force(o):
    """sigma, the tails and the pseudo-spectrum on tiny inputs against pure-Python loops: a
    sharded bank (global indices), a constant (degenerate) run, a NaN, both norms, and
    kappa = 0 with the centred norm (every non-degenerate pair is a tail, no degenerate one
    is)."""
    p = BankParams(fs=16.0, L=7, n_f0=3, n_fdot=2, f0_min=1.5, f0_max=4.0,
                   fdot_min=-3.0, fdot_max=5.0, shard_index=1, shard_count=2)
    rng = np.random.default_rng(15)
    x = rng.standard_normal(44)
    x[18:26] = -0.4           # windows 18, 19 are degenerate
    x[37] = np.nan            # windows 31..37 hold a NaN
    for norm in ("centred", "raw"):
        rho, deg, kg, bins = _brute_rho(x, p, norm)
        n_ok = sum(1 for d in deg if not d)
        K = len(kg)
        sig = [math.sqrt(sum(row[k] ** 2 for row in rho) / n_ok) for k in range(K)]
        # kappa = 0 only with the centred norm: under the raw norm a constant window is not
        # degenerate and its rho is a rounding residue (~1e-17) whose sign depends on the
        # summation order
        for kappa in ((0.0, 1.0, 1.7) if norm == "centred" else (0.5, 1.0, 1.7)):
            want = sorted((t, kg[k], rho[t][k]) for t in range(len(rho)) for k in range(K)
                          if abs(rho[t][k]) > kappa * sig[k])
            counts = [0] * (max(bins) + 1)
            for t in range(len(rho)):
                for k in range(K):
                    if abs(rho[t][k]) > kappa * sig[k]:
                        counts[bins[k]] += 1
            r = o.sigma_tails(x, p, kappa, norm)
            assert r["n_ok"] == n_ok
            assert np.allclose(r["sigma"], sig, rtol=0, atol=1e-13)
            assert list(r["tau"]) == [w[0] for w in want]
            assert list(r["k"]) == [w[1] for w in want]
            assert np.allclose(r["rho"], [w[2] for w in want], rtol=0, atol=1e-13)
            assert list(r["counts"]) == counts


def pin_tails_parseval(o):
    """A series of period L: every window holds one whole period, so E is the same for every
    offset and, over W = L offsets, the numerator is the circular cross-correlation of the
    template with one period.  Parseval's theorem then gives
    sigma_k^2 = sum_f |H_k(f)|^2 |X(f)|^2 / (L^2 E) with L-point DFTs (numpy.fft)."""
    p = _small_bank(L=32)
    L = p.L
    per = np.random.default_rng(16).standard_normal(L) + 0.3
    x = np.concatenate([per, per[:L - 1]])
    H = o.bank_templates(p)
    Hf = np.abs(np.fft.fft(H, axis=1)) ** 2
    Xf = np.abs(np.fft.fft(per)) ** 2
    for norm in ("centred", "raw"):
        E = float(((per - per.mean()) ** 2).sum()) if norm == "centred" else float((per ** 2).sum())
        want = np.sqrt((Hf * Xf[None, :]).sum(axis=1) / (L * L * E))
        r = o.sigma_tails(x, p, 2.0, norm)
        assert r["n_ok"] == L
        assert np.allclose(r["sigma"], want, rtol=1e-12, atol=0), (norm, r["sigma"], want)


def pin_tails_invariants(o):
    """Every tail exceeds kappa sigma and is at most the butterfly maximum of its offset; the
    counts add up to the tails; an offset whose maximum exceeds kappa sigma of its argmax
    template contributes that tail; an affine map of x changes nothing (centred norm); for
    iid Gaussian data the mean of sigma_k^2 over the bank is 1/(L-1) (statistical, ~3%)."""
    p = _small_bank(L=32)
    g = o.grid(p)
    x = np.random.default_rng(17).standard_normal(20000)
    kappa = 2.5
    r = o.sigma_tails(x, p, kappa)
    s = o.search(x, p)
    kl = r["k"] - int(g.k_global[0])
    assert np.all(np.abs(r["rho"]) > kappa * r["sigma"][kl])
    assert np.all(np.abs(r["rho"]) <= s["m"][r["tau"]] + 1e-13)
    assert int(r["counts"].sum()) == r["tau"].size > 0
    pairs = set(zip(r["tau"].tolist(), r["k"].tolist()))
    hit = np.nonzero(s["m"] > kappa * r["sigma"][s["a"] - int(g.k_global[0])])[0]
    assert hit.size > 0 and all((int(t), int(s["a"][t])) in pairs for t in hit)
    r2 = o.sigma_tails(2.0 * x - 3.0, p, kappa)
    assert np.allclose(r2["sigma"], r["sigma"], rtol=1e-12, atol=0)
    assert np.array_equal(r2["tau"], r["tau"]) and np.array_equal(r2["k"], r["k"])
    est = float((r["sigma"] ** 2).mean())
    assert abs(est * (p.L - 1) - 1.0) < 0.1, est * (p.L - 1)


# ---------------------------------------------------------------------------------------
# several series at once, the top-2 margin, |rho| at given pairs
# ---------------------------------------------------------------------------------------
def _brute_reduce(rho, deg, kg, bins, nb, hist_bins=8):
    """Reductions of a brute-force rho table, in plain loops: m, a (first maximum in
    increasing k), the second largest |rho| (ties count twice), S, histogram."""
    m, a, second, S = [], [], [], []
    for row, d_ in zip(rho, deg):
        if d_:
            m.append(0.0)
            a.append(-1)
            second.append(0.0)
            S.append([0.0] * nb)
            continue
        best, arg = -1.0, -1
        Srow = [0.0] * nb
        for k, v in enumerate(row):
            if abs(v) > best:
                best, arg = abs(v), kg[k]
            Srow[bins[k]] = max(Srow[bins[k]], abs(v))
        vals = sorted((abs(v) for v in row), reverse=True)
        m.append(best)
        a.append(arg)
        second.append(vals[1] if len(vals) > 1 else -1.0)
        S.append(Srow)
    hist = [0] * hist_bins
    for v, d_ in zip(m, deg):
        if not d_:
            hist[min(hist_bins - 1, max(0, int(math.floor(v * hist_bins))))] += 1
    return np.array(m), np.array(a), np.array(second), np.array(S), np.array(hist)


def pin_search_many_brute_force(o):
    """Three series of uneven length (constant runs, a NaN) searched together on a sharded
    bank, on all or on a subset of their offsets, with the bank applied in one, two or four
    chunks: m, a, the runner-up |rho|, S and the histograms equal pure-Python loops, and each
    series equals its own single search bit for bit."""
    p = BankParams(fs=16.0, L=7, n_f0=8, n_fdot=3, f0_min=1.5, f0_max=6.0,
                   fdot_min=-3.0, fdot_max=5.0, shard_index=1, shard_count=2)
    rng = np.random.default_rng(21)
    xs = [rng.standard_normal(40), 0.3 + 2.0 * rng.standard_normal(23), rng.standard_normal(31)]
    xs[0][12:21] = 0.5              # windows 12..14 degenerate
    xs[1][9] = np.nan               # windows 3..9 hold a NaN
    xs[2][20:31] = 0.0              # windows 20..24 degenerate (all zero)
    offs = [None, np.array([0, 2, 3, 9, 10, 16]), None]
    for norm in ("centred", "raw"):
        for kc in (3, 6, None):
            many = o.search_many(xs, p, offs, norm=norm, hist_bins=8, k_chunk=kc)
            for x, of, r in zip(xs, offs, many):
                rho, deg, kg, bins = _brute_rho(x, p, norm)
                sel = np.arange(len(rho)) if of is None else of
                m, a, second, S, hist = _brute_reduce([rho[t] for t in sel],
                                                      [deg[t] for t in sel], kg, bins, 4)
                assert np.array_equal(r["offsets"], sel)
                assert np.array_equal(r["degen"], np.array([deg[t] for t in sel]))
                assert np.allclose(r["m"], m, rtol=0, atol=1e-13), (norm, kc)
                assert np.array_equal(r["a"], a), (norm, kc, r["a"], a)
                assert np.allclose(r["second"], second, rtol=0, atol=1e-13), (norm, kc)
                assert np.allclose(r["S"], S, rtol=0, atol=1e-13)
                assert np.array_equal(r["hist"], hist)
                one = o.search(x, p, offsets=of, norm=norm, hist_bins=8, k_chunk=kc)
                for key in ("m", "a", "second", "S", "hist", "spectrum", "degen"):
                    assert np.array_equal(one[key], r[key]), (key, norm, kc)


def pin_second_ties(o):
    """Duplicate templates tie exactly: the runner-up equals the maximum (margin 0), within a
    chunk and across chunks; with distinct templates the margin is positive."""
    q = BankParams(fs=64.0, L=20, n_f0=2, n_fdot=3, f0_min=6.0, f0_max=6.0,
                   fdot_min=1.0, fdot_max=1.0)
    x = np.random.default_rng(22).standard_normal(120)
    for kc in (3, 6):
        r = o.search(x, q, k_chunk=kc)
        assert np.array_equal(r["second"], r["m"])
    p = _small_bank(L=20)
    r = o.search(x, p)
    assert np.all(r["m"] - r["second"] > 0)


def pin_rho_at_brute_force(o):
    """|rho| at given (offset, global template) pairs on a sharded bank against pure-Python
    loops, with degenerate windows (0) and k = -1 entries (0), both norms."""
    p = BankParams(fs=16.0, L=7, n_f0=5, n_fdot=3, f0_min=1.5, f0_max=4.0,
                   fdot_min=-3.0, fdot_max=5.0, shard_index=1, shard_count=2)
    rng = np.random.default_rng(23)
    x = rng.standard_normal(40) - 0.8
    x[15:24] = 1.5            # windows 15..17 degenerate (centred)
    x[30] = np.inf            # windows 24..30 hold an inf
    for norm in ("centred", "raw"):
        rho, deg, kg, _ = _brute_rho(x, p, norm)
        taus = rng.integers(0, len(rho), 60)
        ks = rng.integers(0, len(kg), 60)
        want = np.array([abs(rho[t][k]) for t, k in zip(taus, ks)])
        kglob = np.array([kg[k] for k in ks])
        kglob[::7] = -1
        want[::7] = 0.0
        got = o.rho_at(x, p, taus, kglob, norm=norm)
        assert np.allclose(got, want, rtol=0, atol=1e-13), norm
        assert np.any(got > 0) and np.all(got[np.array([deg[t] for t in taus])] == 0.0)


# ---------------------------------------------------------------------------------------
# two-detector coincidence of tails
# ---------------------------------------------------------------------------------------
def _brute_coincidences(ta, ka, tb, kb, p, dtau, df):
    """Pure-Python pairwise loops over unsorted lists; f0 from the linspace formula."""
    f0s = [p.f0_min + i * (p.f0_max - p.f0_min) / (p.n_f0 - 1) for i in range(p.n_f0)]
    f0s[-1] = p.f0_max
    lo = p.shard_index * p.n_f0 // p.shard_count
    nb = (p.shard_index + 1) * p.n_f0 // p.shard_count - lo
    ca, cb = [0] * nb, [0] * nb
    hb = [False] * len(tb)
    pairs = 0
    for i in range(len(ta)):
        hit = False
        for j in range(len(tb)):
            if abs(ta[i] - tb[j]) <= dtau and \
                    abs(f0s[ka[i] // p.n_fdot] - f0s[kb[j] // p.n_fdot]) <= df:
                hit = True
                hb[j] = True
                pairs += 1
        if hit:
            ca[ka[i] // p.n_fdot - lo] += 1
    for j in range(len(tb)):
        if hb[j]:
            cb[kb[j] // p.n_fdot - lo] += 1
    return ca, cb, pairs


def pin_coincidence_brute_force(o):
    """Random tail lists of two channels on a sharded bank against pure-Python pairwise
    loops, for several offset windows and frequency widths, including a width equal to
    the f0 spacing (pairs exactly df apart count)."""
    p = BankParams(fs=256.0, L=40, n_f0=9, n_fdot=5, f0_min=10.0, f0_max=70.0,
                   fdot_min=-20.0, fdot_max=20.0, shard_index=1, shard_count=2)
    lo = 1 * 9 // 2
    hi = 2 * 9 // 2
    rng = np.random.default_rng(18)
    ka = rng.integers(lo * 5, hi * 5, 60)
    kb = rng.integers(lo * 5, hi * 5, 50)
    ta = rng.integers(0, 30, 60)
    tb = rng.integers(0, 30, 50)
    for dtau, df in ((0, 0.0), (0, 7.5), (2, 7.5), (1, 16.0), (5, 100.0)):
        r = o.coincidences({"tau": ta, "k": ka}, {"tau": tb, "k": kb}, p, dtau, df)
        ca, cb, pairs = _brute_coincidences(ta.tolist(), ka.tolist(), tb.tolist(), kb.tolist(),
                                            p, dtau, df)
        assert list(r["counts_a"]) == ca and list(r["counts_b"]) == cb, (dtau, df)
        assert r["n_pairs"] == pairs, (dtau, df)


def pin_coincidence_limits(o):
    """Swapping the channels swaps the counts; a channel against itself with dtau = 0 and
    df = 0 makes every tail coincident with itself; an empty channel makes none."""
    p = _small_bank()
    rng = np.random.default_rng(19)
    a = {"tau": rng.integers(0, 50, 40), "k": rng.integers(0, 12, 40)}
    b = {"tau": rng.integers(0, 50, 30), "k": rng.integers(0, 12, 30)}
    r1 = o.coincidences(a, b, p, 1, 7.5)
    r2 = o.coincidences(b, a, p, 1, 7.5)
    assert np.array_equal(r1["counts_a"], r2["counts_b"])
    assert np.array_equal(r1["counts_b"], r2["counts_a"]) and r1["n_pairs"] == r2["n_pairs"]
    r3 = o.coincidences(a, a, p, 0, 0.0)
    assert np.array_equal(r3["counts_a"], np.bincount(a["k"] // p.n_fdot, minlength=p.n_f0))
    empty = {"tau": np.zeros(0, np.int64), "k": np.zeros(0, np.int64)}
    r4 = o.coincidences(a, empty, p, 3, 1e9)
    assert r4["n_pairs"] == 0 and not r4["counts_a"].any()


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
