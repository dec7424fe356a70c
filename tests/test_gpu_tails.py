"""GPU parity of the kappa-sigma tails (sigma per template, the tails above kappa * sigma
and their per-f0-bin counts) against the FP64 oracle, through the C ABI.

sigma must match the oracle to the precision form's tolerance.  A tail's membership is a
floating-point decision, so the GPU and FP64 sets may differ only on pairs within a band
of the threshold: every FP64 tail clear of the band is found, every GPU tail reaches the
threshold within the band, shared tails agree in value and sign to tolerance.  The counts
equal the binning of the GPU's own list exactly; lists, sigma and counts are identical bit
for bit alone and in a batch; the search outputs equal those of a plain search.  The
two-detector coincidence counts are integer work on tail lists: they must equal the
oracle's counts on the GPU's own lists exactly.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bfly_oracle as O  # noqa: E402
from synth import BankParams, bank_params, small_strain_series, time_randomised, white_noise  # noqa: E402
from tests.parity_util import TOL, to_np  # noqa: E402

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16x3", "f16x2", "fp8", "fft", "f16f8", "f16f6"]

SMALL = BankParams(fs=128.0, L=48, n_f0=5, n_fdot=7, f0_min=3.0, f0_max=40.0,
                   fdot_min=-30.0, fdot_max=25.0)


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_01685_amd import bfly
    bfly.lib()
    return bfly


def _edge_series(n, seed, L):
    x = white_noise(n, seed)
    x[n // 3: n // 3 + L + 5] = 1.25            # constant run -> degenerate windows
    x[(2 * n) // 3] = np.nan                     # NaN -> L degenerate windows
    return x.astype(np.float32)


def _tails_np(t: dict) -> dict:
    r = {k: v.detach().cpu().numpy() for k, v in t.items()}
    n = int(r["n_tails"][0])
    m = min(n, r["tau"].shape[0])
    order = np.lexsort((r["k"][:m], r["tau"][:m]))
    return {"sigma": r["sigma"], "tau": r["tau"][:m][order].astype(np.int64),
            "k": r["k"][:m][order].astype(np.int64), "rho": r["rho"][:m][order],
            "counts": r["bin_counts"].view(np.uint32).astype(np.int64), "n": n}


def _search_tails(bf, bank, xs32, kappa, capacity, prm=None):
    xs = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda() for x in xs32]
    outs, tails = bf.search_tails(bank, xs, kappa, capacity, prm)
    torch.cuda.synchronize()
    return [to_np(o) for o in outs], [_tails_np(t) for t in tails]


def check_tails(x64, p, g: dict, orc: dict, kappa: float, tol: float, label: str) -> dict:
    grid = O.grid(p)
    floor = 1.0 / np.sqrt(p.L)
    # sigma
    s64 = orc["sigma"]
    pos = s64 > 0
    rel = np.abs(g["sigma"][pos].astype(np.float64) - s64[pos]) / s64[pos]
    assert rel.max(initial=0.0) <= tol, f"{label}: sigma rel error {rel.max():.3e}"
    assert np.all(g["sigma"][~pos] == 0.0)
    # every GPU tail is counted, in its f0 bin
    assert g["n"] == g["tau"].shape[0], f"{label}: list truncated"
    kl = g["k"] - int(grid.k_global[0])
    assert np.array_equal(g["counts"], np.bincount(grid.bin[kl], minlength=grid.n_bins))
    thr64 = kappa * s64
    # FP64 tails clear of the band are found
    ok_kl = orc["k"] - int(grid.k_global[0])
    r64 = np.abs(orc["rho"])
    band_o = 2 * tol * np.maximum(np.maximum(r64, thr64[ok_kl]), floor)
    gset = set(zip(g["tau"].tolist(), g["k"].tolist()))
    clear = r64 > thr64[ok_kl] + band_o
    missing = [(int(t), int(k)) for t, k, c in zip(orc["tau"], orc["k"], clear)
               if c and (int(t), int(k)) not in gset]
    assert not missing, f"{label}: {len(missing)} clear FP64 tails missing, e.g. {missing[:3]}"
    # every GPU tail reaches the FP64 threshold within the band
    r_at = O.rho_at(x64, p, g["tau"], g["k"])
    band_g = 2 * tol * np.maximum(np.maximum(r_at, thr64[kl]), floor)
    low = r_at <= thr64[kl] - band_g
    assert not low.any(), f"{label}: {int(low.sum())} GPU tails below the FP64 threshold"
    # shared tails: value and sign
    oidx = {(int(t), int(k)): i for i, (t, k) in enumerate(zip(orc["tau"], orc["k"]))}
    both = [(i, oidx[(int(t), int(k))]) for i, (t, k) in enumerate(zip(g["tau"], g["k"]))
            if (int(t), int(k)) in oidx]
    if both:
        gi, oi = np.array(both).T
        rg = g["rho"][gi].astype(np.float64)
        ro = orc["rho"][oi]
        err = np.abs(rg - ro) / np.maximum(np.abs(ro), floor)
        assert err.max() <= tol, f"{label}: tail rho rel error {err.max():.3e}"
        assert np.all(np.sign(rg) == np.sign(ro))
    n_border = len(gset ^ set(oidx))
    return {"n_gpu": int(g["n"]), "n_fp64": int(orc["tau"].shape[0]), "borderline": n_border,
            "max_rel_sigma": float(rel.max(initial=0.0))}


@pytest.mark.parametrize("prec", PRECS)
def test_tails_small_with_edges(bf, prec):
    """48-tap bank of 35 templates, 1500 samples with degenerate windows, kappa = 2.5."""
    p = SMALL
    x32 = _edge_series(1500, 7, p.L)
    bank = bf.bank_create(p, prec)
    outs, tails = _search_tails(bf, bank, [x32], 2.5, 1 << 16)
    orc = O.sigma_tails(x32.astype(np.float64), p, 2.5)
    st = check_tails(x32.astype(np.float64), p, tails[0], orc, 2.5, TOL[prec], f"small/{prec}")
    print(prec, st)
    # the search outputs of the tail search are those of a plain search
    plain = to_np(bf.search_segment(bank, torch.from_numpy(x32).cuda(), bf.make_params()))
    torch.cuda.synchronize()
    for key in plain:
        assert np.array_equal(plain[key].view(np.uint8), outs[0][key].view(np.uint8)), key


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fft"])
def test_tails_small_strain(bf, prec):
    """4 s at 512 Hz with a chirp, bank 16 x 16, L = 512, kappa = 4: every offset."""
    p = bank_params("small_strain")
    x32 = small_strain_series().astype(np.float32)
    bank = bf.bank_create(p, prec)
    _, tails = _search_tails(bf, bank, [x32], 4.0, 1 << 18)
    orc = O.sigma_tails(x32.astype(np.float64), p, 4.0)
    st = check_tails(x32.astype(np.float64), p, tails[0], orc, 4.0, TOL[prec], f"small_strain/{prec}")
    print(prec, st)
    assert st["n_fp64"] > 0


@pytest.mark.parametrize("prec", PRECS)
def test_tails_batch_equals_single_and_truncation(bf, prec):
    """Uneven series and a control in one batch give the lists, sigma and counts of each
    searched alone; a short list keeps its count and counts, and holds a subset."""
    p = BankParams(fs=256.0, L=96, n_f0=6, n_fdot=20, f0_min=5.0, f0_max=90.0,
                   fdot_min=-70.0, fdot_max=70.0)
    xs = [_edge_series(3000, 1, p.L), white_noise(96, 2).astype(np.float32),
          white_noise(1777, 3).astype(np.float32)]
    xs.append(time_randomised(xs[2], 103))
    bank = bf.bank_create(p, prec)
    _, batch = _search_tails(bf, bank, xs, 3.0, 1 << 16)
    for i, x in enumerate(xs):
        _, alone = _search_tails(bf, bank, [x], 3.0, 1 << 16)
        for key in ("sigma", "tau", "k", "rho", "counts"):
            assert np.array_equal(np.asarray(batch[i][key]).view(np.uint8),
                                  np.asarray(alone[0][key]).view(np.uint8)), (i, key)
    full = batch[0]
    cap = full["n"] // 3
    assert cap > 0
    _, short = _search_tails(bf, bank, [xs[0]], 3.0, cap)
    assert short[0]["n"] == full["n"]
    assert np.array_equal(short[0]["counts"], full["counts"])
    got = set(zip(short[0]["tau"].tolist(), short[0]["k"].tolist()))
    assert len(got) == cap and got <= set(zip(full["tau"].tolist(), full["k"].tolist()))


def _tails_run(bf, bank, xs32, kappa, env, monkeypatch):
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    try:
        return _search_tails(bf, bank, xs32, kappa, 1 << 18)
    finally:
        for k in env:
            monkeypatch.delenv(k, raising=False)


@pytest.mark.parametrize("prec", ["fft", "f16f6", "fp32", "bf16x3", "fp8"])
@pytest.mark.parametrize("shape", [(6, 10), (5, 7)])
def test_single_pass_equals_two_pass(bf, prec, shape, monkeypatch):
    """Sec. 2.2 predicts sigma before the search (Parseval): the single-pass tail search keeps
    the pairs above a predicted lower threshold while it sums rho^2 and selects the tails
    among them afterwards.  Its search outputs, sigma, tails and counts equal the two-pass
    search's bit for bit -- by default, when its check of the prediction fails (margin above
    1: every series falls back to the tails pass) and when its candidates overflow.  The
    5 x 7 bank gives odd template counts per bin range (the FFT form's single pass transforms
    two templates at a time)."""
    from synth import chirp_samples
    p = BankParams(fs=1024.0, L=1024, n_f0=shape[0], n_fdot=shape[1], f0_min=40.0,
                   f0_max=300.0, fdot_min=-150.0, fdot_max=150.0)   # L = 1024: N = 8192
    gr = O.grid(p)
    sig, _ = chirp_samples(30000, p.fs, 7000 / p.fs, gr.f0[23], gr.fdot[23])
    a = (white_noise(30000, 41) + 0.4 * sig).astype(np.float32)
    a[20000:20000 + p.L + 9] = 0.5                        # degenerate windows
    b = (3.0 * white_noise(20011, 42) + 100.0).astype(np.float32)
    bank = bf.bank_create(p, prec)
    kappa = 3.5
    runs = {name: _tails_run(bf, bank, [a, b], kappa, env, monkeypatch)
            for name, env in (("one", {}), ("two", {"BF_TAILS_TWO_PASS": "1"}),
                              ("redo", {"BF_TAILS_MARGIN": "4.0"}),
                              ("overflow", {"BF_TAILS_CAND_CAP": "4"}))}
    ref_out, ref_t = runs["two"]
    assert all(t["n"] > 0 for t in ref_t)
    for name in ("one", "redo", "overflow"):
        out, t = runs[name]
        for i in range(2):
            for key in ref_out[i]:
                assert np.array_equal(ref_out[i][key].view(np.uint8), out[i][key].view(np.uint8)), \
                    (name, i, key)
            for key in ("sigma", "tau", "k", "rho", "counts"):
                assert np.array_equal(np.asarray(ref_t[i][key]).view(np.uint8),
                                      np.asarray(t[i][key]).view(np.uint8)), (name, i, key)
            assert ref_t[i]["n"] == t[i]["n"], (name, i)
    # and the single-pass tails are right
    st = check_tails(a.astype(np.float64), p, runs["one"][1][0],
                     O.sigma_tails(a.astype(np.float64), p, kappa), kappa, TOL[prec],
                     f"single-pass/{prec}")
    print(prec, st)


def test_tails_kappa_zero_and_all_degenerate(bf):
    """kappa = 0: every non-degenerate pair is a tail.  A constant series: no non-degenerate
    offset, sigma = 0 and no tails."""
    p = SMALL
    K = p.n_f0 * p.n_fdot
    x = white_noise(400, 21).astype(np.float32)
    bank = bf.bank_create(p, "fp32")
    _, t = _search_tails(bf, bank, [x], 0.0, 1 << 16)
    W = 400 - p.L + 1
    assert t[0]["n"] == W * K
    assert np.array_equal(t[0]["counts"], np.full(p.n_f0, W * p.n_fdot))
    c = np.full(300, 0.75, np.float32)
    outs, t = _search_tails(bf, bank, [c], 3.0, 1024)
    assert t[0]["n"] == 0 and np.all(t[0]["sigma"] == 0.0) and np.all(t[0]["counts"] == 0)
    assert int(outs[0]["n_degenerate"][0]) == 300 - p.L + 1


def test_tails_errors(bf):
    p = SMALL
    bank = bf.bank_create(p, "fp32")
    x = torch.from_numpy(white_noise(400, 22).astype(np.float32)).cuda()
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(bf.BflyError) as e:
            bf.search_tails(bank, [x], bad, 16)
        assert e.value.status == bf.BF_EINVAL


def _coinc_np(c: dict) -> dict:
    return {"counts_a": c["counts_a"].cpu().numpy().view(np.uint32).astype(np.int64),
            "counts_b": c["counts_b"].cpu().numpy().view(np.uint32).astype(np.int64),
            "n_pairs": int(c["n_pairs"].cpu().numpy()[0])}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fft"])
def test_coincidence_two_channels(bf, prec):
    """Two simultaneous channels (independent noise, one common chirp at sample 1500):
    the GPU's coincidence counts equal the oracle's on the GPU's own tail lists, exactly,
    for several offset windows and frequency widths; the common chirp is coincident."""
    from synth import chirp_samples
    p = BankParams(fs=1024.0, L=1024, n_f0=24, n_fdot=24, f0_min=40.0, f0_max=300.0,
                   fdot_min=-150.0, fdot_max=150.0)
    gr = O.grid(p)
    k0 = 9 * 24 + 17
    n = 6000
    sig, _ = chirp_samples(n, p.fs, 1500 / p.fs, gr.f0[k0], gr.fdot[k0])
    a = (white_noise(n, 31) + 0.3 * sig).astype(np.float32)
    b = (white_noise(n, 32) + 0.3 * sig).astype(np.float32)
    bank = bf.bank_create(p, prec)
    xs = [torch.from_numpy(v).cuda() for v in (a, b)]
    _, tails = bf.search_tails(bank, xs, 3.5, 1 << 16)
    torch.cuda.synchronize()
    tn = [_tails_np(t) for t in tails]
    W = n - p.L + 1
    step = (p.f0_max - p.f0_min) / (p.n_f0 - 1)
    for dtau, df in ((0, 0.0), (0, 50.0), (3, 50.0), (10, step), (2, float("inf"))):
        c = _coinc_np(bf.coincidence(bank, tails[0], tails[1], W, dtau, df))
        torch.cuda.synchronize()
        want = O.coincidences(tn[0], tn[1], p, dtau, df)
        assert np.array_equal(c["counts_a"], want["counts_a"]), (dtau, df)
        assert np.array_equal(c["counts_b"], want["counts_b"]), (dtau, df)
        assert c["n_pairs"] == want["n_pairs"], (dtau, df)
        if (dtau, df) == (0, 0.0):
            assert c["counts_a"][9] > 0 and c["counts_b"][9] > 0    # the common chirp
    # swapping the channels swaps the counts
    c1 = _coinc_np(bf.coincidence(bank, tails[0], tails[1], W, 3, 50.0))
    c2 = _coinc_np(bf.coincidence(bank, tails[1], tails[0], W, 3, 50.0))
    assert np.array_equal(c1["counts_a"], c2["counts_b"]) and c1["n_pairs"] == c2["n_pairs"]


def test_coincidence_errors(bf):
    p = SMALL
    bank = bf.bank_create(p, "fp32")
    x = torch.from_numpy(white_noise(400, 22).astype(np.float32)).cuda()
    _, t = bf.search_tails(bank, [x, x], 3.0, 64)
    for dtau, df in ((-1, 1.0), (0, -1.0), (0, float("nan"))):
        with pytest.raises(bf.BflyError) as e:
            bf.coincidence(bank, t[0], t[1], 400 - p.L + 1, dtau, df)
        assert e.value.status == bf.BF_EINVAL


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fft", "f16f6"])
def test_tails_light_curve_share_sampled_templates(bf, prec, monkeypatch):
    """The tail search at full size, as the benchmark runs it: one GPU's 720,000-template
    share (L = 2000) against the 64 s light curve and its control at kappa = 5.  The FP64
    oracle forms rho at every offset for 16 seeded templates of each series (its sigma needs
    them all; 8 templates with GPU tails, 8 at random): their sigma and their tails are
    checked with the band rule of check_tails.
    The single pass is also held to the two-pass search bit for bit on the whole output."""
    from synth import light_curve_series
    p = bank_params("light_curve_share")
    xs = [light_curve_series(), light_curve_series(control=True)]
    kappa = 5.0
    bank = bf.bank_create(p, prec)
    outs1, t1 = _search_tails(bf, bank, xs, kappa, 1 << 20)
    outs2, t2 = _tails_run(bf, bank, xs, kappa, {"BF_TAILS_TWO_PASS": "1"}, monkeypatch)
    del bank
    torch.cuda.empty_cache()
    for i in range(2):
        for key in outs2[i]:
            assert np.array_equal(outs1[i][key].view(np.uint8), outs2[i][key].view(np.uint8)), \
                (i, key)
        for key in ("sigma", "tau", "k", "rho", "counts"):
            assert np.array_equal(np.asarray(t1[i][key]).view(np.uint8),
                                  np.asarray(t2[i][key]).view(np.uint8)), (i, key)
        assert t1[i]["n"] == t2[i]["n"] and t1[i]["n"] <= (1 << 20)
    grid = O.grid(p)
    K = grid.f0.shape[0]
    tol = TOL[prec]
    floor = 1.0 / np.sqrt(p.L)
    rng = np.random.default_rng(77)
    for i, (x32, g) in enumerate(zip(xs, t1)):
        x = x32.astype(np.float64)
        # 8 templates that have GPU tails and 8 at random
        with_tails = np.unique(g["k"] - int(grid.k_global[0]))
        ks = np.unique(np.concatenate([rng.choice(with_tails, min(8, with_tails.shape[0]),
                                                  replace=False),
                                       rng.choice(K, 8, replace=False)]))
        H = O.templates(p.fs, p.L, grid.f0[ks], grid.fdot[ks])
        r, degen = O.rho(x, H)                           # [W, 16], FP64
        ok = ~degen
        s64 = np.sqrt((r[ok] ** 2).sum(axis=0) / ok.sum())
        rel = np.abs(g["sigma"][ks].astype(np.float64) - s64) / s64
        assert rel.max() <= tol, f"series {i}: sigma rel error {rel.max():.3e}"
        thr = kappa * s64
        for j, k in enumerate(ks):
            kg = int(grid.k_global[k])
            mine = g["tau"][g["k"] == kg]
            a = np.abs(r[:, j])
            band = 2 * tol * np.maximum(np.maximum(a, thr[j]), floor)
            clear = np.nonzero(a > thr[j] + band)[0]
            assert np.isin(clear, mine).all(), f"series {i} k {kg}: clear FP64 tails missing"
            assert np.all(a[mine] > thr[j] - band[mine]), f"series {i} k {kg}: GPU tail below"
            rg = g["rho"][g["k"] == kg].astype(np.float64)
            err = np.abs(rg - r[mine, j]) / np.maximum(np.abs(r[mine, j]), floor)
            assert err.max(initial=0.0) <= tol, f"series {i} k {kg}: tail rho error"
        print(f"light-curve share {prec} series {i}: {g['n']} tails, sigma rel err "
              f"{rel.max():.2e}, sampled templates' tails {sum(int((g['k'] == int(grid.k_global[k])).sum()) for k in ks)}")


def test_fft_tails_with_many_templates_per_bin(bf):
    """An FFT bank whose f0 bin holds 65,535 templates: the single pass keeps each bin's
    argmax as a 16-bit offset, so such a bank takes the two-pass route (its rho^2 sums by
    atomics).  sigma and the tails of 16 sampled templates against FP64 rho at every offset,
    and the search outputs equal those of a plain search."""
    from synth import chirp_samples
    p = BankParams(fs=1024.0, L=1024, n_f0=1, n_fdot=65535, f0_min=60.0, f0_max=60.0,
                   fdot_min=-200.0, fdot_max=200.0)
    gr = O.grid(p)
    sig, _ = chirp_samples(20000, p.fs, 9000 / p.fs, gr.f0[40000], gr.fdot[40000])
    x = (white_noise(20000, 61) + 0.5 * sig).astype(np.float32)
    bank = bf.bank_create(p, "fft")
    kappa = 4.0
    outs, tails = _search_tails(bf, bank, [x], kappa, 1 << 20)
    plain = to_np(bf.search_segment(bank, torch.from_numpy(x).cuda(), bf.make_params()))
    torch.cuda.synchronize()
    del bank
    for key in plain:
        assert np.array_equal(plain[key].view(np.uint8), outs[0][key].view(np.uint8)), key
    g = tails[0]
    assert g["n"] > 0 and g["n"] <= (1 << 20)
    tol = TOL["fft"]
    floor = 1.0 / np.sqrt(p.L)
    rng = np.random.default_rng(62)
    with_tails = np.unique(g["k"] - int(gr.k_global[0]))
    ks = np.unique(np.concatenate([rng.choice(with_tails, min(8, with_tails.shape[0]),
                                              replace=False), [40000],
                                   rng.choice(gr.f0.shape[0], 8, replace=False)]))
    H = O.templates(p.fs, p.L, gr.f0[ks], gr.fdot[ks])
    r, degen = O.rho(x.astype(np.float64), H)
    ok = ~degen
    s64 = np.sqrt((r[ok] ** 2).sum(axis=0) / ok.sum())
    rel = np.abs(g["sigma"][ks].astype(np.float64) - s64) / s64
    assert rel.max() <= tol, f"sigma rel error {rel.max():.3e}"
    for j, k in enumerate(ks):
        kg = int(gr.k_global[k])
        mine = g["tau"][g["k"] == kg]
        a = np.abs(r[:, j])
        thr = kappa * s64[j]
        band = 2 * tol * np.maximum(np.maximum(a, thr), floor)
        assert np.isin(np.nonzero(a > thr + band)[0], mine).all(), f"k {kg}: FP64 tails missing"
        assert np.all(a[mine] > thr - band[mine]), f"k {kg}: GPU tail below the threshold"
    print(f"65,535 templates per bin: {g['n']} tails, sigma rel err {rel.max():.2e}")


@pytest.mark.parametrize("points", [2048, 4096])
def test_fft_tails_shorter_transforms(bf, points, monkeypatch):
    """The FFT form's three-pass tail search on the general kernel (BF_FFT_POINTS = N < 8192):
    the L = 512 small strain-like bank with a chirp at kappa = 4, every offset against FP64;
    the search outputs of the tail search equal a plain search bit for bit."""
    monkeypatch.setenv("BF_FFT_POINTS", str(points))
    p = bank_params("small_strain")
    x32 = small_strain_series().astype(np.float32)
    bank = bf.bank_create(p, "fft")
    outs, tails = _search_tails(bf, bank, [x32], 4.0, 1 << 18)
    orc = O.sigma_tails(x32.astype(np.float64), p, 4.0)
    st = check_tails(x32.astype(np.float64), p, tails[0], orc, 4.0, TOL["fft"],
                     f"small_strain/N={points}")
    assert st["n_fp64"] > 0
    plain = to_np(bf.search_segment(bank, torch.from_numpy(x32).cuda(), bf.make_params()))
    torch.cuda.synchronize()
    for key in plain:
        assert np.array_equal(plain[key].view(np.uint8), outs[0][key].view(np.uint8)), key
    print(points, st)


@pytest.mark.parametrize("prec", ["fft", "f16f6", "fp32"])
def test_tails_any_workspace_contents(bf, prec):
    """The tail search does not depend on what its workspace held before: a workspace of all
    one bits (every stale word flagged, every stale count huge) and one of zeros give the
    same search outputs, sigma, tails and counts bit for bit.  A 5 x 7 bank leaves 29
    padding templates in its 64-template granule."""
    p = BankParams(fs=1024.0, L=1024, n_f0=5, n_fdot=7, f0_min=40.0, f0_max=300.0,
                   fdot_min=-150.0, fdot_max=150.0)
    xs = [torch.from_numpy(white_noise(20000, 51).astype(np.float32)).cuda(),
          torch.from_numpy(white_noise(15000, 52).astype(np.float32)).cuda()]
    bank = bf.bank_create(p, "fft" if prec == "fft" else prec)
    prm = bf.make_params()
    nbytes = bf.tails_workspace_bytes(bank, [int(x.shape[0]) for x in xs], prm)
    res = []
    for fill in (0x00, 0xFF):
        ws = torch.full((nbytes,), fill, dtype=torch.uint8, device="cuda")
        outs, tails = bf.search_tails(bank, xs, 3.0, 1 << 16, prm, workspace=ws)
        torch.cuda.synchronize()
        res.append(([to_np(o) for o in outs], [_tails_np(t) for t in tails]))
    (o0, t0), (o1, t1) = res
    assert all(t["n"] > 0 for t in t0)
    for i in range(2):
        for key in o0[i]:
            assert np.array_equal(o0[i][key].view(np.uint8), o1[i][key].view(np.uint8)), (i, key)
        for key in ("sigma", "tau", "k", "rho", "counts"):
            assert np.array_equal(np.asarray(t0[i][key]).view(np.uint8),
                                  np.asarray(t1[i][key]).view(np.uint8)), (i, key)
        assert t0[i]["n"] == t1[i]["n"]
