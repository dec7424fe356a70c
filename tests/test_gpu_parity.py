"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle.

Tolerances (max relative error of the butterfly output m and of the spectrogram S over
non-degenerate offsets): FP32 1e-5, BF16 hi/lo split 1e-4, FP16 template split (fp16 data)
1e-3 and FP8 (e4m3 with power-of-two template and strip scales) 0.2, the stated bounds of
those two; the FFT-correlation form (float32 spectra and transforms) 1e-5.  Relative errors
are taken
against max(value, 1/sqrt(L)).  Argmax: the template the GPU
reports must reach the FP64 maximum within 2*tol (so it must be the oracle's template
wherever the FP64 top-2 margin exceeds 2*tol*m).  Histograms: exact against the floor-rule
binning of the GPU's own maxima, and equal to the FP64 histogram except for maxima within
tol of a bin edge.  Integer and index outputs of batched and single searches must be
identical bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bfly_oracle as O  # noqa: E402
from synth import (BankParams, bank_params, small_strain_series, strain_series, light_curve_series,  # noqa: E402
                   chirp_samples, time_randomised, white_noise)
from tests.parity_util import TOL, check_against_oracle, check_hist, to_np, tolerance  # noqa: E402

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16x3", "f16x2", "fp8", "fft", "f16f8", "f16f6"]


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_01685_amd import bfly
    bfly.lib()
    return bfly


def _run(bf, p, x32, prec, t_block=1, norm="centred", hist_bins=256, lo=0.0, hi=1.0):
    bank = bf.bank_create(p, prec)
    prm = bf.make_params(norm=norm, t_block=t_block, hist_bins=hist_bins, hist_lo=lo, hist_hi=hi)
    x = torch.from_numpy(np.ascontiguousarray(x32, dtype=np.float32)).cuda()
    out = bf.search_segment(bank, x, prm)
    torch.cuda.synchronize()
    return to_np(out), bank


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("offset", [1000.0, -250.0])
@pytest.mark.parametrize("norm", ["centred", "raw"])
def test_constant_offset(bf, prec, offset, norm):
    """The centred correlation does not depend on a constant added to the series (an
    invariant the oracle pins); every form stays within its tolerance when the 4 s, 512 Hz
    unit-variance strain-like series is raised or lowered far past its fluctuations.  Under
    the raw normalisation the level enters the normaliser and rho shrinks accordingly; the
    forms keep the raw frame there and are held to the same bound."""
    p = bank_params("small_strain")
    x32 = (small_strain_series() + offset).astype(np.float32)
    x64 = x32.astype(np.float64)
    g, _ = _run(bf, p, x32, prec, norm=norm)
    orc = O.search(x64, p, norm=norm)
    st = check_against_oracle(x64, p, g, orc, prec, f"offset {offset}/{norm}/{prec}",
                              norm=norm)
    print(f"offset {offset} {norm} {prec}: {st}")


@pytest.mark.parametrize("prec", PRECS)
def test_small_strain_full(bf, prec):
    """4 s at 512 Hz, bank 16x16, L = 512: every one of the 1537 offsets."""
    p = bank_params("small_strain")
    x32 = small_strain_series().astype(np.float32)
    x64 = x32.astype(np.float64)
    g, _ = _run(bf, p, x32, prec)
    orc = O.search(x64, p)
    st = check_against_oracle(x64, p, g, orc, prec, f"small_strain/{prec}")
    check_hist(g, orc["m"], orc["degen"], TOL[prec], 256, 0.0, 1.0, f"small_strain/{prec}")
    assert np.allclose(g["spectrum"], orc["spectrum"], rtol=TOL[prec], atol=0)
    print(f"small_strain {prec}: {st}")


def _edge_series(n, seed, L):
    x = white_noise(n, seed)
    x[n // 3: n // 3 + L + 5] = 1.25            # constant run -> degenerate windows
    x[n // 2: n // 2 + L + 2] = 0.0             # zero run -> degenerate windows
    x[(2 * n) // 3] = np.nan                     # NaN -> L windows degenerate
    x[(2 * n) // 3 + 3 * L] = np.inf
    return x.astype(np.float32)


SMALL = {
    # name: (bank, n, norm, t_block, edge cases)
    "ragged": (BankParams(fs=128.0, L=48, n_f0=5, n_fdot=7, f0_min=3.0, f0_max=40.0,
                          fdot_min=-30.0, fdot_max=25.0), 1500, "centred", 1, True),
    "L_odd": (BankParams(fs=100.0, L=37, n_f0=3, n_fdot=40, f0_min=4.0, f0_max=30.0,
                         fdot_min=-50.0, fdot_max=50.0), 700, "centred", 1, False),
    "W_is_1": (BankParams(fs=64.0, L=64, n_f0=4, n_fdot=16, f0_min=2.0, f0_max=20.0,
                          fdot_min=-10.0, fdot_max=10.0), 64, "centred", 1, False),
    "sharded_raw": (BankParams(fs=256.0, L=100, n_f0=7, n_fdot=24, f0_min=5.0, f0_max=80.0,
                               fdot_min=-60.0, fdot_max=60.0, shard_index=1, shard_count=3),
                    2000, "raw", 1, True),
    "t_block": (BankParams(fs=200.0, L=50, n_f0=6, n_fdot=9, f0_min=3.0, f0_max=60.0,
                           fdot_min=-40.0, fdot_max=40.0), 1600, "centred", 7, True),
    "wide_bins": (BankParams(fs=128.0, L=64, n_f0=3, n_fdot=150, f0_min=5.0, f0_max=50.0,
                             fdot_min=-80.0, fdot_max=80.0), 1200, "centred", 1, False),
}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", sorted(SMALL))
def test_small_shapes(bf, name, prec):
    p, n, norm, t_block, edges = SMALL[name]
    x32 = _edge_series(n, 7, p.L) if edges else white_noise(n, 8).astype(np.float32)
    x64 = x32.astype(np.float64)
    g, bank = _run(bf, p, x32, prec, t_block=t_block, norm=norm, hist_bins=64)
    orc = O.search(x64, p, norm=norm, hist_bins=64)
    st = check_against_oracle(x64, p, g, orc, prec, f"{name}/{prec}", t_block=t_block,
                              norm=norm)
    check_hist(g, orc["m"], orc["degen"], TOL[prec], 64, 0.0, 1.0, f"{name}/{prec}")
    if edges:
        assert st["n_degenerate"] > 0
    if t_block > 1:
        want = O.decimate(orc["S"], t_block)
        got = g["spec"].T.astype(np.float64)
        pos = want > 0
        floor = 1.0 / np.sqrt(p.L)
        tol = float(tolerance(prec, x64, p.L, orc["offsets"]).max())
        assert np.all(np.abs(got[pos] - want[pos]) <= tol * np.maximum(want[pos], floor))
        assert np.all(got[~pos] == 0.0)
    W = n - p.L + 1
    # spectrum: time mean of the undecimated spectrogram
    assert np.allclose(g["spectrum"], orc["spectrum"], rtol=TOL[prec], atol=1e-12)
    assert bank.k_offset == O.grid(p).k_global[0]
    assert g["max_abs"].shape == (W,)


@pytest.mark.parametrize("prec", PRECS)
def test_batch_equals_single_bitwise(bf, prec):
    """Uneven series (and a time-randomised control) in one batch give exactly the outputs
    of searching each alone."""
    p = BankParams(fs=256.0, L=96, n_f0=6, n_fdot=20, f0_min=5.0, f0_max=90.0,
                   fdot_min=-70.0, fdot_max=70.0)
    xs = [_edge_series(3000, 1, p.L), white_noise(96, 2).astype(np.float32),
          white_noise(1777, 3).astype(np.float32)]
    xs.append(time_randomised(xs[2], 103))
    bank = bf.bank_create(p, prec)
    prm = bf.make_params(t_block=3, hist_bins=32)
    xt = [torch.from_numpy(x).cuda() for x in xs]
    batch = [to_np(o) for o in bf.search_batch(bank, xt, prm)]
    single = [to_np(bf.search_segment(bank, x, prm)) for x in xt]
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(batch, single)):
        for k in a:
            assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), (i, k)


def test_determinism(bf):
    p = bank_params("small_strain")
    x32 = small_strain_series().astype(np.float32)
    a, _ = _run(bf, p, x32, "bf16x3")
    b, _ = _run(bf, p, x32, "bf16x3")
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


@pytest.mark.parametrize("prec", PRECS)
def test_on_grid_recovery(bf, prec):
    """A bank template's chirp (amplitude 0.5) injected at sample 666 into unit noise is
    found at exactly that offset and template."""
    p = bank_params("small_strain")
    gr = O.grid(p)
    k = 3 * 16 + 11
    for seed in (1, 2):
        x = white_noise(2048, seed)
        sig, _ = chirp_samples(2048, p.fs, 666 / p.fs, gr.f0[k], gr.fdot[k])
        x32 = (x + 0.5 * sig).astype(np.float32)
        g, _ = _run(bf, p, x32, prec)
        i = int(np.argmax(g["max_abs"]))
        assert i == 666 and g["argmax"][i] == k, (seed, i, g["argmax"][i])


def _glitch_series():
    """4 s at 512 Hz of unit noise with a stretch 64 times quieter (offsets 1500..2999) and a
    short burst of loud samples just before it, inside the same work item's strip and the
    same FFT block: windows of the quiet stretch see a strip peak ~250 times their RMS."""
    x = white_noise(4096, 41)
    x[1500:3000] /= 64.0
    x[1480:1484] = [40.0, -55.0, 62.0, -47.0]
    return x.astype(np.float32)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("norm", ["centred", "raw"])
def test_glitch_next_to_quiet_windows(bf, prec, norm):
    """Every offset of a series whose strips mix a loud burst with quiet windows, every form
    against its bound (F16F6's grows with the strip peak-to-window-RMS ratio)."""
    p = bank_params("small_strain")
    x32 = _glitch_series()
    x64 = x32.astype(np.float64)
    g, _ = _run(bf, p, x32, prec, norm=norm)
    orc = O.search(x64, p, norm=norm)
    st = check_against_oracle(x64, p, g, orc, prec, f"glitch/{norm}/{prec}", norm=norm)
    print(f"glitch {norm} {prec}: {st}")


def _sample_offsets(W, centre, n_block, n_rand, seed):
    rng = np.random.default_rng(seed)
    blk = np.arange(max(0, centre - n_block // 2), min(W, centre + n_block // 2))
    rnd = rng.choice(W, n_rand, replace=False)
    return np.unique(np.concatenate([blk, rnd, [0, W - 1]]))


@pytest.fixture(scope="module")
def strain_oracle():
    """The FP64 oracle on 2,048 offsets of the strain-like series (a block of 512 around the
    injection, seeded random picks, both ends), computed once for every form."""
    p = bank_params("strain")
    x32 = strain_series()
    W = x32.shape[0] - p.L + 1
    offs = _sample_offsets(W, 49152, 512, 1534, seed=22)
    print(f"strain oracle: {offs.shape[0]} offsets", flush=True)
    return p, x32, O.search(x32.astype(np.float64), p, offsets=offs)


@pytest.mark.parametrize("prec", PRECS)
def test_strain_full_size_sampled(bf, prec, strain_oracle):
    """32 s at 4096 Hz against 65,536 templates of L = 4096, at full size; the oracle checks
    2,048 offsets: a contiguous block around the injection, random offsets and the two
    ends."""
    p, x32, orc = strain_oracle
    x64 = x32.astype(np.float64)
    g, _ = _run(bf, p, x32, prec)
    W = x32.shape[0] - p.L + 1
    st = check_against_oracle(x64, p, g, orc, prec, f"strain/{prec}")
    # properties at every offset
    assert np.array_equal(g["hist"], O.histogram(g["max_abs"].astype(np.float64),
                                                 g["argmax"] < 0, 256, 0.0, 1.0))
    spec = g["spec"].T.astype(np.float64)          # [offset][bin]
    assert np.array_equal(spec.max(axis=1), g["max_abs"].astype(np.float64))
    assert np.allclose(g["spectrum"] * W, spec.sum(axis=0), rtol=1e-9, atol=0)
    assert np.all(g["max_abs"] <= 1.0 + 1e-5)
    print(f"strain {prec}: {st}")


@pytest.fixture(scope="module")
def light_curve_oracle():
    """The FP64 oracle on 1,024 offsets of the light curve and 1,024 of its control (a block
    of 256 plus seeded random picks and the ends of each), computed once for every form."""
    p = bank_params("light_curve_share")
    x = light_curve_series()
    xc = light_curve_series(control=True)
    W = x.shape[0] - p.L + 1
    offs = [_sample_offsets(W, W // 2, 256, 766, seed=33), _sample_offsets(W, W // 3, 256, 766, 34)]
    print(f"light-curve oracle: {[o.shape[0] for o in offs]} offsets", flush=True)
    orcs = O.search_many([x.astype(np.float64), xc.astype(np.float64)], p, offs)
    return p, x, xc, orcs


@pytest.mark.parametrize("prec", PRECS)
def test_light_curve_share_with_control_sampled(bf, prec, light_curve_oracle):
    """One GPU's 720,000-template share (L = 2000) against the 64 s light curve and its
    time-randomised control in one batch; the oracle checks 1,024 sampled offsets of each."""
    p, x, xc, orcs = light_curve_oracle
    bank = bf.bank_create(p, prec)
    prm = bf.make_params()
    outs = bf.search_batch(bank, [torch.from_numpy(x).cuda(), torch.from_numpy(xc).cuda()], prm)
    torch.cuda.synchronize()
    g = [to_np(o) for o in outs]
    del bank
    for gi, oi, xi, lab in zip(g, orcs, (x, xc), ("data", "control")):
        st = check_against_oracle(xi.astype(np.float64), p, gi, oi, prec, f"light_curve/{lab}/{prec}")
        assert np.array_equal(gi["hist"], O.histogram(gi["max_abs"].astype(np.float64),
                                                      gi["argmax"] < 0, 256, 0.0, 1.0))
        print(f"light_curve {lab} {prec}: {st}")
    # the control keeps the value histogram of the data
    assert np.array_equal(np.sort(x), np.sort(xc))


SHAPES = {"fp32": ["2x4", "1x8"], "bf16x3": ["2x4", "1x8", "2x8", "2x4i", "2x8i"],
          "f16x2": ["2x4", "2x8", "2x8i"]}


@pytest.mark.parametrize("prec,shape", [(p, s) for p in SHAPES for s in SHAPES[p]])
def test_tile_shapes_bitwise_equal(bf, prec, shape, monkeypatch):
    """Every compiled tile shape of the contraction kernel gives bit-identical outputs: the
    accumulation order of each correlation does not depend on the tiling, and every merge of
    partial maxima and sums is exact."""
    p, n, norm, t_block, edges = SMALL["ragged"]
    x32 = _edge_series(3000, 11, p.L)
    monkeypatch.setenv("BF_TILE", "2x4")
    ref, _ = _run(bf, p, x32, prec, t_block=3, hist_bins=64)
    monkeypatch.setenv("BF_TILE", shape)
    got, _ = _run(bf, p, x32, prec, t_block=3, hist_bins=64)
    for k in ref:
        assert np.array_equal(ref[k].view(np.uint8), got[k].view(np.uint8)), (shape, k)
    big = bank_params("small_strain")
    xb = small_strain_series().astype(np.float32)
    monkeypatch.setenv("BF_TILE", shape)
    g, _ = _run(bf, big, xb, prec)
    orc = O.search(xb.astype(np.float64), big)
    check_against_oracle(xb.astype(np.float64), big, g, orc, prec, f"small_strain/{prec}/{shape}")


def test_search_on_a_side_stream(bf):
    """A search enqueued on another stream than torch's current one, with the workspace and
    outputs allocated by the binding: memory allocated and written on the current stream right
    after the call must not reuse those buffers while the search runs."""
    p, n, norm, t_block, edges = SMALL["ragged"]
    x32 = _edge_series(20000, 12, p.L)
    bank = bf.bank_create(p, "fp32")
    prm = bf.make_params(t_block=1, hist_bins=64)
    x = torch.from_numpy(x32).cuda()
    ref = to_np(bf.search_segment(bank, x, prm))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        out = bf.search_segment(bank, x, prm, stream=side)
        # the binding dropped its workspace at return; fill fresh memory on the current stream
        junk = [torch.full((1 << 16,), float("nan"), device="cuda") for _ in range(64)]
        side.synchronize()
        torch.cuda.synchronize()
        got = to_np(out)
        for k in ref:
            assert np.array_equal(ref[k].view(np.uint8), got[k].view(np.uint8)), k
        del junk, out


@pytest.mark.parametrize("points", [1024, 2048, 4096])
def test_fft_shorter_transforms(bf, points, monkeypatch):
    """The FFT form's general kernel, selected by BF_FFT_POINTS = N < 8192 (the library uses
    N = 8192 for every template length): the L = 512 small strain-like bank at every offset,
    and the ragged 48-tap shape with degenerate windows, against the FP64 oracle."""
    monkeypatch.setenv("BF_FFT_POINTS", str(points))
    p = bank_params("small_strain")
    x32 = small_strain_series().astype(np.float32)
    x64 = x32.astype(np.float64)
    g, bank = _run(bf, p, x32, "fft")
    assert bf.bank_bytes(bf.make_desc(p, "fft")) == 256 * (points // 2 + 2) * 8 + 256
    orc = O.search(x64, p)
    st = check_against_oracle(x64, p, g, orc, "fft", f"small_strain/N={points}")
    assert np.allclose(g["spectrum"], orc["spectrum"], rtol=TOL["fft"], atol=0)
    pr, n, norm, t_block, _ = SMALL["ragged"]
    xr = _edge_series(n, 7, pr.L)
    gr, _ = _run(bf, pr, xr, "fft", t_block=t_block, norm=norm, hist_bins=64)
    orr = O.search(xr.astype(np.float64), pr, norm=norm, hist_bins=64)
    st2 = check_against_oracle(xr.astype(np.float64), pr, gr, orr, "fft", f"ragged/N={points}",
                               norm=norm)
    assert st2["n_degenerate"] > 0
    print(f"N = {points}: {st}; ragged {st2}")
