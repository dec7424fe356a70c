"""GPU tests of the batched light-curve workload: 42 seeded light curves of uneven length and
their time-randomised controls searched in one launch (Fig. 1 caption: a spectrum averaged over
42 light curves).

* All 84 series in one bf_search_batch against the 512 x 512 bank (262,144 templates,
  L = 2000), for the BF16 split and plain FP32: four series (two light curves, two controls,
  the longest among them) against the FP64 oracle on sampled offsets, one batch member against
  the same series searched alone, bit for bit, and every histogram complete.
* The six shortest light curves and their controls against an 8 x 8 bank on the same ranges:
  every offset of every series against the oracle, each series' spectrum, and the spectrum
  averaged over the six light curves against the oracle's average of its full-length spectra.
"""
import os
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bfly_oracle as O  # noqa: E402
from synth import bank_params, light_curve_batch  # noqa: E402
from tests.parity_util import TOL, check_against_oracle, to_np, tolerance  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_01685_amd import bfly
    bfly.lib()
    return bfly


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _wait_with_progress(torch, label, poll_s=10.0):
    """Waits for the current stream while appending a line per poll to a progress file (when
    the run keeps a gpurun_out folder), so that a long search is not mistaken for a hang."""
    ev = torch.cuda.Event()
    ev.record()
    t0 = time.time()
    prog = os.path.join(ROOT, "gpurun_out")
    while not ev.query():
        time.sleep(0.05 if time.time() - t0 < poll_s else poll_s)
        if os.path.isdir(prog):
            with open(os.path.join(prog, "test_progress.log"), "a") as f:
                f.write(f"{label}: {time.time() - t0:.0f} s\n")
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def batch84():
    """The 84 series and the FP64 oracle on 96 sampled offsets (a block of 32 plus random
    picks) of four of them: the longest light curve, the shortest control, and two more."""
    p = bank_params("light_curve_batch")
    batch = light_curve_batch()
    lengths = [e["x"].shape[0] for e in batch]
    data = [i for i, e in enumerate(batch) if not e["control"]]
    ctl = [i for i, e in enumerate(batch) if e["control"]]
    checks = [max(data, key=lambda i: lengths[i]), min(ctl, key=lambda i: lengths[i]),
              data[17], ctl[30]]
    rng = np.random.default_rng(48)
    offs = []
    for i in checks:
        W = lengths[i] - p.L + 1
        blk = np.arange(W // 2, W // 2 + 32)
        offs.append(np.unique(np.concatenate([blk, rng.choice(W, 64, replace=False),
                                              [0, W - 1]])))
    print(f"batch oracle: series {checks}", flush=True)
    orcs = O.search_many([batch[i]["x"].astype(np.float64) for i in checks], p, offs)
    return p, batch, checks, orcs


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fft", "bf16x3", "fp32"])
def test_all_84_series_in_one_batch(bf, prec, batch84):
    p, batch, checks, orcs = batch84
    bank = bf.bank_create(p, prec)
    prm = bf.make_params(t_block=256)
    xs = [torch.from_numpy(e["x"]).cuda() for e in batch]
    print(f"84-series batch {prec}: {sum(x.shape[0] for x in xs)} samples", flush=True)
    outs_t = bf.search_batch(bank, xs, prm)
    _wait_with_progress(torch, f"84-series batch {prec}")
    outs = [to_np(o) for o in outs_t]
    del outs_t
    for i, orc in zip(checks, orcs):
        st = check_against_oracle(batch[i]["x"].astype(np.float64), p, outs[i], orc, prec,
                                  f"batch84/{batch[i]['name']}/{prec}", t_block=256)
        print(batch[i]["name"], st)
    # every offset of every series is counted once
    for o, e in zip(outs, batch):
        W = e["x"].shape[0] - p.L + 1
        assert int(o["hist"].sum()) + int(o["n_degenerate"][0]) == W
        assert o["spec"].shape == (p.n_f0, -(-W // 256))
    # a batch member equals the same series searched alone
    j = checks[2]
    alone = to_np(bf.search_segment(bank, xs[j], prm))
    torch.cuda.synchronize()
    for k in alone:
        assert np.array_equal(alone[k].view(np.uint8), outs[j][k].view(np.uint8)), k
    avg = O.average_spectrum([o["spectrum"] for o, e in zip(outs, batch) if not e["control"]])
    assert avg.shape == (p.n_f0,) and np.all(avg > 0)


@pytest.fixture(scope="module")
def small_bank_oracle():
    """Twelve uneven series: the opening 6,000 + 1,500 i samples of the six shortest light
    curves and of their controls (i = 0..5), and the FP64 oracle on every offset of each
    against an 8 x 8 bank on the batch ranges."""
    p = bank_params("light_curve_batch").with_(n_f0=8, n_fdot=8)
    batch = light_curve_batch()
    series = sorted({e["series"] for e in batch},
                    key=lambda i: batch[2 * i]["x"].shape[0])[:6]
    picked = []
    for r, i in enumerate(series):
        n = 6000 + 1500 * r
        for e in (batch[2 * i], batch[2 * i + 1]):
            picked.append({"name": e["name"], "control": e["control"], "x": e["x"][:n].copy()})
    orcs = [O.search(e["x"].astype(np.float64), p) for e in picked]
    return p, picked, orcs


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fft", "f16f6"])
def test_average_spectrum_small_bank(bf, prec, small_bank_oracle):
    p, picked, orcs = small_bank_oracle
    bank = bf.bank_create(p, prec)
    prm = bf.make_params(t_block=1)
    xs = [torch.from_numpy(e["x"]).cuda() for e in picked]
    outs = [to_np(o) for o in bf.search_batch(bank, xs, prm)]
    torch.cuda.synchronize()
    spectra_gpu, spectra_orc = [], []
    for o, e, orc in zip(outs, picked, orcs):
        x64 = e["x"].astype(np.float64)
        check_against_oracle(x64, p, o, orc, prec, f"small_bank/{e['name']}/{prec}")
        tol = float(tolerance(prec, x64, p.L, orc["offsets"]).max())
        assert np.allclose(o["spectrum"], orc["spectrum"], rtol=tol, atol=0), e["name"]
        if not e["control"]:
            spectra_gpu.append(o["spectrum"])
            spectra_orc.append(orc["spectrum"])
    avg_g = O.average_spectrum(spectra_gpu)
    avg_o = O.average_spectrum(spectra_orc)
    rel = np.abs(avg_g - avg_o) / avg_o
    print(f"average spectrum {prec}: max relative error {rel.max():.2e}")
    assert rel.max() <= TOL[prec], rel.max()
