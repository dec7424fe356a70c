"""GPU test of the batched light-curve workload: uneven series and their time-randomised
controls in one search against the 512 x 512 bank (262,144 templates, L = 2000).

The six shortest of the 42 seeded light curves (with their controls, twelve series in one
batch) are searched; two of them are checked against the FP64 oracle on sampled offsets,
one against a single-series search bit for bit, and the averaged spectrum is the mean of the
per-series spectra.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bfly_oracle as O  # noqa: E402
from synth import bank_params, light_curve_batch  # noqa: E402
from tests.parity_util import TOL, check_against_oracle, to_np  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_01685_amd import bfly
    bfly.lib()
    return bfly


@pytest.mark.parametrize("prec", ["bf16x3"])
def test_batched_light_curves_with_controls(bf, prec):
    p = bank_params("light_curve_batch")
    batch = light_curve_batch()
    series = sorted({e["series"] for e in batch},
                    key=lambda i: batch[2 * i]["x"].shape[0])[:6]
    picked = [e for e in batch if e["series"] in series]
    assert len(picked) == 12 and sum(e["control"] for e in picked) == 6
    bank = bf.bank_create(p, prec)
    prm = bf.make_params(t_block=1)
    xs = [torch.from_numpy(e["x"]).cuda() for e in picked]
    outs = [to_np(o) for o in bf.search_batch(bank, xs, prm)]
    torch.cuda.synchronize()
    # two series (a light curve and another's control) against the oracle
    rng = np.random.default_rng(44)
    checks = [0, 7]
    offs, x64s = [], []
    for i in checks:
        W = picked[i]["x"].shape[0] - p.L + 1
        offs.append(np.unique(np.concatenate([np.arange(100, 116), rng.choice(W, 16, replace=False)])))
        x64s.append(picked[i]["x"].astype(np.float64))
    orcs = O.search_many(x64s, p, offs)
    for i, orc, x64 in zip(checks, orcs, x64s):
        st = check_against_oracle(x64, p, outs[i], orc, TOL[prec], f"batch/{picked[i]['name']}")
        print(picked[i]["name"], st)
    # a batch member equals the same series searched alone
    alone = to_np(bf.search_segment(bank, xs[5], prm))
    torch.cuda.synchronize()
    for k in alone:
        assert np.array_equal(alone[k].view(np.uint8), outs[5][k].view(np.uint8)), k
    # the averaged spectrum over the light curves (not the controls)
    data = [o for o, e in zip(outs, picked) if not e["control"]]
    avg = O.average_spectrum([o["spectrum"] for o in data])
    assert np.allclose(avg, np.mean(np.stack([o["spectrum"] for o in data]), axis=0))
    assert avg.shape == (p.n_f0,) and np.all(avg > 0)
    # histograms: every non-degenerate offset counted once, controls included
    for o, e in zip(outs, picked):
        W = e["x"].shape[0] - p.L + 1
        assert int(o["hist"].sum()) + int(o["n_degenerate"][0]) == W
