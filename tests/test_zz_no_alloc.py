"""bf_search_segment_noalloc against bf_search_segment, through the C ABI.

The no-allocation entry point runs the same kernels with the library's device scratch array
as workspace, so its outputs must equal the allocating entry point's bit for bit.  Two calls
in a row, the second on a shorter series, check that what the first call left in the array
does not leak into the second; a series too long for the array is refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import BankParams, white_noise  # noqa: E402

pytestmark = pytest.mark.gpu

FORMS = ["fp32", "bf16x3", "f16f6", "fft"]
KEYS = ("max_abs", "argmax", "spec", "spectrum", "hist", "n_degenerate")


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_01685_amd import bfly
    bfly.lib()
    return bfly


def _series(n, seed, L):
    x = white_noise(n, seed)
    x[n // 3: n // 3 + L + 3] = 0.75          # constant run: degenerate windows
    x[(2 * n) // 3] = np.nan
    return torch.from_numpy(x.astype(np.float32)).cuda()


@pytest.mark.parametrize("prec", FORMS)
def test_noalloc_equals_segment(bf, prec):
    p = BankParams(fs=512.0, L=300, n_f0=9, n_fdot=20, f0_min=10.0, f0_max=150.0,
                   fdot_min=-90.0, fdot_max=90.0)
    bank = bf.bank_create(p, prec)
    prm = bf.make_params(t_block=3, hist_bins=64)
    for n, seed in ((9000, 31), (2500, 32)):          # the second call is shorter
        print(f"noalloc {prec}: n = {n}, seed = {seed}", flush=True)
        x = _series(n, seed, p.L)
        ref = bf.search_segment(bank, x, prm)
        got = bf.alloc_outputs(bank, n, prm, x.device)
        for t in got.values():
            t.fill_(-7)                                 # every output must be written
        bf.search_segment_noalloc(bank, x, got, prm)
        torch.cuda.synchronize()
        for k in KEYS:
            a = ref[k].cpu().numpy()
            b = got[k].cpu().numpy()
            assert a.shape == b.shape, (prec, n, k)
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (prec, n, k)
        assert int(ref["n_degenerate"][0]) > 0


def test_noalloc_refuses_oversized_series(bf):
    p = BankParams(fs=4096.0, L=4096, n_f0=2, n_fdot=4, f0_min=50.0, f0_max=60.0,
                   fdot_min=-5.0, fdot_max=5.0)
    bank = bf.bank_create(p, "fp32")
    prm = bf.make_params()
    n = 1 << 20                                          # needs ~52 MB of workspace
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    out = bf.alloc_outputs(bank, n, prm, x.device)
    with pytest.raises(bf.BflyError) as e:
        bf.search_segment_noalloc(bank, x, out, prm)
    assert e.value.status == bf.BF_EINVAL and "no-allocation" in str(e.value)
