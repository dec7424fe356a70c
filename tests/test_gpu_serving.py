"""GPU tests of the serving loop: continuous batching through the C ABI.

Each request's results must be identical, bit for bit, alone, in a mix of concurrent
requests, and from a direct batched search; admission waits for the HBM budget; cancel,
unknown tickets, over-budget requests and shutdown with pending work behave as declared.
Every tick replays a captured graph, so the mix test also checks many graph replays against
eager searches.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bfly_oracle as O  # noqa: E402
from synth import BankParams, white_noise, chirp_samples  # noqa: E402
from tests.parity_util import check_against_oracle  # noqa: E402

pytestmark = pytest.mark.gpu

P = BankParams(fs=1024.0, L=256, n_f0=24, n_fdot=20, f0_min=20.0, f0_max=400.0,
               fdot_min=-300.0, fdot_max=300.0)


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_01685_amd import bfly
    bfly.lib()
    return bfly


def _series(i, n):
    x = white_noise(n, 900 + i)
    if i % 3 == 0:
        sig, _ = chirp_samples(n, P.fs, 0.3 * n / P.fs, 100.0 + 5 * i, 50.0 - 7 * i)
        x = x + 0.4 * sig
    return x.astype(np.float32)


def _wait(bf, srv, tickets, timeout=120.0):
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            st = bf.poll(srv, t)[0]
            if st in ("done", "failed", "cancelled"):
                pending.discard(t)
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(pending)} requests still pending")
        time.sleep(0.001)


def _direct(bf, bank, x, prm):
    out = bf.search_segment(bank, torch.from_numpy(x).cuda(), prm)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in out.items()}
    r["hist"] = r["hist"].view(np.uint32)
    return r


def _same(a, b, label):
    for k in ("max_abs", "argmax", "spec", "spectrum", "hist", "n_degenerate"):
        assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), \
            (label, k)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fft", "f16f6", "f16f8", "f16x2", "fp8"])
def test_alone_equals_mix_equals_direct(bf, prec):
    bank = bf.bank_create(P, prec)
    prm = bf.make_params(t_block=4, hist_bins=64)
    srv = bf.server_create(bank, hbm_budget_bytes=256 << 20, max_slots=8, ticks_in_flight=2,
                           params=prm)
    lengths = [1000 + 733 * i for i in range(20)]
    xs = [_series(i, n) for i, n in enumerate(lengths)]
    probe = 7
    t = bf.submit(srv, xs[probe])
    _wait(bf, srv, [t])
    alone = bf.fetch(srv, t, lengths[probe])
    tickets = [bf.submit(srv, x) for x in xs]          # arrive while others run
    _wait(bf, srv, tickets)
    stats = bf.server_stats(srv)
    mix = [bf.fetch(srv, t, n) for t, n in zip(tickets, lengths)]
    _same(alone, mix[probe], "alone vs mix")
    for i in (0, 5, probe, 19):
        _same(mix[i], _direct(bf, bank, xs[i], prm), f"mix vs direct {i}")
    assert stats["ticks"] >= 3 and stats["done"] == 21
    # and the served results are right
    x64 = xs[probe].astype(np.float64)
    orc = O.search(x64, P)
    check_against_oracle(x64, P, mix[probe], orc, prec, f"served/{prec}", t_block=4)
    bf.server_destroy(srv)


def test_server_budget_beyond_device_memory(bf):
    """A budget larger than the device's memory cannot be allocated: BF_ENOMEM, and the
    library keeps working (a server created next serves a request correctly)."""
    bank = bf.bank_create(P, "bf16x3")
    prm = bf.make_params()
    total = torch.cuda.get_device_properties(0).total_memory
    with pytest.raises(bf.BflyError) as e:
        bf.server_create(bank, hbm_budget_bytes=4 * total, params=prm)
    assert e.value.status == bf.BF_ENOMEM
    srv = bf.server_create(bank, hbm_budget_bytes=64 << 20, max_slots=2, params=prm)
    x = _series(1, 5000)
    t = bf.submit(srv, x)
    _wait(bf, srv, [t])
    _same(bf.fetch(srv, t, 5000), _direct(bf, bank, x, prm), "after ENOMEM")
    bf.server_destroy(srv)


def test_budget_defers_admission(bf):
    bank = bf.bank_create(P, "bf16x3")
    prm = bf.make_params()
    n = 30000
    tmp = bf.server_create(bank, 64 << 20, params=prm)
    per = bf.server_request_bytes(tmp, n)
    bf.server_destroy(tmp)
    srv = bf.server_create(bank, hbm_budget_bytes=2 * per + 4096, max_slots=16,
                           ticks_in_flight=2, params=prm)
    xs = [_series(i, n) for i in range(8)]
    tickets = [bf.submit(srv, x) for x in xs]
    _wait(bf, srv, tickets)
    st = bf.server_stats(srv)
    assert st["done"] == 8 and st["queued"] == 0 and st["on_device"] == 0
    assert st["ticks"] >= 4          # at most two fit at a time
    # A request is stamped done before its memory is released, and one admitted into that
    # memory is stamped started after its launch: no instant sees three on the device.
    events = []
    for t in tickets:
        _, _, t_start, t_done = bf.poll(srv, t)
        assert 0 < t_start <= t_done
        events += [(t_start, 1), (t_done, -1)]
    live, peak = 0, 0
    for _, d in sorted(events, key=lambda e: (e[0], e[1])):   # ends before starts on ties
        live += d
        peak = max(peak, live)
    assert peak <= 2
    ref = _direct(bf, bank, xs[3], prm)
    _same(bf.fetch(srv, tickets[3], n), ref, "budget")
    bf.server_destroy(srv)


def test_errors_cancel_and_shutdown(bf):
    bank = bf.bank_create(P, "bf16x3")
    prm = bf.make_params()
    srv = bf.server_create(bank, hbm_budget_bytes=8 << 20, max_slots=2, ticks_in_flight=1,
                           params=prm)
    big = np.zeros(4_000_000, np.float32)
    with pytest.raises(bf.BflyError) as e:
        bf.submit(srv, big)
    assert e.value.status == bf.BF_EBUDGET
    with pytest.raises(bf.BflyError) as e:
        bf.submit(srv, np.zeros(100, np.float32))       # shorter than L
    assert e.value.status == bf.BF_EINVAL
    with pytest.raises(bf.BflyError) as e:
        bf.poll(srv, 123456)
    assert e.value.status == bf.BF_ENOTFOUND
    xs = [_series(i, 20000) for i in range(6)]
    tickets = [bf.submit(srv, x) for x in xs]
    bf.cancel(srv, tickets[-1])                        # still queued: dropped
    _wait(bf, srv, tickets)
    assert bf.poll(srv, tickets[-1])[0] == "cancelled"
    with pytest.raises(bf.BflyError) as e:
        bf.fetch(srv, tickets[-1], 20000)
    assert e.value.status == bf.BF_ECANCELED
    with pytest.raises(bf.BflyError) as e:
        bf.fetch(srv, tickets[-1], 20000)              # forgotten after the fetch
    assert e.value.status == bf.BF_ENOTFOUND
    r0 = bf.fetch(srv, tickets[0], 20000)
    assert r0["max_abs"].shape == (20000 - P.L + 1,)
    # shutdown with work pending: queued requests are dropped, running ones drain
    more = [bf.submit(srv, x) for x in xs]
    assert len(more) == 6
    t0 = time.time()
    bf.server_destroy(srv)
    assert time.time() - t0 < 60


def test_serving_trace_segments_against_oracle(bf):
    """Segments of the seeded two-channel strain trace (1-64 s at 4096 Hz, 30% with an
    injected chirp) served against the 512 x 512 bank of L = 4096 in the BF16 split form:
    sampled offsets of the two shortest injected and two shortest plain segments match the
    FP64 oracle, and a strong injected chirp's offset carries a larger maximum than the noise
    around it."""
    from synth import bank_params, serving_segment, serving_trace
    p = bank_params("serving")
    trace = serving_trace(64)
    inj = sorted([e for e in trace if e["inject"]], key=lambda e: e["n"])[:2]
    plain = sorted([e for e in trace if not e["inject"]], key=lambda e: e["n"])[:2]
    picked = inj + plain
    bank = bf.bank_create(p, "bf16x3")
    prm = bf.make_params(t_block=256)
    srv = bf.server_create(bank, hbm_budget_bytes=8 << 30, max_slots=8, ticks_in_flight=2,
                           params=prm)
    xs = [serving_segment(e) for e in picked]
    tickets = [bf.submit(srv, x) for x in xs]
    _wait(bf, srv, tickets, timeout=300.0)
    outs = [bf.fetch(srv, t, x.shape[0]) for t, x in zip(tickets, xs)]
    bf.server_destroy(srv)
    rng = np.random.default_rng(55)
    offs, x64s = [], []
    for e, x in zip(picked, xs):
        W = x.shape[0] - p.L + 1
        extra = [int(round(e["start"] * p.fs))] if e["inject"] else []
        o = np.unique(np.concatenate([rng.choice(W, 12, replace=False),
                                      [v for v in extra if 0 <= v < W], [0, W - 1]]))
        offs.append(o)
        x64s.append(x.astype(np.float64))
    orcs = O.search_many(x64s, p, offs)
    for e, out, orc, x64 in zip(picked, outs, orcs, x64s):
        g = {"max_abs": out["max_abs"], "argmax": out["argmax"]}
        st = check_against_oracle(x64, p, g, orc, "bf16x3", f"trace{e['i']}",
                                  check_spec=False)
        print(e["i"], e["inject"], st)
    for e, out in zip(inj, outs[:2]):
        t0 = int(round(e["start"] * p.fs))
        W = out["max_abs"].shape[0]
        if 0 <= t0 < W and e["snr"] >= 7.5:   # clear of grid mismatch at lower SNR
            near = out["max_abs"][max(0, t0 - 8):t0 + 9].max()
            lo, hi = max(0, t0 - 4096), min(W, t0 + 4096)
            ring = np.concatenate([out["max_abs"][lo:max(lo, t0 - 64)],
                                   out["max_abs"][min(hi, t0 + 64):hi]])
            assert near > np.median(ring), (e["i"], near, np.median(ring))
