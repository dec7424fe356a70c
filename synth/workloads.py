"""The five workloads: bank parameters and seeded series, traces and controls.

Seeds: the small strain-like series draws its noise from seed 1, the 32 s strain-like series
from seed 2 (control permutation seed 102), the 64 s light curve from seed 3 (control 103);
the 42-light-curve batch draws per-series data seeds 400 + i and control seeds 1400 + i;
the serving trace draws its arrivals from seed 500 and each segment's noise from 5000 + i.
"""

from __future__ import annotations

from dataclasses import dataclass, asdict, replace

import numpy as np

from .series import chirp_samples, white_noise, kolmogorov_light_curve, time_randomised


@dataclass(frozen=True)
class BankParams:
    """An (f0, fdot) grid of 1 s chirp templates, f0-major.

    Both axes are inclusive linspaces.  Shard ``shard_index`` of ``shard_count`` owns the
    contiguous f0 index range [s*n_f0//S, (s+1)*n_f0//S); (0, 1) is the whole bank.
    """
    fs: float
    L: int
    n_f0: int
    n_fdot: int
    f0_min: float
    f0_max: float
    fdot_min: float
    fdot_max: float
    shard_index: int = 0
    shard_count: int = 1

    def as_dict(self) -> dict:
        return asdict(self)

    def with_(self, **kw) -> "BankParams":
        return replace(self, **kw)

    @property
    def f0_lo(self) -> int:
        return self.shard_index * self.n_f0 // self.shard_count

    @property
    def f0_hi(self) -> int:
        return (self.shard_index + 1) * self.n_f0 // self.shard_count

    @property
    def n_bins(self) -> int:
        return self.f0_hi - self.f0_lo

    @property
    def K(self) -> int:
        return self.n_bins * self.n_fdot


_BANKS = {
    "small_strain": BankParams(fs=512.0, L=512, n_f0=16, n_fdot=16, f0_min=20.0,
                               f0_max=200.0, fdot_min=-100.0, fdot_max=100.0),
    "strain": BankParams(fs=4096.0, L=4096, n_f0=256, n_fdot=256, f0_min=50.0, f0_max=2000.0,
                         fdot_min=-2000.0, fdot_max=2000.0),
    # One GPU's share of an 8.64M-template bank: 2880 f0 x 3000 fdot split 12 ways by f0.
    "light_curve_share": BankParams(fs=2000.0, L=2000, n_f0=2880, n_fdot=3000, f0_min=10.0,
                                    f0_max=1000.0, fdot_min=-1000.0, fdot_max=1000.0,
                                    shard_index=0, shard_count=12),
    "light_curve_batch": BankParams(fs=2000.0, L=2000, n_f0=512, n_fdot=512, f0_min=10.0,
                                    f0_max=1000.0, fdot_min=-1000.0, fdot_max=1000.0),
    "serving": BankParams(fs=4096.0, L=4096, n_f0=512, n_fdot=512, f0_min=50.0, f0_max=2000.0,
                          fdot_min=-2000.0, fdot_max=2000.0),
}

WORKLOADS = {
    "small_strain": "4 s at 512 Hz, f64 white noise + chirp (60 Hz, +40 Hz/s, A=0.5, "
                    "t=1.3 s); bank 16x16 L=512",
    "strain": "strain-like: 32 s at 4096 Hz, f32 white noise + chirp (100 Hz, +150 Hz/s, "
              "SNR 8, t=12 s); bank 256x256 L=4096",
    "light_curve_share": "light-curve bank share: 64 s Poisson counts in 0.5 ms bins, 2000/s, "
                         "Kolmogorov envelope; shard 0/12 of 2880x3000 (720,000 templates) "
                         "L=2000; + shuffled control",
    "light_curve_batch": "batch: 42 light curves 20-200 s, 500-5000 counts/s, each + "
                         "shuffled control; bank 512x512 L=2000",
    "serving": "serving: two-channel 4096 Hz strain segments 1-64 s, 30% with chirps, 50/s "
               "Poisson arrivals; bank 512x512 L=4096",
}


def bank_params(workload: str) -> BankParams:
    return _BANKS[workload]


def small_strain_series() -> np.ndarray:
    """2048 samples (4 s at 512 Hz), float64: unit white noise + 0.5 * chirp(60, +40) at 1.3 s."""
    x = white_noise(2048, seed=1)
    sig, _ = chirp_samples(2048, 512.0, start=1.3, f0=60.0, fdot=40.0)
    return x + 0.5 * sig


def _snr_amplitude(fs: float, f0: float, fdot: float, snr: float) -> float:
    """Amplitude A with A*||c|| = snr for the unit-amplitude 1 s chirp c at unit noise."""
    n = int(round(fs))
    c, _ = chirp_samples(n, fs, 0.0, f0, fdot)
    return snr / float(np.linalg.norm(c))


def strain_series() -> np.ndarray:
    """131072 samples (32 s at 4096 Hz), float32: unit noise + SNR-8 chirp(100, +150) at 12 s."""
    fs = 4096.0
    x = white_noise(131072, seed=2)
    sig, _ = chirp_samples(131072, fs, start=12.0, f0=100.0, fdot=150.0)
    x = x + _snr_amplitude(fs, 100.0, 150.0, 8.0) * sig
    return x.astype(np.float32)


def light_curve_series(control: bool = False) -> np.ndarray:
    """128000 standardised photon-count bins (64 s at 0.5 ms), float32; or its control."""
    x = kolmogorov_light_curve(128000, rate=2000.0, seed=3)
    return time_randomised(x, seed=103) if control else x


def light_curve_batch() -> list[dict]:
    """42 light curves of 20-200 s at 500-5000 counts/s, each followed by its control.

    Returns 84 dicts {name, x, series, control} in the order data_0, control_0, data_1, ...
    """
    rng = np.random.default_rng(4)
    dur = rng.uniform(20.0, 200.0, 42)
    rate = rng.uniform(500.0, 5000.0, 42)
    out = []
    for i in range(42):
        n = int(round(dur[i] * 2000.0))
        x = kolmogorov_light_curve(n, rate=float(rate[i]), seed=400 + i)
        out.append({"name": f"grb{i:02d}", "x": x, "series": i, "control": False})
        out.append({"name": f"grb{i:02d}_ctl", "x": time_randomised(x, seed=1400 + i),
                    "series": i, "control": True})
    return out


def serving_trace(n_segments: int = 256, rate_scale: float = 1.0) -> list[dict]:
    """Seeded arrival trace: Poisson arrivals at 50/s (times ``rate_scale``).

    Each entry: arrival time (s), channel, n samples, and an optional chirp injection
    (f0, fdot, snr, start).  Draw order per segment is fixed so the trace is reproducible.
    """
    rng = np.random.default_rng(500)
    t = 0.0
    out = []
    for i in range(n_segments):
        t += rng.exponential(0.02 / rate_scale)
        ch = int(rng.integers(0, 2))
        dur = rng.uniform(1.0, 64.0)
        inj = bool(rng.random() < 0.3)
        f0 = rng.uniform(50.0, 1000.0)
        fdot = rng.uniform(-500.0, 500.0)
        snr = rng.uniform(6.0, 12.0)
        start = rng.uniform(0.0, max(dur - 1.0, 0.0))
        out.append({"i": i, "t_arrival": t, "channel": ch, "n": int(round(4096.0 * dur)),
                    "inject": inj, "f0": f0, "fdot": fdot, "snr": snr, "start": start})
    return out


def serving_segment(entry: dict) -> np.ndarray:
    """The float32 samples of one trace entry: unit noise (seed 5000+i) + optional chirp."""
    fs = 4096.0
    n = entry["n"]
    x = white_noise(n, seed=5000 + entry["i"])
    if entry["inject"]:
        sig, _ = chirp_samples(n, fs, entry["start"], entry["f0"], entry["fdot"])
        x = x + _snr_amplitude(fs, entry["f0"], entry["fdot"], entry["snr"]) * sig
    return x.astype(np.float32)
