"""Elementary seeded generators: noise, injected chirps, photon-count light curves, controls.

The paper's inputs are BeppoSAX gamma-ray light curves (0.5 ms bins, about 1.26 photons per
bin on average; Sec. 2.1) and LIGO H1/L1 strain at 4096 Hz in 16 s segments (Sec. 2.2 and
the Fig. 5 caption).  Neither dataset is available here, so these functions make seeded
stand-ins with the same sampling, length and value statistics.
"""

from __future__ import annotations

import numpy as np


def chirp_samples(n_total: int, fs: float, start: float, f0: float, fdot: float,
                  duration: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """A unit-amplitude chirp placed in a series of ``n_total`` samples.

    The waveform is cos(2*pi*(f0*t' + fdot*t'**2/2)) with t' = n/fs - start, on the samples
    where 0 <= t' < duration (zero elsewhere).  Returns (signal[n_total], mask[n_total]).
    A non-integer ``start * fs`` is honoured: t' is evaluated at the sample times.
    """
    n = np.arange(n_total, dtype=np.float64)
    tp = n / fs - start
    mask = (tp >= 0.0) & (tp < duration)
    sig = np.zeros(n_total, dtype=np.float64)
    t = tp[mask]
    sig[mask] = np.cos(2.0 * np.pi * (f0 * t + 0.5 * fdot * t * t))
    return sig, mask


def white_noise(n: int, seed: int) -> np.ndarray:
    """Unit-variance white Gaussian noise (float64) from ``default_rng(seed)``.

    Whitened strain has a flat spectrum, so whitening is the identity on this stand-in.
    """
    return np.random.default_rng(seed).standard_normal(n)


def kolmogorov_envelope(n: int, rng: np.random.Generator) -> np.ndarray:
    """Zero-mean, unit-std Gaussian process with power spectrum proportional to f**(-5/3).

    Complex Gaussian Fourier coefficients are weighted by f**(-5/6) (the square root of the
    power law), the DC term is zeroed and the inverse real FFT is standardised.
    """
    nf = n // 2 + 1
    coef = rng.standard_normal(nf) + 1j * rng.standard_normal(nf)
    f = np.arange(nf, dtype=np.float64)
    w = np.zeros(nf)
    w[1:] = f[1:] ** (-5.0 / 6.0)
    g = np.fft.irfft(coef * w, n)
    g -= g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def kolmogorov_light_curve(n: int, rate: float, seed: int, dt: float = 5e-4,
                           depth: float = 0.5) -> np.ndarray:
    """Photon counts in bins of ``dt`` seconds, standardised and cast to float32.

    The rate is r(t) = rate * exp(depth*g - depth**2/2) with g the Kolmogorov envelope, a
    log-normal modulation whose mean is ``rate``.  Counts are Poisson(r*dt).  The series
    returned is (counts - mean)/std as float32 (mean-subtracted and normalised).
    """
    rng = np.random.default_rng(seed)
    g = kolmogorov_envelope(n, rng)
    r = rate * np.exp(depth * g - 0.5 * depth * depth)
    counts = rng.poisson(r * dt).astype(np.float64)
    c = counts - counts.mean()
    sd = c.std()
    if sd > 0:
        c /= sd
    return c.astype(np.float32)


def time_randomised(x: np.ndarray, seed: int) -> np.ndarray:
    """Time-randomised control: the samples of ``x`` in a seeded uniform random order.

    A permutation keeps the value histogram exactly (Sec. 2.2: time randomisation gives
    maximal-entropy data with the same histogram).  The permutation is drawn here, by the
    harness, and the permuted copy is then searched as an ordinary series.
    """
    perm = np.random.default_rng(seed).permutation(x.shape[0])
    return x[perm]
