"""The identity behind the single-pass tail search's prediction of sigma (Sec. 2.2: the
variance of the matched-filter output follows from the spectra by Parseval's theorem).

For a template h of L taps and a series z (zero outside its samples), the sum over every
shift tau of (sum_n h[n] z[tau + n])^2 equals sum over the lags |l| < L of R_h(l) R_z(l),
R the autocorrelations, and, on N >= 2L - 1 points, (1/N) sum_f |H(f)|^2 Q(f) with Q the
cosine transform of R_z over those lags.  The library computes exactly these three
ingredients (the lag sums of the locally normalised series, their cosine transform, and the
template power spectrum) to bound which correlations its single pass keeps; the pass's
results never depend on the prediction, only its running time does, so the GPU path is
checked by equality with the two-pass search instead (tests/test_gpu_tails.py).  Here the
identity itself is checked by brute force in float64, with N the library's choice for the
direct forms (the power of two >= 2L - 1 within [1024, 8192]) and for the FFT form (8192).
"""
import numpy as np
import pytest


def _brute(h, z):
    # every shift with any overlap: full correlation of the zero-padded series
    c = np.correlate(np.concatenate([np.zeros(len(h) - 1), z, np.zeros(len(h) - 1)]), h, "valid")
    return float(np.sum(c * c))


def _lags(v, L):
    n = len(v)
    return np.array([np.dot(v[: n - l], v[l:]) for l in range(L)])


def _parseval(h, z, N):
    L = len(h)
    rz = _lags(z, L)                                   # R_z(l), l = 0 .. L - 1
    f = np.arange(N // 2 + 1)
    ang = 2.0 * np.pi * np.outer(f, np.arange(L)) / N
    q = rz[0] + 2.0 * np.sum(rz[None, 1:] * np.cos(ang[:, 1:]), axis=1)   # Q(f), real
    H = np.fft.rfft(h, N)
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    if N % 2 == 0:
        w[-1] = 1.0                                    # f = 0 and N / 2 appear once
    return float(np.sum(w * np.abs(H) ** 2 * q) / N)


def _lag_form(h, z):
    L = len(h)
    rh, rz = _lags(h, L), _lags(z, L)
    return float(rh[0] * rz[0] + 2.0 * np.sum(rh[1:] * rz[1:]))


@pytest.mark.parametrize("L,n,N", [(37, 300, 1024), (500, 2000, 1024), (1000, 3000, 2048),
                                   (2000, 9000, 8192)])
def test_parseval_prediction_identity(L, n, N):
    rng = np.random.default_rng(L + n)
    h = rng.standard_normal(L)
    h -= h.mean()
    h /= np.linalg.norm(h)
    z = rng.standard_normal(n) * (1.0 + 0.5 * np.sin(np.arange(n) / 97.0))
    brute = _brute(h, z)
    assert _lag_form(h, z) == pytest.approx(brute, rel=1e-11)
    assert _parseval(h, z, N) == pytest.approx(brute, rel=1e-10)


def test_parseval_needs_enough_points():
    """With fewer than 2L - 1 points the lags wrap round and the identity fails: the reason
    the library never predicts on fewer."""
    rng = np.random.default_rng(5)
    L = 700
    h = rng.standard_normal(L)
    z = rng.standard_normal(2500)
    brute = _brute(h, z)
    assert _parseval(h, z, 2048) == pytest.approx(brute, rel=1e-10)
    assert abs(_parseval(h, z, 1024) - brute) > 1e-6 * abs(brute)
