"""FP64 CPU oracle for butterfly filtering -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this module.
The GPU library never calls it and shares no code with it.

It computes, plainly and slowly, what the butterfly-filtering search computes (van Putten,
"GPU-accelerated broadband analysis of multi-messenger light curves of GRBs", Sec. 2):

* a bank of 1 s chirp templates over an (f0, fdot) grid covering ascending and descending
  chirps (Sec. 2.1; abstract);
* matched filtering of a series against every template at every time offset (Sec. 2.1),
  normalised per window to a correlation coefficient rho;
* the butterfly output: per offset, max |rho| over the bank and the template reaching it,
  whose maxima are histogrammed beside a time-randomised control (Fig. 2 caption; Sec. 2.2);
* the chirp-based spectrogram: per offset and f0 bin, max |rho| over the fdot templates of
  that bin, and its time average, the broadband spectrum (Sec. 2.1; Fig. 1 caption).

The paper gives no formula for the template, the normalisation, the grid, the spectrogram or
the tie rule.  The readings used (one chirp per template with phase f0 t + fdot t^2/2 from the
template start, zero-mean unit-norm templates, centred window norm, inclusive f0-major
linspace grid, f0 grid index as the spectrogram frequency key, lowest index on ties,
degenerate-window rule) are listed with their reasons in the design notes; each function
below names the reading it applies.

Everything is float64.  The correlation numerator is a plain matrix product of the template
matrix with the window (Hankel) matrix; the window energy is a two-pass centred sum per
window (no prefix sums), so it is independent of how the GPU computes it.

Parity status: every function is pinned by the CPU tests (tests/pins.py), none is "parity
unpinned": templates by hand-derived closed forms and mean/norm identities; the numerator by
numpy.correlate, scipy's FFT correlation and its own FFT path; search and search_many (one
core: several series, chunks of the bank, sharded banks, the runner-up |rho|) by pure-Python
brute force and invariants; rho_at by brute force at given pairs; sigma and the tails by
brute force and Parseval's theorem; the coincidence by pairwise loops.  Planted mistakes in
each (tests/test_oracle_mutants.py) fail at least one pin.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

DEGENERATE_REL = 1e-12  # a window is degenerate when E <= DEGENERATE_REL * R (reading 13)


# ---------------------------------------------------------------------------------------
# O1: the grid.
# ---------------------------------------------------------------------------------------
@dataclass(frozen=True)
class Grid:
    f0: np.ndarray        # [K] start frequency of template k (Hz)
    fdot: np.ndarray      # [K] frequency slope of template k (Hz/s)
    bin: np.ndarray       # [K] spectrogram bin = local f0 index
    k_global: np.ndarray  # [K] index in the unsharded f0-major bank
    n_bins: int
    n_fdot: int


def grid(p) -> Grid:
    """The (f0, fdot) template grid of bank parameters ``p`` (reading 5: inclusive linspace,
    f0-major, k = i*n_fdot + j; a shard owns a contiguous f0 index range)."""
    f0_axis = np.linspace(p.f0_min, p.f0_max, p.n_f0)
    fd_axis = np.linspace(p.fdot_min, p.fdot_max, p.n_fdot)
    lo = p.shard_index * p.n_f0 // p.shard_count
    hi = (p.shard_index + 1) * p.n_f0 // p.shard_count
    nb = hi - lo
    f0 = np.repeat(f0_axis[lo:hi], p.n_fdot)
    fdot = np.tile(fd_axis, nb)
    b = np.repeat(np.arange(nb), p.n_fdot)
    kg = lo * p.n_fdot + np.arange(nb * p.n_fdot)
    return Grid(f0=f0, fdot=fdot, bin=b, k_global=kg, n_bins=nb, n_fdot=p.n_fdot)


# ---------------------------------------------------------------------------------------
# O2: templates.
# ---------------------------------------------------------------------------------------
def templates(fs: float, L: int, f0: np.ndarray, fdot: np.ndarray) -> np.ndarray:
    """Zero-mean, unit-L2-norm chirp templates, float64 [K, L] (Sec. 2.1; readings 1, 2).

    Template k samples cos(2 pi phi) at t_n = n/fs, n = 0..L-1, with phi = f0 t + fdot t^2/2
    (phase zero at the template start; rectangular window).  The phase is reduced mod 1
    before the cosine.  The mean over the L samples is removed and the result scaled to
    unit norm.  A template whose centred norm vanishes cannot be normalised and is rejected.
    """
    f0 = np.asarray(f0, dtype=np.float64).reshape(-1, 1)
    fdot = np.asarray(fdot, dtype=np.float64).reshape(-1, 1)
    t = np.arange(L, dtype=np.float64) / fs
    phi = f0 * t + 0.5 * fdot * (t * t)
    phi = phi - np.floor(phi)
    c = np.cos(2.0 * np.pi * phi)
    c = c - c.mean(axis=1, keepdims=True)
    nrm = np.sqrt((c * c).sum(axis=1, keepdims=True))
    if np.any(nrm <= 1e-9 * math.sqrt(L)):
        raise ValueError("degenerate template: zero centred norm")
    return c / nrm


def bank_templates(p, k_lo: int = 0, k_hi: int | None = None) -> np.ndarray:
    """Templates of the (local) bank index range [k_lo, k_hi) of parameters ``p``."""
    g = grid(p)
    k_hi = g.f0.shape[0] if k_hi is None else k_hi
    return templates(p.fs, p.L, g.f0[k_lo:k_hi], g.fdot[k_lo:k_hi])


# ---------------------------------------------------------------------------------------
# O3: correlation numerator.
# ---------------------------------------------------------------------------------------
def windows(x: np.ndarray, L: int, offsets: np.ndarray | None = None) -> np.ndarray:
    """The Hankel window matrix X[tau, n] = x[tau + n], float64 [len(offsets), L]."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[0] < L:
        raise ValueError("series shorter than the template")
    v = sliding_window_view(x, L)
    return v if offsets is None else v[np.asarray(offsets)]


def numerator(x: np.ndarray, H: np.ndarray, offsets: np.ndarray | None = None) -> np.ndarray:
    """d[tau, k] = sum_n H[k, n] x[tau + n] (matched filtering, Sec. 2.1), float64."""
    Xw = windows(x, H.shape[1], offsets)
    return Xw @ H.T


def numerator_fft(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """The same numerator for one template through zero-padded FFTs (Sec. 2.2 computes the
    correlations with the FFT).  Linear correlation: size >= N + L - 1.  Returns d[W]."""
    x = np.asarray(x, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    n, L = x.shape[0], h.shape[0]
    size = 1 << int(math.ceil(math.log2(n + L - 1)))
    X = np.fft.rfft(x, size)
    Hf = np.fft.rfft(h, size)
    full = np.fft.irfft(X * np.conj(Hf), size)
    return full[: n - L + 1]


# ---------------------------------------------------------------------------------------
# O4, O5: window energies and degenerate windows.
# ---------------------------------------------------------------------------------------
def window_energy(x: np.ndarray, L: int, offsets: np.ndarray | None = None,
                  norm: str = "centred") -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Per-window energy E, raw energy R and the degenerate flag (readings 3 and 13).

    Centred (default): E = sum_n (x[tau+n] - mean_tau)^2, two passes per window.
    Raw: E = R = sum_n x[tau+n]^2.
    Degenerate: R == 0, or E <= 1e-12 * R, or the window holds a non-finite value.
    """
    Xw = windows(x, L, offsets)
    finite = np.all(np.isfinite(Xw), axis=1)
    Xf = np.where(np.isfinite(Xw), Xw, 0.0)
    R = (Xf * Xf).sum(axis=1)
    if norm == "centred":
        mu = Xf.sum(axis=1, keepdims=True) / L
        dev = Xf - mu
        E = (dev * dev).sum(axis=1)
    elif norm == "raw":
        E = R.copy()
    else:
        raise ValueError(norm)
    degen = (~finite) | (R == 0.0) | (E <= DEGENERATE_REL * R)
    return E, R, degen


# ---------------------------------------------------------------------------------------
# O6-O9: correlation coefficient, butterfly output, spectrogram, histogram.
# ---------------------------------------------------------------------------------------
def rho(x: np.ndarray, H: np.ndarray, offsets: np.ndarray | None = None,
        norm: str = "centred") -> tuple[np.ndarray, np.ndarray]:
    """rho[tau, k] = d[tau, k] / sqrt(E_tau); rows of degenerate windows are 0 (reading 13).
    Returns (rho, degenerate)."""
    E, _, degen = window_energy(x, H.shape[1], offsets, norm)
    Xw = windows(x, H.shape[1], offsets)
    Xw = np.where(np.isfinite(Xw), Xw, 0.0)
    d = Xw @ H.T
    r = np.zeros_like(d)
    ok = ~degen
    r[ok] = d[ok] / np.sqrt(E[ok])[:, None]
    return r, degen


def hist_bin(v: np.ndarray, bins: int, lo: float, hi: float) -> np.ndarray:
    """Bin index min(B-1, max(0, floor((v - lo)/(hi - lo) * B))) (reading 11)."""
    q = np.floor((np.asarray(v, dtype=np.float64) - lo) / (hi - lo) * bins)
    return np.clip(q, 0, bins - 1).astype(np.int64)


def histogram(m: np.ndarray, degen: np.ndarray, bins: int = 256, lo: float = 0.0,
              hi: float = 1.0) -> np.ndarray:
    """Histogram of the butterfly maxima over non-degenerate offsets (Fig. 2 caption)."""
    b = hist_bin(m[~degen], bins, lo, hi)
    return np.bincount(b, minlength=bins).astype(np.int64)


def decimate(S: np.ndarray, t_block: int) -> np.ndarray:
    """Row-block maximum of a spectrogram: out[r, i] = max over tau in block r of S[tau, i]."""
    W = S.shape[0]
    nr = -(-W // t_block)
    out = np.zeros((nr, S.shape[1]), dtype=S.dtype)
    for r in range(nr):
        out[r] = S[r * t_block:(r + 1) * t_block].max(axis=0)
    return out


def search(x: np.ndarray, p, offsets: np.ndarray | None = None, norm: str = "centred",
           hist_bins: int = 256, hist_lo: float = 0.0, hist_hi: float = 1.0,
           k_chunk: int | None = None) -> dict:
    """The whole search of one series on the offsets given (all W offsets when ``offsets``
    is None); ``search_many`` with a single series.

    Returns a dict with
      m[T]        max_k |rho(tau, k)|           (butterfly output; 0 on degenerate windows)
      a[T]        the smallest global k reaching m (reading 12); -1 on degenerate windows
      second[T]   the second largest |rho(tau, k)| over the bank (equal to m when two
                  templates tie for the maximum; -1 for a one-template bank; 0 on degenerate
                  windows): m - second is the top-2 margin that decides where an argmax is
                  unique at a given tolerance (reading 22)
      S[T, B]     max over the fdot templates of f0 bin i of |rho|  (chirp spectrogram)
      degen[T]    degenerate-window flags
      hist[B_h]   histogram of m over non-degenerate offsets
      n_degenerate
      spectrum[B] time mean of S over the offsets given (over all W: the broadband spectrum)
      offsets[T]
    """
    return search_many([x], p, [offsets], norm, hist_bins, hist_lo, hist_hi, k_chunk)[0]


def search_many(xs: list, p, offsets_list: list | None = None, norm: str = "centred",
                hist_bins: int = 256, hist_lo: float = 0.0, hist_hi: float = 1.0,
                k_chunk: int | None = None) -> list:
    """``search`` for several series (each on its own offsets, None = all), generating each
    template chunk once for all of them.  Returns one dict per series, as ``search``.

    Templates are generated and applied in chunks of whole f0 bins (``k_chunk`` templates,
    rounded down to whole bins; by default sized to bound memory); the reductions merge the
    chunks in increasing k with strict comparisons, so ties keep the smallest k."""
    g = grid(p)
    L = p.L
    nb, nfd = g.n_bins, g.n_fdot
    if offsets_list is None:
        offsets_list = [None] * len(xs)
    series = []
    for x, offs in zip(xs, offsets_list):
        x = np.asarray(x, dtype=np.float64)
        W = x.shape[0] - L + 1
        if W < 1:
            raise ValueError("series shorter than the template")
        offs = np.arange(W) if offs is None else np.asarray(offs, dtype=np.int64)
        T = offs.shape[0]
        E, _, degen = window_energy(x, L, offs, norm)
        Xw = windows(x, L, offs)
        Xw = np.where(np.isfinite(Xw), Xw, 0.0)
        scale = np.zeros(T)
        scale[~degen] = 1.0 / np.sqrt(E[~degen])
        series.append({"Xw": Xw, "scale": scale, "degen": degen, "offsets": offs,
                       "m": np.full(T, -1.0), "second": np.full(T, -1.0),
                       "a": np.full(T, -1, dtype=np.int64), "S": np.zeros((T, nb))})

    T_all = sum(q["offsets"].shape[0] for q in series)
    if k_chunk is None:
        k_chunk = max(nfd, (1 << 22) // max(T_all, 1) // nfd * nfd)
    bins_per_chunk = max(1, k_chunk // nfd)
    for b0 in range(0, nb, bins_per_chunk):
        b1 = min(nb, b0 + bins_per_chunk)
        k0, k1 = b0 * nfd, b1 * nfd
        H = templates(p.fs, L, g.f0[k0:k1], g.fdot[k0:k1])
        for q in series:
            T = q["offsets"].shape[0]
            r = np.abs((q["Xw"] @ H.T) * q["scale"][:, None])          # |rho|
            q["S"][:, b0:b1] = r.reshape(T, b1 - b0, nfd).max(axis=2)
            j = np.argmax(r, axis=1)                          # first maximum in this chunk
            v = r[np.arange(T), j]
            # the chunk's second largest value (ties count twice)
            c2 = np.partition(r, -2, axis=1)[:, -2] if k1 - k0 > 1 else np.full(T, -1.0)
            # top two of {m, second, v, c2}: the larger maximum, and the larger of the
            # smaller maximum and both runners-up
            q["second"] = np.maximum(np.minimum(q["m"], v), np.maximum(q["second"], c2))
            better = v > q["m"]
            q["m"][better] = v[better]
            q["a"][better] = g.k_global[k0 + j[better]]

    out = []
    for q in series:
        degen = q["degen"]
        m, a, S, second = q["m"], q["a"], q["S"], q["second"]
        m[degen] = 0.0
        a[degen] = -1
        S[degen] = 0.0
        second[degen] = 0.0
        out.append({
            "m": m, "a": a, "second": second, "S": S, "degen": degen,
            "hist": histogram(m, degen, hist_bins, hist_lo, hist_hi),
            "n_degenerate": int(degen.sum()),
            "spectrum": S.mean(axis=0),
            "offsets": q["offsets"],
        })
    return out


def average_spectrum(spectra: list[np.ndarray]) -> np.ndarray:
    """Mean of per-series spectra (Fig. 1 caption: a spectrum averaged over 42 light curves;
    reading 10: each series contributes its own time mean, uneven lengths are not pooled)."""
    return np.mean(np.stack(spectra), axis=0)


def rho_at(x: np.ndarray, p, offsets: np.ndarray, k_global: np.ndarray,
           norm: str = "centred") -> np.ndarray:
    """|rho(tau_i, k_i)| in float64 for given (offset, global template index) pairs; used to
    check that a reported argmax really reaches the reported maximum.  k_i = -1 gives 0, as
    does a degenerate window."""
    x = np.asarray(x, dtype=np.float64)
    g = grid(p)
    offs = np.asarray(offsets, dtype=np.int64)
    kg = np.asarray(k_global, dtype=np.int64)
    out = np.zeros(offs.shape[0])
    ok = kg >= 0
    if not ok.any():
        return out
    kl = kg[ok] - int(g.k_global[0])
    if np.any(kl < 0) or np.any(kl >= g.f0.shape[0]):
        raise ValueError("template index outside the bank")
    H = templates(p.fs, p.L, g.f0[kl], g.fdot[kl])
    E, _, degen = window_energy(x, p.L, offs[ok], norm)
    Xw = windows(x, p.L, offs[ok])
    Xw = np.where(np.isfinite(Xw), Xw, 0.0)
    d = np.einsum("ij,ij->i", Xw, H)
    r = np.zeros(d.shape[0])
    r[~degen] = np.abs(d[~degen]) / np.sqrt(E[~degen])
    out[ok] = r
    return out


# ---------------------------------------------------------------------------------------
# O14-O15: sigma of rho per template, the kappa-sigma tails and their pseudo-spectrum
# (Sec. 2.2; Fig. 5 and Fig. 6 captions).
# ---------------------------------------------------------------------------------------
def sigma_tails(x: np.ndarray, p, kappa: float, norm: str = "centred") -> dict:
    """Per-template sigma, the tails above kappa * sigma, and the tail counts per f0 bin.

    sigma_k = sqrt(mean over the non-degenerate offsets of rho_k(tau)^2): the spread of the
    matched-filter output of template k over the series (Sec. 2.2, Fig. 5 caption).  A zero-
    mean template gives an output of zero mean, so its mean square is its variance -- the
    energy the paper obtains from the spectra by Parseval's theorem (reading 23).
    Tails: every (tau, k) with |rho_k(tau)| > kappa * sigma_k, strictly (reading 24; the
    magnitude, as for every other reduction, reading 4).
    Pseudo-spectrum: the number of tails per f0 bin (Fig. 6 caption; reading 9's key).

    Returns sigma[K], n_ok, the tails sorted by (tau, k): tau[T], k[T] (global index),
    rho[T] (signed), counts[n_bins], and degen[W].
    """
    x = np.asarray(x, dtype=np.float64)
    g = grid(p)
    L = p.L
    W = x.shape[0] - L + 1
    if W < 1:
        raise ValueError("series shorter than the template")
    E, _, degen = window_energy(x, L, None, norm)
    ok = ~degen
    n_ok = int(ok.sum())
    Xw = windows(x, L)
    Xw = np.where(np.isfinite(Xw), Xw, 0.0)
    scale = np.zeros(W)
    scale[ok] = 1.0 / np.sqrt(E[ok])
    K = g.f0.shape[0]
    nfd = g.n_fdot
    sig = np.zeros(K)
    counts = np.zeros(g.n_bins, dtype=np.int64)
    taus, ks, rhos = [], [], []
    step = max(nfd, (1 << 22) // W // nfd * nfd)
    for k0 in range(0, K, step):
        k1 = min(K, k0 + step)
        H = templates(p.fs, L, g.f0[k0:k1], g.fdot[k0:k1])
        r = (Xw @ H.T) * scale[:, None]                  # rho [W, k1-k0], 0 if degenerate
        s = np.sqrt((r * r).sum(axis=0) / n_ok) if n_ok else np.zeros(k1 - k0)
        sig[k0:k1] = s
        t, j = np.nonzero(np.abs(r) > kappa * s[None, :])
        taus.append(t)
        ks.append(g.k_global[k0 + j])
        rhos.append(r[t, j])
        counts += np.bincount(g.bin[k0 + j], minlength=g.n_bins)
    tau = np.concatenate(taus).astype(np.int64)
    k = np.concatenate(ks).astype(np.int64)
    rh = np.concatenate(rhos)
    order = np.lexsort((k, tau))
    return {"sigma": sig, "n_ok": n_ok, "tau": tau[order], "k": k[order], "rho": rh[order],
            "counts": counts, "degen": degen}


# ---------------------------------------------------------------------------------------
# O16: two-detector coincidence of tails (Fig. 6 caption).
# ---------------------------------------------------------------------------------------
def template_f0(p, k_global: np.ndarray) -> np.ndarray:
    """Start frequency f0 of global template indices (reading 5: inclusive f0-major grid)."""
    i = np.asarray(k_global, dtype=np.int64) // p.n_fdot
    f0_axis = np.linspace(p.f0_min, p.f0_max, p.n_f0)
    return f0_axis[i]


def coincidences(tails_a: dict, tails_b: dict, p, dtau: int, df: float) -> dict:
    """Tails of two simultaneous channels (e.g. two detectors) searched with the same bank.

    A tail (tau, k) of channel A is coincident when channel B has a tail (tau', k') with
    |tau - tau'| <= dtau and |f0(k) - f0(k')| <= df (reading 25: "simultaneous" means within
    dtau offsets, the frequency key is the template's f0).  Returns, per f0 bin, the number
    of coincident tails of A (counts_a) and of B (counts_b) -- the pseudo-spectra by
    simultaneous counts -- and the number of coincident pairs.
    Plain double loop over the two lists, grouped by offset.
    """
    g = grid(p)
    ta, ka = np.asarray(tails_a["tau"], np.int64), np.asarray(tails_a["k"], np.int64)
    tb, kb = np.asarray(tails_b["tau"], np.int64), np.asarray(tails_b["k"], np.int64)
    fa, fb = template_f0(p, ka), template_f0(p, kb)
    lo = int(g.k_global[0]) // p.n_fdot                    # first f0 index of the share
    hit_a = np.zeros(ta.shape[0], dtype=bool)
    hit_b = np.zeros(tb.shape[0], dtype=bool)
    n_pairs = 0
    by_tau = {}
    for j, t in enumerate(tb.tolist()):
        by_tau.setdefault(t, []).append(j)
    for i in range(ta.shape[0]):
        for t in range(int(ta[i]) - dtau, int(ta[i]) + dtau + 1):
            for j in by_tau.get(t, ()):
                if abs(fa[i] - fb[j]) <= df:
                    hit_a[i] = True
                    hit_b[j] = True
                    n_pairs += 1
    counts_a = np.bincount(ka[hit_a] // p.n_fdot - lo, minlength=g.n_bins).astype(np.int64)
    counts_b = np.bincount(kb[hit_b] // p.n_fdot - lo, minlength=g.n_bins).astype(np.int64)
    return {"counts_a": counts_a, "counts_b": counts_b, "n_pairs": n_pairs}
