"""Helpers for comparing the GPU library's outputs with the FP64 oracle.

Error bounds (max relative error of the butterfly output m and of the spectrogram S, over
non-degenerate offsets, relative to max(value, floor)), fixed from each form's rounding model
before any measurement and not tuned to measured errors:

* FP32 1e-5, BF16 hi/lo split 1e-4 (the bounds stated for the method); the FFT form computes in
  float32: 1e-5.  F16F8 and F16F6 are held to the BF16 split's 1e-4.
* Rounding model for the two forms whose data are rounded coarsely.  A form that rounds each
  operand value with relative error at most u (uniform, independent) perturbs
  d = sum_n h_n x_n by a sum of L independent terms; for a unit-norm template of amplitude
  about sqrt(2/L) the perturbation of rho has standard deviation u_eff * sqrt(2/3) / sqrt(L),
  u_eff^2 the sum of u^2 over the rounded operands.  Relative to the floor 1/sqrt(L) (the noise
  scale of |rho|) six standard deviations are 6 sqrt(2/3) u_eff = 4.9 u_eff:
    F16X2: data as one fp16 (u = 2^-11), templates split to ~2^-22:   4.9 * 2^-11  = 2.4e-3
    FP8:   template and data e4m3 codes (u = 2^-4 each):           4.9 * 2^-3.5 = 0.43
* Forms that round against a scale shared by many windows lose accuracy on a quiet window next
  to loud samples, in proportion to the ratio of that scale to the window's RMS:
  F16F6 codes the data residual y - fp16(y) in e2m3 at a fixed quantum: the strip is scaled so
  that its largest sample lies in (7680, 15360], and a residual below 1 keeps an absolute error
  up to 1/16, but never more than the residual itself (at most the fp16 rounding, F16X2's
  bound).  A window whose RMS is PR times below its strip's peak therefore carries an extra
  error of 6 * (1/16) / sqrt(3) * PR / 7680 = 2.8e-5 * PR relative to the floor; its bound is
  max(1e-4, min(2.8e-5 * PR, 2.5e-3)).  PR is the largest |x - mu| within one work item
  (1024 offsets) before the window and one work item plus the template length after it, over
  the window's RMS about the series mean mu.
  The FFT form transforms whole overlap-save blocks in float32: an output's rounding error is
  about u sqrt(2 log2 N) times the block's RMS for each of the three transforms it passes
  (template, block, inverse), u = 2^-24, N = 8192: 6 sqrt(3) * 2^-24 * sqrt(26) * BR =
  3.2e-6 * BR relative to the floor, BR the RMS of the block over the window's RMS; its bound
  is max(1e-5, 3.2e-6 * BR), BR taken from the largest energy of any N consecutive samples
  within N of the window.

The floor is the noise scale of |rho| for the window: 1/sqrt(L) under the centred norm, and
nu/sqrt(L) under the raw norm, nu^2 = (E_c + L (mean_tau - mu)^2) / R, the share of the raw
window energy R held by its fluctuation about the series mean mu (E_c its centred energy).
Every form stages the series minus its (rounded) mean, so its rounding acts on exactly that
fluctuation.

Argmax (reading 22): wherever the FP64 top-2 margin m - second exceeds 2 * tol * max(m, floor),
the GPU's template must be the FP64 argmax exactly; everywhere, the template the GPU reports
must reach the FP64 maximum within 2 * tol.  Both agreement rates are returned.
"""

from __future__ import annotations

import numpy as np

from oracle import bfly_oracle as O

TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "f16x2": 2.4e-3, "fp8": 0.43, "fft": 1e-5, "f16f8": 1e-4,
       "f16f6": 1e-4}
F16F6_PR_COEF = 2.8e-5       # F16F6: extra bound per unit of strip peak-to-window-RMS ratio
F16F6_CAP = 2.5e-3           # F16F6: never worse than fp16 data (F16X2's bound)
FFT_BR_COEF = 3.2e-6         # FFT form: bound per unit of block-RMS-to-window-RMS ratio
STRIP_REACH = 1024           # offsets of one work item: the strip reaches this far past tau
FFT_N = 8192                 # largest real FFT length of the FFT form


def to_np(out: dict) -> dict:
    r = {}
    for k, v in out.items():
        a = v.detach().cpu().numpy()
        if k == "hist":
            a = a.view(np.uint32).astype(np.int64)
        r[k] = a
    return r


def window_floor(x64, L: int, offs: np.ndarray, norm: str) -> np.ndarray:
    """The comparison floor of each offset (see the module docstring)."""
    if norm == "centred":
        return np.full(offs.shape[0], 1.0 / np.sqrt(L))
    x = np.asarray(x64, dtype=np.float64)
    fin = np.isfinite(x)
    mu = float(x[fin].mean()) if fin.any() else 0.0
    Ec, R, _ = O.window_energy(x, L, offs, "centred")
    Xw = O.windows(x, L, offs)
    mean_tau = np.where(np.isfinite(Xw), Xw, 0.0).sum(axis=1) / L
    nu2 = (Ec + L * (mean_tau - mu) ** 2) / np.where(R > 0, R, 1.0)
    return np.sqrt(np.clip(nu2, 0.0, 1.0)) / np.sqrt(L)


def peak_ratio(x64, L: int, offs: np.ndarray) -> np.ndarray:
    """Per offset: the largest |x - mu| within the reach of its strip over the window's RMS
    about mu (mu the series mean over finite samples); inf for an all-zero window."""
    x = np.asarray(x64, dtype=np.float64)
    fin = np.isfinite(x)
    mu = float(x[fin].mean()) if fin.any() else 0.0
    dev = np.where(fin, np.abs(x - mu), 0.0)
    n = x.shape[0]
    out = np.empty(offs.shape[0])
    sq = np.concatenate([[0.0], np.cumsum(dev * dev)])
    for i, t in enumerate(offs):
        lo = max(0, int(t) - STRIP_REACH)
        hi = min(n, int(t) + STRIP_REACH + L)
        rms = np.sqrt((sq[t + L] - sq[t]) / L)
        out[i] = dev[lo:hi].max() / rms if rms > 0 else np.inf
    return out


def block_ratio(x64, L: int, offs: np.ndarray) -> np.ndarray:
    """Per offset: the RMS of the loudest FFT_N consecutive samples within FFT_N of the window,
    over the window's RMS (both about the series mean); inf for an all-zero window."""
    x = np.asarray(x64, dtype=np.float64)
    fin = np.isfinite(x)
    mu = float(x[fin].mean()) if fin.any() else 0.0
    d2 = np.where(fin, (x - mu) ** 2, 0.0)
    n = x.shape[0]
    sq = np.concatenate([[0.0], np.cumsum(d2)])
    nb = min(FFT_N, n)
    blk = sq[nb:] - sq[:-nb]                     # energy of x[i, i + nb)
    out = np.empty(offs.shape[0])
    for i, t in enumerate(offs):
        lo = max(0, int(t) - FFT_N)
        hi = min(blk.shape[0], int(t) + FFT_N)
        e_w = (sq[t + L] - sq[t]) / L
        out[i] = np.sqrt(blk[lo:hi].max() / nb / e_w) if e_w > 0 else np.inf
    return out


def tolerance(prec: str, x64, L: int, offs: np.ndarray) -> np.ndarray:
    """Per-offset bound of a form (see the module docstring)."""
    tol = np.full(offs.shape[0], TOL[prec])
    if prec == "f16f6":
        tol = np.maximum(tol, np.minimum(F16F6_PR_COEF * peak_ratio(x64, L, offs), F16F6_CAP))
    elif prec == "fft":
        tol = np.maximum(tol, FFT_BR_COEF * block_ratio(x64, L, offs))
    return tol


def check_against_oracle(x64, p, g: dict, orc: dict, prec: str, label: str,
                         t_block: int = 1, check_spec: bool = True,
                         norm: str = "centred") -> dict:
    """Element-by-element comparison on the oracle's offsets for precision form ``prec``
    (bounds, floor and argmax rule: module docstring).  Returns summary statistics."""
    offs = orc["offsets"]
    deg = orc["degen"]
    m_g = g["max_abs"][offs].astype(np.float64)
    a_g = g["argmax"][offs].astype(np.int64)
    assert np.all(a_g[deg] == -1), f"{label}: degenerate windows must report argmax -1"
    assert np.all(m_g[deg] == 0.0), f"{label}: degenerate windows must report m = 0"
    ok = ~deg
    floor = window_floor(x64, p.L, offs, norm)[ok]
    tol = tolerance(prec, x64, p.L, offs)[ok]
    m_o = orc["m"][ok]
    den = np.maximum(m_o, floor)
    rel = np.abs(m_g[ok] - m_o) / den
    max_rel = float(rel.max()) if rel.size else 0.0
    excess = rel / tol
    assert float(excess.max(initial=0.0)) <= 1.0, \
        f"{label}: relative error of m {rel[np.argmax(excess)]:.3e} > {tol[np.argmax(excess)]:.1e}"
    # the reported template reaches the reported value, and the FP64 maximum within 2 tol
    assert np.all(a_g[ok] >= 0)
    r_at = O.rho_at(x64, p, offs[ok], a_g[ok], norm=norm)
    gap = (m_o - r_at) / den
    assert float((gap / tol).max(initial=0.0)) <= 2.0, \
        f"{label}: reported argmax is {gap.max():.3e} below the maximum (> 2 tol)"
    assert np.all(np.abs(r_at - m_g[ok]) <= 2 * tol * den), f"{label}: |rho(a)| != m"
    # argmax must be exact where the FP64 top-2 margin exceeds 2 tol
    agree = a_g[ok] == orc["a"][ok]
    decisive = (m_o - orc["second"][ok]) > 2.0 * tol * den
    assert np.all(agree[decisive]), \
        f"{label}: argmax differs on {int((~agree & decisive).sum())} offsets whose FP64 " \
        f"top-2 margin exceeds 2 tol"
    stats = {"max_rel_m": max_rel, "n": int(offs.shape[0]), "n_degenerate": int(deg.sum()),
             "argmax_agreement": float(agree.mean()) if ok.any() else 1.0,
             "argmax_decisive": int(decisive.sum()),
             "argmax_agreement_decisive": float(agree[decisive].mean()) if decisive.any() else 1.0}
    if check_spec and t_block == 1 and "spec" in g:
        S_g = g["spec"][:, offs].T.astype(np.float64)       # spec is bin-major
        S_o = orc["S"]
        assert np.all(S_g[deg] == 0.0)
        relS = np.abs(S_g[ok] - S_o[ok]) / np.maximum(S_o[ok], floor[:, None])
        stats["max_rel_S"] = float(relS.max()) if relS.size else 0.0
        assert float((relS / tol[:, None]).max(initial=0.0)) <= 1.0, \
            f"{label}: max relative error of S {relS.max():.3e}"
    return stats


def check_hist(g: dict, orc_m: np.ndarray, orc_deg: np.ndarray, tol: float, bins: int,
               lo: float, hi: float, label: str) -> None:
    """The GPU histogram equals the floor-rule binning of the GPU's own m values exactly; and
    differs from the FP64 histogram only by entries within tol of a bin edge."""
    m = g["max_abs"].astype(np.float64)
    deg = g["argmax"] < 0
    assert np.array_equal(deg, orc_deg), f"{label}: degenerate sets differ"
    want = O.histogram(m, deg, bins, lo, hi)
    assert np.array_equal(g["hist"], want), f"{label}: histogram != binning of GPU m"
    ref = O.histogram(orc_m, orc_deg, bins, lo, hi)
    q = (orc_m[~orc_deg] - lo) / (hi - lo) * bins
    near = np.abs(q - np.round(q)) <= tol * bins * np.abs(orc_m[~orc_deg]) + 1e-12
    assert int(np.abs(g["hist"] - ref).sum()) <= 2 * int(near.sum()), \
        f"{label}: histogram differs beyond edge cases"
    assert int(g["n_degenerate"][0]) == int(orc_deg.sum())
