"""Helpers for comparing the GPU library's outputs with the FP64 oracle."""

from __future__ import annotations

import numpy as np

from oracle import bfly_oracle as O

# FP32 and the BF16 split: the bounds stated for the method.  The FP16 template split keeps
# the data as one fp16 (11-bit significand): each sample carries up to 2^-11 relative
# rounding, measured at up to 5.2e-4 relative on m and 6.6e-4 on small spectrogram entries
# (relative to the 1/sqrt(L) floor) on templates of 37-512 taps; its stated bound is 1e-3.
# FP8 (e4m3, 3 mantissa bits): a stated number.  Template and data
# codes each carry up to 2^-4 relative rounding, so a correlation carries a random error of
# about 0.05 / sqrt(L) in rho: about 1% of m at the median, and up to ~7% of m (~15% of a
# small spectrogram entry, relative to the 1/sqrt(L) floor) on templates of 37-64 taps.
# The FFT form computes in float32 (spectra, transforms, products): the FP32 bound.
TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "f16x2": 1e-3, "fp8": 0.2, "fft": 1e-5, "f16f8": 1e-4,
       "f16f6": 1e-4}


def to_np(out: dict) -> dict:
    r = {}
    for k, v in out.items():
        a = v.detach().cpu().numpy()
        if k == "hist":
            a = a.view(np.uint32).astype(np.int64)
        r[k] = a
    return r


def check_against_oracle(x64, p, g: dict, orc: dict, tol: float, label: str,
                         t_block: int = 1, check_spec: bool = True,
                         norm: str = "centred") -> dict:
    """Element-by-element comparison on the oracle's offsets.

    m: max relative error over non-degenerate offsets <= tol; the template the GPU reports
    reaches its value within 2*tol of the FP64 maximum (so argmax must agree wherever the
    FP64 top-2 margin exceeds 2*tol*m); degenerate windows give m = 0, a = -1, S = 0.
    S: relative error per entry <= tol (undecimated spectrogram, t_block == 1).
    Relative errors are taken against max(value, 1/sqrt(L)): 1/sqrt(L) is the scale of |rho|
    for noise, and it only binds where rho vanishes identically (e.g. a constant window under
    the raw norm, where every zero-mean template gives d = 0 up to rounding).
    Returns summary statistics."""
    offs = orc["offsets"]
    deg = orc["degen"]
    m_g = g["max_abs"][offs].astype(np.float64)
    a_g = g["argmax"][offs].astype(np.int64)
    assert np.all(a_g[deg] == -1), f"{label}: degenerate windows must report argmax -1"
    assert np.all(m_g[deg] == 0.0), f"{label}: degenerate windows must report m = 0"
    ok = ~deg
    floor = 1.0 / np.sqrt(p.L)
    m_o = orc["m"][ok]
    den = np.maximum(m_o, floor)
    rel = np.abs(m_g[ok] - m_o) / den
    max_rel = float(rel.max()) if rel.size else 0.0
    assert max_rel <= tol, f"{label}: max relative error of m {max_rel:.3e} > {tol:.1e}"
    # the reported template reaches the reported value
    r_at = O.rho_at(x64, p, offs[ok], a_g[ok], norm=norm)
    gap = (m_o - r_at) / den
    assert np.all(a_g[ok] >= 0)
    assert float(gap.max(initial=0.0)) <= 2 * tol, \
        f"{label}: reported argmax is {gap.max():.3e} below the maximum (> 2 tol)"
    assert np.all(np.abs(r_at - m_g[ok]) <= 2 * tol * den), f"{label}: |rho(a)| != m"
    agree = float(np.mean(a_g[ok] == orc["a"][ok])) if ok.any() else 1.0
    stats = {"max_rel_m": max_rel, "argmax_agreement": agree, "n": int(offs.shape[0]),
             "n_degenerate": int(deg.sum())}
    if check_spec and t_block == 1 and "spec" in g:
        S_g = g["spec"][:, offs].T.astype(np.float64)       # spec is bin-major
        S_o = orc["S"]
        assert np.all(S_g[deg] == 0.0)
        relS = np.abs(S_g[ok] - S_o[ok]) / np.maximum(S_o[ok], floor)
        stats["max_rel_S"] = float(relS.max()) if relS.size else 0.0
        assert stats["max_rel_S"] <= tol, f"{label}: max relative error of S {relS.max():.3e}"
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
