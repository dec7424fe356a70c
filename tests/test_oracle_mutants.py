"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutant replaces one snippet of the oracle's source (a dropped term, a wrong sign or
index, a transposed operand, a wrong reduction) and is executed as a separate module; the
real oracle is untouched.  A snippet that no longer exists fails the test loudly.
"""
import os
import sys
import types

import pytest

from tests.pins import ALL_PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "bfly_oracle.py")

MUTANTS = {
    "average_pooled": ("return np.mean(np.stack(spectra), axis=0)",
                       "return np.mean(np.stack(spectra), axis=0) * 0 + np.median(np.stack(spectra), axis=0)"),
    "no_mean_removal": ("c = c - c.mean(axis=1, keepdims=True)", "c = c"),
    "dropped_half": ("phi = f0 * t + 0.5 * fdot * (t * t)", "phi = f0 * t + fdot * (t * t)"),
    "fdot_sign": ("phi = f0 * t + 0.5 * fdot * (t * t)", "phi = f0 * t - 0.5 * fdot * (t * t)"),
    "t_in_samples": ("t = np.arange(L, dtype=np.float64) / fs", "t = np.arange(L, dtype=np.float64)"),
    "convolution": ('r = np.abs((q["Xw"] @ H.T) * q["scale"][:, None])          # |rho|',
                    'r = np.abs((q["Xw"][:, ::-1] @ H.T) * q["scale"][:, None])          # |rho|'),
    "numerator_flip": ("    return Xw @ H.T\n", "    return Xw @ H[:, ::-1].T\n"),
    "raw_energy": ("dev = Xf - mu", "dev = Xf"),
    "norm_not_sqrt": ("scale[~degen] = 1.0 / np.sqrt(E[~degen])\n        series.append",
                      "scale[~degen] = 1.0 / E[~degen]\n        series.append"),
    "argmax_last": ("j = np.argmax(r, axis=1)                          # first",
                    "j = r.shape[1] - 1 - np.argmax(r[:, ::-1], axis=1)  # first"),
    "merge_ge": ('better = v > q["m"]', 'better = v >= q["m"]'),
    "fdot_major": ("f0 = np.repeat(f0_axis[lo:hi], p.n_fdot)\n    fdot = np.tile(fd_axis, nb)",
                   "f0 = np.tile(f0_axis[lo:hi], p.n_fdot)\n    fdot = np.repeat(fd_axis, nb)"),
    "linspace_open": ("fd_axis = np.linspace(p.fdot_min, p.fdot_max, p.n_fdot)",
                      "fd_axis = np.linspace(p.fdot_min, p.fdot_max, p.n_fdot, endpoint=False)"),
    "shard_index": ("kg = lo * p.n_fdot + np.arange(nb * p.n_fdot)", "kg = np.arange(nb * p.n_fdot)"),
    "hist_round": ("q = np.floor(", "q = np.round("),
    "hist_with_degenerate": ("b = hist_bin(m[~degen], bins, lo, hi)", "b = hist_bin(m, bins, lo, hi)"),
    "spec_transposed": ('q["S"][:, b0:b1] = r.reshape(T, b1 - b0, nfd).max(axis=2)',
                        'q["S"][:, b0:b1] = r.reshape(T, nfd, b1 - b0).max(axis=1)'),
    "nan_not_degenerate": ("degen = (~finite) | (R == 0.0)", "degen = (R == 0.0)"),
    "no_rel_threshold": ("| (E <= DEGENERATE_REL * R)", "| (E < 0.0)"),
    "window_shift": ("return v if offsets is None else v[np.asarray(offsets)]",
                     "return v[1:] if offsets is None else v[np.asarray(offsets) + 1]"),
    "spectrum_max": ('"spectrum": S.mean(axis=0)', '"spectrum": S.max(axis=0)'),
    "sigma_all_offsets": ("s = np.sqrt((r * r).sum(axis=0) / n_ok) if n_ok",
                          "s = np.sqrt((r * r).sum(axis=0) / W) if n_ok"),
    "sigma_squared": ("s = np.sqrt((r * r).sum(axis=0) / n_ok) if n_ok",
                      "s = ((r * r).sum(axis=0) / n_ok) if n_ok"),
    "sigma_of_numerator": ("r = (Xw @ H.T) * scale[:, None]                  # rho",
                           "r = (Xw @ H.T) * (scale[:, None] > 0)            # rho"),
    "tails_one_sided": ("t, j = np.nonzero(np.abs(r) > kappa * s[None, :])",
                        "t, j = np.nonzero(r > kappa * s[None, :])"),
    "tails_ge": ("t, j = np.nonzero(np.abs(r) > kappa * s[None, :])",
                 "t, j = np.nonzero(np.abs(r) >= kappa * s[None, :])"),
    "tails_local_index": ("ks.append(g.k_global[k0 + j])", "ks.append(k0 + j)"),
    "tail_counts_by_fdot": ("counts += np.bincount(g.bin[k0 + j], minlength=g.n_bins)",
                            "counts += np.bincount((k0 + j) // nfd % g.n_bins, minlength=g.n_bins)[::-1]"),
    "many_chunk_offset": ('q["a"][better] = g.k_global[k0 + j[better]]',
                          'q["a"][better] = g.k_global[j[better]]'),
    "many_degenerate_argmax": ("        a[degen] = -1\n        S[degen] = 0.0",
                               "        S[degen] = 0.0"),
    "many_mixed_series": ('r = np.abs((q["Xw"] @ H.T) * q["scale"][:, None])',
                          'r = np.abs((q["Xw"] @ H.T) * series[0]["scale"][:1, None])'),
    "second_forgets_smaller_max": (
        'q["second"] = np.maximum(np.minimum(q["m"], v), np.maximum(q["second"], c2))',
        'q["second"] = np.maximum(q["second"], c2)'),
    "second_is_smaller_max": (
        'q["second"] = np.maximum(np.minimum(q["m"], v), np.maximum(q["second"], c2))',
        'q["second"] = np.minimum(q["m"], v)'),
    "second_third_largest": ("c2 = np.partition(r, -2, axis=1)[:, -2] if k1 - k0 > 1",
                             "c2 = np.partition(r, -3, axis=1)[:, -3] if k1 - k0 > 2"),
    "rho_at_local_index": ("kl = kg[ok] - int(g.k_global[0])", "kl = kg[ok]"),
    "rho_at_signed": ("r[~degen] = np.abs(d[~degen]) / np.sqrt(E[~degen])",
                      "r[~degen] = d[~degen] / np.sqrt(E[~degen])"),
    "rho_at_not_degenerate": ("r[~degen] = np.abs(d[~degen]) / np.sqrt(E[~degen])",
                              "r = np.abs(d) / np.sqrt(np.maximum(E, 1e-300))"),
    "rho_at_window_shift": ("Xw = windows(x, p.L, offs[ok])", "Xw = windows(x, p.L, offs[ok] + 1)"),
    "coinc_strict_df": ("if abs(fa[i] - fb[j]) <= df:", "if abs(fa[i] - fb[j]) < df:"),
    "coinc_no_dtau": ("for t in range(int(ta[i]) - dtau, int(ta[i]) + dtau + 1):",
                      "for t in range(int(ta[i]), int(ta[i]) + 1):"),
    "coinc_one_sided_dtau": ("for t in range(int(ta[i]) - dtau, int(ta[i]) + dtau + 1):",
                             "for t in range(int(ta[i]), int(ta[i]) + dtau + 1):"),
    "coinc_index_as_frequency": ("fa, fb = template_f0(p, ka), template_f0(p, kb)",
                                 "fa, fb = ka.astype(float), kb.astype(float)"),
    "coinc_fdot_as_f0_index": ("i = np.asarray(k_global, dtype=np.int64) // p.n_fdot",
                               "i = np.asarray(k_global, dtype=np.int64) % p.n_f0"),
    "coinc_unsharded_bins": ("lo = int(g.k_global[0]) // p.n_fdot", "lo = 0"),
}


def _load_mutant(name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutant {name}: snippet not found in the oracle"
    mod = types.ModuleType(f"oracle_mutant_{name}")
    mod.__file__ = SRC
    sys.modules[mod.__name__] = mod        # dataclasses resolve their module by name
    try:
        exec(compile(src.replace(old, new), SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    mod = _load_mutant(name, old, new)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(mod)
        except Exception as e:  # AssertionError, or the mutant crashing on a pin's input
            failed.append((pin.__name__, type(e).__name__))
    assert failed, f"no pin catches mutant {name}"
