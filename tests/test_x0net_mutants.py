"""Plant plausible mistakes in a copy of the network reference and check that the pins
catch each (source-level edits loaded as a fresh module; the real file is untouched)."""
import os
import sys
import types

import pytest

from tests import x0net_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "x0net_oracle.py")

MUTANTS = {
    "bf16_truncates": ("r = ((u + 0x7FFF + lsb) >> 16) << 16", "r = (u >> 16) << 16"),
    "bf16_ties_up": ("r = ((u + 0x7FFF + lsb) >> 16) << 16", "r = ((u + 0x8000) >> 16) << 16"),
    "conv_convolution_not_correlation": ("out += _shift(x, dz, dy, dx) @ w[:, t, :].T",
                                         "out += _shift(x, -dz, -dy, -dx) @ w[:, t, :].T"),
    "conv_weight_transposed_taps": ("TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]",
                                    "TAPS = [(dz, dy, dx) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]"),
    "dgrad_wrong_direction": ("gx += _shift(gout @ w[:, t, :], -dz, -dy, -dx)",
                              "gx += _shift(gout @ w[:, t, :], dz, dy, dx)"),
    "wgrad_unshifted_input": ("gw[:, t, :] = flat_g.T @ xs.reshape(-1, cin)",
                              "gw[:, t, :] = flat_g.T @ x.reshape(-1, cin)"),
    "pool_backward_unscaled": ("return upsample2(g) / 8.0", "return upsample2(g)"),
    "relu_backward_uses_input_sign": ("return np.where(y > 0.0, gy, 0.0)", "return np.where(y >= 0.0, gy, 0.0)"),
    "skip_gradient_dropped": ("            g = g + gskip[i]", "            g = g"),
    "decoder_split_swapped": ("gskip[i] = gcat[..., cup:]", "gskip[i] = gcat[..., :gcat.shape[3] - cup]"),
    "loss_alpha_missing": ("        L = 1.0 - u * u / (v * c)", "        L = 1.0 - u / c"),
    "regression_cross_term_sign": ("L = (sigma * sigma * v - 2.0 * sigma * u + c) / c",
                                   "L = (sigma * sigma * v + 2.0 * sigma * u + c) / c"),
    "regression_grad_scale": ("grad = (2.0 / c) * (sigma * sigma * Ay - sigma * P1b)",
                              "grad = (2.0 / c) * (sigma * Ay - sigma * P1b)"),
    "loss_grad_sign": ("grad = (2.0 * u / (v * c)) * ((u / v) * Ay - P1b)",
                       "grad = (2.0 * u / (v * c)) * (P1b - (u / v) * Ay)"),
    "wl2_unweighted_denominator": ("den = float(np.sum(dv * tv * tv))", "den = float(np.sum(tv * tv))"),
    "diag_missing_z_faces": ("+ tz[:-1] + tz[1:]", ""),
    "adam_no_bias_correction": ("    mh = m / (1.0 - b1 ** t)", "    mh = m"),
    "input_not_standardised": ("lk = (lk - lk.mean()) / max(lk.std(), 1e-12)", "lk = lk - lk.mean()"),
}


def _load(name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    src = src.replace(old, new, 1)
    modname = "x0net_mutant_" + name
    mod = types.ModuleType(modname)
    sys.modules[modname] = mod
    try:
        exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    finally:
        sys.modules.pop(modname, None)
    return mod


def _caught(mod):
    for pin in sorted(k for k in dir(P) if k.startswith("pin_")):
        fn = getattr(P, pin)
        try:
            if pin == "pin_network_gradient_finite_differences":
                fn(mod, False)
                fn(mod, True)
            else:
                fn(mod)
        except Exception:
            return pin
    return None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    pin = _caught(_load(name, old, new))
    assert pin is not None, f"no pin catches the planted mistake {name}"
