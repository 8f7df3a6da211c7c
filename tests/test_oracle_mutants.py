"""Plant plausible mistakes in a copy of the CPU oracle and check that the pins catch each.

Every mutant is a source-level edit of oracle/psl_oracle.py loaded as a fresh module on
the CPU; the real oracle is never modified. A mutant that passed every pin would mean
the pins cannot tell that slip from the correct method.
"""
import importlib.util
import os
import sys
import types

import pytest

from tests import oracle_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "psl_oracle.py")

MUTANTS = {
    "arithmetic_mean_face": ("out[nz] = 2.0 * Ka[nz] * Kb[nz] / s[nz]", "out[nz] = 0.5 * s[nz]"),
    "dirichlet_full_cell": ("Tx[:, :, 0] = 2.0 * k[:, :, 0]", "Tx[:, :, 0] = 1.0 * k[:, :, 0]"),
    "dropped_z_faces": ("+ Tz[:-1, :, :] + Tz[1:, :, :]).reshape(-1)", ").reshape(-1)"),
    "wrong_offdiag_sign": ("vals += [-t, -t]", "vals += [t, t]"),
    "subdomain_ceil": ("bx = (ix * sx) // nx", "bx = -((-ix * sx) // nx)"),
    "subdomain_axes_swapped": ("return (bx + sx * (by + sy * bz))", "return (by + sy * (bx + sx * bz))"),
    "strict_threshold": ("c += (K >= t)", "c += (K > t)"),
    "coarse_is_ZtZ": ("return np.asarray((Z.T @ (A @ Z)).todense())",
                      "return np.asarray((Z.T @ Z).todense())"),
    "P1_sign": ("return v - A @ coarse.correction(v)", "return v + A @ coarse.correction(v)"),
    "P1_without_A": ("return v - A @ coarse.correction(v)", "return v - coarse.correction(v)"),
    "no_projection_back": ("x = xhat + coarse.correction(b - A @ xhat)", "x = xhat.copy()"),
    "projection_of_b_only": ("x = xhat + coarse.correction(b - A @ xhat)",
                             "x = xhat + coarse.correction(b)"),
    "jacobi_multiplies": ("y = rhat / dg\n        rho_new", "y = rhat * dg\n        rho_new"),
    "beta_inverted": ("beta = rho_new / rho", "beta = rho / rho_new"),
    "alpha_uses_q": ("pw = p @ w", "pw = p @ q"),
    "x_update_uses_w": ("xhat += alpha * p", "xhat += alpha * w"),
    "projector_P1_P2_swapped": ("P1 = np.eye(n) - A @ Z @ Einv @ Z.T\n    P2 = np.eye(n) - Z @ Einv @ Z.T @ A",
                                "P2 = np.eye(n) - A @ Z @ Einv @ Z.T\n    P1 = np.eye(n) - Z @ Einv @ Z.T @ A"),
    "no_initial_deflation": ("rhat = P1(b - A @ xhat)", "rhat = b - A @ xhat"),
    "components_ignore_class": ("key = (sub * ncls + c).reshape(nz, ny, nx)",
                                "key = (sub * ncls + 0 * c).reshape(nz, ny, nx)"),
    "components_no_z_faces": ("for axis in (2, 1, 0):", "for axis in (2, 1):"),
    "gmres_left_preconditioned": ("        return P1(A @ Minv(v))", "        return Minv(P1(A @ v))"),
    "gmres_update_without_Minv": ("xm = xm + Minv(np.array(basis[:k]).T @ y)",
                                  "xm = xm + np.array(basis[:k]).T @ y"),
    "gmres_rotation_sign": ("            g[k + 1] = -sn[k] * g[k]", "            g[k + 1] = sn[k] * g[k] * 0.5"),
    "gmres_earlier_rotations_skipped": ("            for i in range(k):\n                h[i], h[i + 1]",
                                        "            for i in range(0):\n                h[i], h[i + 1]"),
    "gmres_no_projection_back": ("x = xm + coarse.correction(b - A @ xm)", "x = xm.copy()"),
    "cheb_rho_sign": ("rho_next = 1.0 / (2.0 * sigma - rho)", "rho_next = 1.0 / (2.0 * sigma + rho)"),
    "cheb_step_without_jacobi": ("(2.0 * rho_next / delta) * (res / dg)", "(2.0 * rho_next / delta) * res"),
    "cheb_residual_of_d": ("res = r - A @ y", "res = r - A @ d"),
    "poly_beta_inverted": ("p = y + (rho_new / rho) * p", "p = y + (rho / rho_new) * p"),
    "gmres_poly_degree_ignored": ("        if degree <= 1:\n            return v / dg\n",
                                  "        if True:\n            return v / dg\n"),
    "components_reverse_order": ("order[np.argsort(first, kind=\"stable\")] = np.arange(ncomp)",
                                 "order[np.argsort(-first, kind=\"stable\")] = np.arange(ncomp)"),
}


def _load_mutant(name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    src = src.replace(old, new, 1)
    modname = "oracle_mutant_" + name
    mod = types.ModuleType(modname)
    sys.modules[modname] = mod          # dataclasses look their module up by name
    try:
        exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    finally:
        sys.modules.pop(modname, None)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    O = _load_mutant(name, old, new)
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(O)
        except Exception as exc:  # AssertionError or a crash both count as caught
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} passes every pin"
