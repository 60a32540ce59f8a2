"""Pointwise viscosity at physical points.

Sec. 2 gives the generalised Newtonian law
    eta(gdot) = eta_inf + (eta_0 - eta_inf) [kappa + (lambda gdot)^a]^((b-1)/a)
with the shear rate gdot = sqrt(2 grad^S u : grad^S u); Sec. 4 and 4.1 store
the viscosity pointwise at the integration points.  Besides the law, smooth
prescribed fields mu(x) are supported (Sec. 2 allows an analytic function of
space).  The fields' random modes come from the ``workloads`` generators.
"""
from __future__ import annotations

import numpy as np


def _logfield(law, x):
    k = np.asarray(law["k"], dtype=np.float64)
    r = np.cos(2 * np.pi * (x @ k.T) + np.asarray(law["phi"])) @ np.asarray(law["a"])
    s = np.clip((r - law["rmin"]) / (law["rmax"] - law["rmin"]), 0.0, 1.0)
    return law["contrast"] ** s


def shear_rate_of_modes(law, x):
    """gdot = sqrt(2 eps(w):eps(w)) of w = sum_m v_m cos(2 pi k_m.x + phi_m)."""
    k = np.asarray(law["k"], dtype=np.float64)
    v = np.asarray(law["v"], dtype=np.float64)
    arg = 2 * np.pi * (x @ k.T) + np.asarray(law["phi"])  # (P, M)
    # grad w [p, i, j] = d w_i / d x_j = -sum_m v_mi 2 pi k_mj sin(arg_m)
    gw = -2 * np.pi * np.einsum("pm,mi,mj->pij", np.sin(arg), v, k)
    eps = 0.5 * (gw + np.swapaxes(gw, 1, 2))
    return np.sqrt(2.0 * np.einsum("pij,pij->p", eps, eps))


def generalized_newtonian(law, gdot):
    """eta(gdot) of Sec. 2 with (eta_0, eta_inf, lambda, kappa, a, b) =
    (mu0, mu_inf, lam, kappa, a_exp, n_exp)."""
    return law["mu_inf"] + (law["mu0"] - law["mu_inf"]) * (
        law["kappa"] + (law["lam"] * gdot) ** law["a_exp"]) ** ((law["n_exp"] - 1.0) / law["a_exp"])


def viscosity(law, x: np.ndarray) -> np.ndarray:
    """mu at physical points x (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    shp = x.shape[:-1]
    P = x.reshape(-1, 3)
    if callable(law):
        out = law(P)
    else:
        kind = law["kind"]
        if kind == "const":
            out = np.full(P.shape[0], law["mu"])
        elif kind == "sine":
            out = law["mu"] * (1.0 + law["amp"] * np.sin(2 * np.pi * P[:, 0])
                               * np.sin(2 * np.pi * P[:, 1]) * np.sin(2 * np.pi * P[:, 2]))
        elif kind == "logfield":
            out = _logfield(law, P)
        elif kind == "carreau":
            out = generalized_newtonian(law, shear_rate_of_modes(law, P))
        else:
            raise ValueError(f"unknown law {kind}")
    return np.asarray(out, dtype=np.float64).reshape(shp)
