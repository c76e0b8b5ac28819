"""Oracle of the discrepancy principle for the regularisation parameter (test infrastructure only).

§3 leaves the choice of alpha open; Morozov's rule is the classical a-posteriori choice: with
f_alpha the quasi-boundary-value reconstruction from mu_eps and F the direct map f -> u(., T) of
§6.1 (the forward substitution with A-hat), take the largest alpha on a grid whose discrepancy
||F f_alpha - mu_eps||_2 is at most tau * delta, delta = ||mu_eps - mu||_2."""
from __future__ import annotations

import dataclasses

import numpy as np

from .system import Problem, dense_A, dense_Ahat, rhs_z, rhs_zhat


def recovered_f(p: Problem) -> np.ndarray:
    return np.linalg.solve(dense_A(p), rhs_z(p))[p.S * p.Nd:]


def forward_data(p: Problem, f: np.ndarray) -> np.ndarray:
    """u(., T) = v^(S) of the direct problem A-hat v = z-hat(f)."""
    v = np.linalg.solve(dense_Ahat(p), rhs_zhat(p, f))
    return v[(p.S - 1) * p.Nd:]


def residuals(p: Problem, alphas) -> list:
    out = []
    for a in alphas:
        q = dataclasses.replace(p, alpha=float(a))
        out.append(float(np.linalg.norm(forward_data(q, recovered_f(q)) - q.mu)))
    return out


def select(alphas, res, delta: float, tau: float = 1.1):
    ok = [a for a, r in zip(alphas, res) if r <= tau * delta]
    return max(ok) if ok else None
