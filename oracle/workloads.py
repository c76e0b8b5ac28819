"""Problems built from the seeded inputs, with the final-time data made by the
oracle's own forward solve (the 'direct problem' of §6.1: mu = v^(S) of
A-hat v = z-hat, then the noise of the input set is added)."""
from __future__ import annotations

from typing import Optional

import numpy as np

from paper_2507_02809_amd.inputs import Inputs

from . import matfree
from .system import Problem


def problem(inp: Inputs, mu: Optional[np.ndarray] = None,
            stencil: Optional[np.ndarray] = None) -> Problem:
    """A Problem with the input set's fields; mu defaults to zeros (fill it with with_data)."""
    return Problem(d=inp.d, N=inp.N, S=inp.M, T=inp.T, beta=inp.beta, omega=inp.omega,
                   alpha=inp.alpha, gamma1=inp.gamma1, gamma2=inp.gamma2, q=inp.q,
                   rho=inp.rho, mu=np.zeros(inp.Nd) if mu is None else mu,
                   length=inp.length, stencil=stencil)


def with_data(inp: Inputs, inner: str = "dense", inner_tol: float = 1e-14,
              stencil: Optional[np.ndarray] = None) -> Problem:
    """Forward-solve A-hat v = z-hat with f = f_true (§6.1), take mu = v^(S), add the
    input set's noise, and return the inverse problem with mu_eps."""
    from .system import rhs_zhat
    p = problem(inp, stencil=stencil)
    v = matfree.forward_solve(p, rhs_zhat(p, inp.f_true), inner=inner, inner_tol=inner_tol)
    mu = v.reshape(p.S, p.Nd)[-1]
    p.mu = inp.noisy(mu)
    return p
