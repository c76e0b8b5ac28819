"""Reference Krylov solvers in FP64 (the paper solves eq. lin-syst with GMRES,
§5 'Implementation' and §6: zero initial guess, tolerance 1e-8, at most
min(size, 1000) iterations).

  gmres   textbook GMRES (Saad & Schultz 1986): Arnoldi with modified Gram-Schmidt,
          Givens rotations on the Hessenberg matrix, no restart.  Preconditioning
          on the left (residual measured on the preconditioned system, the convention
          of MATLAB's gmres with a preconditioner) or on the right.
  fgmres  flexible, restarted GMRES (Saad 1993): right preconditioning whose action
          may change between iterations; the preconditioned directions z_j are kept
          and the iterate is x0 + Z y.  Stops on ||b - A x|| / ||b||.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def gmres(A: Callable, b: np.ndarray, tol: float, maxit: int,
          M_left: Optional[Callable] = None, M_right: Optional[Callable] = None,
          x0: Optional[np.ndarray] = None):
    """Full GMRES.  Returns (x, iterations, relres_history).  The stopping test is
    ||r_k|| <= tol * ||r_0-reference|| where r is the residual of the system actually
    iterated on: M^{-1}(b - A x) relative to ||M^{-1} b|| for left preconditioning,
    b - A x relative to ||b|| otherwise."""
    n = b.shape[0]
    x0 = np.zeros(n) if x0 is None else x0.copy()
    L = M_left if M_left is not None else (lambda v: v)
    R = M_right if M_right is not None else (lambda v: v)
    op = lambda v: L(A(R(v)))
    r0 = L(b - A(x0))
    bref = np.linalg.norm(L(b))
    beta = np.linalg.norm(r0)
    hist = [beta / bref]
    if beta <= tol * bref:
        return x0, 0, hist
    m = maxit
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[0] = r0 / beta
    k_done = 0
    for j in range(m):
        w = op(V[j])
        for i in range(j + 1):
            H[i, j] = float(V[i] @ w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] != 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k_done = j + 1
        hist.append(abs(g[j + 1]) / bref)
        if abs(g[j + 1]) <= tol * bref or H[j, j] == 0.0:
            break
    k = k_done
    yk = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = x0 + R(V[:k].T @ yk)
    return x, k, hist


def fgmres(A: Callable, M: Callable, b: np.ndarray, tol: float, restart: int, maxit: int,
           x0: Optional[np.ndarray] = None):
    """Restarted flexible GMRES with right preconditioner M (applied as z_j = M(v_j)).
    Returns (x, total_iterations, relres_history) with relres = ||b - A x||/||b|| as
    estimated by the least-squares residual, recomputed exactly at every restart."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), 0, [0.0]
    total = 0
    hist = []
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bn)
        if beta <= tol * bn or total >= maxit:
            return x, total, hist
        m = min(restart, maxit - total)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = float(V[i] @ w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            total += 1
            if abs(g[j + 1]) <= tol * bn:
                break
        yk = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ yk


def arnoldi_cgs2(op: Callable, b: np.ndarray, k: int):
    """k steps of Arnoldi on op from b, classical Gram-Schmidt applied twice (the solver's
    orthogonalisation).  Returns (H, V): H (k+1) x k upper Hessenberg, V n x (k+1) orthonormal,
    op(V[:, :k]) = V H."""
    n = b.shape[0]
    V = np.zeros((n, k + 1))
    H = np.zeros((k + 1, k))
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(k):
        w = op(V[:, j])
        h1 = V[:, :j + 1].T @ w
        w = w - V[:, :j + 1] @ h1
        h2 = V[:, :j + 1].T @ w
        w = w - V[:, :j + 1] @ h2
        H[:j + 1, j] = h1 + h2
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            return H[:j + 2, :j + 1], V[:, :j + 2]
        V[:, j + 1] = w / H[j + 1, j]
    return H, V
