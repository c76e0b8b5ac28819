"""Oracle of the transposed problem (test infrastructure only: the HIP library never imports it).

The gradients of the recovered source f~ = R A^{-1} z (R keeps the last block, §5 eq. lin-syst)
with respect to the final-time data mu_eps and the regularisation parameter alpha (§3), by the
adjoint method written out with dense matrices:
    lam = A^{-T} R^T g,   dL/dmu = lam^(S+1)   (z^(S+1) = mu_eps, the other blocks of z do not
                                                depend on mu),
    dL/dalpha = -lam^T (dA/dalpha) y,  where only c_f = alpha / h^omega depends on alpha, so
                dA/dalpha is zero except its last diagonal block (c_f/alpha) D_2^(S) B.
P^{-T} is the transpose of the block lower-triangular P of §5.1, applied by a dense solve."""
from __future__ import annotations

import numpy as np

from .system import Problem, dense_A, dense_B, dense_P, rhs_z


def apply_AT(p: Problem, lam: np.ndarray) -> np.ndarray:
    """A^T lam with A assembled densely."""
    return dense_A(p).T @ lam


def matvec_T_entry(p: Problem, w: np.ndarray, m: int, j: int) -> float:
    """Entry (m, j) of A^T w (0-based slice m, flat spatial index j), summed down column (m, j) of the
    blocks of A in eq. lin-syst (§5), with the stencil sum written out (no FFT, no dense matrix):
        m < S:  sum_{s=m}^{S-1} e_{s-m} gamma1^(s)_j w^(s)_j + c_t sum_i a_{i-j} gamma2^(m)_i w^(m)_i
                + [m = S-1] w^(S)_j
        m = S:  -eta sum_s q^(s) w^(s)_j + c_f sum_i a_{i-j} gamma2^(S)_i w^(S)_i
    (1-based slices of the paper shifted by one; the last block column multiplies f~)."""
    S, N, d = p.S, p.N, p.d
    W = w.reshape(S + 1, p.Nd)
    a = p.a()
    if d == 1:
        lag = np.abs(np.arange(N) - j)
        Bcol = lambda v: float(np.dot(a[lag], v))
    else:
        j1, j2 = divmod(j, N)
        l1 = np.abs(np.arange(N) - j1)
        l2 = np.abs(np.arange(N) - j2)
        Bcol = lambda v: float(np.sum(a[l1[:, None], l2[None, :]] * v.reshape(N, N)))
    if m == S:
        return (-p.eta * float(np.dot(p.q, W[:S, j]))
                + p.c_f * Bcol(p.gamma2[S - 1] * W[S]))
    e = p.e()
    hist = sum(e[s - m] * p.gamma1[s, j] * W[s, j] for s in range(m, S))
    out = hist + p.c_t * Bcol(p.gamma2[m] * W[m])
    if m == S - 1:
        out += W[S, j]
    return float(out)


def PT_solve(p: Problem, g: np.ndarray) -> np.ndarray:
    """P^{-T} g by a dense solve."""
    return np.linalg.solve(dense_P(p).T, g)


def adjoint_solve(p: Problem, g: np.ndarray) -> np.ndarray:
    """A^{-T} g by a dense solve."""
    return np.linalg.solve(dense_A(p).T, g)


def dA_dalpha(p: Problem) -> np.ndarray:
    """dA/dalpha: (c_f/alpha) D_2^(S) B in the last diagonal block, zero elsewhere."""
    D = np.zeros((p.n_tot, p.n_tot))
    S, Nd = p.S, p.Nd
    D[S * Nd:, S * Nd:] = (p.c_f / p.alpha) * p.gamma2[S - 1][:, None] * dense_B(p)
    return D


def vjp(p: Problem, gf: np.ndarray):
    """(dL/dmu, dL/dalpha) for a loss L(f~) with dL/df~ = gf, and the solution y of A y = z."""
    A = dense_A(p)
    y = np.linalg.solve(A, rhs_z(p))
    g = np.zeros(p.n_tot)
    g[p.S * p.Nd:] = gf
    lam = np.linalg.solve(A.T, g)
    return lam[p.S * p.Nd:].copy(), float(-lam @ (dA_dalpha(p) @ y)), y


def grad_gamma2(p: Problem, gf: np.ndarray) -> np.ndarray:
    """dL/dgamma2 (S x N^d, the gamma2 samples at t_1..t_S): gamma2^(s) multiplies the B term of
    diagonal block s (coefficient c_t) and, for s = S, also that of the last block (coefficient c_f),
    so dL/dgamma2^(s) = -c_t lam^(s) .* B y^(s) - [s = S] c_f lam^(S+1) .* B y^(S+1)."""
    A = dense_A(p)
    B = dense_B(p)
    S, Nd = p.S, p.Nd
    y = np.linalg.solve(A, rhs_z(p)).reshape(S + 1, Nd)
    g = np.zeros(p.n_tot)
    g[S * Nd:] = gf
    lam = np.linalg.solve(A.T, g).reshape(S + 1, Nd)
    G = np.empty((S, Nd))
    for s in range(S):
        G[s] = -p.c_t * lam[s] * (B @ y[s])
    G[S - 1] -= p.c_f * lam[S] * (B @ y[S])
    return G
