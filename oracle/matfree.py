"""Matrix-free products with A_{n,S} and P_{n,S} (paper §5 'Implementation'
paragraphs), in FP64 NumPy.

  matvec        z = A y by the paper's per-slice algorithm: the time-history sum,
                the Toeplitz product through a circulant embedding and the FFT,
                the -eta q^(s) f~ coupling, and the last block row (§5).
  apply_B       B v by circulant embedding + FFT (§5, step 1(b) of the matvec).
  P_solve       y = P^{-1} z by the paper's forward substitution over time (§5.1),
                diagonal blocks solved either densely (the paper's backslash) or by
                conjugate gradients on the symmetrised block (an approximation with
                a stated tolerance, for sizes where dense blocks do not fit).
  forward_solve the direct problem A-hat v = z-hat (§6.1): the first S steps of the
                same forward substitution.
  T_solve       y = T_{n,S}^{-1} z (§5.1 Remark, with the frozen-coefficient reading of
                system.dense_T): the same forward substitution, each block solved exactly
                by the orthonormal DST-I.
  S_solve       y = S_{n,S}^{-1} z (§5.1 Remark, Strang blocks under the same reading,
                system.dense_S): each block solved exactly by the d-dimensional FFT.

The embedding size used here is 2N per direction (the smallest even size
>= 2N-1); any size >= 2N-1 gives the same product in exact arithmetic.  The
transforms are SciPy's real FFTs on all host cores (WORKERS); the time-history
sums are products with the lower-triangular Toeplitz matrix of the e_m weights.
"""
from __future__ import annotations

import os
from typing import Callable, Optional

import numpy as np
import scipy.fft as sfft
import scipy.sparse.linalg as spla

from . import coeffs
from .system import Problem, dense_B, tau_sigma

WORKERS = os.cpu_count() or 1  # threads of the FFTs (scipy.fft workers)


# --------------------------------------------------------------------------
# B v through a circulant embedding (§5, matvec step 1(b))
# --------------------------------------------------------------------------

def circulant_symbol(p: Problem) -> np.ndarray:
    """Eigenvalues of the d-level circulant of size (2N)^d whose leading N^d block is B:
    the FFT of the first column c = [a_0, ..., a_{N-1}, 0, a_{N-1}, ..., a_1] per direction."""
    a = p.a()
    N = p.N
    L = 2 * N
    if p.d == 1:
        c = np.zeros(L)
        c[:N] = a
        c[L - N + 1:] = a[1:][::-1]
        return np.fft.fft(c).real
    c = np.zeros((L, L))
    idx = np.concatenate([np.arange(N), [0], np.arange(N - 1, 0, -1)])  # lag for each position
    mask = np.ones(L, dtype=bool)
    mask[N] = False
    A2 = a[idx[:, None], idx[None, :]]
    A2[~mask, :] = 0.0
    A2[:, ~mask] = 0.0
    c[:, :] = A2
    return np.fft.fft2(c).real


def apply_B(p: Problem, v: np.ndarray, symbol: Optional[np.ndarray] = None) -> np.ndarray:
    """B v for v of shape (..., Nd): zero-pad each direction to 2N, multiply by the circulant
    symbol in Fourier space, crop (§5, matvec step 1(b)).  v is real and the symbol is real and
    even, so the half spectrum of the real transform carries the whole product."""
    if symbol is None:
        symbol = circulant_symbol(p)
    N = p.N
    L = 2 * N
    lead = v.shape[:-1]
    if p.d == 1:
        V = sfft.rfft(v, n=L, axis=-1, workers=WORKERS)
        return sfft.irfft(V * symbol[:N + 1], n=L, axis=-1, workers=WORKERS)[..., :N]
    vv = v.reshape(lead + (N, N))
    V = sfft.rfftn(vv, s=(L, L), axes=(-2, -1), workers=WORKERS)
    out = sfft.irfftn(V * symbol[:, :N + 1], s=(L, L), axes=(-2, -1), workers=WORKERS)[..., :N, :N]
    return out.reshape(lead + (N * N,))


def history_matrix(p: Problem) -> np.ndarray:
    """The S x S lower-triangular Toeplitz matrix E with E[s, m] = e_{s-m} (m <= s): block (s, m)
    of the time part of A is e_{s-m} D_1^(s) (§5, eq. lin-syst), so the history sums of all
    slices are D_1 (E Y)."""
    e = p.e()
    s = np.arange(p.S)
    lag = s[:, None] - s[None, :]
    return np.where(lag >= 0, e[np.clip(lag, 0, None)], 0.0)


# --------------------------------------------------------------------------
# z = A y (§5, the matvec algorithm)
# --------------------------------------------------------------------------

def matvec(p: Problem, y: np.ndarray, symbol: Optional[np.ndarray] = None) -> np.ndarray:
    """z = A_{n,S} y following the paper's steps: for s = 1..S
         w^(s) = D_1^(s) (e_{s-1} y^(1) + ... + e_0 y^(s))
         z^(s) = w^(s) + (eta/h^omega) D_2^(s) B y^(s) - eta q^(s) y^(S+1)
       (the paper's step 1(c) prints y^(s); the last block column of A_{n,S} multiplies
        y^(S+1), which is what is subtracted here), and
         z^(S+1) = (lambda/h^omega) D_2^(S) B y^(S+1) + y^(S)."""
    S, Nd = p.S, p.Nd
    Y = y.reshape(S + 1, Nd)
    if symbol is None:
        symbol = circulant_symbol(p)
    BY = apply_B(p, Y, symbol)
    W = history_matrix(p) @ Y[:S]  # W[s] = sum_{m <= s} e_{s-m} y^(m)
    Z = np.empty_like(Y)
    for s in range(S):
        Z[s] = p.gamma1[s] * W[s] + p.c_t * p.gamma2[s] * BY[s] - p.eta * p.q[s] * Y[S]
    Z[S] = p.c_f * p.gamma2[S - 1] * BY[S] + Y[S - 1]
    return Z.reshape(-1)


def matvec_entry(p: Problem, y: np.ndarray, s: int, j: int) -> float:
    """One entry z^(s+1)_j of A y (0-based slice s, flat spatial index j), computed straight
    from eq. numer-scheme with the stencil sum written out (no FFT)."""
    S, N, d = p.S, p.N, p.d
    Y = y.reshape(S + 1, p.Nd)
    a = p.a()
    if d == 1:
        lag = np.abs(np.arange(N) - j)
        Bv = lambda v: float(np.dot(a[lag], v))
    else:
        j1, j2 = divmod(j, N)
        l1 = np.abs(np.arange(N) - j1)
        l2 = np.abs(np.arange(N) - j2)
        Bv = lambda v: float(np.sum(a[l1[:, None], l2[None, :]] * v.reshape(N, N)))
    if s == S:
        return p.c_f * p.gamma2[S - 1, j] * Bv(Y[S]) + Y[S - 1, j]
    e = p.e()
    hist = sum(e[s - m] * Y[m, j] for m in range(s + 1))
    return (p.gamma1[s, j] * hist + p.c_t * p.gamma2[s, j] * Bv(Y[s])
            - p.eta * p.q[s] * Y[S, j])


# --------------------------------------------------------------------------
# y = P^{-1} z by forward substitution (§5.1 'Implementation')
# --------------------------------------------------------------------------

def _cg(apply: Callable, rhs: np.ndarray, x0: np.ndarray, tol: float, maxit: int,
        prec: Optional[Callable] = None):
    """Plain (preconditioned) conjugate gradients, relative residual tol."""
    x = x0.copy()
    r = rhs - apply(x)
    bn = np.linalg.norm(rhs)
    if bn == 0.0:
        return np.zeros_like(rhs), 0
    z = prec(r) if prec else r
    pdir = z.copy()
    rz = float(r @ z)
    for it in range(1, maxit + 1):
        if np.linalg.norm(r) <= tol * bn:
            return x, it - 1
        q = apply(pdir)
        al = rz / float(pdir @ q)
        x += al * pdir
        r -= al * q
        z = prec(r) if prec else r
        rz_new = float(r @ z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    return x, maxit


def tau_block_preconditioner(p: Problem, sigma: float, c: float) -> Callable:
    """r -> (sigma I + c tau(B))^{-1} r with tau(B) = S diag(lambda) S, S the orthonormal DST-I over
    every level (§5.1 Remark): an SPD approximation of the block sigma I + c B, used only to speed up
    the CG of P_solve (the block system and its solution are unchanged)."""
    lam = coeffs.tau_eigenvalues(p.a())
    shape = (p.N,) * p.d
    diag = sigma + c * lam

    def apply(r):
        t = sfft.dstn(r.reshape(shape), type=1, norm="ortho", workers=WORKERS)
        return sfft.dstn(t / diag, type=1, norm="ortho", workers=WORKERS).reshape(-1)
    return apply


def P_solve(p: Problem, z: np.ndarray, inner: str = "dense", inner_tol: float = 1e-14,
            inner_maxit: int = 2000, last_block: bool = True) -> np.ndarray:
    """y = P_{n,S}^{-1} z by the forward substitution of §5.1:
         s = 1:      (e_0 D_1^(1) + c_t D_2^(1) B) y^(1) = z^(1)
         s = 2..S:   (e_0 D_1^(s) + c_t D_2^(s) B) y^(s) = z^(s) - D_1^(s)(e_{s-1} y^(1) + ... + e_1 y^(s-1))
         s = S+1:    c_f D_2^(S) B y^(S+1) = z^(S+1) - y^(S)
    inner = 'dense': each block solved by LU of the assembled block (the paper's backslash);
    inner = 'cg':    each block solved by CG on the SPD form (D_2^-1 D_1 e_0 + c_t B) y = D_2^-1 r
                     (respectively B y = r / (c_f gamma_2)) to relative residual inner_tol —
                     an approximation of P^{-1}, used only where dense blocks do not fit;
    inner = 'pcg':   the same CG preconditioned by the tau matrix of the block with its diagonal
                     frozen at the slice mean (tau_block_preconditioner), for the large sizes."""
    S, Nd = p.S, p.Nd
    Z = z.reshape(-1, Nd)
    e = p.e()
    Y = np.zeros((S + 1, Nd))
    if inner == "dense":
        B = dense_B(p)
    else:
        symbol = circulant_symbol(p)
        Bop = lambda v: apply_B(p, v, symbol)
    for s in range(S):
        r = Z[s].copy()
        if s > 0:
            hist = e[s:0:-1] @ Y[:s]  # sum_{m < s} e_{s-m} y^(m)
            r -= p.gamma1[s] * hist
        if inner == "dense":
            K = e[0] * np.diag(p.gamma1[s]) + p.c_t * p.gamma2[s][:, None] * B
            Y[s] = np.linalg.solve(K, r)
        else:
            dg = e[0] * p.gamma1[s] / p.gamma2[s]
            x0 = Y[s - 1] if s > 0 else np.zeros(Nd)
            prec = tau_block_preconditioner(p, float(np.mean(dg)), p.c_t) if inner == "pcg" else None
            Y[s], _ = _cg(lambda v: dg * v + p.c_t * Bop(v), r / p.gamma2[s], x0,
                          inner_tol, inner_maxit, prec)
    if not last_block:
        return Y[:S].reshape(-1)
    r = Z[S] - Y[S - 1]
    if inner == "dense":
        Y[S] = np.linalg.solve(p.c_f * p.gamma2[S - 1][:, None] * B, r)
    else:
        prec = tau_block_preconditioner(p, 0.0, 1.0) if inner == "pcg" else None
        Y[S], _ = _cg(Bop, r / (p.c_f * p.gamma2[S - 1]), np.zeros(Nd), inner_tol, inner_maxit, prec)
    return Y.reshape(-1)


def forward_solve(p: Problem, zhat: np.ndarray, inner: str = "dense",
                  inner_tol: float = 1e-14) -> np.ndarray:
    """v = A-hat^{-1} z-hat (§6.1 direct problem), i.e. the first S block steps of the
    forward substitution for P (A-hat is the leading S x S block part of P)."""
    zz = np.concatenate([zhat, np.zeros(p.Nd)])
    return P_solve(p, zz, inner=inner, inner_tol=inner_tol, last_block=False)


# --------------------------------------------------------------------------
# y = T_{n,S}^{-1} z (§5.1 Remark; blocks as in system.dense_T)
# --------------------------------------------------------------------------
def T_solve(p: Problem, z: np.ndarray, last_block: bool = True) -> np.ndarray:
    """Forward substitution with the blocks of T_{n,S}:
         s = 1..S:  r = (z^(s) - D_1^(s) sum_{m<s} e_{s-m} y^(m)) / gamma2^(s),
                    y^(s) = S diag(1/(sigma_s + c_t lambda)) S r
         s = S+1:   y^(S+1) = S diag(1/lambda) S (z^(S+1) - y^(S)) / (c_f gamma2^(S))
    with S the orthonormal DST-I over every level and lambda the tau eigenvalues of B_n."""
    S_, Nd = p.S, p.Nd
    shape = (p.N,) * p.d
    lam = coeffs.tau_eigenvalues(p.a())
    sig = tau_sigma(p)
    e = p.e()
    Z = z.reshape(-1, Nd)
    Y = np.zeros((S_ + 1, Nd))

    def dst(v):
        return sfft.dstn(v.reshape(shape), type=1, norm="ortho")

    for s in range(S_):
        hist = np.zeros(Nd)
        for m in range(s):
            hist += e[s - m] * Y[m]
        r = (Z[s] - p.gamma1[s] * hist) / p.gamma2[s]
        Y[s] = dst(dst(r) / (sig[s] + p.c_t * lam)).reshape(-1)
    if last_block:
        r = (Z[S_] - Y[S_ - 1]) / (p.c_f * p.gamma2[S_ - 1])
        Y[S_] = dst(dst(r) / lam).reshape(-1)
    return Y.reshape(-1)


def S_solve(p: Problem, z: np.ndarray, last_block: bool = True) -> np.ndarray:
    """Forward substitution with the blocks of S_{n,S}: as T_solve, with the block solves
         s = 1..S:  y^(s) = F^{-1} diag(1/(sigma_s + c_t lambda)) F r
         s = S+1:   y^(S+1) = F^{-1} diag(1/lambda) F (z^(S+1) - y^(S)) / (c_f gamma2^(S))
    where F is the d-dimensional DFT and lambda the eigenvalues of Strang's circulant s(B_n)."""
    S_, Nd = p.S, p.Nd
    shape = (p.N,) * p.d
    lam = coeffs.strang_eigenvalues(p.a())
    sig = tau_sigma(p)
    e = p.e()
    Z = z.reshape(-1, Nd)
    Y = np.zeros((S_ + 1, Nd))

    def solve(r, diag):
        return np.fft.ifftn(np.fft.fftn(r.reshape(shape)) / diag).real.reshape(-1)

    for s in range(S_):
        hist = np.zeros(Nd)
        for m in range(s):
            hist += e[s - m] * Y[m]
        r = (Z[s] - p.gamma1[s] * hist) / p.gamma2[s]
        Y[s] = solve(r, sig[s] + p.c_t * lam)
    if last_block:
        r = (Z[S_] - Y[S_ - 1]) / (p.c_f * p.gamma2[S_ - 1])
        Y[S_] = solve(r, lam)
    return Y.reshape(-1)
