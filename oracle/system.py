"""Problem data and the dense all-at-once matrices (paper §4 eq. numer-scheme, §5).

Layout (paper §2 multi-index rule, §5 eq. lin-syst): a solution vector is
y = [v^(1); ...; v^(S); f~], S+1 slices of Nd = N^d reals, slice-major, and
inside a slice the multi-index j = (j_1, ..., j_d) runs lexicographically
with the last index fastest.

Readings of the paper taken here (each is a choice the paper leaves open):
  * grid: n interior points per direction, h = L/(n+1), x_j = j h on
    Omega = (0, L)^d (§4 grid definition; reproduces the printed condition
    numbers of the 1D and 2D tables of §6);
  * row s of the scheme uses gamma_1, gamma_2, q at t_s, s = 1..S; the
    regularised final condition uses gamma_2 at t_S (§4 eq. numer-scheme);
  * the stencil of B is a_l for 0 <= l_i <= n-1, mirrored to negative l by
    evenness of the generating function (§4 eq. gen-func, §5).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import math

import numpy as np

from . import coeffs


@dataclasses.dataclass
class Problem:
    """Inputs of the regularised discrete problem (§4 eq. numer-scheme).

    gamma1, gamma2: (S, Nd) samples at (x_j, t_s), s = 1..S
    q:              (S,)   samples q(t_s)
    rho:            (Nd,)  initial state v^(0)
    mu:             (Nd,)  noisy final-time data mu_eps
    alpha:          the regularisation parameter (lambda in the paper)
    length:         Omega = (0, length)^d
    stencil:        optional a_l table, shape (N,)*d; computed from omega if None
    """
    d: int
    N: int
    S: int
    T: float
    beta: float
    omega: float
    alpha: float
    gamma1: np.ndarray
    gamma2: np.ndarray
    q: np.ndarray
    rho: np.ndarray
    mu: np.ndarray
    length: float = 1.0
    stencil: Optional[np.ndarray] = None

    @property
    def Nd(self) -> int:
        return self.N ** self.d

    @property
    def n_tot(self) -> int:
        return (self.S + 1) * self.Nd

    @property
    def h(self) -> float:
        return self.length / (self.N + 1)

    @property
    def dt(self) -> float:
        return self.T / self.S

    @property
    def eta(self) -> float:
        return coeffs.eta(self.beta, self.dt)

    @property
    def c_t(self) -> float:
        """eta / h^omega, the factor of D_2^(s) B in the diagonal blocks (§5)."""
        return self.eta / self.h ** self.omega

    @property
    def c_f(self) -> float:
        """lambda / h^omega, the factor of D_2^(S) B in the last block row (§5)."""
        return self.alpha / self.h ** self.omega

    def a(self) -> np.ndarray:
        if self.stencil is None:
            self.stencil = coeffs.stencil(self.omega, self.d, self.N)
        return self.stencil

    def e(self) -> np.ndarray:
        return coeffs.l1_e(self.beta, self.S)

    def b(self) -> np.ndarray:
        return coeffs.l1_b(self.beta, self.S)


def dense_B(p: Problem) -> np.ndarray:
    """B_n: the d-level symmetric Toeplitz matrix with entries a_{i-j} (§2, §5)."""
    a = p.a()
    N = p.N
    i = np.arange(N)
    lag = np.abs(i[:, None] - i[None, :])
    if p.d == 1:
        return a[lag]
    # 2-level: entry ((i1,i2),(j1,j2)) = a[|i1-j1|, |i2-j2|], last index fastest
    B4 = a[lag[:, None, :, None], lag[None, :, None, :]]  # (i1, i2, j1, j2)
    return B4.reshape(N * N, N * N)


def dense_A(p: Problem, B: Optional[np.ndarray] = None) -> np.ndarray:
    """A_{n,S} of eq. lin-syst (§5), assembled block by block.  B overrides the spatial
    matrix B_n (used to form the paper's T_{n,S}: every B_n replaced by its tau matrix)."""
    Nd, S = p.Nd, p.S
    e = p.e()
    B = dense_B(p) if B is None else B
    A = np.zeros((p.n_tot, p.n_tot))
    I = np.eye(Nd)
    for s in range(S):  # block row s+1 of the paper
        D1 = p.gamma1[s]
        D2 = p.gamma2[s]
        for m in range(s):
            A[s * Nd:(s + 1) * Nd, m * Nd:(m + 1) * Nd] = e[s - m] * np.diag(D1)
        A[s * Nd:(s + 1) * Nd, s * Nd:(s + 1) * Nd] = e[0] * np.diag(D1) + p.c_t * D2[:, None] * B
        A[s * Nd:(s + 1) * Nd, S * Nd:] = -p.eta * p.q[s] * I
    A[S * Nd:, (S - 1) * Nd:S * Nd] = I
    A[S * Nd:, S * Nd:] = p.c_f * p.gamma2[S - 1][:, None] * B
    return A


def dense_P(p: Problem, B: Optional[np.ndarray] = None) -> np.ndarray:
    """P_{n,S} (§5.1): A_{n,S} with the upper-right block column (rows 1..S of the
    last block column) replaced by zeros.  B overrides B_n as in dense_A."""
    P = dense_A(p, B)
    P[:p.S * p.Nd, p.S * p.Nd:] = 0.0
    return P


def dst1_matrix(n: int) -> np.ndarray:
    """The orthonormal DST-I matrix sqrt(2/(n+1)) sin(pi j k/(n+1)), j, k = 1..n (symmetric,
    its own inverse)."""
    j = np.arange(1, n + 1)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * math.pi / (n + 1))


def dense_tauB(p: Problem) -> np.ndarray:
    """tau(B_n), the natural tau matrix of B_n (§5.1 Remark; Bini–Capovani): S diag(lambda) S with
    S the orthonormal DST-I (tensor product over the d levels) and lambda the truncated symbol
    (coeffs.tau_eigenvalues)."""
    from .coeffs import tau_eigenvalues
    lam = tau_eigenvalues(p.a())
    S1 = dst1_matrix(p.N)
    S = S1 if p.d == 1 else np.kron(S1, S1)
    return S @ np.diag(lam.reshape(-1)) @ S


def tau_sigma(p: Problem) -> np.ndarray:
    """sigma_s = mean over the grid of e_0 gamma1^(s)/gamma2^(s), s = 1..S: the coefficient
    ratio of block s frozen at its mean (the reading under which T_{n,S} stays fast-invertible
    for variable coefficients)."""
    e0 = p.e()[0]
    return np.array([np.mean(e0 * p.gamma1[s] / p.gamma2[s]) for s in range(p.S)])


def dense_T(p: Problem) -> np.ndarray:
    """T_{n,S} of the §5.1 Remark, with variable coefficients read as follows: P_{n,S} with
    B_n replaced by tau(B_n) and each diagonal block e_0 D_1 + c_t D_2 B_n replaced by
    D_2 (sigma_s I + c_t tau(B_n)), sigma_s = mean(e_0 gamma1^(s)/gamma2^(s)).  For constant
    coefficients this is exactly P_{n,S} with every B_n replaced by tau(B_n)."""
    Nd, S = p.Nd, p.S
    T = dense_P(p, dense_tauB(p))
    tB = dense_tauB(p)
    sig = tau_sigma(p)
    I = np.eye(Nd)
    for s in range(S):
        T[s * Nd:(s + 1) * Nd, s * Nd:(s + 1) * Nd] = p.gamma2[s][:, None] * (sig[s] * I + p.c_t * tB)
    return T


def dense_strangB(p: Problem) -> np.ndarray:
    """s(B_n), Strang's circulant (§5.1 Remark): along every level the entry at lag l is
    c_{l mod n} of coeffs.strang_first_column, i.e. a d-level circulant."""
    from .coeffs import strang_first_column
    c = strang_first_column(p.a())
    N = p.N
    i = np.arange(N)
    lag = (i[:, None] - i[None, :]) % N
    if p.d == 1:
        return c[lag]
    return c[lag[:, None, :, None], lag[None, :, None, :]].reshape(N * N, N * N)


def dense_S(p: Problem) -> np.ndarray:
    """S_{n,S} of the §5.1 Remark under the reading of dense_T: P_{n,S} with B_n replaced by
    s(B_n) and each diagonal block replaced by D_2 (sigma_s I + c_t s(B_n)).  For constant
    coefficients this is exactly P_{n,S} with every B_n replaced by s(B_n)."""
    Nd, S = p.Nd, p.S
    sB = dense_strangB(p)
    Sm = dense_P(p, sB)
    sig = tau_sigma(p)
    I = np.eye(Nd)
    for s in range(S):
        Sm[s * Nd:(s + 1) * Nd, s * Nd:(s + 1) * Nd] = p.gamma2[s][:, None] * (sig[s] * I + p.c_t * sB)
    return Sm


def rhs_z(p: Problem) -> np.ndarray:
    """z of eq. lin-syst: z^(s) = b_{s-1} D_1^(s) rho for s = 1..S, z^(S+1) = mu_eps."""
    b = p.b()
    z = np.empty((p.S + 1, p.Nd))
    for s in range(p.S):
        z[s] = b[s] * p.gamma1[s] * p.rho
    z[p.S] = p.mu
    return z.reshape(-1)


def dense_Ahat(p: Problem) -> np.ndarray:
    """A-hat (§6.1 direct problem): the top-left S x S block part of P_{n,S}."""
    return dense_P(p)[:p.S * p.Nd, :p.S * p.Nd]


def rhs_zhat(p: Problem, f: np.ndarray) -> np.ndarray:
    """z-hat (§6.1): b_{s-1} D_1^(s) rho + eta q^(s) f, s = 1..S."""
    b = p.b()
    zh = np.empty((p.S, p.Nd))
    for s in range(p.S):
        zh[s] = b[s] * p.gamma1[s] * p.rho + p.eta * p.q[s] * f
    return zh.reshape(-1)


def with_mu(p: Problem, mu: np.ndarray) -> Problem:
    return dataclasses.replace(p, mu=np.asarray(mu, dtype=np.float64).copy())
