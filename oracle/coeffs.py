"""Scalar weights and stencils of the discretisation, in FP64.

Paper sections cited:
  §4  L1 formula (eq. L1-formula) and the b_m weights; the e_m weights built
      from them; the fractional centred difference (eq. discrete-laplacian)
      whose stencil a_l is the Fourier coefficient (eq. fourier-coeff) of the
      generating function (eq. gen-func); the 1D closed form
      (eq. fourier-coeff-1d) and Lemma 1.
  §5  eta = dt^beta * Gamma(2 - beta).
  §5 Remark  the tau preconditioner of a (multilevel) symmetric Toeplitz
      matrix, diagonalised by the sine transform.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
from scipy import special


# --------------------------------------------------------------------------
# time weights (§4)
# --------------------------------------------------------------------------

def l1_b(beta: float, count: int) -> np.ndarray:
    """b_m = (m+1)^(1-beta) - m^(1-beta), m = 0..count-1 (§4, under eq. L1-formula)."""
    m = np.arange(count, dtype=np.float64)
    return (m + 1.0) ** (1.0 - beta) - m ** (1.0 - beta)


def l1_e(beta: float, S: int) -> np.ndarray:
    """e_0 = b_0 and e_m = b_m - b_{m-1} for 1 <= m <= S-1 (§4, the e_m definition
    right before eq. numer-scheme).  e_m is written out from the second-difference
    form (m+1)^(1-beta) - 2 m^(1-beta) + (m-1)^(1-beta) that the paper also gives."""
    e = np.empty(S, dtype=np.float64)
    e[0] = 1.0  # b_0 = 1^(1-beta) - 0 = 1
    m = np.arange(1, S, dtype=np.float64)
    e[1:] = (m + 1.0) ** (1.0 - beta) - 2.0 * m ** (1.0 - beta) + (m - 1.0) ** (1.0 - beta)
    return e


def eta(beta: float, dt: float) -> float:
    """eta = dt^beta * Gamma(2 - beta) (§5, start of the matrix formulation)."""
    return dt ** beta * math.gamma(2.0 - beta)


# --------------------------------------------------------------------------
# fractional-Laplacian stencil (§4)
# --------------------------------------------------------------------------

def c_omega(omega: float, d: int) -> float:
    """Normalisation constant of the hypersingular integral (§1, eq. fractional-laplacian)."""
    return (2.0 ** omega * math.gamma((omega + d) / 2.0)
            / (math.pi ** (d / 2.0) * abs(math.gamma(-omega / 2.0))))


def stencil_1d_closed(omega: float, n: int) -> np.ndarray:
    """a_l, l = 0..n-1, from the closed form (eq. fourier-coeff-1d):
        a_l = (-1)^l Gamma(omega+1) / (Gamma(omega/2 - l + 1) Gamma(omega/2 + l + 1)),
    evaluated with 40-digit arithmetic and rounded once to FP64."""
    with mpmath.workdps(40):
        w = mpmath.mpf(omega)
        g = mpmath.gamma(w + 1)
        out = np.empty(n, dtype=np.float64)
        for l in range(n):
            v = (-1) ** l * g * mpmath.rgamma(w / 2 - l + 1) * mpmath.rgamma(w / 2 + l + 1)
            out[l] = float(v)
    return out


def stencil_1d_recursion(omega: float, n: int) -> np.ndarray:
    """a_l, l = 0..n-1, from Lemma 1: a_0 = Gamma(omega+1)/Gamma(omega/2+1)^2 (part a)
    and a_{l+1} = (1 - (omega+1)/(omega/2 + l + 1)) a_l (part b).  FP64 throughout."""
    a = np.empty(n, dtype=np.float64)
    a[0] = math.gamma(omega + 1.0) / math.gamma(omega / 2.0 + 1.0) ** 2
    for l in range(n - 1):
        a[l + 1] = (1.0 - (omega + 1.0) / (omega / 2.0 + l + 1.0)) * a[l]
    return a


def _i0_minus_one_series(tau: np.ndarray) -> np.ndarray:
    """I_0(2 tau) - 1 = sum_{k>=1} tau^(2k) / (k!)^2, summed without cancellation (tau <= 1)."""
    out = np.zeros_like(tau)
    term = np.ones_like(tau)
    for k in range(1, 40):
        term = term * tau * tau / (k * k)
        out = out + term
    return out


def _bessel_asymptotic_coeffs(nu: np.ndarray, K: int) -> np.ndarray:
    """Coefficients s_k(nu) of  e^{-x} I_nu(x) ~ (2 pi x)^(-1/2) sum_k s_k x^(-k)  for large x
    (Hankel's expansion: s_k = (-1)^k prod_{j=1..k} (4 nu^2 - (2j-1)^2) / (k! 8^k)).
    Returns an array of shape (K+1, len(nu))."""
    mu = 4.0 * nu.astype(np.float64) ** 2
    s = np.empty((K + 1, len(nu)), dtype=np.float64)
    s[0] = 1.0
    for k in range(1, K + 1):
        s[k] = -s[k - 1] * (mu - (2 * k - 1) ** 2) / (k * 8.0)
    return s


def stencil_subordination(omega: float, d: int, n: int) -> np.ndarray:
    """a_l for 0 <= l_i <= n-1 (an array of shape (n,)*d) from the Fourier-coefficient
    definition (eq. fourier-coeff) rewritten through Bochner subordination.

    With alpha = omega/2 in (0,1) and s = sum_i 4 sin^2(theta_i/2) >= 0,
        s^alpha = |Gamma(-alpha)|^-1 * int_0^inf (1 - exp(-tau s)) tau^(-1-alpha) dtau,
    and exp(-tau * 4 sin^2(theta/2)) = exp(-2 tau) exp(2 tau cos theta) has Fourier
    coefficients e^{-2 tau} I_l(2 tau) (modified Bessel functions).  Hence
        a_l = |Gamma(-alpha)|^-1 int_0^inf (delta_{l,0} - prod_i e^{-2tau} I_{l_i}(2tau)) tau^(-1-alpha) dtau.
    This route shares nothing with the FFT-of-samples route the GPU library uses.

    Quadrature: Gauss-Jacobi (weight tau^-alpha) on [0, 1]; Gauss-Legendre panels in
    u = log tau on [1, tau_1]; on [tau_1, inf) Hankel's large-argument expansion,
    integrated term by term in closed form."""
    alpha = omega / 2.0
    C = 1.0 / abs(math.gamma(-alpha))
    ls = np.arange(n)
    total = np.zeros((n,) * d, dtype=np.float64)

    def accumulate(weights, F_vecs, delta_part):
        # F_vecs: (Q, n) values of e^{-2tau} I_l(2tau) (or their tau-scaled versions);
        # adds  sum_q w_q (delta_{l0} * delta_part_q - prod_i F_vecs[q, l_i])
        nonlocal total
        if d == 1:
            prod = weights @ F_vecs
        elif d == 2:
            prod = (F_vecs * weights[:, None]).T @ F_vecs
        else:
            raise ValueError("d must be 1 or 2")
        total -= prod
        total[(0,) * d] += float(np.sum(weights * delta_part))

    # --- region 1: tau in (0, 1].  The integrand is tau^-alpha * G(tau) with
    # G = (delta - F)/tau analytic; its value G(0) is integrated in closed form
    # (int_0^1 tau^-alpha = 1/(1-alpha)) and the remainder tau^-alpha (G - G(0)) = O(tau^(1-alpha))
    # by Gauss-Legendre on panels [2^-(k+1), 2^-k], k = 0..79, graded towards 0.
    tau0 = 1.0
    xl, wl = special.roots_legendre(20)
    tq_list, wq_list = [], []
    for k in range(80):
        lo, hi = tau0 * 2.0 ** (-k - 1), tau0 * 2.0 ** (-k)
        tq_list.append((hi - lo) / 2.0 * xl + (hi + lo) / 2.0)
        wq_list.append(wl * (hi - lo) / 2.0)
    tq = np.concatenate(tq_list)
    wq = np.concatenate(wq_list) * tq ** (-alpha)
    F = special.ive(ls[None, :], 2.0 * tq[:, None])  # (Q, n)
    Fs = F / tq[:, None]  # one factor divided by tau: prod_i F_{l_i} / tau stays smooth
    # G(0) of prod_i F_{l_i}/tau: 1 when |l|_1 = 1, else 0
    G0 = np.zeros((n,) * d)
    if n > 1:
        for i in range(d):
            idx = [0] * d
            idx[i] = 1
            G0[tuple(idx)] = 1.0
    if d == 1:
        r1 = wq @ Fs
    else:
        r1 = (Fs * wq[:, None]).T @ F
    r1 = r1 - G0 * float(np.sum(wq)) + G0 * tau0 ** (1.0 - alpha) / (1.0 - alpha)
    # l = 0: integrand (1 - F_0(tau))/tau with G(0) = 2d; 1 - F_0 from the series of I_0
    # (no cancellation for small tau)
    one_minus_F0 = -np.expm1(d * (np.log1p(_i0_minus_one_series(tq)) - 2.0 * tq))
    r1[(0,) * d] = -(float(np.sum(wq * (one_minus_F0 / tq - 2.0 * d)))
                     + 2.0 * d * tau0 ** (1.0 - alpha) / (1.0 - alpha))
    total -= r1

    # --- region 2: tau in [1, tau1], u = log tau, integrand (delta - F) e^{-alpha u}
    tau1 = max(200.0, 20.0 * float(n - 1) ** 2)
    u0, u1 = math.log(tau0), math.log(tau1)
    npan = int(math.ceil((u1 - u0) / 0.25))
    xl, wl = special.roots_legendre(24)
    edges = np.linspace(u0, u1, npan + 1)
    for p in range(npan):
        a_, b_ = edges[p], edges[p + 1]
        u = (b_ - a_) / 2.0 * xl + (a_ + b_) / 2.0
        w = wl * (b_ - a_) / 2.0
        tau = np.exp(u)
        wt = w * np.exp(-alpha * u)
        Fp = special.ive(ls[None, :], 2.0 * tau[:, None])
        accumulate(wt, Fp, np.ones_like(tau))

    # --- region 3: tau in [tau1, inf)
    # delta term: int tau^(-1-alpha) = tau1^-alpha / alpha
    total[(0,) * d] += tau1 ** (-alpha) / alpha
    K = 10
    s = _bessel_asymptotic_coeffs(ls, K)  # (K+1, n), series in x^-k with x = 2 tau
    if d == 1:
        coef = s  # c_m(l)
    else:
        coef = np.zeros((2 * K + 1, n, n))
        for k1 in range(K + 1):
            for k2 in range(K + 1):
                coef[k1 + k2] += np.outer(s[k1], s[k2])
    # F(tau) ~ (4 pi tau)^(-d/2) sum_m c_m (2 tau)^(-m)
    for m in range(coef.shape[0]):
        p = alpha + d / 2.0 + m
        integral = (4.0 * math.pi) ** (-d / 2.0) * 2.0 ** (-m) * tau1 ** (-p) / p
        total -= coef[m] * integral
    return C * total


def stencil(omega: float, d: int, n: int) -> np.ndarray:
    """The stencil table a_l, 0 <= l_i <= n-1, shape (n,)*d: the 1D closed form for
    d = 1 (eq. fourier-coeff-1d), the subordination integral for d = 2 (eq. fourier-coeff)."""
    if d == 1:
        return stencil_1d_closed(omega, n)
    if d == 2:
        return stencil_subordination(omega, 2, n)
    raise ValueError("d must be 1 or 2")


def tau_eigenvalues(a: np.ndarray) -> np.ndarray:
    """Eigenvalues of the natural tau matrix tau(B) = B - (Hankel part) of the (multilevel)
    symmetric Toeplitz matrix with stencil a (§5 Remark, tau preconditioner): the truncated
    symbol  sum_{|l_i| < n} a_|l| prod_i cos(l_i theta_{k_i})  at theta_k = k pi/(n+1),
    k = 1..n.  tau(B) = S diag(lambda) S with S the orthonormal DST-I."""
    n = a.shape[0]
    d = a.ndim
    k = np.arange(1, n + 1)
    l = np.arange(n)
    theta = k * math.pi / (n + 1)
    w = np.where(l == 0, 1.0, 2.0)
    Cm = w[:, None] * np.cos(np.outer(l, theta))  # (n_l, n_k)
    if d == 1:
        return Cm.T @ a
    return Cm.T @ a @ Cm


def strang_first_column(a: np.ndarray) -> np.ndarray:
    """First column of Strang's circulant s(B) of the (multilevel) symmetric Toeplitz matrix with
    stencil a (§5.1 Remark, the Strang preconditioner): along every level the central diagonals of
    B are kept and wrapped around the circle, c_l = a_l for 0 <= l <= n//2 and c_l = a_{n-l} for
    n//2 < l < n.  Shape (n,)*d like a."""
    n = a.shape[0]
    l = np.arange(n)
    f = np.where(l <= n // 2, l, n - l)
    if a.ndim == 1:
        return a[f]
    return a[f[:, None], f[None, :]]


def strang_eigenvalues(a: np.ndarray) -> np.ndarray:
    """Eigenvalues of s(B): the d-dimensional DFT of its first column, index k the frequency of
    the Fourier vector exp(2 pi i k.j / n) (real because the column is even along every level)."""
    return np.fft.fftn(strang_first_column(a)).real
