"""Pins of the oracle's coefficient routines against closed forms, invariants and
special cases fixed by the paper (§4 eqs. L1-formula, fourier-coeff, fourier-coeff-1d,
Lemma 1) and by textbook mathematics."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import coeffs


@pytest.mark.parametrize("beta", [0.1, 0.5, 0.6, 0.9])
def test_l1_weights_invariants(beta):
    S = 300
    b = coeffs.l1_b(beta, S)
    e = coeffs.l1_e(beta, S)
    s = np.arange(1, S + 1)
    # telescoping: sum_{m<s} b_m = s^(1-beta)
    np.testing.assert_allclose(np.cumsum(b), s ** (1.0 - beta), rtol=1e-13)
    # e_0 = b_0 = 1 and e_m = b_m - b_{m-1}: the two printed forms agree
    assert e[0] == 1.0 == b[0]
    np.testing.assert_allclose(e[1:], b[1:] - b[:-1], rtol=1e-10, atol=1e-16)
    # sum_{m<s} e_m = b_{s-1}
    np.testing.assert_allclose(np.cumsum(e), b, rtol=1e-12, atol=1e-15)
    # e_m < 0 for m >= 1 (b_m is strictly decreasing for beta in (0,1))
    assert np.all(e[1:] < 0.0)


@pytest.mark.parametrize("beta", [0.2, 0.6, 0.9])
def test_l1_formula_exact_on_linear_functions(beta):
    """The L1 formula interpolates piecewise linearly, so it is exact on v(t) = a + c t:
    Caputo derivative c t^(1-beta)/Gamma(2-beta).  In the e-weight form of eq. numer-scheme:
        e_0 v_s + sum_{m=1}^{s-1} e_{s-m} v_m - b_{s-1} v_0 = c dt s^(1-beta)."""
    S, T, a, c = 64, 1.7, 0.3, -2.1
    dt = T / S
    t = dt * np.arange(S + 1)
    v = a + c * t
    e = coeffs.l1_e(beta, S)
    b = coeffs.l1_b(beta, S)
    for s in range(1, S + 1):
        lhs = sum(e[s - m] * v[m] for m in range(1, s + 1)) - b[s - 1] * v[0]
        exact = c * dt ** beta * math.gamma(2 - beta) * t[s] ** (1 - beta) / math.gamma(2 - beta)
        assert abs(lhs - exact) <= 1e-13 * max(1.0, abs(exact))
        # with the eta scaling of §5: eta * D^beta t = c * dt * s^(1-beta)
        assert abs(lhs - c * dt * s ** (1 - beta)) <= 1e-13


def test_eta():
    assert coeffs.eta(0.5, 0.25) == pytest.approx(0.5 * math.gamma(1.5), rel=1e-15)


@pytest.mark.parametrize("omega", [1.05, 1.2, 1.5, 1.6, 1.8, 1.95])
def test_stencil_1d_closed_form_vs_lemma1(omega):
    n = 600
    a = coeffs.stencil_1d_closed(omega, n)
    r = coeffs.stencil_1d_recursion(omega, n)
    np.testing.assert_allclose(a, r, rtol=2e-13, atol=0)
    # Lemma 1(a): a_0 = Gamma(omega+1)/Gamma(omega/2+1)^2 >= 0, a_l < 0 for l != 0
    assert a[0] == pytest.approx(math.gamma(omega + 1) / math.gamma(omega / 2 + 1) ** 2, rel=1e-15)
    assert np.all(a[1:] < 0)
    # Lemma 1(c): coefficients sum to zero; the partial sums decay like the tail
    # 2 c_omega L^-omega / omega of the far field -c_omega |l|^(-1-omega)
    for L in (100, 400, 599):
        partial = a[0] + 2 * a[1:L + 1].sum()
        tail = 2 * coeffs.c_omega(omega, 1) * L ** (-omega) / omega
        assert partial > 0
        assert partial == pytest.approx(tail, rel=0.02)


def test_stencil_1d_special_cases():
    # omega = 1: the Fourier coefficients of |2 sin(theta/2)| are 4/(pi (1 - 4 l^2))
    a = coeffs.stencil_1d_closed(1.0, 50)
    l = np.arange(50)
    np.testing.assert_allclose(a, 4 / (math.pi * (1 - 4 * l ** 2)), rtol=1e-14)
    # omega = 2: 4 sin^2(theta/2) = 2 - 2 cos(theta): the second difference [-1, 2, -1]
    a = coeffs.stencil_1d_closed(2.0, 10)
    np.testing.assert_allclose(a, [2, -1, 0, 0, 0, 0, 0, 0, 0, 0], atol=1e-15)


@pytest.mark.parametrize("omega", [1.1, 1.5, 1.6, 1.9])
def test_subordination_route_reproduces_1d_closed_form(omega):
    """The d-dimensional route (Bochner subordination + modified Bessel functions), run at
    d = 1, against eq. fourier-coeff-1d: this pins the quadrature the 2D table relies on."""
    n = 300
    np.testing.assert_allclose(coeffs.stencil_subordination(omega, 1, n),
                               coeffs.stencil_1d_closed(omega, n), rtol=1e-13, atol=5e-15)


@pytest.fixture(scope="module")
def a2d():
    return {om: coeffs.stencil_subordination(om, 2, 128) for om in (1.1, 1.6, 1.9)}


@pytest.mark.parametrize("omega", [1.1, 1.6, 1.9])
def test_stencil_2d_parseval(a2d, omega):
    """sum_{l in Z^2} a_l^2 = (2 pi)^-2 int g^2 (Parseval for eq. fourier-coeff).  The table
    covers |l_i| <= 127; the omitted tail is O(127^(-2-2 omega)) < 1e-9."""
    a = a2d[omega]
    w = np.where(np.arange(a.shape[0]) == 0, 1.0, 2.0)
    lhs = float(w @ (a ** 2) @ w)
    g2 = lambda t2, t1: (4 * math.sin(t1 / 2) ** 2 + 4 * math.sin(t2 / 2) ** 2) ** omega
    val, err = integrate.dblquad(g2, 0, math.pi, 0, math.pi, epsabs=1e-13, epsrel=1e-13)
    rhs = 4 * val / (2 * math.pi) ** 2
    assert lhs == pytest.approx(rhs, rel=2e-9)


@pytest.mark.parametrize("omega", [1.1, 1.6, 1.9])
def test_stencil_2d_structure_and_far_field(a2d, omega):
    a = a2d[omega]
    np.testing.assert_allclose(a, a.T, rtol=1e-13, atol=0)  # g symmetric in (theta_1, theta_2)
    assert a[0, 0] > 0 and np.all(a.ravel()[1:] < 0)
    # the stencil discretises c_omega * int (u(x)-u(y))/|x-y|^(d+omega): a_l ~ -c_omega |l|^(-2-omega)
    c = coeffs.c_omega(omega, 2)
    for l1, l2, tol in ((40, 30, 2e-3), (100, 60, 5e-4)):
        assert a[l1, l2] == pytest.approx(-c * math.hypot(l1, l2) ** (-2 - omega), rel=tol)
    # a_0 = (2 pi)^-2 int g
    val, _ = integrate.dblquad(lambda t2, t1: (4 * math.sin(t1 / 2) ** 2 + 4 * math.sin(t2 / 2) ** 2)
                               ** (omega / 2), 0, math.pi, 0, math.pi, epsabs=1e-14, epsrel=1e-14)
    assert a[0, 0] == pytest.approx(4 * val / (2 * math.pi) ** 2, rel=1e-12)


def test_tau_eigenvalues_match_natural_tau_matrix():
    """tau(T) = T - H (H the Hankel part built from t_2..t_{n-1}) is diagonalised by the DST-I
    and its eigenvalues are the truncated symbol at k pi/(n+1) (§5 Remark, tau preconditioner)."""
    import scipy.linalg as sl
    n = 20
    t = coeffs.stencil_1d_closed(1.5, n)
    T = sl.toeplitz(t)
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            k = i + j
            if k <= n - 3:
                H[i, j] = t[k + 2]
            elif k >= n + 1:
                H[i, j] = t[2 * n - k]
    Sm = math.sqrt(2 / (n + 1)) * np.sin(np.outer(np.arange(1, n + 1), np.arange(1, n + 1)) * math.pi / (n + 1))
    D = Sm @ (T - H) @ Sm
    assert np.abs(D - np.diag(np.diag(D))).max() < 1e-13
    np.testing.assert_allclose(np.diag(D), coeffs.tau_eigenvalues(t), rtol=1e-13)
    # 2-level: for a separable stencil the tau matrix is the Kronecker product
    a2 = np.outer(t[:8], t[:8])
    lam1 = coeffs.tau_eigenvalues(t[:8])
    np.testing.assert_allclose(coeffs.tau_eigenvalues(a2), np.outer(lam1, lam1), rtol=1e-13)


@pytest.mark.parametrize("d,omega", [(1, 1.5), (1, 1.8), (2, 1.6)])
def test_stencil_consistency_with_closed_form_fractional_laplacian(d, omega):
    """(-Delta)^(omega/2) (1-|x|^2)_+^(omega/2) = 2^omega Gamma(1+omega/2) Gamma((d+omega)/2)/Gamma(d/2)
    on the unit ball.  The discrete operator h^-omega sum_l a_l v_{j+l} (eq. discrete-laplacian) on
    (-1,1)^d must approach it at |x| <= 1/2 as h halves."""
    from oracle.system import Problem
    from oracle.matfree import apply_B
    K = 2 ** omega * math.gamma(1 + omega / 2) * math.gamma((d + omega) / 2) / math.gamma(d / 2)
    errs = []
    Ns = (63, 127, 255, 511) if d == 1 else (31, 63, 127)
    for N in Ns:
        h = 2.0 / (N + 1)
        x = -1 + h * np.arange(1, N + 1)
        if d == 1:
            r2 = x ** 2
        else:
            X1, X2 = np.meshgrid(x, x, indexing="ij")
            r2 = (X1 ** 2 + X2 ** 2).ravel()
        v = np.clip(1 - r2, 0, None) ** (omega / 2)
        p = Problem(d=d, N=N, S=1, T=1.0, beta=0.5, omega=omega, alpha=1.0, gamma1=np.ones((1, N ** d)),
                    gamma2=np.ones((1, N ** d)), q=np.ones(1), rho=np.zeros(N ** d), mu=np.zeros(N ** d),
                    length=2.0)
        Lv = apply_B(p, v) / h ** omega
        inner = r2 <= 0.25
        errs.append(np.abs(Lv[inner] - K).max() / K)
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.05, errs
