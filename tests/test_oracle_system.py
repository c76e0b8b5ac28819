"""Pins of the oracle's assembly, products and solvers: brute force on tiny inputs,
invariants of §5, and the printed condition numbers / GMRES iteration counts of §6."""
import dataclasses
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import krylov, matfree, system, workloads
from paper_2507_02809_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(line.split())
    return rows


PAIRS = [(0.1, 1.9), (0.5, 1.5), (0.9, 1.1)]


def paper_problem(d, n, S, beta, omega, lam=5e-3, eps=0.01):
    inp = inputs.paper_problem(d, n, S, beta, omega, lam, eps)
    return workloads.with_data(inp)


@pytest.fixture(scope="module")
def small1d():
    return workloads.with_data(inputs.small(1, 12, 7))


@pytest.fixture(scope="module")
def small2d():
    return workloads.with_data(inputs.small(2, 6, 5, beta=0.6, omega=1.6, alpha=1e-3))


def test_A_time_structure_exact_on_linear_in_t(small1d):
    """A applied to v^(s) = psi (a + c t_s), f~ = 0: block row s minus its spatial part
    c_t D_2 B v^(s) equals D_1^(s) psi (c dt s^(1-beta) + a b_{s-1})  (L1 exactness, §4)."""
    p = small1d
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(p.Nd)
    a, c = 0.7, -1.3
    t = p.dt * np.arange(1, p.S + 1)
    Y = np.zeros((p.S + 1, p.Nd))
    Y[:p.S] = np.outer(a + c * t, psi)
    Z = (system.dense_A(p) @ Y.ravel()).reshape(p.S + 1, p.Nd)
    B = system.dense_B(p)
    b = p.b()
    for s in range(p.S):
        hist = Z[s] - p.c_t * p.gamma2[s] * (B @ Y[s])
        expect = p.gamma1[s] * psi * (c * p.dt * (s + 1) ** (1 - p.beta) + a * b[s])
        np.testing.assert_allclose(hist, expect, rtol=1e-12, atol=1e-12)
    # last block row: y^(S) + c_f D_2^(S) B f~ with f~ = 0
    np.testing.assert_allclose(Z[p.S], Y[p.S - 1], rtol=0, atol=0)


@pytest.mark.parametrize("which", ["small1d", "small2d"])
def test_rhs_rho_term_completes_the_L1_formula(which, request):
    """The initial state rho = v^(0) enters z^(s) = b_{s-1} D_1^(s) rho (§5, eq. lin-syst): with
    rho = a psi and v^(s) = psi (a + c t_s), f~ = 0, block row s of A y - z minus its spatial
    part c_t D_2^(s) B v^(s) is the L1 formula (§4, eq. L1-formula) applied to a + c t with its
    v^(0) term, which is exact on functions linear in t: D_1^(s) psi c dt s^(1-beta)."""
    p0 = request.getfixturevalue(which)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(p0.Nd)
    a, c = 1.9, -0.8
    p = dataclasses.replace(p0, rho=a * psi)
    t = p.dt * np.arange(1, p.S + 1)
    Y = np.zeros((p.S + 1, p.Nd))
    Y[:p.S] = np.outer(a + c * t, psi)
    R = (matfree.matvec(p, Y.ravel()) - system.rhs_z(p)).reshape(p.S + 1, p.Nd)
    BY = matfree.apply_B(p, Y[:p.S])
    for s in range(p.S):
        hist = R[s] - p.c_t * p.gamma2[s] * BY[s]
        expect = p.gamma1[s] * psi * c * p.dt * (s + 1) ** (1 - p.beta)
        np.testing.assert_allclose(hist, expect, rtol=0, atol=1e-12 * np.abs(psi).max())
    # without the rho term of z the a-part of the L1 formula would remain: a b_{s-1} D_1 psi
    R0 = (matfree.matvec(p, Y.ravel()) - system.rhs_z(dataclasses.replace(p, rho=0 * psi))).reshape(p.S + 1, p.Nd)
    assert np.abs(R0[p.S - 1] - R[p.S - 1]).max() > 0.1 * a * np.abs(psi).max() * p.b()[p.S - 1]


@pytest.mark.parametrize("which", ["small1d", "small2d"])
def test_matvec_matches_dense(which, request):
    p = request.getfixturevalue(which)
    A = system.dense_A(p)
    rng = np.random.default_rng(1)
    for _ in range(3):
        y = rng.standard_normal(p.n_tot)
        ref = A @ y
        np.testing.assert_allclose(matfree.matvec(p, y), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        for s, j in [(0, 0), (p.S - 1, p.Nd - 1), (p.S, 3), (2, p.Nd // 2)]:
            assert matfree.matvec_entry(p, y, s, j) == pytest.approx(ref[s * p.Nd + j], rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("which", ["small1d", "small2d"])
def test_P_solve_matches_dense_lu(which, request):
    p = request.getfixturevalue(which)
    P = system.dense_P(p)
    rng = np.random.default_rng(2)
    z = rng.standard_normal(p.n_tot)
    ref = np.linalg.solve(P, z)
    np.testing.assert_allclose(matfree.P_solve(p, z), ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(matfree.P_solve(p, z, inner="cg", inner_tol=1e-14), ref,
                               rtol=0, atol=1e-9 * np.abs(ref).max())


def test_forward_solve_is_Ahat_inverse(small2d):
    p = small2d
    rng = np.random.default_rng(3)
    f = rng.standard_normal(p.Nd)
    zh = system.rhs_zhat(p, f)
    v = matfree.forward_solve(p, zh)
    np.testing.assert_allclose(system.dense_Ahat(p) @ v, zh, rtol=0, atol=1e-11 * np.abs(zh).max())


def test_P_inverse_A_structure(small2d):
    """P^{-1} A = [[I, U], [0, Y]]: A - P is nonzero only in the last block column of rows 1..S,
    so rank(A - P) = Nd and the first S*Nd columns of P^{-1}A are identity columns (§5.1)."""
    p = small2d
    A = system.dense_A(p)
    P = system.dense_P(p)
    R = A - P
    assert np.linalg.matrix_rank(R) == p.Nd
    M = np.linalg.solve(P, A)
    k = p.S * p.Nd
    np.testing.assert_allclose(M[:, :k], np.eye(p.n_tot)[:, :k], atol=1e-12)
    ev = np.linalg.eigvals(M)
    assert np.sum(np.abs(ev - 1) < 1e-8) >= k


def test_c1_solvers_agree():
    """Dense LU vs textbook GMRES (none / left / right) vs FGMRES on the d=1, N=63, M=32 workload."""
    p = workloads.with_data(inputs.c1())
    A = system.dense_A(p)
    P = system.dense_P(p)
    b = system.rhs_z(p)
    x_lu = np.linalg.solve(A, b)
    f_lu = x_lu[p.S * p.Nd:]
    lu = sl.lu_factor(P)
    Pinv = lambda v: sl.lu_solve(lu, v)
    Aop = lambda v: A @ v
    for kw in ({"M_left": Pinv}, {"M_right": Pinv}):
        x, it, _ = krylov.gmres(Aop, b, 1e-13, 400, **kw)
        assert np.linalg.norm(x[p.S * p.Nd:] - f_lu) <= 1e-10 * np.linalg.norm(f_lu)
    x, it, _ = krylov.fgmres(Aop, Pinv, b, 1e-13, 50, 400)
    assert np.linalg.norm(x[p.S * p.Nd:] - f_lu) <= 1e-10 * np.linalg.norm(f_lu)
    x, it, _ = krylov.fgmres(lambda v: matfree.matvec(p, v), lambda v: matfree.P_solve(p, v), b,
                             1e-13, 50, 400)
    assert np.linalg.norm(x[p.S * p.Nd:] - f_lu) <= 1e-10 * np.linalg.norm(f_lu)
    # the reconstruction is meaningful: noise 1e-3, alpha = 1e-3
    assert np.linalg.norm(f_lu - inputs.c1().f_true) < 0.2 * np.linalg.norm(inputs.c1().f_true)


def test_tiny_2d_solvers_agree(small2d):
    p = small2d
    A = system.dense_A(p)
    b = system.rhs_z(p)
    x_lu = np.linalg.solve(A, b)
    x, it, _ = krylov.gmres(lambda v: A @ v, b, 1e-13, p.n_tot)
    assert np.linalg.norm(x - x_lu) <= 1e-9 * np.linalg.norm(x_lu)
    x, it, _ = krylov.fgmres(lambda v: matfree.matvec(p, v), lambda v: matfree.P_solve(p, v), b,
                             1e-13, 30, 300)
    assert np.linalg.norm(x - x_lu) <= 1e-10 * np.linalg.norm(x_lu)


def test_noise_free_recovery_improves_with_smaller_alpha():
    errs = []
    for alpha in (1e-2, 1e-4, 1e-6):
        inp = inputs.synthetic(1, 31, 16, 0.5, 1.5, alpha, config_id=7, modes=3, noise_level=0.0)
        p = workloads.with_data(inp)
        x = np.linalg.solve(system.dense_A(p), system.rhs_z(p))
        errs.append(np.linalg.norm(x[p.S * p.Nd:] - inp.f_true) / np.linalg.norm(inp.f_true))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def _t1_rows():
    out = []
    for r in read_table("paper_1d_condnum.txt"):
        n, S = int(r[0]), int(r[1])
        if n * (S + 1) <= 2100:
            for k, (beta, omega) in enumerate(PAIRS):
                out.append((n, S, beta, omega, float(r[2 + 2 * k]), float(r[3 + 2 * k])))
    return out


@pytest.mark.parametrize("n,S,beta,omega,condA,condPA", _t1_rows())
def test_paper_1d_condition_numbers(n, S, beta, omega, condA, condPA):
    """The 1D table of 2-norm condition numbers in §6.1 (lambda = 5e-3): pins the grid
    (h = pi/(n+1)), eta, the e_m weights, the 1D stencil and the block structure of A and P."""
    p = workloads.problem(inputs.paper_problem(1, n, S, beta, omega, 5e-3))
    A = system.dense_A(p)
    P = system.dense_P(p)
    cA = np.linalg.cond(A)
    cPA = np.linalg.cond(np.linalg.solve(P, A))
    assert abs(cA - condA) <= max(0.51, 1e-3 * condA)
    assert abs(cPA - condPA) <= max(0.51, 1e-3 * condPA)


def _t2_rows():
    out = []
    for r in read_table("paper_1d_gmres.txt"):
        n, S = int(r[0]), int(r[1])
        if n * (S + 1) <= 2100:
            for k, (beta, omega) in enumerate(PAIRS):
                out.append((n, S, beta, omega, r[2 + 4 * k], int(r[3 + 4 * k])))
    return out


@pytest.mark.parametrize("n,S,beta,omega,it_none,it_P", _t2_rows())
def test_paper_1d_gmres_iterations(n, S, beta, omega, it_none, it_P):
    """The 1D GMRES table of §6.1: preconditioned iteration counts within 2 (left preconditioning,
    MATLAB's convention; x0 = 0, tol 1e-8, maxit = min(size, 1000); noise 0.01 * ||mu|| * U(-1,1))."""
    p = paper_problem(1, n, S, beta, omega)
    A = system.dense_A(p)
    lu = sl.lu_factor(system.dense_P(p))
    b = system.rhs_z(p)
    maxit = min(p.n_tot, 1000)
    _, it, _ = krylov.gmres(lambda v: A @ v, b, 1e-8, maxit, M_left=lambda v: sl.lu_solve(lu, v))
    assert abs(it - it_P) <= 2
    if n == 16 and S == 16:
        _, it0, _ = krylov.gmres(lambda v: A @ v, b, 1e-8, maxit)
        assert abs(it0 - int(it_none)) <= 0.05 * int(it_none)


@pytest.mark.xfail(strict=True, reason=(
    "The 2D tables of §6.2 are not reproduced by the stated 2D setup (Omega=(0,pi)^2, "
    "gamma1=t e^(x1+x2), gamma2=t^2 x1 x2, q=t^2, lambda=5e-3, h=pi/(n+1), stencil of eq. "
    "fourier-coeff); the 1D tables are reproduced exactly by the same code.  The 2D assembly is "
    "pinned instead by the dense/FFT matvec agreement, the stencil pins and the closed-form "
    "fractional Laplacian consistency."))
def test_paper_2d_gmres_iterations_16_16():
    r = read_table("paper_2d_gmres.txt")[0]
    assert int(r[0]) == 16 and int(r[1]) == 16
    beta, omega = PAIRS[0]
    p = paper_problem(2, 16, 16, beta, omega)
    A = system.dense_A(p)
    lu = sl.lu_factor(system.dense_P(p))
    _, it, _ = krylov.gmres(lambda v: A @ v, system.rhs_z(p), 1e-8, 1000,
                            M_left=lambda v: sl.lu_solve(lu, v))
    assert abs(it - int(r[3])) <= 2


# ---------------------------------------------------------------------------
# T_{n,S} (§5.1 Remark): B_n replaced by its tau matrix
# ---------------------------------------------------------------------------
def _hankel_part(a1: np.ndarray) -> np.ndarray:
    """H of the natural tau splitting T = tau(T) + H for a symmetric Toeplitz matrix with first
    column a1 (Bini–Capovani), 0-based with k = i + j: H_ij = a_{k+2} for k <= n-3 (upper-left
    anti-diagonals) and a_{2n-k} for k >= n+1 (lower-right), zero in between."""
    n = a1.shape[0]
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            k = i + j
            if k <= n - 3:
                H[i, j] = a1[k + 2]
            elif k >= n + 1:
                H[i, j] = a1[2 * n - k]
    return H


def test_dense_tauB_is_the_natural_tau_matrix_1d():
    """1D: dense_tauB = B - H, the natural tau matrix written out from the Toeplitz entries."""
    p = workloads.problem(inputs.small(1, 17, 4))
    B = system.dense_B(p)
    np.testing.assert_allclose(system.dense_tauB(p), B - _hankel_part(p.a()), atol=1e-14)


def test_dense_tauB_2d_is_diagonalised_by_the_2d_sine_transform():
    """2D: tau(B) is diagonalised by S (x) S with the truncated symbol as its eigenvalues (the
    symbol itself is pinned against the natural tau matrix in test_oracle_coeffs)."""
    p = workloads.problem(inputs.small(2, 6, 3))
    tB = system.dense_tauB(p)
    S1 = system.dst1_matrix(p.N)
    S = np.kron(S1, S1)
    D = S @ tB @ S
    np.testing.assert_allclose(D, np.diag(np.diag(D)), atol=1e-12)
    np.testing.assert_allclose(np.diag(D), system.coeffs.tau_eigenvalues(p.a()).reshape(-1), rtol=1e-12)
    np.testing.assert_allclose(tB, tB.T, atol=1e-14)


def test_dense_T_constant_coefficients_is_P_with_tau():
    """For constant gamma1, gamma2 the frozen-coefficient T equals P with every B replaced by
    tau(B) — the paper's T_{n,S} exactly."""
    inp = inputs.small(2, 5, 4)
    p = workloads.problem(inp)
    p = dataclasses.replace(p, gamma1=np.full_like(p.gamma1, 1.3), gamma2=np.full_like(p.gamma2, 0.7))
    np.testing.assert_allclose(system.dense_T(p), system.dense_P(p, system.dense_tauB(p)), atol=1e-13)


@pytest.mark.parametrize("d,N,M", [(1, 15, 6), (2, 7, 4)])
def test_T_solve_matches_dense_T(d, N, M):
    """Matrix-free T_{n,S}^{-1} (DST-I block solves) against LU of the assembled T."""
    p = workloads.problem(inputs.small(d, N, M))
    z = np.random.default_rng(3).standard_normal(p.n_tot)
    np.testing.assert_allclose(matfree.T_solve(p, z), np.linalg.solve(system.dense_T(p), z),
                               rtol=1e-11, atol=1e-12 * np.abs(z).max())


def test_fgmres_with_T_reaches_the_dense_solution():
    """T_{n,S} as a right preconditioner changes only the path of the Krylov solve."""
    p = workloads.problem(inputs.small(2, 7, 5))
    b = system.rhs_z(p)
    x_lu = np.linalg.solve(system.dense_A(p), b)
    A = system.dense_A(p)
    x, its, _ = krylov.fgmres(lambda v: A @ v, lambda v: matfree.T_solve(p, v), b, tol=1e-13, restart=60,
                              maxit=300)
    np.testing.assert_allclose(x, x_lu, rtol=1e-9, atol=1e-10 * np.abs(x_lu).max())


@pytest.mark.parametrize("d,N", [(1, 9), (1, 10), (2, 5), (2, 6)])
def test_dense_strangB_is_a_symmetric_circulant_keeping_the_central_diagonals(d, N):
    """s(B) is a d-level circulant, symmetric, and equal to B wherever every per-level lag is at
    most N//2 (Strang's construction), checked entry by entry against dense_B."""
    p = workloads.problem(inputs.small(d, N, 2))
    C = system.dense_strangB(p)
    B = system.dense_B(p)
    np.testing.assert_allclose(C, C.T, atol=0)
    idx = np.indices((N,) * d).reshape(d, -1).T  # multi-index of every row, last level fastest
    for r in range(0, C.shape[0], 3):
        for c in range(C.shape[1]):
            lag = np.abs(idx[r] - idx[c])
            if np.all(lag <= N // 2):
                assert C[r, c] == B[r, c]
            shifted = ((idx[r] + 1) % N, (idx[c] + 1) % N)  # one step along every level
            rr = np.ravel_multi_index(tuple(shifted[0]), (N,) * d)
            cc = np.ravel_multi_index(tuple(shifted[1]), (N,) * d)
            assert C[rr, cc] == C[r, c]


@pytest.mark.parametrize("d,N", [(1, 9), (1, 10), (2, 6), (2, 7)])
def test_strang_eigenvalues_match_a_dense_eigensolver(d, N):
    """The DFT eigenvalues of s(B) against LAPACK's symmetric eigensolver on the assembled matrix."""
    p = workloads.problem(inputs.small(d, N, 2))
    lam = np.sort(system.coeffs.strang_eigenvalues(p.a()).reshape(-1))
    ref = np.linalg.eigvalsh(system.dense_strangB(p))
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert lam.min() > 0.0  # s(B) of the fractional stencil is SPD


def test_dense_S_constant_coefficients_is_P_with_strang():
    """For constant gamma1, gamma2 the frozen-coefficient S equals P with every B replaced by
    s(B) — the paper's S_{n,S} exactly."""
    p = workloads.problem(inputs.small(2, 5, 4))
    p = dataclasses.replace(p, gamma1=np.full_like(p.gamma1, 1.3), gamma2=np.full_like(p.gamma2, 0.7))
    np.testing.assert_allclose(system.dense_S(p), system.dense_P(p, system.dense_strangB(p)), atol=1e-13)


@pytest.mark.parametrize("d,N,M", [(1, 15, 6), (1, 12, 5), (2, 7, 4), (2, 6, 3)])
def test_S_solve_matches_dense_S(d, N, M):
    """Matrix-free S_{n,S}^{-1} (FFT block solves) against LU of the assembled S."""
    p = workloads.problem(inputs.small(d, N, M))
    z = np.random.default_rng(4).standard_normal(p.n_tot)
    np.testing.assert_allclose(matfree.S_solve(p, z), np.linalg.solve(system.dense_S(p), z),
                               rtol=1e-11, atol=1e-12 * np.abs(z).max())


def test_fgmres_with_S_reaches_the_dense_solution():
    """S_{n,S} as a right preconditioner changes only the path of the Krylov solve."""
    p = workloads.problem(inputs.small(2, 7, 5))
    b = system.rhs_z(p)
    A = system.dense_A(p)
    x_lu = np.linalg.solve(A, b)
    x, its, _ = krylov.fgmres(lambda v: A @ v, lambda v: matfree.S_solve(p, v), b, tol=1e-13, restart=60,
                              maxit=300)
    np.testing.assert_allclose(x, x_lu, rtol=1e-9, atol=1e-10 * np.abs(x_lu).max())
