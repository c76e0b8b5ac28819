"""Pins of the adjoint oracle (oracle/adjoint.py) against what does not depend on its formulas:
the adjoint identity with the matrix-free product A y of the paper's algorithm, central finite
differences of f~ in alpha, and the exact linearity of f~ in mu."""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint, matfree, system, workloads
from paper_2507_02809_amd import inputs

CASES = [
    ("1d", lambda: inputs.small(1, 12, 7)),
    ("2d", lambda: inputs.small(2, 6, 5, beta=0.6, omega=1.6)),
    ("2d_odd", lambda: inputs.small(2, 7, 4, beta=0.3, omega=1.2)),
]


@pytest.fixture(params=CASES, ids=[c[0] for c in CASES])
def prob(request):
    return workloads.with_data(request.param[1]())


def f_tilde(p):
    return np.linalg.solve(system.dense_A(p), system.rhs_z(p))[p.S * p.Nd:]


def test_transpose_satisfies_adjoint_identity(prob):
    """<A x, w> = <x, A^T w> with A x by the FFT-based matrix-free product (not the dense matrix)."""
    rng = np.random.default_rng(5)
    for _ in range(3):
        x = rng.standard_normal(prob.n_tot)
        w = rng.standard_normal(prob.n_tot)
        lhs = float(matfree.matvec(prob, x) @ w)
        rhs = float(x @ adjoint.apply_AT(prob, w))
        assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(x) * np.linalg.norm(w) * prob.c_t * 10 + abs(lhs))


def test_grad_alpha_matches_central_difference(prob):
    rng = np.random.default_rng(6)
    gf = rng.standard_normal(prob.Nd)
    _, ga, _ = adjoint.vjp(prob, gf)
    h = 1e-5 * prob.alpha
    lp = gf @ f_tilde(dataclasses.replace(prob, alpha=prob.alpha + h))
    lm = gf @ f_tilde(dataclasses.replace(prob, alpha=prob.alpha - h))
    fd = (lp - lm) / (2 * h)
    assert ga == pytest.approx(fd, rel=1e-6)


def test_grad_mu_is_exact_for_the_linear_map(prob):
    """f~ is linear in mu_eps, so gf . (f~(mu + d) - f~(mu)) = grad_mu . d exactly (up to rounding)."""
    rng = np.random.default_rng(7)
    gf = rng.standard_normal(prob.Nd)
    gmu, _, _ = adjoint.vjp(prob, gf)
    d = rng.standard_normal(prob.Nd)
    lhs = gf @ (f_tilde(system.with_mu(prob, prob.mu + d)) - f_tilde(prob))
    assert lhs == pytest.approx(gmu @ d, rel=1e-9)


def test_PT_solve_inverts_the_transposed_block_triangle(prob):
    """P^{-T} g solves the block upper-triangular P^T: back-substituted block by block from the
    last block, with the blocks of P (not a dense solve of the whole matrix)."""
    rng = np.random.default_rng(8)
    g = rng.standard_normal(prob.n_tot)
    lam = adjoint.PT_solve(prob, g)
    PT = system.dense_P(prob).T
    S, Nd = prob.S, prob.Nd
    ref = np.zeros(prob.n_tot)
    for s in range(S, -1, -1):
        blk = slice(s * Nd, (s + 1) * Nd)
        r = g[blk] - PT[blk, (s + 1) * Nd:] @ ref[(s + 1) * Nd:]
        ref[blk] = np.linalg.solve(PT[blk, blk], r)
    assert np.abs(lam - ref).max() <= 1e-10 * np.abs(ref).max()
    # P^T is block upper triangular: nothing below the diagonal blocks
    for s in range(S + 1):
        assert not PT[(s + 1) * Nd:, s * Nd:(s + 1) * Nd].any()


def test_grad_gamma2_matches_central_differences(prob):
    """Sampled entries of dL/dgamma2 against central differences of gf . f~ in that one sample
    (including the last time level, where gamma2 also scales the final-condition block)."""
    rng = np.random.default_rng(9)
    gf = rng.standard_normal(prob.Nd)
    G = adjoint.grad_gamma2(prob, gf)
    S, Nd = prob.S, prob.Nd
    # samples where the gradient is well above the finite differences' rounding noise
    samples = [(s, int(np.argmax(np.abs(G[s])))) for s in (0, S // 2, S - 1)]
    big = np.flatnonzero(np.abs(G[S - 1]) > 0.1 * np.abs(G[S - 1]).max())
    samples.append((S - 1, int(big[len(big) // 2])))
    for s, j in samples:
        h = 1e-6 * prob.gamma2[s, j]
        vals = []
        for sign in (1, -1):
            g2 = prob.gamma2.copy()
            g2[s, j] += sign * h
            vals.append(gf @ f_tilde(dataclasses.replace(prob, gamma2=g2)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert G[s, j] == pytest.approx(fd, rel=1e-5)


@pytest.mark.parametrize("d,N,M", [(1, 9, 6), (2, 5, 4)])
def test_matvec_T_entry_matches_dense_transpose(d, N, M):
    """Entries of A^T w summed down the columns of the block definition agree with the dense A^T."""
    inp = inputs.small(d, N, M, beta=0.4, omega=1.7)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    w = np.random.default_rng(7).standard_normal(p.n_tot)
    ref = system.dense_A(p).T @ w
    for m in range(p.S + 1):
        for j in range(p.Nd):
            assert abs(adjoint.matvec_T_entry(p, w, m, j) - ref[m * p.Nd + j]) <= 1e-12 * np.abs(ref).max()
