"""Spectral properties the solver relies on (§5.1): P^{-1} A differs from the identity by a matrix of
rank at most N^d (A - P is the upper-right block column), so at least n_tot - N^d of its eigenvalues
equal 1; and the oracle's Arnoldi (classical Gram-Schmidt twice) satisfies the Arnoldi relation and
recovers that spectrum when run to full dimension."""
import numpy as np
import pytest

from oracle import krylov, system, workloads
from paper_2507_02809_amd import inputs

CASES = [
    ("1d", lambda: inputs.small(1, 6, 5)),
    ("2d", lambda: inputs.small(2, 3, 4, beta=0.6, omega=1.6)),
]


@pytest.fixture(params=CASES, ids=[c[0] for c in CASES])
def prob(request):
    return workloads.with_data(request.param[1]())


def test_preconditioned_matrix_is_identity_plus_low_rank(prob):
    A, P = system.dense_A(prob), system.dense_P(prob)
    K = np.linalg.solve(P, A)
    assert np.linalg.matrix_rank(K - np.eye(prob.n_tot), tol=1e-9 * np.abs(K).max()) <= prob.Nd
    ev = np.linalg.eigvals(K)
    assert np.sum(np.abs(ev - 1.0) < 1e-7) >= prob.n_tot - prob.Nd


def test_arnoldi_relation_and_full_dimension_ritz_values(prob):
    A, P = system.dense_A(prob), system.dense_P(prob)
    op = lambda v: A @ np.linalg.solve(P, v)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(prob.n_tot)
    k = 8
    H, V = krylov.arnoldi_cgs2(op, b, k)
    m = H.shape[1]
    AV = np.column_stack([op(V[:, j]) for j in range(m)])
    assert np.abs(AV - V[:, :m + 1] @ H).max() <= 1e-10 * np.abs(AV).max()
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() <= 1e-12
    # the Krylov space of A P^{-1} = I + low rank from b closes after N^d + 1 steps (the next
    # subdiagonal entry vanishes up to rounding), and the Ritz values are then eigenvalues of A P^{-1}
    # (which has the spectrum of P^{-1} A)
    kf = prob.Nd + 1
    Hf, _ = krylov.arnoldi_cgs2(op, b, kf)
    assert Hf.shape[1] == kf and abs(Hf[kf, kf - 1]) <= 1e-8 * np.abs(Hf).max()
    ritz = np.linalg.eigvals(Hf[:kf, :])
    ev = np.linalg.eigvals(np.linalg.solve(P, A))
    for r in ritz:
        assert np.min(np.abs(ev - r)) <= 1e-7 * max(1.0, abs(r))
