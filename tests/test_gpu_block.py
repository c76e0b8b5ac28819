"""GPU: block FGMRES on several right-hand sides of one problem (tsfde_gmres_solve_block,
tsfde_recover_f_block) against the plain definition X = A^{-1} B (LU of the oracle's assembled A),
and against single-right-hand-side solves.  The block Gram-Schmidt products run on the matrix cores;
the shapes below give vector lengths that leave a ragged last chunk of 256 values, and block sizes
and restarts whose basis spans one, two, four and eight 16-vector tiles per Gram workgroup."""
import numpy as np
import pytest

from oracle import system, workloads
from paper_2507_02809_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no ROCm device", allow_module_level=True)

from paper_2507_02809_amd import tsfde  # noqa: E402

DEV = "cuda"


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _case(d, N, M, **kw):
    inp = inputs.small(d, N, M, **kw)
    p = workloads.with_data(inp)
    return inp, p


@pytest.mark.parametrize("d,N,M,nrhs,restart", [
    (1, 12, 7, 1, 10),      # n = 96: a single partial chunk
    (1, 100, 20, 3, 30),    # basis up to 90 vectors: Gram tiles 1, 2, 4, 8 per workgroup
    (2, 7, 9, 16, 5),       # 16 columns: full MFMA column width, basis up to 80 vectors
    (2, 15, 6, 5, 4),       # restarts (4 block steps per cycle)
])
def test_block_gmres_matches_dense_lu(d, N, M, nrhs, restart):
    inp, p = _case(d, N, M, beta=0.45, omega=1.35)
    A = system.dense_A(p)
    rng = np.random.default_rng(41)
    B = rng.standard_normal((nrhs, p.n_tot))
    ref = np.linalg.solve(A, B.T).T
    opts = tsfde.default_opts(tol=1e-12, restart=restart, inner_tol=1e-13, inner_maxit=500)
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a()) as g:
        X, st, rel = g.gmres_solve_block(torch.tensor(B, device=DEV), opts=opts, raise_noconv=True)
        X = X.cpu().numpy()
    assert st.converged == 1 and np.all(rel <= 1e-12)
    for c in range(nrhs):
        assert rel_err(X[c], ref[c]) <= 1e-9, c
        # the reported residual is the true one
        r = np.linalg.norm(B[c] - A @ X[c]) / np.linalg.norm(B[c])
        assert r <= 2e-12


def test_block_gmres_initial_guess_and_zero_column():
    """X's initial guesses are used (an exact guess converges with no step), and a zero right-hand
    side yields a zero column next to nonzero ones."""
    inp, p = _case(1, 40, 10)
    A = system.dense_A(p)
    rng = np.random.default_rng(43)
    B = rng.standard_normal((3, p.n_tot))
    B[1] = 0.0
    ref = np.linalg.solve(A, B.T).T
    opts = tsfde.default_opts(tol=1e-12, restart=20, inner_tol=1e-13, inner_maxit=500)
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a()) as g:
        X, st, rel = g.gmres_solve_block(torch.tensor(B, device=DEV), opts=opts, raise_noconv=True)
        Xn = X.cpu().numpy()
        assert np.abs(Xn[1]).max() <= 1e-12 * np.abs(Xn).max()
        assert rel_err(Xn[0], ref[0]) <= 1e-9 and rel_err(Xn[2], ref[2]) <= 1e-9
        X0 = torch.tensor(np.ascontiguousarray(ref), device=DEV)
        X2, st2, _ = g.gmres_solve_block(torch.tensor(B, device=DEV), X=X0, opts=opts, raise_noconv=True)
        assert st2.iters == 0 and st2.converged == 1


def test_recover_f_block_matches_single_solves():
    """f~ for several data sets mu_c in one block solve against single recover_f calls with set_mu
    and the dense LU of each system; the block needs fewer P^{-1} applications per data set."""
    inp, p = _case(2, 15, 8, beta=0.6, omega=1.6)
    rng = np.random.default_rng(47)
    k = 4
    mus = np.stack([inp.noisy(p.mu) if c == 0 else p.mu * (1 + 0.1 * c) + 1e-3 * rng.standard_normal(inp.Nd)
                    for c in range(k)])
    opts = tsfde.default_opts(tol=1e-11, restart=30, inner_tol=1e-12, inner_maxit=500)
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a()) as g:
        F, st, rel = g.recover_f_block(torch.tensor(mus, device=DEV), opts=opts, raise_noconv=True)
        F = F.cpu().numpy()
        single_iters = 0
        for c in range(k):
            g.set_mu(mus[c])
            f1, s1 = g.recover_f(opts, raise_noconv=True)
            single_iters += s1.iters
            pc = workloads.problem(inp, mu=mus[c])
            f_lu = np.linalg.solve(system.dense_A(pc), system.rhs_z(pc))[pc.S * pc.Nd:]
            assert rel_err(F[c], f_lu) <= 1e-8, c
            assert rel_err(F[c], f1.cpu().numpy()) <= 1e-8, c
    assert st.converged == 1 and np.all(rel <= 1e-11)
    assert st.iters * k <= single_iters


def test_block_gmres_fp32_preconditioner():
    inp, p = _case(2, 31, 5, beta=0.4, omega=1.3)
    A = system.dense_A(p)
    B = np.random.default_rng(53).standard_normal((2, p.n_tot))
    ref = np.linalg.solve(A, B.T).T
    opts = tsfde.default_opts(tol=1e-11, restart=40, precision=tsfde.PREC_F32)
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a()) as g:
        X, st, rel = g.gmres_solve_block(torch.tensor(B, device=DEV), opts=opts, raise_noconv=True)
    assert st.converged == 1
    for c in range(2):
        assert rel_err(X[c].cpu().numpy(), ref[c]) <= 1e-8


def test_block_gmres_argument_errors():
    inp, p = _case(1, 12, 7)
    B = torch.zeros(17, p.n_tot, dtype=torch.float64, device=DEV)
    with tsfde.Problem.from_inputs(inp, mu=p.mu) as g:
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.gmres_solve_block(B)  # 17 columns
        assert ei.value.status == tsfde.ENOTIMPL
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.gmres_solve_block(B[:2], opts=tsfde.default_opts(precision=tsfde.MIXED))
        assert ei.value.status == tsfde.ENOTIMPL
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.gmres_solve_block(B[:8], opts=tsfde.default_opts(restart=200))  # 1600 basis vectors
        assert ei.value.status == tsfde.ENOTIMPL
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.gmres_solve_block(B[:2], X=B[1:3])  # overlapping
        assert ei.value.status == tsfde.EINVAL
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.gmres_solve_block(B[:4] + 1.0, opts=tsfde.default_opts(max_device_bytes=g.device_bytes() + 1000))
        assert ei.value.status == tsfde.ENOMEM
