"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the same seeded
inputs.  Solver parity is isolated from coefficient parity by handing the oracle's stencil to
the library (create_problem_ex override); the library's own stencil is compared with the
oracle's separately (tests/test_abi.py and test_library_stencil_used_by_problem below)."""
import functools

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import adjoint, matfree, system, workloads
from paper_2507_02809_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no ROCm device", allow_module_level=True)

from paper_2507_02809_amd import tsfde  # noqa: E402

DEV = "cuda"


def gpu_problem(inp, p):
    """Library problem with the oracle problem's data (mu) and stencil."""
    return tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a())


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


SMALL_DENSE = [
    ("1d_12x7", lambda: inputs.small(1, 12, 7)),
    ("1d_c1", lambda: inputs.c1()),
    ("2d_6x5_padded_tau", lambda: inputs.small(2, 6, 5, beta=0.6, omega=1.6)),
    ("2d_7x9", lambda: inputs.small(2, 7, 9, beta=0.3, omega=1.2)),
]


@pytest.fixture(scope="module", params=SMALL_DENSE, ids=[n for n, _ in SMALL_DENSE])
def dense_case(request):
    inp = request.param[1]()
    p = workloads.with_data(inp)
    return inp, p, system.dense_A(p), system.dense_P(p)


def test_apply_A_fp64_matches_dense(dense_case):
    inp, p, A, _ = dense_case
    rng = np.random.default_rng(11)
    y = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        z = g.apply_A(torch.tensor(y, device=DEV)).cpu().numpy()
    assert rel_err(z, A @ y) <= 1e-13


def test_apply_A_fp32_matches_dense(dense_case):
    inp, p, A, _ = dense_case
    rng = np.random.default_rng(12)
    y = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        z = g.apply_A(torch.tensor(y, device=DEV, dtype=torch.float32)).cpu().double().numpy()
    assert rel_err(z, A @ y.astype(np.float32).astype(np.float64)) <= 2e-5


def test_apply_P_inv_matches_dense(dense_case):
    inp, p, _, P = dense_case
    rng = np.random.default_rng(13)
    zz = rng.standard_normal(p.n_tot)
    ref = np.linalg.solve(P, zz)
    with gpu_problem(inp, p) as g:
        o = tsfde.default_opts(inner_tol=1e-14, inner_maxit=500)
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=o).cpu().numpy()
        y32 = g.apply_P_inv(torch.tensor(zz, device=DEV, dtype=torch.float32)).cpu().double().numpy()
    assert rel_err(y, ref) <= 1e-10
    assert rel_err(y32, ref) <= 5e-4


def test_gmres_fp64_and_mixed_match_dense_lu(dense_case):
    inp, p, A, _ = dense_case
    b = system.rhs_z(p)
    x_lu = np.linalg.solve(A, b)
    f_lu = x_lu[p.S * p.Nd:]
    with gpu_problem(inp, p) as g:
        # 3e-13: near the attainable FP64 residual of these systems
        f, st = g.recover_f(tsfde.default_opts(tol=3e-13, inner_tol=1e-14, inner_maxit=500), raise_noconv=True)
        assert st.converged == 1 and st.rel_res <= 3e-13
        assert rel_err(f.cpu().numpy(), f_lu) <= 1e-10
        fm, sm = g.recover_f(tsfde.default_opts(tol=1e-12, precision=tsfde.MIXED), raise_noconv=True)
        assert sm.converged == 1 and sm.refinements >= 1
        assert rel_err(fm.cpu().numpy(), f_lu) <= 1e-8
        # FP64 Krylov solve with the preconditioner applied in FP32: same FP64 residual target
        fp, sp = g.recover_f(tsfde.default_opts(tol=3e-13, precision=tsfde.PREC_F32), raise_noconv=True)
        assert sp.converged == 1 and sp.rel_res <= 3e-13
        assert rel_err(fp.cpu().numpy(), f_lu) <= 1e-10
        # explicit right-hand side and initial guess through gmres_solve
        x, st2 = g.gmres_solve(torch.tensor(b, device=DEV), opts=tsfde.default_opts(tol=3e-13, inner_tol=1e-14))
        assert np.linalg.norm(x.cpu().numpy() - x_lu) <= 1e-10 * np.linalg.norm(x_lu)


def test_mixed_refinement_checks_the_last_correction():
    """MIXED with a single refinement sweep: the residual of the corrected x is computed, so a sweep
    that reaches the tolerance reports convergence (and the statistics describe the returned x).  One
    FP32 sweep ends near 1e-4 here (8e-5 to 1.4e-4 depending on the FP32 rounding order), so the
    tolerance is 1e-3."""
    inp = inputs.small(1, 12, 7)
    p = workloads.with_data(inp)
    x_lu = np.linalg.solve(system.dense_A(p), system.rhs_z(p))
    with gpu_problem(inp, p) as g:
        f, st = g.recover_f(tsfde.default_opts(tol=1e-3, precision=tsfde.MIXED, max_refine=1, refine_tol=1e-5),
                            raise_noconv=True)
        assert st.converged == 1 and st.refinements == 1 and st.rel_res <= 1e-3
        assert rel_err(f.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-2
        # two refinement sweeps to a tight tolerance, repeated on the same problem (problem-owned buffers)
        for _ in range(2):
            f2, s2 = g.recover_f(tsfde.default_opts(tol=1e-12, precision=tsfde.MIXED), raise_noconv=True)
            assert s2.converged == 1 and s2.rel_res <= 1e-12
            assert rel_err(f2.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-8


def test_barrier_timeout_returns_edevice_and_recovers(monkeypatch):
    """A device-wide barrier wait of the persistent P^-1 that outlasts its bound ends the grid normally
    and the call reports EDEVICE; the bound is forced from the host (0 us, so the first workgroup to
    wait gives up at once).  With the default bound the next call on the same problem is exact."""
    inp = inputs.small(2, 15, 9, beta=0.5, omega=1.5)
    p = workloads.with_data(inp)
    P = system.dense_P(p)
    zz = np.random.default_rng(41).standard_normal(p.n_tot)
    ref = np.linalg.solve(P, zz)
    o = tsfde.default_opts(inner_tol=1e-14, inner_maxit=500)
    with gpu_problem(inp, p) as g:
        monkeypatch.setenv("TSFDE_PINV_BLOCKS", "4")
        monkeypatch.setenv("TSFDE_BARRIER_TIMEOUT_US", "0")
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(inner_tol=1e-14, inner_maxit=5))
        assert ei.value.status == tsfde.EDEVICE
        assert "timed out" in str(ei.value)
        monkeypatch.delenv("TSFDE_BARRIER_TIMEOUT_US")
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=o).cpu().numpy()
    assert rel_err(y, ref) <= 1e-10


@pytest.mark.parametrize("restart", [3, 70])
def test_gmres_unpreconditioned_restarts_match_dense_lu(restart):
    """Arnoldi without the preconditioner: restart 70 takes the Gram-Schmidt sweeps past 64 basis
    vectors (split into passes of at most 64), restart 3 restarts many times."""
    inp = inputs.small(1, 12, 7)
    p = workloads.with_data(inp)
    A = system.dense_A(p)
    b = system.rhs_z(p)
    x_lu = np.linalg.solve(A, b)
    with gpu_problem(inp, p) as g:
        o = tsfde.default_opts(tol=1e-11, use_precond=0, restart=restart, maxit=20000)
        x, st = g.gmres_solve(torch.tensor(b, device=DEV), opts=o, raise_noconv=True)
        assert st.converged == 1 and st.rel_res <= 1e-11
        if restart == 70:
            assert st.iters > 64
        else:
            assert st.restarts >= 2
        assert np.linalg.norm(A @ x.cpu().numpy() - b) <= 1e-10 * np.linalg.norm(b)
        assert rel_err(x.cpu().numpy(), x_lu) <= 1e-6


def test_forward_solve_matches_oracle():
    inp = inputs.c1()
    p = workloads.problem(inp)
    zh = system.rhs_zhat(p, inp.f_true)
    ref = matfree.forward_solve(p, zh)
    with tsfde.Problem.from_inputs(inp, stencil=p.a()) as g:
        v = g.forward_solve(torch.tensor(inp.f_true, device=DEV), opts=tsfde.default_opts(inner_tol=1e-14))
    assert rel_err(v.cpu().numpy(), ref) <= 1e-11


@pytest.mark.parametrize("d,N,M", [(1, 12, 7), (2, 6, 5), (2, 15, 9)])
def test_initial_state_rho_matches_dense(d, N, M):
    """A nonzero initial state rho = v^(0): the library builds z^(s) = b_{s-1} D_1^(s) rho (§5, eq.
    lin-syst) and z-hat of the direct problem (§6.1) itself; the whole solution y of recover_f and
    the direct solve are checked against the dense LU solutions with the oracle's z and z-hat."""
    import dataclasses
    inp = inputs.small(d, N, M, beta=0.4, omega=1.7, alpha=1e-3)
    rng = np.random.default_rng(31)
    inp = dataclasses.replace(inp, rho=1.0 + rng.standard_normal(inp.Nd))
    p = workloads.with_data(inp)
    assert np.abs(p.rho).max() > 0.5
    x_lu = np.linalg.solve(system.dense_A(p), system.rhs_z(p))
    v_lu = np.linalg.solve(system.dense_Ahat(p), system.rhs_zhat(p, inp.f_true))
    with gpu_problem(inp, p) as g:
        work = torch.zeros(p.n_tot, dtype=torch.float64, device=DEV)
        f, st = g.recover_f(tsfde.default_opts(tol=3e-13, inner_tol=1e-14, inner_maxit=500), work=work,
                            raise_noconv=True)
        v = g.forward_solve(torch.tensor(inp.f_true, device=DEV), opts=tsfde.default_opts(inner_tol=1e-14))
        y = work.cpu().numpy()
    assert st.converged == 1
    assert rel_err(y, x_lu) <= 1e-10
    assert rel_err(f.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-10
    assert rel_err(v.cpu().numpy(), v_lu) <= 1e-11


@pytest.mark.parametrize("shape", [(1, 100, 70), (1, 255, 130), (2, 13, 70), (2, 31, 20)])
def test_apply_A_ragged_tiles_match_oracle_matvec(shape):
    """Sizes that span several history tiles (64 points x 64 steps) with ragged tails and several
    FFT row pairs, against the oracle's FFT matvec."""
    d, N, M = shape
    inp = inputs.small(d, N, M, beta=0.7, omega=1.8)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    rng = np.random.default_rng(14)
    y = rng.standard_normal(p.n_tot)
    ref = matfree.matvec(p, y)
    with gpu_problem(inp, p) as g:
        z = g.apply_A(torch.tensor(y, device=DEV)).cpu().numpy()
    assert rel_err(z, ref) <= 1e-13


@pytest.mark.parametrize("which", ["c2a", "c3"])
def test_apply_A_full_size_sampled(which):
    """apply_A at the full workload sizes in the launch configuration the benchmark uses, checked
    on sampled entries that the oracle computes one by one from the scheme's definition."""
    inp = inputs.c2(0) if which == "c2a" else inputs.c3()
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    rng = np.random.default_rng(15)
    y = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        z = g.apply_A(torch.tensor(y, device=DEV)).cpu().numpy()
    samples = [(0, 0), (p.S - 1, p.Nd - 1), (p.S, 0), (p.S, p.Nd - 1), (p.S // 2, p.Nd // 2)]
    samples += [(int(rng.integers(0, p.S + 1)), int(rng.integers(0, p.Nd))) for _ in range(40)]
    scale = np.abs(z).max()
    for s, j in samples:
        ref = matfree.matvec_entry(p, y, s, j)
        assert abs(z[s * p.Nd + j] - ref) <= 1e-13 * scale, (s, j)


def test_library_stencil_used_by_problem():
    inp = inputs.small(2, 15, 4, beta=0.5, omega=1.5)
    p = workloads.problem(inp)
    with tsfde.Problem.from_inputs(inp) as g:
        a = g.stencil()
        sc = g.scalars()
    assert np.abs(a - p.a()).max() <= 5e-15 * p.a()[0, 0]
    assert sc["h"] == pytest.approx(p.h, rel=1e-15)
    assert sc["eta"] == pytest.approx(p.eta, rel=1e-14)
    assert sc["c_t"] == pytest.approx(p.c_t, rel=1e-14)
    assert sc["c_f"] == pytest.approx(p.c_f, rel=1e-14)


@pytest.fixture
def pinv_path(monkeypatch):
    def set_path(persistent: bool, extrap: int = 0):
        monkeypatch.setenv("TSFDE_PINV", "1" if persistent else "0")
        monkeypatch.setenv("TSFDE_EXTRAP", str(int(extrap)))
    return set_path


@pytest.mark.parametrize("persistent,extrap", [(True, 0), (True, 1), (True, 2), (True, 3), (False, 0)])
def test_apply_P_inv_paths_match_dense(dense_case, pinv_path, persistent, extrap):
    """Both implementations of the forward substitution (one persistent cooperative kernel, or one
    launch per CG phase), with each initial guess of the block CG (previous time level; linear,
    quadratic, half-linear extrapolation), against dense P^{-1}."""
    pinv_path(persistent, extrap)
    inp, p, _, P = dense_case
    rng = np.random.default_rng(16)
    zz = rng.standard_normal(p.n_tot)
    ref = np.linalg.solve(P, zz)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(inner_tol=1e-14, inner_maxit=500))
    assert rel_err(y.cpu().numpy(), ref) <= 1e-10


def test_apply_P_inv_zero_rhs_and_warm_start_exact(pinv_path):
    """z = 0 gives y = 0 exactly; a z whose blocks are already solved by the warm start still works."""
    pinv_path(True)
    inp = inputs.small(2, 15, 12, beta=0.5, omega=1.5)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.zeros(p.n_tot, dtype=torch.float64, device=DEV))
        assert float(y.abs().max()) == 0.0


@functools.lru_cache(maxsize=1)
def _n127_case():
    inp = inputs.small(2, 127, 6, beta=0.7, omega=1.3)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    zz = np.random.default_rng(19).standard_normal(p.n_tot)
    return inp, p, zz, matfree.P_solve(p, zz, inner="cg", inner_tol=1e-13)


@pytest.mark.parametrize("fixed", [True, False])
def test_apply_P_inv_fixed_length_kernel_matches_oracle(pinv_path, monkeypatch, fixed):
    """N = 127 (L = 256), where the 2D sine-transform path has a kernel compiled for that length;
    it and the run-time-length kernel (TSFDE_PINV_FIXED=0) against the oracle's forward
    substitution with CG inner solves, both to an inner tolerance far below the bound."""
    pinv_path(True)
    monkeypatch.setenv("TSFDE_PINV_FIXED", "1" if fixed else "0")
    inp, p, zz, ref = _n127_case()
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(inner_tol=1e-13, inner_maxit=500))
        y32 = g.apply_P_inv(torch.tensor(zz, device=DEV, dtype=torch.float32))
    assert rel_err(y.cpu().numpy(), ref) <= 1e-9
    assert rel_err(y32.cpu().double().numpy(), ref) <= 5e-4


def test_apply_P_inv_full_size_c3_residual():
    """P^{-1} at the full d=2, N=255^2, M=256 size (persistent kernel), checked through the oracle:
    (P y - z) on sampled entries, with (P y)_s = (A y)_s + eta q_s y_{M+1} for s <= M."""
    inp = inputs.c3()
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    rng = np.random.default_rng(17)
    zz = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV),
                          opts=tsfde.default_opts(inner_tol=1e-12)).cpu().numpy()
    samples = [(0, 0), (1, 5), (p.S - 1, p.Nd - 1), (p.S, 0), (p.S, p.Nd // 3)]
    samples += [(int(rng.integers(0, p.S + 1)), int(rng.integers(0, p.Nd))) for _ in range(30)]
    for s, j in samples:
        py = matfree.matvec_entry(p, y, s, j)
        if s < p.S:
            py += p.eta * p.q[s] * y[p.S * p.Nd + j]
        assert abs(py - zz[s * p.Nd + j]) <= 1e-8 * np.abs(zz).max(), (s, j)


@pytest.mark.parametrize("which", ["c3", "c2a"])
def test_gmres_full_size_true_residual(which):
    """Solves at full size (c3: the headline d=2, N=255^2, M=256; c2a: d=1, N=4095, M=1024) in the
    benchmark's configuration (FGMRES(50), tol 1e-7, block CG to 0.1 from the previous time
    level), checked through the oracle: its FFT matvec gives the true relative residual
    ||z - A x|| / ||z||, which must meet the tolerance and agree with the library's own FP64
    figure."""
    inp = inputs.c3() if which == "c3" else inputs.c2(0)
    p = workloads.problem(inp, mu=1e-3 * np.asarray(inp.f_true))
    opts = tsfde.default_opts(tol=1e-7, inner_tol=0.1, maxit=300, warm_start=tsfde.WARM_PREVIOUS)
    with gpu_problem(inp, p) as g:
        x, st = g.gmres_solve(opts=opts, raise_noconv=True)
        x = x.cpu().numpy()
    z = system.rhs_z(p)
    res = float(np.linalg.norm(z - matfree.matvec(p, x)) / np.linalg.norm(z))
    assert st.converged == 1
    assert res <= 1.05e-7
    assert abs(res - st.rel_res) <= 1e-3 * res


# ---------------------------------------------------------------------------
# T_{n,S}: the tau-block form of the preconditioner (opts.block_solver = BLOCK_TAU)
# ---------------------------------------------------------------------------
def test_apply_P_inv_tau_blocks_matches_dense_T(dense_case):
    """y = T^{-1} z (each block solved by sine transforms: FFT-based in the persistent kernels for d = 2
    with 2(N+1) a power of two, dense sine passes for d = 1 and other N) against LU of the assembled T."""
    inp, p, _, _ = dense_case
    rng = np.random.default_rng(21)
    zz = rng.standard_normal(p.n_tot)
    o = tsfde.default_opts(block_solver=tsfde.BLOCK_TAU)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=o).cpu().numpy()
        y32 = g.apply_P_inv(torch.tensor(zz, device=DEV, dtype=torch.float32), opts=o).cpu().double().numpy()
    ref = np.linalg.solve(system.dense_T(p), zz)
    assert rel_err(y, ref) <= 1e-12
    assert rel_err(y32, ref) <= 1e-5


def test_gmres_tau_blocks_reaches_dense_lu(dense_case):
    """FGMRES preconditioned by T reaches the same solution as dense LU of A."""
    inp, p, A, _ = dense_case
    x_lu = np.linalg.solve(A, system.rhs_z(p))
    with gpu_problem(inp, p) as g:
        f, st = g.recover_f(tsfde.default_opts(tol=3e-13, block_solver=tsfde.BLOCK_TAU), raise_noconv=True)
        assert st.converged == 1 and st.inner_iters == 0
        fp, sp = g.recover_f(tsfde.default_opts(tol=3e-13, block_solver=tsfde.BLOCK_TAU,
                                                precision=tsfde.PREC_F32), raise_noconv=True)
        assert sp.converged == 1
    assert rel_err(f.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-10
    assert rel_err(fp.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-10


@pytest.mark.parametrize("shape", [(1, 100, 20), (1, 255, 12), (2, 37, 6), (2, 63, 5)])
def test_tau_blocks_any_shape_match_oracle(shape, monkeypatch):
    """T^{-1} at shapes beyond the dense LU (1D, and 2D with 2(N+1) a power of two or not) against the
    oracle's matrix-free T^{-1} (orthonormal DST-I of size N); for N = 63 in 2D also the dense sine
    passes (persistent kernels switched off) against the FFT-based persistent path."""
    from oracle import matfree
    d, N, M = shape
    inp = inputs.small(d, N, M, beta=0.45, omega=1.35)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    zz = np.random.default_rng(24).standard_normal(p.n_tot)
    ref = matfree.T_solve(p, zz)
    o = tsfde.default_opts(block_solver=tsfde.BLOCK_TAU)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=o).cpu().numpy()
        assert rel_err(y, ref) <= 1e-12
        if d == 2 and N == 63:
            monkeypatch.setenv("TSFDE_PINV", "0")
            y2 = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=o).cpu().numpy()
            assert rel_err(y2, ref) <= 1e-12


@pytest.mark.parametrize("fixed", [True, False])
def test_apply_P_inv_tau_blocks_n127_matches_oracle(monkeypatch, fixed):
    """N = 127 (fixed-length and run-time-length kernels) against the oracle's matrix-free T^{-1}."""
    monkeypatch.setenv("TSFDE_PINV_FIXED", "1" if fixed else "0")
    inp, p, zz, _ = _n127_case()
    ref = matfree.T_solve(p, zz)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=tsfde.BLOCK_TAU))
    assert rel_err(y.cpu().numpy(), ref) <= 1e-12


# ---------------------------------------------------------------------------
# S_{n,S}: the Strang-block form of the preconditioner (opts.block_solver = BLOCK_STRANG)
# ---------------------------------------------------------------------------
def test_apply_P_inv_strang_blocks_matches_dense_S(dense_case):
    """y = S^{-1} z (each block solved by Hartley transforms) against LU of the assembled S, in
    FP64 and FP32; every shape (any N, d = 1, 2) is covered."""
    inp, p, _, _ = dense_case
    rng = np.random.default_rng(23)
    zz = rng.standard_normal(p.n_tot)
    o = tsfde.default_opts(block_solver=tsfde.BLOCK_STRANG)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=o).cpu().numpy()
        y32 = g.apply_P_inv(torch.tensor(zz, device=DEV, dtype=torch.float32), opts=o).cpu().double().numpy()
    ref = np.linalg.solve(system.dense_S(p), zz)
    assert rel_err(y, ref) <= 1e-12
    assert rel_err(y32, ref) <= 1e-5


def test_gmres_strang_blocks_reaches_dense_lu(dense_case):
    """FGMRES preconditioned by S reaches the same solution as dense LU of A, with no inner
    iterations; also with S^{-1} applied in FP32."""
    inp, p, A, _ = dense_case
    x_lu = np.linalg.solve(A, system.rhs_z(p))
    with gpu_problem(inp, p) as g:
        f, st = g.recover_f(tsfde.default_opts(tol=3e-13, block_solver=tsfde.BLOCK_STRANG), raise_noconv=True)
        assert st.converged == 1 and st.inner_iters == 0
        fp, sp = g.recover_f(tsfde.default_opts(tol=3e-13, block_solver=tsfde.BLOCK_STRANG,
                                                precision=tsfde.PREC_F32), raise_noconv=True)
        assert sp.converged == 1
    assert rel_err(f.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-10
    assert rel_err(fp.cpu().numpy(), x_lu[p.S * p.Nd:]) <= 1e-10


@pytest.mark.parametrize("d,N,M", [(1, 700, 5), (2, 100, 4), (2, 255, 3)])
def test_apply_P_inv_strang_blocks_matches_oracle(d, N, M):
    """Several transform tiles with ragged tails (64 outputs and 4 rows per workgroup, sums unrolled by 8), up to the
    255 x 255 slices of the headline workload, against the oracle's FFT forward substitution.

    Bound: the smallest eigenvalues of s(B) come from sums that cancel down to lambda_max / cond;
    the oracle's FFT gets them to about eps log2(N^d) lambda_max absolute, i.e. eps log2(N^d) cond
    relative, and the solve's dominant components inherit that (the library sums in extended
    precision).  8 eps log2(N^d) cond, at least 1e-12."""
    inp = inputs.small(d, N, M, beta=0.6, omega=1.7)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    zz = np.random.default_rng(29).standard_normal(p.n_tot)
    ref = matfree.S_solve(p, zz)
    lam = system.coeffs.strang_eigenvalues(p.a())
    tol = max(1e-12, 8 * np.finfo(float).eps * np.log2(p.Nd) * lam.max() / lam.min())
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=tsfde.BLOCK_STRANG))
    assert rel_err(y.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("kind", ["strang", "tau"])
@pytest.mark.parametrize("d,N,M", [(1, 300, 37), (2, 37, 37), (2, 66, 17)])
def test_dense_block_solvers_persistent_matches_pass_launches(monkeypatch, kind, d, N, M):
    """The persistent dense-transform block solver (one launch per segment of 16 steps, two device-wide
    barriers per step) against the one-launch-per-pass form, over several segments with a ragged last
    one, and against the oracle's S^{-1} / T^{-1}."""
    inp = inputs.small(d, N, M, beta=0.35, omega=1.45)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    zz = np.random.default_rng(33).standard_normal(p.n_tot)
    bs = tsfde.BLOCK_STRANG if kind == "strang" else tsfde.BLOCK_TAU
    ref = matfree.S_solve(p, zz) if kind == "strang" else matfree.T_solve(p, zz)
    if kind == "tau" and d == 2 and N == 63:
        monkeypatch.setenv("TSFDE_PINV", "0")
    with gpu_problem(inp, p) as g:
        monkeypatch.setenv("TSFDE_DENSE_PERSISTENT", "1")
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=bs)).cpu().numpy()
        monkeypatch.setenv("TSFDE_DENSE_PERSISTENT", "0")
        y0 = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=bs)).cpu().numpy()
    assert rel_err(y, y0) <= 1e-13
    assert rel_err(y, ref) <= 1e-11


@pytest.mark.parametrize("kind", ["strang", "tau"])
@pytest.mark.parametrize("N,M", [(1, 3), (17, 16), (37, 17), (100, 33), (255, 3)])
def test_dense_block_solvers_mfma_passes_match_lds_passes(monkeypatch, kind, N, M):
    """2D, FP64: the block solves as products on the matrix cores (16 x 16 tiles, the sum over j split
    over four waves, a ragged last tile) against the passes that read the table from LDS, and both
    against the oracle's S^{-1} / T^{-1}.  M = 16 puts the last row at the start of a block of steps
    (its right-hand side formed by the first pass), M = 17 and 33 inside one (formed by the previous
    step's last pass)."""
    inp = inputs.small(2, N, M, beta=0.35, omega=1.45)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    zz = np.random.default_rng(35).standard_normal(p.n_tot)
    bs = tsfde.BLOCK_STRANG if kind == "strang" else tsfde.BLOCK_TAU
    ref = matfree.S_solve(p, zz) if kind == "strang" else matfree.T_solve(p, zz)
    monkeypatch.setenv("TSFDE_DENSE_PERSISTENT", "0")
    monkeypatch.setenv("TSFDE_PINV", "0")  # tau: the dense sine passes, also where 2(N+1) is a power of two
    with gpu_problem(inp, p) as g:
        monkeypatch.setenv("TSFDE_DENSE_MFMA", "1")
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=bs)).cpu().numpy()
        monkeypatch.setenv("TSFDE_DENSE_MFMA", "0")
        y0 = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=bs)).cpu().numpy()
    assert rel_err(y, y0) <= 1e-13
    assert rel_err(y, ref) <= 1e-11


@pytest.mark.parametrize("d,N,M", [(1, 1, 3), (2, 1, 2), (1, 2, 4), (2, 2, 3), (2, 9, 1)])
def test_apply_P_inv_strang_blocks_degenerate_shapes(d, N, M):
    """One or two points per direction (a single-entry circulant, a 2 x 2 one) and a single time
    level, against LU of the assembled S."""
    inp = inputs.small(d, N, M)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    zz = np.random.default_rng(31).standard_normal(p.n_tot)
    ref = np.linalg.solve(system.dense_S(p), zz)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=tsfde.BLOCK_STRANG))
    assert rel_err(y.cpu().numpy(), ref) <= 1e-12


def test_strang_blocks_reject_an_indefinite_circulant():
    """A stencil whose Strang circulant is not positive definite is refused with ENOTIMPL before
    anything is launched (its block solves would divide by a zero or negative eigenvalue)."""
    inp = inputs.small(1, 9, 3)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    bad = p.a().copy()
    bad[1:] = -bad[0]  # row sums far below zero
    zz = np.ones(p.n_tot)
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=bad) as g:
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(block_solver=tsfde.BLOCK_STRANG))
        assert ei.value.status == tsfde.ENOTIMPL


BATCH_CASES = [
    lambda: inputs.small(1, 12, 7),
    lambda: inputs.small(2, 7, 9, beta=0.3, omega=1.2),
    lambda: inputs.c1(),
    lambda: inputs.small(2, 15, 6, beta=0.6, omega=1.6),
    lambda: inputs.small(2, 31, 5, beta=0.4, omega=1.3),
]


@pytest.mark.parametrize("inflight", [2, 4])
def test_recover_f_batch_matches_single_solves_and_dense_lu(inflight):
    """The batch solves each problem exactly as a single call does (same kernels, same reduction
    order), several at a time on worker streams; each f~ also matches the oracle's dense LU."""
    cases = [mk() for mk in BATCH_CASES]
    opts = tsfde.default_opts(tol=1e-11, inner_tol=1e-12, inner_maxit=500)
    probs, refs = [], []
    try:
        for inp in cases:
            p = workloads.with_data(inp)
            probs.append(gpu_problem(inp, p))
            b = system.rhs_z(p)
            refs.append(np.linalg.solve(system.dense_A(p), b)[p.S * p.Nd:])
        single = [g.recover_f(opts, raise_noconv=True) for g in probs]
        out = tsfde.recover_f_batch(probs, opts, max_inflight=inflight, raise_noconv=True)
        for (f1, s1), (fb, sb), f_lu in zip(single, out, refs):
            assert sb.converged == 1 and sb.iters == s1.iters
            assert np.array_equal(fb.cpu().numpy(), f1.cpu().numpy())
            assert rel_err(fb.cpu().numpy(), f_lu) <= 1e-8
    finally:
        for g in probs:
            g.close()


def test_recover_f_batch_strang_blocks_matches_single_solves():
    """S_{n,S}-preconditioned solves in a batch (worker streams, 3 in flight) give bit for bit the
    single-call results, and each f~ matches the oracle's dense LU."""
    cases = [mk() for mk in BATCH_CASES]
    opts = tsfde.default_opts(tol=1e-11, maxit=400, block_solver=tsfde.BLOCK_STRANG)
    probs, refs = [], []
    try:
        for inp in cases:
            p = workloads.with_data(inp)
            probs.append(gpu_problem(inp, p))
            refs.append(np.linalg.solve(system.dense_A(p), system.rhs_z(p))[p.S * p.Nd:])
        single = [g.recover_f(opts, raise_noconv=True) for g in probs]
        out = tsfde.recover_f_batch(probs, opts, max_inflight=3, raise_noconv=True)
        for (f1, s1), (fb, sb), f_lu in zip(single, out, refs):
            assert sb.converged == 1 and sb.iters == s1.iters and sb.inner_iters == 0
            assert np.array_equal(fb.cpu().numpy(), f1.cpu().numpy())
            assert rel_err(fb.cpu().numpy(), f_lu) <= 1e-8
    finally:
        for g in probs:
            g.close()


def test_recover_f_batch_rejects_bad_batches():
    inp = inputs.small(1, 12, 7)
    p = workloads.with_data(inp)
    with gpu_problem(inp, p) as g:
        with pytest.raises(tsfde.TsfdeError) as e:
            tsfde.recover_f_batch([g, g])
        assert e.value.status == tsfde.EINVAL and "twice" in str(e.value)
        with pytest.raises(tsfde.TsfdeError) as e:
            tsfde.recover_f_batch([g], max_inflight=9)
        assert e.value.status == tsfde.EINVAL
        assert tsfde.recover_f_batch([]) == []


@pytest.mark.parametrize("N", [12, 64, 100, 300])
def test_apply_P_inv_1d_padded_tau_matches_dense(N, pinv_path):
    """d = 1 with 2(N+1) not a power of two: the persistent kernel preconditions its block CG with
    the tau matrix of the next size 2^k - 1 on the zero-padded residual (N = 64 also doubles the
    circulant embedding to that transform length).  P^{-1} still matches dense P, and the block
    CG needs far fewer iterations than the diagonal preconditioner of the multi-launch path."""
    pinv_path(True)
    inp = inputs.small(1, N, 6, beta=0.7, omega=1.8)
    p = workloads.with_data(inp)
    P = system.dense_P(p)
    A = system.dense_A(p)
    rng = np.random.default_rng(N)
    zz = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(inner_tol=1e-13, inner_maxit=500))
        assert rel_err(y.cpu().numpy(), np.linalg.solve(P, zz)) <= 1e-9
        o = tsfde.default_opts(tol=1e-11, inner_tol=1e-8, inner_maxit=500)
        b = system.rhs_z(p)
        x, st = g.gmres_solve(torch.tensor(b, device=DEV), opts=o, raise_noconv=True)
        assert np.linalg.norm(A @ x.cpu().numpy() - b) <= 1e-10 * np.linalg.norm(b)
        pinv_path(False)
        _, st_diag = g.gmres_solve(torch.tensor(b, device=DEV), opts=o, raise_noconv=True)
    if N >= 64:
        assert 3 * st.inner_iters < st_diag.inner_iters, (st.inner_iters, st_diag.inner_iters)


@pytest.mark.parametrize("N", [6, 12, 16, 20])
def test_apply_P_inv_2d_padded_tau_matches_dense(N, pinv_path):
    """d = 2 with 2(N+1) not a power of two: the fused tau-preconditioned CG of the persistent kernel
    runs with sine transforms of the next size 2^k - 1 per direction on zero-padded rows and columns
    (N = 16 also doubles the circulant embedding).  P^{-1} matches dense P, and FGMRES through it
    needs far fewer block-CG iterations than with the diagonal preconditioner."""
    pinv_path(True)
    inp = inputs.small(2, N, 4, beta=0.6, omega=1.8)
    p = workloads.with_data(inp)
    P = system.dense_P(p)
    A = system.dense_A(p)
    rng = np.random.default_rng(100 + N)
    zz = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        y = g.apply_P_inv(torch.tensor(zz, device=DEV), opts=tsfde.default_opts(inner_tol=1e-13, inner_maxit=500))
        assert rel_err(y.cpu().numpy(), np.linalg.solve(P, zz)) <= 1e-9
        o = tsfde.default_opts(tol=1e-11, inner_tol=1e-8, inner_maxit=500)
        b = system.rhs_z(p)
        x, st = g.gmres_solve(torch.tensor(b, device=DEV), opts=o, raise_noconv=True)
        assert np.linalg.norm(A @ x.cpu().numpy() - b) <= 1e-10 * np.linalg.norm(b)
        pinv_path(False)
        _, st_diag = g.gmres_solve(torch.tensor(b, device=DEV), opts=o, raise_noconv=True)
    if N >= 12:
        assert 2 * st.inner_iters < st_diag.inner_iters, (st.inner_iters, st_diag.inner_iters)


@pytest.mark.parametrize("d,N,M", [(1, 1, 1), (1, 2, 1), (1, 3, 2), (1, 5, 1), (2, 1, 1), (2, 2, 3), (2, 3, 1),
                                   (2, 4, 2)])
def test_degenerate_shapes_match_dense(d, N, M):
    """One time step, one or a few grid points (transforms of length 8, single-thread transform
    groups): A y, P^{-1} z and the recovered f~ against the oracle's dense matrices."""
    inp = inputs.small(d, N, M, beta=0.55, omega=1.45)
    p = workloads.with_data(inp)
    A, P = system.dense_A(p), system.dense_P(p)
    rng = np.random.default_rng(1000 + 100 * d + 10 * N + M)
    y = rng.standard_normal(p.n_tot)
    b = system.rhs_z(p)
    with gpu_problem(inp, p) as g:
        z = g.apply_A(torch.tensor(y, device=DEV)).cpu().numpy()
        assert rel_err(z, A @ y) <= 1e-13
        w = g.apply_P_inv(torch.tensor(y, device=DEV), opts=tsfde.default_opts(inner_tol=1e-14, inner_maxit=500))
        assert rel_err(w.cpu().numpy(), np.linalg.solve(P, y)) <= 1e-10
        f, st = g.recover_f(tsfde.default_opts(tol=1e-12, inner_tol=1e-14, inner_maxit=500), raise_noconv=True)
        assert rel_err(f.cpu().numpy(), np.linalg.solve(A, b)[p.S * p.Nd:]) <= 1e-9


# ---------------------------------------------------------------------------
# transposed problem (gradients)
# ---------------------------------------------------------------------------
def test_apply_AT_and_PT_inv_match_dense(dense_case):
    inp, p, A, P = dense_case
    rng = np.random.default_rng(31)
    lam = rng.standard_normal(p.n_tot)
    with gpu_problem(inp, p) as g:
        z = g.apply_AT(torch.tensor(lam, device=DEV)).cpu().numpy()
        assert rel_err(z, A.T @ lam) <= 1e-13
        w = g.apply_PT_inv(torch.tensor(lam, device=DEV), opts=tsfde.default_opts(inner_tol=1e-14, inner_maxit=500))
        assert rel_err(w.cpu().numpy(), np.linalg.solve(P.T, lam)) <= 1e-10


@pytest.mark.parametrize("shape", [(1, 60, 37), (2, 15, 40), (2, 12, 20), (2, 7, 17), (1, 5, 1), (2, 9, 16)])
def test_apply_PT_inv_persistent_sweep_matches_host_loop_and_oracle(monkeypatch, shape):
    """P^{-T} g on the persistent kernels (the backward substitution as a forward sweep in reversed
    step order, history weights per earlier step) against the one-launch-per-CG-phase loop, over
    several blocks of 16 steps with ragged ends (M = 1, 16, 17, 20, 37, 40; 1D, 2D with the sine
    preconditioner and with its padded form), and against the oracle's dense P^T solve where that
    fits."""
    d, N, M = shape
    inp = inputs.small(d, N, M, beta=0.55, omega=1.45)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    g_np = np.random.default_rng(37).standard_normal(p.n_tot)
    o = tsfde.default_opts(inner_tol=1e-14, inner_maxit=500)
    with gpu_problem(inp, p) as g:
        gt = torch.tensor(g_np, device=DEV)
        w = g.apply_PT_inv(gt, opts=o).cpu().numpy()
        monkeypatch.setenv("TSFDE_PTINV", "0")
        w0 = g.apply_PT_inv(gt, opts=o).cpu().numpy()
    assert rel_err(w, w0) <= 1e-10
    if p.n_tot <= 3000:
        assert rel_err(w, np.linalg.solve(system.dense_P(p).T, g_np)) <= 1e-10


@pytest.mark.parametrize("shape", [(1, 100, 70), (2, 13, 70), (2, 31, 20), (2, 64, 9)])
def test_apply_AT_adjoint_identity_ragged(shape):
    """<A x, w> (oracle, FFT matvec) = <x, A^T w> (library) at sizes past the dense oracle: several
    history tiles with ragged tails, and the doubled embedding of N = 64."""
    d, N, M = shape
    inp = inputs.small(d, N, M, beta=0.7, omega=1.8)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    rng = np.random.default_rng(32)
    with gpu_problem(inp, p) as g:
        for _ in range(2):
            x = rng.standard_normal(p.n_tot)
            w = rng.standard_normal(p.n_tot)
            lhs = float(matfree.matvec(p, x) @ w)
            rhs = float(x @ g.apply_AT(torch.tensor(w, device=DEV)).cpu().numpy())
            assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(matfree.matvec(p, x)) * np.linalg.norm(w)


def test_apply_AT_full_size_c3_adjoint_identity():
    """c3 (d = 2, N = 255, M = 256): <A x, w> = <x, A^T w> with both products on the GPU."""
    inp = inputs.c3()
    with tsfde.Problem.from_inputs(inp) as g:
        gen = torch.Generator(device=DEV).manual_seed(33)
        x = torch.randn(g.n_tot, dtype=torch.float64, device=DEV, generator=gen)
        w = torch.randn(g.n_tot, dtype=torch.float64, device=DEV, generator=gen)
        ax = g.apply_A(x)
        lhs = float(torch.dot(ax, w))
        rhs = float(torch.dot(x, g.apply_AT(w)))
        assert abs(lhs - rhs) <= 1e-12 * float(ax.norm() * w.norm())


def test_vjp_full_size_c5_through_the_oracle():
    """The gradient workload at full size (d = 2, N = 127, M = 128), checked with the oracle's FFT
    matvec.  With r_lam = A^T lam - g and r_x = A x - z the two solves' residuals (g = R^T gf,
    z = R^T mu since rho = 0):
      <lam, A y> - <g, y> = <r_lam, y>                                   (random y)
      <g, x> - <lam, z>   = <lam, r_x> - <r_lam, x>,  <g, x> = gf . f~,  <lam, z> = grad_mu . mu
    so both gaps are bounded by the solve tolerance times the norms involved (plus rounding of the
    inner products, 64 eps times the same norms)."""
    inp = inputs.c5()
    mu = 1e-3 * np.asarray(inp.f_true)
    p = workloads.problem(inp, mu=mu)
    assert not np.any(p.rho)
    rng = np.random.default_rng(35)
    gf = rng.standard_normal(p.Nd)
    gvec = np.zeros(p.n_tot)
    gvec[p.S * p.Nd:] = gf
    tol = 1e-11
    eps = np.finfo(float).eps
    o = tsfde.default_opts(tol=tol, maxit=400)
    with gpu_problem(inp, p) as g:
        lam, st = g.adjoint_solve(torch.tensor(gvec, device=DEV), opts=o, raise_noconv=True)
        x, sx = g.gmres_solve(opts=o, raise_noconv=True)
        gmu, _, sv = g.recover_f_vjp(x, torch.tensor(gf, device=DEV), opts=o, raise_noconv=True)
        lam, x, gmu = lam.cpu().numpy(), x.cpu().numpy(), gmu.cpu().numpy()
    assert rel_err(gmu, lam[p.S * p.Nd:]) <= 1e-8  # the VJP's adjoint is this adjoint solve
    ng, nl, nx, nz = (np.linalg.norm(v) for v in (gvec, lam, x, mu))
    for _ in range(2):
        y = rng.standard_normal(p.n_tot)
        ay = matfree.matvec(p, y)
        gap = float(lam @ ay - gvec @ y)
        assert abs(gap) <= 2 * tol * ng * np.linalg.norm(y) + 64 * eps * (nl * np.linalg.norm(ay) + ng * np.linalg.norm(y))
    lhs, rhs = float(gf @ x[p.S * p.Nd:]), float(gmu @ mu)
    assert abs(lhs - rhs) <= 2 * tol * (ng * nx + nl * nz) + 64 * eps * (ng * nx + nl * nz)


def test_adjoint_solve_and_vjp_match_oracle(dense_case):
    inp, p, A, _ = dense_case
    rng = np.random.default_rng(34)
    gf = rng.standard_normal(p.Nd)
    gmu_ref, ga_ref, y_ref = adjoint.vjp(p, gf)
    gvec = np.zeros(p.n_tot)
    gvec[p.S * p.Nd:] = gf
    # 3e-13: near the attainable FP64 residual of these systems
    o = tsfde.default_opts(tol=3e-13, inner_tol=1e-12, inner_maxit=500)
    with gpu_problem(inp, p) as g:
        lam, st = g.adjoint_solve(torch.tensor(gvec, device=DEV), opts=o, raise_noconv=True)
        assert st.converged == 1
        assert rel_err(lam.cpu().numpy(), np.linalg.solve(A.T, gvec)) <= 1e-9
        y = torch.empty(p.n_tot, dtype=torch.float64, device=DEV)
        g.recover_f(o, work=y, raise_noconv=True)
        assert rel_err(y.cpu().numpy(), y_ref) <= 1e-9
        gmu, ga, _ = g.recover_f_vjp(y, torch.tensor(gf, device=DEV), opts=o, raise_noconv=True)
        gmu2, ga2, gg2, _ = g.recover_f_vjp(y, torch.tensor(gf, device=DEV), opts=o, raise_noconv=True, gamma2=True)
    assert rel_err(gmu.cpu().numpy(), gmu_ref) <= 1e-9
    assert ga == pytest.approx(ga_ref, rel=1e-8)
    assert rel_err(gmu2.cpu().numpy(), gmu_ref) <= 1e-9 and ga2 == pytest.approx(ga_ref, rel=1e-8)
    assert rel_err(gg2.cpu().numpy(), adjoint.grad_gamma2(p, gf)) <= 1e-8


def test_recover_f_autograd_gradient_in_mu():
    """torch.autograd through recover_f: the gradient of ||f~ - f_true||^2 in mu against the oracle."""
    inp = inputs.small(2, 7, 9, beta=0.3, omega=1.2)
    p = workloads.with_data(inp)
    f_ref = np.linalg.solve(system.dense_A(p), system.rhs_z(p))[p.S * p.Nd:]
    gmu_ref, ga_ref, _ = adjoint.vjp(p, 2.0 * (f_ref - inp.f_true))
    o = tsfde.default_opts(tol=3e-13, inner_tol=1e-12, inner_maxit=500)
    with gpu_problem(inp, p) as g:
        mu = torch.tensor(p.mu, device=DEV, requires_grad=True)
        f = tsfde.recover_f_autograd(g, mu, opts=o, adjoint_opts=o)
        loss = ((f - torch.tensor(inp.f_true, device=DEV)) ** 2).sum()
        (gmu,) = torch.autograd.grad(loss, mu)
        assert rel_err(gmu.cpu().numpy(), gmu_ref) <= 1e-8
        assert g.last_grad_alpha == pytest.approx(ga_ref, rel=1e-7)


def test_discrepancy_sweep_matches_oracle():
    """set_alpha + recover_f + forward_solve over an alpha grid: the discrepancies against the
    oracle's dense solves, and the same alpha chosen by the discrepancy principle."""
    from oracle import discrepancy
    inp = inputs.small(2, 7, 9, beta=0.3, omega=1.2)
    p = workloads.with_data(inp)
    alphas = list(np.logspace(-7, -2, 6))
    ref = discrepancy.residuals(p, alphas)
    mu0 = discrepancy.forward_data(p, inp.f_true)
    delta = float(np.linalg.norm(p.mu - mu0))
    o = tsfde.default_opts(tol=3e-13, inner_tol=1e-13, inner_maxit=500)
    fo = tsfde.default_opts(inner_tol=1e-13, inner_maxit=500)
    with gpu_problem(inp, p) as g:
        res, _ = tsfde.discrepancy_curve(g, alphas, opts=o, fwd_opts=fo)
    for r, rr in zip(res, ref):
        assert r == pytest.approx(rr, rel=1e-7)
    assert tsfde.select_alpha(alphas, res, delta) == discrepancy.select(alphas, ref, delta)


def test_arnoldi_hessenberg_matches_oracle(dense_case):
    """tsfde_arnoldi on A P^{-1} from z against the oracle's Arnoldi (classical Gram-Schmidt twice)
    on the dense operator."""
    from oracle import krylov
    inp, p, A, P = dense_case
    k = min(10, p.n_tot - 1)
    H_ref, _ = krylov.arnoldi_cgs2(lambda v: A @ np.linalg.solve(P, v), system.rhs_z(p), k)
    with gpu_problem(inp, p) as g:
        H, m = g.arnoldi(k, opts=tsfde.default_opts(inner_tol=1e-14, inner_maxit=500))
    assert m == H_ref.shape[1]
    assert np.abs(H - H_ref).max() <= 1e-9 * np.abs(H_ref).max()


def test_arnoldi_ritz_values_are_eigenvalues_of_preconditioned_matrix():
    """A P^{-1} = I + rank N^d: N^d + 1 Arnoldi steps give eigenvalues of P^{-1} A."""
    inp = inputs.small(1, 6, 5)
    p = workloads.with_data(inp)
    A, P = system.dense_A(p), system.dense_P(p)
    ev = np.linalg.eigvals(np.linalg.solve(P, A))
    with gpu_problem(inp, p) as g:
        H, m = g.arnoldi(p.Nd + 1, opts=tsfde.default_opts(inner_tol=1e-14, inner_maxit=500))
    for r in tsfde.ritz_values(H):
        assert np.min(np.abs(ev - r)) <= 1e-6 * max(1.0, abs(r))


@pytest.mark.parametrize("d,N,M", [(1, 40, 70), (2, 15, 33)])
def test_apply_A_time_operator_exact_on_linear_in_t(d, N, M):
    """The L1 time operator is exact on functions linear in t (closed form, not the oracle): with
    y_s = psi (a + b t_s) and f~ = 0, (A y)_s minus its spatial part, divided by gamma1_s, equals
    psi (b_{s-1} a + b dt s^{1-beta}).  The spatial part c_t gamma2_s .* B psi (a + b t_s) uses
    B psi from the last block row of A [0; psi], which is c_f gamma2_M .* B psi."""
    inp = inputs.small(d, N, M, beta=0.45, omega=1.5)
    Nd, dt, beta = inp.Nd, inp.T / M, inp.beta
    rng = np.random.default_rng(41)
    psi = rng.standard_normal(Nd)
    a, b = 0.7, -1.3
    t = dt * np.arange(1, M + 1)
    y = np.zeros((M + 1) * Nd)
    for s in range(M):
        y[s * Nd:(s + 1) * Nd] = psi * (a + b * t[s])
    e_last = np.zeros((M + 1) * Nd)
    e_last[M * Nd:] = psi
    with tsfde.Problem.from_inputs(inp) as g:
        sc = g.scalars()
        z = g.apply_A(torch.tensor(y, device=DEV)).cpu().numpy().reshape(M + 1, Nd)
        zl = g.apply_A(torch.tensor(e_last, device=DEV)).cpu().numpy().reshape(M + 1, Nd)
    Bpsi = zl[M] / (sc["c_f"] * inp.gamma2[M - 1])
    s1 = np.arange(1, M + 1)
    bw = s1 ** (1 - beta) - (s1 - 1) ** (1 - beta)  # b_{s-1}
    for s in range(M):
        hist = (z[s] - sc["c_t"] * inp.gamma2[s] * (a + b * t[s]) * Bpsi) / inp.gamma1[s]
        ref = psi * (bw[s] * a + b * dt * (s + 1) ** (1 - beta))
        assert np.abs(hist - ref).max() <= 1e-10 * np.abs(psi).max() * (1 + sc["c_t"]), s


def test_recover_f_vjp_batch_matches_single_calls():
    """Forward batch, then the gradient batch on the problems' own solutions: the same numbers as one
    problem at a time (same kernels and reduction order), and the oracle's gradients."""
    cases = [inputs.small(1, 12, 7), inputs.small(2, 7, 9, beta=0.3, omega=1.2), inputs.small(2, 15, 6)]
    o = tsfde.default_opts(tol=3e-13, inner_tol=1e-12, inner_maxit=500)
    rng = np.random.default_rng(51)
    probs, gfs, refs = [], [], []
    try:
        for inp in cases:
            p = workloads.with_data(inp)
            probs.append(gpu_problem(inp, p))
            gf = rng.standard_normal(p.Nd)
            gfs.append(torch.tensor(gf, device=DEV))
            refs.append(adjoint.vjp(p, gf))
        tsfde.recover_f_batch(probs, o, max_inflight=3, raise_noconv=True)
        out = tsfde.recover_f_vjp_batch(probs, gfs, opts=o, max_inflight=3, gamma2=True, raise_noconv=True)
        for g, gf, (gm_b, ga_b, gg_b, _), (gm_ref, ga_ref, _) in zip(probs, gfs, out, refs):
            y = torch.empty(g.n_tot, dtype=torch.float64, device=DEV)
            g.recover_f(o, work=y, raise_noconv=True)
            gm, ga, gg, _ = g.recover_f_vjp(y, gf, opts=o, raise_noconv=True, gamma2=True)
            assert torch.equal(gm, gm_b) and ga == ga_b and torch.equal(gg, gg_b)
            assert rel_err(gm_b.cpu().numpy(), gm_ref) <= 1e-9
            assert ga_b == pytest.approx(ga_ref, rel=1e-8)
    finally:
        for g in probs:
            g.close()


def test_nonconvergence_reports_enoconv_and_the_last_iterate():
    """maxit reached: TSFDE_ENOCONV, converged = 0, the iterate's true residual is the reported one
    and below the starting residual (GMRES minimises it over the Krylov space)."""
    inp = inputs.small(1, 12, 7)
    p = workloads.with_data(inp)
    A = system.dense_A(p)
    b = system.rhs_z(p)
    with gpu_problem(inp, p) as g:
        o = tsfde.default_opts(tol=1e-12, use_precond=0, maxit=3)
        with pytest.raises(tsfde.TsfdeError) as e:
            g.gmres_solve(torch.tensor(b, device=DEV), opts=o, raise_noconv=True)
        assert e.value.status == tsfde.ENOCONV
        x, st = g.gmres_solve(torch.tensor(b, device=DEV), opts=o)
        assert st.converged == 0 and st.iters == 3
        rel = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
        assert rel == pytest.approx(st.rel_res, rel=1e-6) and rel < 1.0
