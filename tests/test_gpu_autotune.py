"""GPU: the autotuner (tsfde_autotune) and the alternatives it chooses between.  Every 2D matvec FFT
tiling is checked against the oracle's matrix-free matvec at several transform lengths; the tuned
problem solves to the same f~ as the untuned one; the chosen solver settings are among
the candidates and converge."""
import numpy as np
import pytest

from oracle import matfree, workloads
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


@pytest.mark.parametrize("N,M", [(31, 3), (100, 3), (255, 2), (300, 2)])
def test_every_matvec_tiling_matches_oracle(monkeypatch, N, M):
    """L = 64, 256, 512 and 1024: each tiling the autotuner may pick (8, 16, 32 values per thread, the
    fixed-length 512 kernels) against the oracle's FFT matvec, FP64 and FP32."""
    inp = inputs.small(2, N, M, beta=0.55, omega=1.45)
    p = workloads.problem(inp, mu=np.zeros(inp.Nd))
    y = np.random.default_rng(61).standard_normal(p.n_tot)
    ref = matfree.matvec(p, y, matfree.circulant_symbol(p))
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a()) as g:
        _, t = g.autotune(tsfde.default_opts(), what=1)
        ids = [int(t.mv_ids[i]) for i in range(t.n_mv)]
        assert t.n_mv >= 1 and t.mv_variant in ids
        yt = torch.tensor(y, device=DEV)
        for v in ids:
            monkeypatch.setenv("TSFDE_MV_VARIANT", str(v))
            z = g.apply_A(yt).cpu().numpy()
            z32 = g.apply_A(yt.float()).cpu().double().numpy()
            assert rel_err(z, ref) <= 1e-13, v
            assert rel_err(z32, ref) <= 5e-6, v
        if N == 255:
            assert set(ids) == {0, 1, 2, 3, 4}


def test_autotune_keeps_results_and_picks_a_candidate():
    inp = inputs.small(2, 63, 12, beta=0.5, omega=1.5)
    p = workloads.with_data(inp)
    base = tsfde.default_opts(tol=1e-10, inner_tol=1e-3)
    with tsfde.Problem.from_inputs(inp, mu=p.mu, stencil=p.a()) as g:
        f0, s0 = g.recover_f(base, raise_noconv=True)
        o, t = g.autotune(base, what=3)
        assert t.solves >= 2 and t.solve_s > 0
        assert o.restart == t.restart and o.inner_tol == t.inner_tol and o.warm_start == t.warm_start
        assert t.inner_tol in (0.3, 0.1, 0.03, 0.01, base.inner_tol)
        assert t.n_pinv >= 1 and t.pinv_blocks in [int(t.pinv_cand[i]) for i in range(t.n_pinv)]
        f1, s1 = g.recover_f(o, raise_noconv=True)
        assert s1.converged == 1 and s1.iters <= o.restart
    assert rel_err(f1.cpu().numpy(), f0.cpu().numpy()) <= 1e-8


def test_autotune_argument_errors():
    inp = inputs.small(1, 12, 7)
    with tsfde.Problem.from_inputs(inp) as g:
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.autotune(tsfde.default_opts(), what=4)
        assert ei.value.status == tsfde.EINVAL
        o, t = g.autotune(tsfde.default_opts(tol=1e-9), what=1)  # 1D: no 2D tiling, no 2D grid
        assert t.mv_variant == -1 and t.n_mv == 0 and t.n_pinv == 0
