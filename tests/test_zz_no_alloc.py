"""tsfde_apply_P_inv_noalloc (the allocation-free P^-1, work buffers in the library's static device
scratch) against tsfde_apply_P_inv through the C ABI: two calls in a row, the second on a smaller
problem, plus its refusals (a problem larger than the scratch, the Strang form)."""
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
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _pair(inp, zz, opts, stencil=None):
    with tsfde.Problem.from_inputs(inp, stencil=stencil) as g:
        z = torch.tensor(zz, device=DEV)
        y_ref = g.apply_P_inv(z, opts=opts).cpu().numpy()
        y = torch.full_like(z, float("nan"))
        g.apply_P_inv_noalloc(z, y, opts=opts)
        return y.cpu().numpy(), y_ref


def test_noalloc_matches_apply_P_inv_twice_then_smaller():
    o = tsfde.default_opts(inner_tol=1e-12, inner_maxit=500)
    # first call: d = 2, N = 127 (fixed-length transform kernels), 24 time steps
    big = inputs.small(2, 127, 24, beta=0.6, omega=1.6)
    zb = np.random.default_rng(51).standard_normal(big.n_tot)
    y, y_ref = _pair(big, zb, o)
    assert np.all(np.isfinite(y))
    assert rel_err(y, y_ref) <= 1e-12
    # second call right after, on a smaller problem (d = 2, N = 15): against the dense P of the oracle too
    small = inputs.small(2, 15, 9, beta=0.5, omega=1.5)
    p = workloads.problem(small, mu=np.zeros(small.Nd))
    zs = np.random.default_rng(52).standard_normal(p.n_tot)
    o14 = tsfde.default_opts(inner_tol=1e-14, inner_maxit=500)
    y2, y2_ref = _pair(small, zs, o14, stencil=p.a())
    assert rel_err(y2, y2_ref) <= 1e-12
    assert rel_err(y2, np.linalg.solve(system.dense_P(p), zs)) <= 1e-10
    # and a 1D problem, tau-block form on a 2D one
    one = inputs.small(1, 255, 40, beta=0.3, omega=1.2)
    z1 = np.random.default_rng(53).standard_normal(one.n_tot)
    y3, y3_ref = _pair(one, z1, o)
    assert rel_err(y3, y3_ref) <= 1e-12
    ot = tsfde.default_opts(block_solver=tsfde.BLOCK_TAU)
    y4, y4_ref = _pair(small, zs, ot)
    assert rel_err(y4, y4_ref) <= 1e-12


def test_noalloc_refusals():
    # d = 2, N = 400: 160 000 points per slice need more than the 32 MiB scratch
    inp = inputs.small(2, 400, 2, beta=0.5, omega=1.5)
    with tsfde.Problem.from_inputs(inp, stencil=workloads.problem(inp).a()) as g:
        z = torch.zeros(g.n_tot, dtype=torch.float64, device=DEV)
        y = torch.empty_like(z)
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.apply_P_inv_noalloc(z, y)
        assert ei.value.status == tsfde.ENOMEM and "scratch" in str(ei.value)
    small = inputs.small(2, 15, 4)
    with tsfde.Problem.from_inputs(small) as g:
        z = torch.zeros(g.n_tot, dtype=torch.float64, device=DEV)
        with pytest.raises(tsfde.TsfdeError) as ei:
            g.apply_P_inv_noalloc(z, torch.empty_like(z), opts=tsfde.default_opts(block_solver=tsfde.BLOCK_STRANG))
        assert ei.value.status == tsfde.ENOTIMPL
