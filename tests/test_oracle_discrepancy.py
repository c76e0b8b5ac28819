"""Pins of the discrepancy-principle oracle: the discrepancy of the quasi-boundary-value
reconstruction equals the last block row's term c_f ||D_2^(S) B f~_alpha|| (the first S block
rows of A y = z are the direct problem with source f~, so F f~ = y^(S) exactly), and it grows
with alpha."""
import dataclasses

import numpy as np
import pytest

from oracle import discrepancy, system, workloads
from paper_2507_02809_amd import inputs

CASES = [
    ("1d", lambda: inputs.small(1, 12, 7)),
    ("2d", lambda: inputs.small(2, 7, 9, beta=0.3, omega=1.2)),
    ("c1", lambda: inputs.c1()),
]
ALPHAS = np.logspace(-8, -1, 8)


@pytest.fixture(params=CASES, ids=[c[0] for c in CASES])
def prob(request):
    return workloads.with_data(request.param[1]())


def test_discrepancy_equals_final_condition_term(prob):
    res = discrepancy.residuals(prob, ALPHAS)
    B = system.dense_B(prob)
    for a, r in zip(ALPHAS, res):
        q = dataclasses.replace(prob, alpha=float(a))
        f = discrepancy.recovered_f(q)
        ref = q.c_f * np.linalg.norm(q.gamma2[q.S - 1] * (B @ f))
        assert r == pytest.approx(ref, rel=1e-8)


def test_discrepancy_grows_with_alpha_and_vanishes(prob):
    res = discrepancy.residuals(prob, ALPHAS)
    assert all(b > a for a, b in zip(res, res[1:]))
    assert res[0] < 1e-3 * np.linalg.norm(prob.mu)
    # the selected alpha is the largest grid point under tau * delta
    delta = 0.5 * res[4] + 0.5 * res[5]
    assert discrepancy.select(ALPHAS, res, delta, tau=1.0) == ALPHAS[4]
