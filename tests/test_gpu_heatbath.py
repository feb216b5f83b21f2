"""The HIP path on a smooth heat-bath gauge field (Wilson action, beta 6.0)
instead of random links: FP64 Dslash parity with the oracle, and the mixed
AMG solve to 1e-10 checked with the oracle's operator."""
import numpy as np
import pytest

import synthetic as syn
from synthetic import heatbath as hb
from gpu_common import Problem, rel

pytestmark = pytest.mark.gpu


def test_heatbath_field_dslash_parity_and_mixed_solve():
    from paper_2111_05012_amd import PREC_FP64, PREC_MIXED
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = hb.heatbath_field(dims, 6.0, 20, 3)
    prob = Problem(dims, block, kappa=0.1345, csw=1.769, U=U)
    psi = syn.gaussian_vectors(dims, 2, 4)
    out = prob.zeros(psi.shape)
    prob.ctx.apply_D(prob.T(psi), out, 2, PREC_FP64)
    got = prob.N(out)
    for k in range(2):
        assert rel(got[k], prob.op.D(psi[k])) < 1e-12
    V0 = syn.gaussian_vectors(dims, 8, 3)
    prob.ctx.setup(prob.ctx.setup_params(8, PREC_MIXED, init_vectors=prob.T(V0)))
    b = syn.point_sources(dims, 2)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 2, restart=16, tol=1e-10)
    assert rc == 0
    xg = prob.N(x)
    for k in range(2):
        assert info.relres[k] <= 1e-10
        assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10
