"""The no-allocation entry point wcamg_apply_D_noalloc (fixed scratch area
instead of workspaces) against wcamg_apply_D, through the C ABI: two calls in
a row on one context, the second with fewer right-hand sides, in FP64 and
mixed precision, and the size limit rejected on the host."""
import ctypes

import numpy as np
import pytest

import synthetic as syn
from gpu_common import Problem, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('prec', [0, 1])
def test_apply_D_noalloc_matches_apply_D(prec):
    from paper_2111_05012_amd import wcamg
    prob = Problem((8, 8, 8, 8), (4, 4, 4, 4), eps=0.5, seed=2, kappa=0.124, csw=1.1)
    for nrhs, seed in ((3, 91), (1, 92)):
        psi = prob.T(syn.gaussian_vectors(prob.dims, nrhs, seed))
        want = prob.zeros(psi.shape)
        prob.ctx.apply_D(psi, want, nrhs, prec)
        got = prob.zeros(psi.shape)
        got.fill_(float('nan'))  # every output element must be written
        prob.ctx.apply_D_noalloc(psi, got, nrhs, prec)
        g, w = prob.N(got), prob.N(want)
        assert np.isfinite(g).all()
        assert rel(g, w) <= (1e-14 if prec == 0 else 1e-7), (nrhs, rel(g, w))
        if prec == 0:
            # FP64 against the oracle's operator as well
            assert rel(g, prob.op.D(prob.N(psi))) < 1e-13


def test_apply_D_noalloc_rejects_oversized_input():
    from paper_2111_05012_amd import wcamg
    prob = Problem((8, 8, 8, 8), (4, 4, 4, 4), eps=0.5, seed=2, kappa=0.124, csw=1.1)
    V = syn.volume(prob.dims)
    per_rhs = 12 * V * 16
    nrhs = wcamg.NOALLOC_SCRATCH_BYTES // (2 * per_rhs) + 1  # just beyond the limit in FP64
    assert nrhs <= wcamg.MAX_RHS
    psi = prob.zeros((nrhs,) + syn.shape_of(prob.dims) + (4, 3))
    out = prob.zeros(psi.shape)
    rc = prob.ctx.lib.wcamg_apply_D_noalloc(prob.ctx.h, ctypes.c_void_p(psi.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), nrhs, 0)
    assert rc == wcamg.EINVAL
    assert b'scratch' in prob.ctx.lib.wcamg_last_error(prob.ctx.h)
    # the context still works afterwards
    psi1 = prob.T(syn.gaussian_vectors(prob.dims, 1, 93))
    out1 = prob.zeros(psi1.shape)
    prob.ctx.apply_D_noalloc(psi1, out1, 1, 0)
    assert rel(prob.N(out1), prob.op.D(prob.N(psi1))) < 1e-13
