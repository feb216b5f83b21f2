"""The outer FGMRES with its two orthogonalisations of the Arnoldi vectors:
classical Gram-Schmidt twice (ortho=1) and the same with the second pass
delayed into the next step (ortho=0, the default).  Both must reach the
tolerance (residual recomputed with the oracle's D) in the same number of
steps and agree on the solution.  A deliberately weak V-cycle (one SAP
sweep of one MR step, two coarse iterations, 4 test vectors) takes about 35
steps on the 8^4 lattice, so that a cycle of 32 passes the 16-vector chunk
of the Gram-Schmidt sweeps and right-hand sides stop at different steps of
one cycle."""
import numpy as np
import pytest

import synthetic as syn
from gpu_common import Problem

pytestmark = pytest.mark.gpu

WEAK = dict(nv=4, sap_sweeps=1, mr_iters=1, coarse_iters=2)


@pytest.fixture(scope='module')
def p8():
    return Problem((8, 8, 8, 8), (4, 4, 4, 4), eps=0.5, seed=2, kappa=0.124, csw=1.0)


def _setup(prob, prec, nv=8, **kw):
    V0 = syn.gaussian_vectors(prob.dims, nv, 7)
    prob.ctx.setup(prob.ctx.setup_params(nv, prec, init_vectors=prob.T(V0), **kw))


def _rhs(prob):
    """A Z2 source, a Gaussian one and a Gaussian one under a linear ramp."""
    g = syn.gaussian_vectors(prob.dims, 2, 9)
    ramp = np.linspace(0.0, 1.0, g[1].size).reshape(g[1].shape)
    return np.concatenate([syn.z2_source(prob.dims, 4, nrhs=1), g[0:1], (g[1] * ramp)[None]])


def _solve(prob, b, **kw):
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, len(b), tol=1e-10, **kw)
    xg = prob.N(x)
    res = [np.linalg.norm(b[k] - prob.op.D(xg[k])) / max(np.linalg.norm(b[k]), 1e-300) for k in range(len(b))]
    return rc, info, xg, res


@pytest.mark.parametrize('prec,weak,restart', [('fp64', False, 1), ('mixed', False, 2), ('fp64', False, 3),
                                               ('mixed', False, 16), ('fp64', True, 3), ('fp64', True, 16),
                                               ('fp64', True, 32), ('mixed', True, 32)])
def test_delayed_and_classical_gram_schmidt_agree(p8, prec, weak, restart):
    from paper_2111_05012_amd import PREC_FP64, PREC_MIXED
    _setup(p8, PREC_FP64 if prec == 'fp64' else PREC_MIXED, **(WEAK if weak else {}))
    b = _rhs(p8)
    out = []
    for ortho in (0, 1):
        rc, info, xg, res = _solve(p8, b, restart=restart, ortho=ortho)
        its = list(info.iters[:3])
        print(prec, 'weak' if weak else 'default', 'restart', restart, 'ortho', ortho, 'iters', its,
              'residuals', ['%.2e' % r for r in res])
        assert rc == 0 and all(info.converged[:3])
        assert max(res) <= 1e-10
        assert max(info.relres[:3]) <= 1e-10
        out.append((its, xg))
    if weak:
        assert min(out[0][0]) > 17  # the sweeps ran over more than one 16-vector chunk
    assert all(abs(a - c) <= 1 for a, c in zip(out[0][0], out[1][0])), (out[0][0], out[1][0])
    # both solve D x = b to 1e-10: the solutions agree to the conditioning
    assert np.abs(out[0][1] - out[1][1]).max() / np.abs(out[1][1]).max() < 1e-7


@pytest.mark.parametrize('ortho', [0, 1])
def test_batch_members_solve_as_alone(p8, ortho):
    """A batch with a zero right-hand side (stopped before the first step)
    and right-hand sides that stop at different steps of one cycle: each
    nonzero one takes the steps it takes alone and gives the same solution;
    the zero one gives x = 0 after no step."""
    from paper_2111_05012_amd import PREC_FP64
    _setup(p8, PREC_FP64, **WEAK)
    b = _rhs(p8)
    bz = np.concatenate([b[0:1], np.zeros_like(b[0:1]), b[1:3]])
    rc, info, xg, res = _solve(p8, bz, restart=32, ortho=ortho)
    its = list(info.iters[:4])
    print('batch iters', its)
    assert rc == 0 and all(info.converged[:4])
    assert its[1] == 0 and np.abs(xg[1]).max() == 0.0 and info.relres[1] == 0.0
    for k, src in ((0, 0), (2, 1), (3, 2)):
        assert res[k] <= 1e-10
        rc1, info1, x1, res1 = _solve(p8, b[src:src + 1], restart=32, ortho=ortho)
        assert rc1 == 0 and info1.iters[0] == its[k], (k, info1.iters[0], its[k])
        assert np.abs(x1[0] - xg[k]).max() / np.abs(x1[0]).max() < 1e-9


def test_solve_rejects_unknown_orthogonalisation(p8):
    """ortho takes 0 or 1; anything else is an argument error, raised before
    any work."""
    from paper_2111_05012_amd import PREC_FP64, WcamgError, EINVAL
    _setup(p8, PREC_FP64)
    b = _rhs(p8)[:1]
    x = p8.zeros(b.shape)
    for bad in (-1, 2):
        with pytest.raises(WcamgError) as e:
            p8.ctx.solve(p8.T(b), x, 1, ortho=bad)
        assert e.value.code == EINVAL


@pytest.mark.parametrize('prec', ['fp64', 'mixed'])
def test_graph_replays_match_eager(p8, prec):
    """The V-cycle replayed from its captured graphs, over three solves in a
    row (the graphs of every Krylov slot replayed many times, with the outer
    solver's eager kernels and synchronisations in between), gives the
    eager V-cycle's iterations and solution (the kernels reduce in a fixed
    order, so to rounding at most)."""
    from paper_2111_05012_amd import PREC_FP64, PREC_MIXED
    _setup(p8, PREC_FP64 if prec == 'fp64' else PREC_MIXED, **WEAK)
    b = _rhs(p8)
    rc, info, x_eager, _ = _solve(p8, b, restart=16, use_graph=0)
    assert rc == 0
    for rep in range(3):
        rc, info_g, x_g, res = _solve(p8, b, restart=16, use_graph=1)
        assert rc == 0 and max(res) <= 1e-10
        assert list(info_g.iters[:3]) == list(info.iters[:3]), rep
        assert np.abs(x_g - x_eager).max() / np.abs(x_eager).max() < 1e-12, rep
