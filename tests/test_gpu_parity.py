"""Parity of each HIP step with the CPU oracle on the same seeded inputs
(FP64 to rounding; mixed precision within its FP16/FP32 bound)."""
import numpy as np
import pytest

import synthetic as syn
from oracle import amg, dirac as od
from gpu_common import Problem, rel, BC_AP

pytestmark = pytest.mark.gpu

# lattices: a 4^4 with 2^4 blocks (coarse extent 2), a ragged volume (V = 576
# is not a multiple of the 256-site tile) and an 8^4 with 4^4 blocks
GEOMS = [((4, 4, 4, 4), (2, 2, 2, 2)), ((6, 4, 4, 6), (2, 2, 2, 2)), ((8, 8, 8, 8), (4, 4, 4, 4))]


@pytest.fixture(scope='module', params=GEOMS, ids=lambda g: 'x'.join(map(str, g[0])))
def prob(request):
    dims, block = request.param
    return Problem(dims, block, eps=0.5, seed=1, kappa=0.124, csw=1.1)


def test_clover_matches_oracle(prob):
    F = prob.zeros((syn.volume(prob.dims), 2, 6, 6))
    prob.ctx.get_clover(F)
    want = prob.Fb.reshape(-1, 2, 6, 6)
    assert rel(prob.N(F), want) < 1e-13


@pytest.mark.parametrize('nrhs', [1, 3])
def test_apply_D_fp64(prob, nrhs):
    from paper_2111_05012_amd import PREC_FP64
    psi = syn.gaussian_vectors(prob.dims, nrhs, 11)
    out = prob.zeros(psi.shape)
    prob.ctx.apply_D(prob.T(psi), out, nrhs, PREC_FP64)
    want = prob.op.D(psi)
    assert rel(prob.N(out), want) < 1e-13


def test_apply_D_mixed(prob):
    """FP16 links/clover, FP32 spinors: relative error of order the FP16 unit
    roundoff 2^-11 times the few terms summed per component."""
    from paper_2111_05012_amd import PREC_MIXED
    psi = syn.gaussian_vectors(prob.dims, 2, 12)
    out = prob.zeros(psi.shape)
    prob.ctx.apply_D(prob.T(psi), out, 2, PREC_MIXED)
    want = prob.op.D(psi)
    assert rel(prob.N(out), want) < 2e-3


def test_apply_Dsap_fp64(prob):
    from paper_2111_05012_amd import PREC_FP64
    psi = syn.gaussian_vectors(prob.dims, 2, 13)
    out = prob.zeros(psi.shape)
    prob.ctx.apply_Dsap(prob.T(psi), out, 2, PREC_FP64)
    assert rel(prob.N(out), prob.op.Dsap(psi)) < 1e-13


def test_sap_fp64(prob):
    from paper_2111_05012_amd import PREC_FP64
    if any((d // b) % 2 for d, b in zip(prob.dims, prob.block)):
        pytest.skip('SAP colouring needs an even number of domains per direction')
    b = syn.gaussian_vectors(prob.dims, 2, 14)
    x = prob.zeros(b.shape)
    prob.ctx.sap(prob.T(b), x, 2, 4, 6, PREC_FP64)
    want = amg.sap(prob.op, b, 4, 6)
    assert rel(prob.N(x), want) < 1e-11


def test_sap_mixed(prob):
    from paper_2111_05012_amd import PREC_MIXED
    if any((d // b) % 2 for d, b in zip(prob.dims, prob.block)):
        pytest.skip('SAP colouring needs an even number of domains per direction')
    b = syn.gaussian_vectors(prob.dims, 1, 15)
    x = prob.zeros(b.shape)
    prob.ctx.sap(prob.T(b), x, 1, 4, 6, PREC_MIXED)
    want = amg.sap(prob.op, b, 4, 6)
    assert rel(prob.N(x), want) < 1e-2


@pytest.mark.parametrize('nv', [6, 20, 32])
def test_orthonormalize_fp64(prob, nv):
    """FP64 block orthonormalisation (Gram matrices on the FP64 matrix cores;
    nv = 20 and 32 span two 16-row output tiles, whose off-diagonal tile is
    written from its Hermitian mirror)."""
    from paper_2111_05012_amd import PREC_FP64
    V = syn.gaussian_vectors(prob.dims, nv, 16)
    out = prob.zeros(V.shape)
    prob.ctx.orthonormalize(prob.T(V), out, nv, PREC_FP64)
    want = amg.block_orthonormalize(V, prob.dims, prob.block)
    assert rel(prob.N(out), want) < 1e-12


@pytest.mark.parametrize('nv', [6, 20, 32])
def test_orthonormalize_mixed(prob, nv):
    """Mixed precision (FP32 vectors, FP64 Gram on the matrix cores, FP32
    matrix-core update): the result of Cholesky-QR twice agrees with the
    oracle to FP32 rounding amplified by the blocks' condition numbers."""
    from paper_2111_05012_amd import PREC_MIXED
    V = syn.gaussian_vectors(prob.dims, nv, 16)
    out = prob.zeros(V.shape)
    prob.ctx.orthonormalize(prob.T(V), out, nv, PREC_MIXED)
    want = amg.block_orthonormalize(V, prob.dims, prob.block)
    assert rel(prob.N(out), want) < 2e-5


def _hier(prob, nv=4, prec=0, coarse_iters=20, coarse_tol=0.0, seed=17, smoothing=0):
    V = amg.block_orthonormalize(syn.gaussian_vectors(prob.dims, nv, seed), prob.dims, prob.block)
    odd = any((d // b) % 2 for d, b in zip(prob.dims, prob.block))
    p = prob.ctx.setup_params(nv, prec, coarse_iters=coarse_iters, coarse_tol=coarse_tol,
                              sap_sweeps=0 if odd else 4, smoothing=smoothing)
    prob.ctx.set_test_vectors(prob.T(V), p)
    return V


def test_restrict_prolong_fp64(prob):
    V = _hier(prob)
    x = syn.gaussian_vectors(prob.dims, 2, 18)
    nX = amg.n_blocks(prob.dims, prob.block)
    xc = prob.zeros((2, nX, 8))
    prob.ctx.restrict(prob.T(x), xc, 2)
    assert rel(prob.N(xc), amg.restrict(V, x, prob.dims, prob.block)) < 1e-13
    yc = syn.gaussian_coarse(nX, 8, 2, 19)
    y = prob.zeros(x.shape)
    prob.ctx.prolong(prob.T(yc), y, 2)
    assert rel(prob.N(y), amg.prolong(V, yc, prob.dims, prob.block)) < 1e-13


@pytest.mark.parametrize('nrhs', [3, 20])
def test_restrict_prolong_mixed_every_variant(prob, nrhs, tmp_path):
    """Mixed-precision restriction and prolongation (FP16 vectors, FP32
    arithmetic) in every launch variant: the vector-ALU kernels with each
    site tile and the FP32 matrix-core kernels, staged through LDS or (block
    volume divisible by 32) with register operands (20 right-hand sides take
    two column tiles of the stacked real and imaginary parts), forced through
    the tuner's cache file, against the oracle with the same FP16-rounded
    vectors."""
    import json
    from paper_2111_05012_amd import PREC_MIXED
    nv = 12
    cache = str(tmp_path / 'tune.json')
    prob.ctx.autotune(True, cache)
    V = _hier(prob, nv=nv, prec=PREC_MIXED)
    V16 = V.real.astype(np.float16).astype(np.float64) + 1j * V.imag.astype(np.float16).astype(np.float64)
    nX = amg.n_blocks(prob.dims, prob.block)
    x = syn.gaussian_vectors(prob.dims, nrhs, 18)
    yc = syn.gaussian_coarse(nX, 2 * nv, nrhs, 19)
    want_r = amg.restrict(V16, x, prob.dims, prob.block)
    want_p = amg.prolong(V16, yc, prob.dims, prob.block)
    xc = prob.zeros((nrhs, nX, 2 * nv))
    y = prob.zeros(x.shape)
    prob.ctx.restrict(prob.T(x), xc, nrhs)  # tunes and writes the cache
    prob.ctx.prolong(prob.T(yc), y, nrhs)
    keys = json.load(open(cache))
    assert any(k.split('|')[1] == 'restrict' for k in keys) and any(k.split('|')[1] == 'prolong' for k in keys)
    vb = int(np.prod(prob.block))
    rvars = (4, 8, 16, 32, -32) + ((-33,) if vb % 32 == 0 else ())
    for kind, variants in (('restrict', rvars), ('prolong', (0, -32))):
        for v in variants:
            forced = {k: (v if k.split('|')[1] == kind else val) for k, val in keys.items()}
            with open(cache, 'w') as f:
                json.dump(forced, f)
            prob.ctx.autotune(True, cache)
            if kind == 'restrict':
                xc = prob.zeros((nrhs, nX, 2 * nv))
                prob.ctx.restrict(prob.T(x), xc, nrhs)
                assert rel(prob.N(xc), want_r) < 2e-5, (kind, v)
            else:
                y = prob.zeros(x.shape)
                prob.ctx.prolong(prob.T(yc), y, nrhs)
                assert rel(prob.N(y), want_p) < 2e-5, (kind, v)
    prob.ctx.autotune(False, None)


def test_coarse_operator_fp64(prob):
    V = _hier(prob)
    nX = amg.n_blocks(prob.dims, prob.block)
    Dc = prob.zeros((nX, 9, 8, 8))
    prob.ctx.get_coarse_op(Dc, level=1)
    want = amg.coarse_operator(prob.op, V)
    assert rel(prob.N(Dc), want) < 1e-13
    x = syn.gaussian_coarse(nX, 8, 3, 20)
    y = prob.zeros(x.shape)
    prob.ctx.apply_coarse(prob.T(x), y, 3)
    cd = amg.coarse_dims(prob.dims, prob.block)
    assert rel(prob.N(y), amg.coarse_apply(want, x, cd)) < 1e-13


@pytest.mark.parametrize('nv', [4, 12])
def test_coarse_operator_mixed_every_variant(prob, nv, tmp_path):
    """Mixed-precision coarse operator (FP16 vectors, links and clover, FP32
    arithmetic) from both contraction kernels (vector ALU and matrix cores),
    each forced through the tuner's cache file, against the oracle's Galerkin
    product of the same FP16-rounded vectors."""
    import json
    from paper_2111_05012_amd import PREC_MIXED
    cache = str(tmp_path / 'tune.json')
    prob.ctx.autotune(True, cache)
    V = _hier(prob, nv=nv, prec=PREC_MIXED)
    V16 = V.real.astype(np.float16).astype(np.float64) + 1j * V.imag.astype(np.float16).astype(np.float64)
    want = amg.coarse_operator(prob.op, V16)
    nX = amg.n_blocks(prob.dims, prob.block)
    keys = json.load(open(cache))
    assert any(k.split('|')[1] == 'coarse_build' for k in keys)
    for v in (0, 1):
        forced = {k: (v if k.split('|')[1] == 'coarse_build' else val) for k, val in keys.items()}
        with open(cache, 'w') as f:
            json.dump(forced, f)
        prob.ctx.autotune(True, cache)
        _hier(prob, nv=nv, prec=PREC_MIXED)  # rebuilds the coarse operator with the forced kernel
        Dc = prob.zeros((nX, 9, 2 * nv, 2 * nv))
        prob.ctx.get_coarse_op(Dc, level=1)
        assert rel(prob.N(Dc), want) < 3e-3, v
    prob.ctx.autotune(False, None)


@pytest.mark.parametrize('nv', [8, 32])
@pytest.mark.parametrize('nrhs', [3, 12])
def test_apply_coarse_mixed_every_variant(prob, nrhs, nv, tmp_path):
    """Mixed-precision coarse stencil (complex64) in every launch variant
    (right-hand sides per thread and the two matrix-core kernels), forced
    through the tuner's cache file, against the oracle's 9-point stencil with
    the library's own coarse operator."""
    import json
    from paper_2111_05012_amd import PREC_MIXED
    cache = str(tmp_path / 'tune.json')
    prob.ctx.autotune(True, cache)
    _hier(prob, nv=nv, prec=PREC_MIXED)
    nX = amg.n_blocks(prob.dims, prob.block)
    Dc = prob.zeros((nX, 9, 2 * nv, 2 * nv))
    prob.ctx.get_coarse_op(Dc, level=1)
    Dc = prob.N(Dc)
    cd = amg.coarse_dims(prob.dims, prob.block)
    x = syn.gaussian_coarse(nX, 2 * nv, nrhs, 23)
    want = amg.coarse_apply(Dc, x, cd)
    y = prob.zeros(x.shape)
    prob.ctx.apply_coarse(prob.T(x), y, nrhs)
    keys = json.load(open(cache))
    assert any(k.split('|')[1] == 'coarse_mv' for k in keys)
    for v in (1, 4, 8, 12, 16, -1, -2):
        forced = {k: (v if k.split('|')[1] == 'coarse_mv' else val) for k, val in keys.items()}
        with open(cache, 'w') as f:
            json.dump(forced, f)
        prob.ctx.autotune(True, cache)
        y = prob.zeros(x.shape)
        prob.ctx.apply_coarse(prob.T(x), y, nrhs)
        assert rel(prob.N(y), want) < 5e-6, v
    prob.ctx.autotune(False, None)


def test_coarse_solve_fp64(prob):
    V = _hier(prob)
    nX = amg.n_blocks(prob.dims, prob.block)
    cd = amg.coarse_dims(prob.dims, prob.block)
    Dc = amg.coarse_operator(prob.op, V)
    b = syn.gaussian_coarse(nX, 8, 2, 21)
    x = prob.zeros(b.shape)
    prob.ctx.coarse_solve(prob.T(b), x, 2, 12, 0.0)
    for k in range(2):
        want, _ = amg.bicgstab(lambda z: amg.coarse_apply(Dc, z, cd), b[k], 12, 0.0)
        assert rel(prob.N(x)[k], want) < 1e-10


@pytest.mark.parametrize('smoothing', ['post', 'pre', 'both'])
def test_vcycle_fp64(prob, smoothing):
    """The FP64 V-cycle with the smoother after (the paper's choice), before,
    or before and after the coarse-grid step, against the oracle's."""
    if any((d // b) % 2 for d, b in zip(prob.dims, prob.block)):
        pytest.skip('SAP colouring needs an even number of domains per direction')
    code = {'post': 0, 'pre': 1, 'both': 2}[smoothing]
    V = _hier(prob, coarse_iters=10, coarse_tol=0.0, smoothing=code)
    mg = amg.TwoLevel(prob.op, V, 4, 6, coarse_iters=10, coarse_tol=0.0, smoothing=smoothing)
    v = syn.gaussian_vectors(prob.dims, 2, 22)
    out = prob.zeros(v.shape)
    prob.ctx.vcycle(prob.T(v), out, 2)
    assert rel(prob.N(out), mg.vcycle(v)) < 1e-10


def test_setup_and_solve_fp64_c1():
    """Config-1 workload: setup from the same start vectors as the oracle,
    then FGMRES(16) to 1e-10; residual recomputed by the oracle's D and the
    solution checked against dense LU."""
    from paper_2111_05012_amd import PREC_FP64
    c = syn.CONFIGS['c1']
    prob = Problem(c['dims'], c['block'], c['eps'], c['seed'], c['kappa'], c['csw'])
    V0 = syn.gaussian_vectors(prob.dims, c['nv'], c['seed'])
    p = prob.ctx.setup_params(c['nv'], PREC_FP64, n_init=3, n_adapt=3, coarse_iters=50, coarse_tol=0.1,
                              init_vectors=prob.T(V0))
    prob.ctx.setup(p)
    mg = amg.setup(prob.op, V0, n_init=3, n_adapt=3, coarse_iters=50, coarse_tol=0.1)
    Vg = prob.zeros(V0.shape)
    prob.ctx.get_test_vectors(Vg)
    # same setup, same inputs: equal up to rounding
    assert rel(prob.N(Vg), mg.V) < 1e-8
    b = syn.z2_source(prob.dims, c['seed'])
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 1, restart=16, tol=1e-10)
    assert rc == 0 and info.converged[0]
    xg = prob.N(x)
    res = np.linalg.norm(b - prob.op.D(xg)) / np.linalg.norm(b)
    assert res <= 1e-10
    D = od.dense_D(prob.U, prob.Fb, prob.kappa, BC_AP, prob.dims)
    xs = np.linalg.solve(D, b.reshape(-1))
    assert np.linalg.norm(xg.reshape(-1) - xs) / np.linalg.norm(xs) <= 1e-9
    _, its_oracle, _ = amg.fgmres(prob.op.D, mg.vcycle, b[0], tol=1e-10, restart=16)
    assert abs(info.iters[0] - its_oracle) <= 1


def test_setup_and_solve_mixed_c1():
    from paper_2111_05012_amd import PREC_MIXED
    c = syn.CONFIGS['c1']
    prob = Problem(c['dims'], c['block'], c['eps'], c['seed'], c['kappa'], c['csw'])
    V0 = syn.gaussian_vectors(prob.dims, c['nv'], c['seed'])
    p = prob.ctx.setup_params(c['nv'], PREC_MIXED, init_vectors=prob.T(V0))
    prob.ctx.setup(p)
    b = syn.z2_source(prob.dims, c['seed'], nrhs=2)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 2, restart=16, tol=1e-10)
    assert rc == 0
    xg = prob.N(x)
    for k in range(2):
        assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10


# ---------------------------------------------------------------- the paper's outer solver
def test_flexible_bicgstab_fp64_matches_oracle(prob):
    """The paper's flexible BiCGStab (FP64) with the FP64 V-cycle as M,
    against the oracle's flexible BiCGStab with the oracle's V-cycle on the
    same hierarchy: the same outer iteration count and the same solution."""
    from paper_2111_05012_amd import PC_AMG
    if any((d // b) % 2 for d, b in zip(prob.dims, prob.block)):
        pytest.skip('SAP colouring needs an even number of domains per direction')
    V = _hier(prob, coarse_iters=10, coarse_tol=0.0)
    mg = amg.TwoLevel(prob.op, V, 4, 6, coarse_iters=10, coarse_tol=0.0)
    b = syn.z2_source(prob.dims, 3, nrhs=2)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve_bicgstab(prob.T(b), x, 2, tol=1e-10, precond=PC_AMG)
    assert rc == 0
    xg = prob.N(x)
    for k in range(2):
        xo, its, res = amg.flexible_bicgstab(prob.op.D, mg.vcycle, b[k], tol=1e-10)
        assert info.iters[k] == its, (k, info.iters[k], its)
        assert info.relres[k] <= 1e-10
        assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10
        assert rel(xg[k], xo) < 1e-8


@pytest.mark.parametrize('smoothing', [1, 2])
def test_setup_and_solve_mixed_c1_smoothing(smoothing):
    """Config-1 workload with the smoother before (1), or before and after
    (2), the coarse-grid step, in setup and solve: FGMRES(16) to 1e-10."""
    from paper_2111_05012_amd import PREC_MIXED
    c = syn.CONFIGS['c1']
    prob = Problem(c['dims'], c['block'], c['eps'], c['seed'], c['kappa'], c['csw'])
    V0 = syn.gaussian_vectors(prob.dims, c['nv'], c['seed'])
    prob.ctx.setup(prob.ctx.setup_params(c['nv'], PREC_MIXED, init_vectors=prob.T(V0), smoothing=smoothing))
    b = syn.z2_source(prob.dims, c['seed'], nrhs=2)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 2, restart=16, tol=1e-10)
    assert rc == 0
    xg = prob.N(x)
    for k in range(2):
        assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10


def test_setup_and_solve_mixed_even_odd_smoother():
    """8^4 lattice with 4^4 blocks: setup and FGMRES(16) to 1e-10 with the
    even-odd preconditioned SAP block solve; residual by the oracle's D.
    The even-odd variant is rejected in FP64 and for odd block extents."""
    from paper_2111_05012_amd import PREC_MIXED, PREC_FP64, WcamgError, BLOCK_EO_MR, EINVAL
    prob = Problem((8, 8, 8, 8), (4, 4, 4, 4), eps=0.5, seed=1, kappa=0.124, csw=1.0)
    V0 = syn.gaussian_vectors(prob.dims, 8, 5)
    prob.ctx.setup(prob.ctx.setup_params(8, PREC_MIXED, init_vectors=prob.T(V0), sap_eo=1))
    b = syn.z2_source(prob.dims, 6, nrhs=2)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 2, tol=1e-10)
    assert rc == 0
    xg = prob.N(x)
    for k in range(2):
        assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10
    with pytest.raises(WcamgError) as e:
        prob.ctx.setup(prob.ctx.setup_params(8, PREC_FP64, init_vectors=prob.T(V0), sap_eo=1))
    assert e.value.code == EINVAL
    with pytest.raises(WcamgError):
        prob.ctx.sap(prob.T(b), x, 2, 4, 6, PREC_FP64, block_solve=BLOCK_EO_MR)


@pytest.mark.parametrize('prec', [0, 1])
def test_setup_vec_chunk_same_hierarchy(prec):
    """The setup's SAP and V-cycles taken over the test vectors in batches
    (vec_chunk 5 of 12: batches 5, 5, 2) give the hierarchy of the unbatched
    setup: the test vectors agree to rounding (the kernels' variants may
    differ with the batch size), and both solve to 1e-10 in the same number
    of outer iterations."""
    prob = Problem((8, 8, 8, 8), (4, 4, 4, 4), eps=0.5, seed=1, kappa=0.124, csw=1.0)
    import torch
    nv = 12
    V0 = syn.gaussian_vectors(prob.dims, nv, 5)
    b = syn.z2_source(prob.dims, 6, nrhs=2)
    got = []
    for ch in (0, 5):
        prob.ctx.setup(prob.ctx.setup_params(nv, prec, init_vectors=prob.T(V0), vec_chunk=ch))
        Q = torch.zeros((nv,) + syn.shape_of(prob.dims) + (4, 3), dtype=torch.complex128, device=prob.dev)
        prob.ctx.get_test_vectors(Q)
        x = prob.zeros(b.shape)
        rc, info = prob.ctx.solve(prob.T(b), x, 2, tol=1e-10)
        assert rc == 0
        xg = prob.N(x)
        for k in range(2):
            assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10
        got.append((Q.cpu().numpy(), list(info.iters[:2])))
    # FP64: summation orders only; mixed: the FP16 storage of the test
    # vectors can round a batch's vector to the neighbouring FP16 value
    assert rel(got[1][0], got[0][0]) < (1e-10 if prec == 0 else 1e-2)
    if prec == 0:
        assert got[1][1] == got[0][1]
    else:
        assert max(abs(i - j) for i, j in zip(got[1][1], got[0][1])) <= 1


def test_flexible_bicgstab_mixed_amg_and_mbicgs_c1():
    """Config-1 workload: the flexible BiCGStab preconditioned by the mixed
    V-cycle, and the comparison solver (preconditioned by an FP32 BiCGStab on
    D), both to 1e-10; residuals recomputed by the oracle's D.  The
    multigrid preconditioner needs fewer outer iterations."""
    from paper_2111_05012_amd import PREC_MIXED, PC_AMG, PC_BICG32
    c = syn.CONFIGS['c1']
    prob = Problem(c['dims'], c['block'], c['eps'], c['seed'], c['kappa'], c['csw'])
    V0 = syn.gaussian_vectors(prob.dims, c['nv'], c['seed'])
    prob.ctx.setup(prob.ctx.setup_params(c['nv'], PREC_MIXED, init_vectors=prob.T(V0)))
    b = syn.z2_source(prob.dims, c['seed'], nrhs=3)
    its = {}
    for pc in (PC_AMG, PC_BICG32):
        x = prob.zeros(b.shape)
        rc, info = prob.ctx.solve_bicgstab(prob.T(b), x, 3, tol=1e-10, precond=pc, inner_iters=20, inner_tol=0.1)
        assert rc == 0, pc
        xg = prob.N(x)
        for k in range(3):
            assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10, (pc, k)
        its[pc] = max(info.iters[:3])
    assert its[PC_AMG] <= its[PC_BICG32], its


# ---------------------------------------------------------------- three levels
def _three_level_problem(prec=0, nv=4, nv1=4):
    """8^4 with 2^4 blocks (coarse 4^4), level-1 blocks 2^4 (level-2 2^4)."""
    prob = Problem((8, 8, 8, 8), (2, 2, 2, 2), eps=0.5, seed=1, kappa=0.124, csw=1.0)
    V = amg.block_orthonormalize(syn.gaussian_vectors(prob.dims, nv, 51), prob.dims, prob.block)
    p = prob.ctx.setup_params(nv, prec, coarse_iters=8, coarse_tol=0.0, nlevels=3, block1=(2, 2, 2, 2),
                              nv1=nv1, mr1_iters=3)
    prob.ctx.set_test_vectors(prob.T(V), p)
    Dc = amg.coarse_operator(prob.op, V)
    cd = amg.coarse_dims(prob.dims, prob.block)
    cop = amg.CoarseOp(Dc, cd, (2, 2, 2, 2))
    W = amg.coarse_block_orthonormalize(syn.gaussian_coarse(cop.Dc.shape[0], 2 * nv, nv1, 52), cd, cop.block)
    prob.ctx.set_level1_vectors(prob.T(W))
    return prob, V, cop, W


def test_level2_operator_fp64():
    prob, V, cop, W = _three_level_problem()
    want = amg.coarse_coarse_operator(cop, W)
    got = prob.zeros(want.shape)
    prob.ctx.get_coarse_op(got, level=2)
    assert rel(prob.N(got), want) < 1e-12
    Wg = prob.zeros(W.shape)
    prob.ctx.get_level1_vectors(Wg)
    assert rel(prob.N(Wg), W) == 0.0


def test_level2_apply_and_solve_fp64():
    """The coarse matvec and the coarse solve on level 2 of a three-level
    hierarchy through the level argument of the C ABI, against the oracle's
    stencil and stabilised BiCGStab on the oracle's level-2 operator (loaded
    with set_coarse_op)."""
    prob, V, cop, W = _three_level_problem()
    D2 = amg.coarse_coarse_operator(cop, W)
    prob.ctx.set_coarse_op(prob.T(D2), level=2)
    got = prob.zeros(D2.shape)
    prob.ctx.get_coarse_op(got, level=2)
    assert rel(prob.N(got), D2) == 0.0
    n2, dof = D2.shape[0], D2.shape[2]
    cd2 = amg.coarse_dims(cop.cdims, cop.block)
    x = syn.gaussian_coarse(n2, dof, 2, 55)
    y = prob.zeros(x.shape)
    prob.ctx.apply_coarse(prob.T(x), y, 2, level=2)
    assert rel(prob.N(y), amg.coarse_apply(D2, x, cd2)) < 1e-13
    z = prob.zeros(x.shape)
    prob.ctx.coarse_solve(prob.T(x), z, 2, 6, 0.0, level=2)
    for k in range(2):
        want, _ = amg.bicgstab(lambda v: amg.coarse_apply(D2, v, cd2), x[k], 6, 0.0)
        assert rel(prob.N(z)[k], want) < 1e-10


def test_three_level_vcycle_fp64():
    prob, V, cop, W = _three_level_problem()
    lv1 = amg.Level1(cop, W, mr1_iters=3, coarse_iters=8, coarse_tol=0.0)
    mg = amg.ThreeLevel(prob.op, V, lv1, 4, 6)
    v = syn.gaussian_vectors(prob.dims, 2, 53)
    out = prob.zeros(v.shape)
    prob.ctx.vcycle(prob.T(v), out, 2)
    assert rel(prob.N(out), mg.vcycle(v)) < 1e-10


@pytest.mark.parametrize('prec', [0, 1])
def test_three_level_setup_and_solve(prec):
    """Full three-level setup (level-1 start vectors from the library's
    seeded generator) and FGMRES solve; residual recomputed by the oracle."""
    prob = Problem((8, 8, 8, 8), (2, 2, 2, 2), eps=0.5, seed=1, kappa=0.124, csw=1.0)
    V0 = syn.gaussian_vectors(prob.dims, 6, 54)
    p = prob.ctx.setup_params(6, prec, init_vectors=prob.T(V0), nlevels=3, block1=(2, 2, 2, 2), nv1=6,
                              mr1_iters=4, seed1=7)
    prob.ctx.setup(p)
    b = syn.z2_source(prob.dims, 2, nrhs=2)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 2, restart=16, tol=1e-10)
    assert rc == 0
    xg = prob.N(x)
    for k in range(2):
        assert np.linalg.norm(b[k] - prob.op.D(xg[k])) / np.linalg.norm(b[k]) <= 1e-10


def test_dslash_every_launch_variant(tmp_path):
    """All autotuner variants of the fine operator (workgroup sizes and the
    colour-split kernel) give the oracle's result: force each one through the
    tuner's cache file."""
    import json
    from paper_2111_05012_amd import PREC_FP64, PREC_MIXED
    prob = Problem((6, 4, 4, 6), (2, 2, 2, 2), eps=0.5, seed=3, kappa=0.124, csw=1.1)
    cache = str(tmp_path / 'tune.json')
    prob.ctx.autotune(True, cache)
    psi = syn.gaussian_vectors(prob.dims, 2, 61)
    want = prob.op.D(psi)
    for prec, tol in ((PREC_FP64, 1e-13), (PREC_MIXED, 2e-3)):
        out = prob.zeros(psi.shape)
        prob.ctx.apply_D(prob.T(psi), out, 2, prec)  # tunes and writes the cache
        keys = json.load(open(cache))
        for v in (64, 128, 256, 512, -1, -2, -3, -12, -14):
            forced = {k: (v if k.split('|')[1] == 'dslash' else val) for k, val in keys.items()}
            with open(cache, 'w') as f:
                json.dump(forced, f)
            prob.ctx.autotune(True, cache)
            out = prob.zeros(psi.shape)
            prob.ctx.apply_D(prob.T(psi), out, 2, prec)
            assert rel(prob.N(out), want) < tol, (prec, v)


@pytest.mark.parametrize('prec', [0, 1])
def test_solve_phase_times(prec):
    """Table 1's split of the solve time (coarse solve, smoother, R/P, rest of
    the preconditioner, outer solver) through the C ABI: every phase is
    timed, the parts add up, and the timed (graph-free) solve gives the same
    iterations and solution as the graph-replayed one."""
    c = syn.CONFIGS['c1']
    prob = Problem(c['dims'], c['block'], c['eps'], c['seed'], c['kappa'], c['csw'])
    V0 = syn.gaussian_vectors(prob.dims, c['nv'], c['seed'])
    prob.ctx.setup(prob.ctx.setup_params(c['nv'], prec, init_vectors=prob.T(V0)))
    b = syn.z2_source(prob.dims, c['seed'], nrhs=2)
    x0 = prob.zeros(b.shape)
    rc0, inf0 = prob.ctx.solve(prob.T(b), x0, 2, tol=1e-10)
    assert rc0 == 0 and inf0.t_precond == 0.0 and inf0.t_outer == 0.0
    x1 = prob.zeros(b.shape)
    rc1, inf1 = prob.ctx.solve(prob.T(b), x1, 2, tol=1e-10, phase_times=1)
    assert rc1 == 0
    ph = inf1.phases()
    for k in ('t_precond', 't_coarse', 't_smoother', 't_rp', 't_outer'):
        assert ph[k] > 0, (k, ph)
    assert ph['t_coarse'] + ph['t_smoother'] + ph['t_rp'] <= ph['t_precond'] * (1 + 1e-9)
    assert abs(ph['t_prec_other'] - (ph['t_precond'] - ph['t_coarse'] - ph['t_smoother'] - ph['t_rp'])) < 1e-9
    assert abs(ph['t_outer'] - (ph['t_solve'] - ph['t_precond'])) < 1e-9
    assert list(inf1.iters[:2]) == list(inf0.iters[:2])
    assert rel(prob.N(x1), prob.N(x0)) < 1e-12
    # the paper's outer solver splits its time the same way
    x2 = prob.zeros(b.shape)
    rc2, inf2 = prob.ctx.solve_bicgstab(prob.T(b), x2, 2, tol=1e-10, phase_times=1)
    assert rc2 == 0 and inf2.t_precond > 0 and inf2.t_smoother > 0 and inf2.t_coarse > 0
