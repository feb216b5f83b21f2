"""Element-wise parity of the kernels the 32^3x64 benchmark runs, at its
domain shape: 4^3x8 blocks (512-site SAP domains and aggregates, t-slab tiles
of the LDS Dslash shorter than the block), N_v = 32 test vectors (2 N_v = 64
coarse dof) and 12 right-hand sides, on an 8^3x16 lattice (two blocks per
direction, the smallest lattice with this block shape and an even number of
SAP domains per direction) with the benchmark's parameters (eps 0.3, kappa
0.1365, c_sw 1.1).

Mixed-precision results are compared with the FP64 oracle evaluated on the
same FP16-rounded hop matrices -kappa U, clover and test vectors, the same FP32-rounded
inputs and (for the coarse level) the same complex64-rounded coarse
operator.  What remains between the two is the FP32 arithmetic of the
kernels, so the tolerances are FP32-rounding bounds (at most 1e-5 relative
to the max-norm of the result), not FP16 ones.

The oracle runs one right-hand side at a time in NumPy; where it would take
minutes for all 12, the GPU solves all 12 in one launch and the oracle
checks a sample of them (first, middle, last), each an independent system."""
import json

import numpy as np
import pytest

import synthetic as syn
from oracle import amg, dirac as od
from gpu_common import Problem, rel

pytestmark = pytest.mark.gpu

DIMS, BLOCK = (8, 8, 8, 16), (4, 4, 4, 8)
KAPPA, CSW, EPS = 0.1365, 1.1, 0.3
NV, NRHS = 32, 12
SAMPLE = (0, 5, 11)

# FP32 bounds (relative max-norm), see the module docstring and the design doc:
# 2^-24 times the square root of the longest sequential FP32 accumulation
# chain of the step, times a safety factor of about 10 (D: ~100 terms per
# output; restriction: 768-term chains per wavefront of the 3072-term block
# sums; coarse build: block sums of 512 sites; SAP and the coarse solve:
# iterated, whose measured growth stays within the single-step bound)
TOL_D = 2e-6
TOL_RP = 1e-5
TOL_DC = 1e-5
TOL_CMV = 1e-5
TOL_SAP = 2e-6
TOL_CSOLVE = 1e-5
TOL_VCYCLE = 5e-6


def r16(a):
    """Round the real and imaginary parts to FP16 (round to nearest even)."""
    a = np.asarray(a)
    return a.real.astype(np.float16).astype(np.float64) + 1j * a.imag.astype(np.float16).astype(np.float64)


def r32(a):
    """Round to complex64 (round to nearest even)."""
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


@pytest.fixture(scope='module')
def prod():
    prob = Problem(DIMS, BLOCK, eps=EPS, seed=1, kappa=KAPPA, csw=CSW)
    # the oracle's operator on the library's FP16 storage: the hop matrices
    # -kappa U (one rounding of the FP64 product) and the clover term
    prob.op16 = amg.FineOp(r16(-KAPPA * prob.U) / -KAPPA, r16(prob.Fb), KAPPA, prob.bc, BLOCK)
    prob.V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, NV, 71), DIMS, BLOCK)
    prob.V16 = r16(prob.V)
    prob.nX = amg.n_blocks(DIMS, BLOCK)
    prob.cd = amg.coarse_dims(DIMS, BLOCK)
    return prob


@pytest.fixture(scope='module')
def ainv16(prod):
    """The library's FP16 storage of (1 + F)^-1 - 1, as the oracle's blocks of A^-1."""
    return np.eye(6) + r16(amg.clover_inverse(prod.Fb) - np.eye(6))


@pytest.fixture(scope='module')
def dc16(prod):
    """The oracle's coarse operator (eq. (7)) from the FP16 vectors, links and clover."""
    return amg.coarse_operator(prod.op16, prod.V16)


def _install(prob, prec, coarse_iters=8):
    p = prob.ctx.setup_params(NV, prec, coarse_iters=coarse_iters, coarse_tol=0.0)
    prob.ctx.set_test_vectors(prob.T(prob.V), p)


def _force(prob, cache, kind, variant, keys):
    forced = {k: (variant if k.split('|')[1] == kind else v) for k, v in keys.items()}
    with open(cache, 'w') as f:
        json.dump(forced, f)
    prob.ctx.autotune(True, cache)


def test_fp16_storage_rounds_to_nearest_even(prod):
    """FP64 test vectors stored in FP16 equal NumPy's round-to-nearest-even
    conversion bit for bit (the rounding both sides assume)."""
    from paper_2111_05012_amd import PREC_MIXED
    _install(prod, PREC_MIXED)
    got = prod.zeros(prod.V.shape)
    prod.ctx.get_test_vectors(got)
    assert np.array_equal(prod.N(got), prod.V16)


@pytest.mark.parametrize('nrhs', [1, NRHS])
def test_dslash_mixed_every_variant(prod, nrhs, tmp_path):
    """Mixed D (FP16 links and clover, FP32 spinors and arithmetic) in every
    launch variant, including the LDS tiles of 4-slice t-slabs (the block is
    8 long in t) and 2 or 4 right-hand sides per thread."""
    from paper_2111_05012_amd import PREC_MIXED
    cache = str(tmp_path / 'tune.json')
    prod.ctx.autotune(True, cache)
    psi = syn.gaussian_vectors(DIMS, nrhs, 72)
    want = prod.op16.D(r32(psi))
    out = prod.zeros(psi.shape)
    prod.ctx.apply_D(prod.T(psi), out, nrhs, PREC_MIXED)  # tunes
    keys = json.load(open(cache))
    variants = [64, 128, 256, 512, -1, -2, -3] + ([-12, -14] if nrhs >= 4 else [])
    for v in variants:
        _force(prod, cache, 'dslash', v, keys)
        out = prod.zeros(psi.shape)
        prod.ctx.apply_D(prod.T(psi), out, nrhs, PREC_MIXED)
        assert rel(prod.N(out), want) < TOL_D, v
    prod.ctx.autotune(False, None)


def test_dslash_fp64_every_variant(prod, tmp_path):
    from paper_2111_05012_amd import PREC_FP64
    cache = str(tmp_path / 'tune.json')
    prod.ctx.autotune(True, cache)
    psi = syn.gaussian_vectors(DIMS, 2, 73)
    want = prod.op.D(psi)
    out = prod.zeros(psi.shape)
    prod.ctx.apply_D(prod.T(psi), out, 2, PREC_FP64)
    keys = json.load(open(cache))
    for v in (64, 128, 256, 512, -1, -2, -3, -12):
        _force(prod, cache, 'dslash', v, keys)
        out = prod.zeros(psi.shape)
        prod.ctx.apply_D(prod.T(psi), out, 2, PREC_FP64)
        assert rel(prod.N(out), want) < 1e-13, v
    prod.ctx.autotune(False, None)


def test_sap_mixed_12rhs(prod):
    """Mixed SAP(4, 6) on 12 right-hand sides in one call (the 512-site
    domain kernel with its loop over right-hand sides, and the crossing-hop
    correction kernel), against the oracle's SAP listing on the FP16 fields."""
    from paper_2111_05012_amd import PREC_MIXED
    b = syn.gaussian_vectors(DIMS, NRHS, 74)
    x = prod.zeros(b.shape)
    prod.ctx.sap(prod.T(b), x, NRHS, 4, 6, PREC_MIXED)
    xg = prod.N(x)
    for k in SAMPLE:
        want = amg.sap(prod.op16, r32(b[k:k + 1]), 4, 6)[0]
        assert rel(xg[k], want) < TOL_SAP, k


def test_sap_mixed_even_odd_12rhs(prod, ainv16):
    """The even-odd preconditioned block solve (the NEXT-2 smoother variant):
    SAP(4, 6) on 12 right-hand sides against the oracle's SAP with its
    even-odd block solve on the same FP16 hop matrices, clover and inverse
    clover."""
    from paper_2111_05012_amd import PREC_MIXED, BLOCK_EO_MR
    b = syn.gaussian_vectors(DIMS, NRHS, 81)
    x = prod.zeros(b.shape)
    prod.ctx.sap(prod.T(b), x, NRHS, 4, 6, PREC_MIXED, block_solve=BLOCK_EO_MR)
    xg = prod.N(x)
    for k in (0, NRHS - 1):
        want = amg.sap(prod.op16, r32(b[k:k + 1]), 4, 6,
                       block_solver=lambda r: amg.eo_mr_domains(prod.op16, r, 6, ainv16)[0])[0]
        assert rel(xg[k], want) < TOL_SAP, k


def test_sap_fp64_512_site_domains(prod):
    from paper_2111_05012_amd import PREC_FP64
    b = syn.gaussian_vectors(DIMS, 2, 75)
    x = prod.zeros(b.shape)
    prod.ctx.sap(prod.T(b), x, 2, 4, 6, PREC_FP64)
    xg = prod.N(x)
    want = amg.sap(prod.op, b[:1], 4, 6)[0]
    assert rel(xg[0], want) < 1e-11


def test_restrict_prolong_mixed_nv32_every_variant(prod, tmp_path):
    """Restriction and prolongation with N_v = 32 FP16 vectors on 12
    right-hand sides (the matrix-core kernels' full 64-row tiles) in every
    launch variant."""
    from paper_2111_05012_amd import PREC_MIXED
    cache = str(tmp_path / 'tune.json')
    prod.ctx.autotune(True, cache)
    _install(prod, PREC_MIXED)
    x = syn.gaussian_vectors(DIMS, NRHS, 76)
    yc = syn.gaussian_coarse(prod.nX, 2 * NV, NRHS, 77)
    want_r = amg.restrict(prod.V16, r32(x), DIMS, BLOCK)
    want_p = amg.prolong(prod.V16, r32(yc), DIMS, BLOCK)
    xc = prod.zeros(want_r.shape)
    y = prod.zeros(x.shape)
    prod.ctx.restrict(prod.T(x), xc, NRHS)
    prod.ctx.prolong(prod.T(yc), y, NRHS)
    keys = json.load(open(cache))
    for kind, variants in (('restrict', (4, 8, 16, 32, -32, -33)), ('prolong', (0, -32))):
        for v in variants:
            _force(prod, cache, kind, v, keys)
            if kind == 'restrict':
                xc = prod.zeros(want_r.shape)
                prod.ctx.restrict(prod.T(x), xc, NRHS)
                assert rel(prod.N(xc), want_r) < TOL_RP, (kind, v)
            else:
                y = prod.zeros(x.shape)
                prod.ctx.prolong(prod.T(yc), y, NRHS)
                assert rel(prod.N(y), want_p) < TOL_RP, (kind, v)
    prod.ctx.autotune(False, None)


def test_coarse_build_mixed_nv32_both_kernels(prod, dc16, tmp_path):
    """The coarse operator from FP16 vectors, links and clover with N_v = 32
    (both source chiralities per work unit on the matrix cores, and the
    vector-ALU contraction), against the oracle's eq. (7) on the same FP16
    data."""
    from paper_2111_05012_amd import PREC_MIXED
    cache = str(tmp_path / 'tune.json')
    prod.ctx.autotune(True, cache)
    _install(prod, PREC_MIXED)
    keys = json.load(open(cache))
    assert any(k.split('|')[1] == 'coarse_build' for k in keys)
    for v in (1, 0):
        _force(prod, cache, 'coarse_build', v, keys)
        _install(prod, PREC_MIXED)
        Dc = prod.zeros(dc16.shape)
        prod.ctx.get_coarse_op(Dc, level=1)
        assert rel(prod.N(Dc), dc16) < TOL_DC, v
    prod.ctx.autotune(False, None)


def test_coarse_op_roundtrip(prod, dc16):
    """set_coarse_op stores the complex64 rounding of the given operator."""
    from paper_2111_05012_amd import PREC_MIXED
    _install(prod, PREC_MIXED)
    prod.ctx.set_coarse_op(prod.T(dc16))
    got = prod.zeros(dc16.shape)
    prod.ctx.get_coarse_op(got, level=1)
    assert np.array_equal(prod.N(got), r32(dc16))


def test_apply_coarse_mixed_every_variant(prod, dc16, tmp_path):
    """The complex64 coarse stencil with 64 dof per coarse site on 12
    right-hand sides in every launch variant (right-hand sides per thread,
    the two matrix-core kernels), on the oracle's operator."""
    from paper_2111_05012_amd import PREC_MIXED
    cache = str(tmp_path / 'tune.json')
    prod.ctx.autotune(True, cache)
    _install(prod, PREC_MIXED)
    prod.ctx.set_coarse_op(prod.T(dc16))
    x = syn.gaussian_coarse(prod.nX, 2 * NV, NRHS, 78)
    want = amg.coarse_apply(r32(dc16), r32(x), prod.cd)
    y = prod.zeros(x.shape)
    prod.ctx.apply_coarse(prod.T(x), y, NRHS)
    keys = json.load(open(cache))
    for v in (1, 4, 8, 12, 16, -1, -2):
        _force(prod, cache, 'coarse_mv', v, keys)
        y = prod.zeros(x.shape)
        prod.ctx.apply_coarse(prod.T(x), y, NRHS)
        assert rel(prod.N(y), want) < TOL_CMV, v
    prod.ctx.autotune(False, None)


def test_coarse_solve_mixed_fixed_iterations(prod, dc16):
    """Eight iterations of the stabilised BiCGStab (Sec. 3 step (1b)) in FP32
    on the complex64 operator, 12 right-hand sides, against the oracle's
    BiCGStab in FP64 on the same operator and right-hand sides."""
    from paper_2111_05012_amd import PREC_MIXED
    _install(prod, PREC_MIXED)
    prod.ctx.set_coarse_op(prod.T(dc16))
    Dc = r32(dc16)
    b = syn.gaussian_coarse(prod.nX, 2 * NV, NRHS, 79)
    x = prod.zeros(b.shape)
    prod.ctx.coarse_solve(prod.T(b), x, NRHS, 8, 0.0)
    xg = prod.N(x)
    for k in range(NRHS):
        want, its = amg.bicgstab(lambda z: amg.coarse_apply(Dc, z, prod.cd), r32(b[k]), 8, 0.0)
        assert its == 8
        assert rel(xg[k], want) < TOL_CSOLVE, k


def test_vcycle_mixed_12rhs(prod, dc16):
    """The mixed V-cycle (restriction, 8 coarse iterations, prolongation, the
    FP32 residual with the mixed D, SAP(4, 6)) on 12 right-hand sides,
    against the oracle's V-cycle on the FP16 fields and vectors and the same
    complex64 coarse operator."""
    from paper_2111_05012_amd import PREC_MIXED
    _install(prod, PREC_MIXED, coarse_iters=8)
    prod.ctx.set_coarse_op(prod.T(dc16))
    mg = amg.TwoLevel(prod.op16, prod.V16, 4, 6, coarse_iters=8, coarse_tol=0.0)
    mg.Dc = r32(dc16)
    v = syn.gaussian_vectors(DIMS, NRHS, 80)
    out = prod.zeros(v.shape)
    prod.ctx.vcycle(prod.T(v), out, NRHS)
    og = prod.N(out)
    for k in SAMPLE:
        want = mg.vcycle(r32(v[k:k + 1]))[0]
        assert rel(og[k], want) < TOL_VCYCLE, k


def test_vcycle_mixed_12rhs_every_dslash_tile(prod, dc16, tmp_path):
    """The mixed V-cycle of test_vcycle_mixed_12rhs with its residual
    b - D x (the D with a source term) forced onto each LDS-tile variant of
    the mixed D."""
    from paper_2111_05012_amd import PREC_MIXED
    _install(prod, PREC_MIXED, coarse_iters=8)
    prod.ctx.set_coarse_op(prod.T(dc16))
    mg = amg.TwoLevel(prod.op16, prod.V16, 4, 6, coarse_iters=8, coarse_tol=0.0)
    mg.Dc = r32(dc16)
    v = syn.gaussian_vectors(DIMS, NRHS, 81)
    cache = str(tmp_path / 'tune.json')
    prod.ctx.autotune(True, cache)
    out = prod.zeros(v.shape)
    prod.ctx.vcycle(prod.T(v), out, NRHS)
    keys = json.load(open(cache))
    want = {k: mg.vcycle(r32(v[k:k + 1]))[0] for k in (0, NRHS - 1)}
    for var in (-2, -3):
        _force(prod, cache, 'dslash', var, keys)
        out = prod.zeros(v.shape)
        prod.ctx.vcycle(prod.T(v), out, NRHS)
        og = prod.N(out)
        for k, w in want.items():
            assert rel(og[k], w) < TOL_VCYCLE, (var, k)
    prod.ctx.autotune(False, None)


def test_vcycle_mixed_even_odd(prod, dc16, ainv16):
    """The mixed V-cycle with the even-odd preconditioned SAP block solve
    (setup parameter sap_eo) against the oracle's V-cycle with that block
    solve, on 12 right-hand sides (two checked)."""
    from paper_2111_05012_amd import PREC_MIXED
    p = prod.ctx.setup_params(NV, PREC_MIXED, coarse_iters=8, coarse_tol=0.0, sap_eo=1)
    prod.ctx.set_test_vectors(prod.T(prod.V), p)
    prod.ctx.set_coarse_op(prod.T(dc16))
    mg = amg.TwoLevel(prod.op16, prod.V16, 4, 6, coarse_iters=8, coarse_tol=0.0,
                      block_solver=lambda r: amg.eo_mr_domains(prod.op16, r, 6, ainv16)[0])
    mg.Dc = r32(dc16)
    v = syn.gaussian_vectors(DIMS, NRHS, 82)
    out = prod.zeros(v.shape)
    prod.ctx.vcycle(prod.T(v), out, NRHS)
    og = prod.N(out)
    for k in (0, NRHS - 1):
        want = mg.vcycle(r32(v[k:k + 1]))[0]
        assert rel(og[k], want) < TOL_VCYCLE, k
