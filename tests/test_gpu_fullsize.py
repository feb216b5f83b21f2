"""GPU checks at the workloads' full sizes: sampled outputs against the
single-site oracle and properties that hold at any size (32^3x64), solves
checked by the oracle's operator (16^4) or by the parity-tested FP64
operator (32^3x64, 48^3x96)."""
import numpy as np
import pytest

import synthetic as syn
from oracle import dirac as od

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


def _ctx(w):
    from paper_2111_05012_amd import Context
    return Context(w['dims'], w['block'], BC, w['kappa'], w['csw'])


@pytest.fixture(scope='module')
def c3():
    import torch
    w = syn.CONFIGS['c3']
    dev = torch.device('cuda:0')
    U = syn.gauge_field_torch(w['dims'], w['eps'], w['seed'], dev)
    ctx = _ctx(w)
    ctx.load_gauge(U)
    yield w, ctx, U, dev
    ctx.close()
    del U
    torch.cuda.empty_cache()


def _samples(dims, n, seed):
    rng = np.random.default_rng(seed)
    pts = [tuple(int(rng.integers(L)) for L in dims) for _ in range(n)]
    # boundary sites of the lattice and of the blocks
    pts += [(0, 0, 0, 0), tuple(L - 1 for L in dims), (3, 4, 7, 63), (31, 0, 31, 0)]
    return pts


@pytest.mark.parametrize('prec,tol', [(0, 1e-12), (1, 2e-3)])
def test_dslash_c3_sampled_sites(c3, prec, tol):
    """32^3x64, 2 RHS: D psi at sampled sites (random, lattice and block
    boundaries) against the single-site oracle."""
    import torch
    w, ctx, U, dev = c3
    psi = syn.gaussian_vectors_torch(w['dims'], 2, 77, dev)
    out = torch.empty_like(psi)
    ctx.apply_D(psi, out, 2, prec)
    Un = U.cpu().numpy()
    pn = psi.cpu().numpy()
    on = out.cpu().numpy()
    scale = np.abs(on).max()
    for c in _samples(w['dims'], 24, 5):
        for r in range(2):
            want = od.apply_D_site(Un, pn[r], c, w['kappa'], w['csw'], BC)
            got = on[r, c[3], c[2], c[1], c[0]]
            assert np.abs(got - want).max() <= tol * scale


def test_dslash_c3_gamma5_hermiticity(c3):
    """eq. (2) at full size: <phi, D psi> = <g5 D g5 phi, psi>."""
    import torch
    w, ctx, U, dev = c3
    v = syn.gaussian_vectors_torch(w['dims'], 2, 78, dev)
    phi, psi = v[:1].contiguous(), v[1:].contiguous()
    g5 = torch.tensor([1, 1, -1, -1], dtype=torch.float64, device=dev).view(4, 1)
    Dpsi = torch.empty_like(psi)
    ctx.apply_D(psi, Dpsi, 1, 0)
    Dg5phi = torch.empty_like(phi)
    ctx.apply_D((phi * g5).contiguous(), Dg5phi, 1, 0)
    lhs = torch.vdot(phi.reshape(-1), Dpsi.reshape(-1))
    rhs = torch.vdot((Dg5phi * g5).reshape(-1), psi.reshape(-1))
    assert abs(complex(lhs - rhs)) <= 1e-12 * abs(complex(lhs))


def test_dslash_c3_free_field_plane_wave():
    """U = 1 at 32^3x64: a plane wave is an eigenvector with the closed-form
    momentum-space symbol (antiperiodic t)."""
    import torch
    w = syn.CONFIGS['c3']
    dims = w['dims']
    dev = torch.device('cuda:0')
    from paper_2111_05012_amd import Context
    ctx = Context(dims, w['block'], BC, w['kappa'], 0.0)
    U = torch.zeros((4,) + syn.shape_of(dims) + (3, 3), dtype=torch.complex128, device=dev)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    ctx.load_gauge(U)
    p = np.array([2 * np.pi * 3 / 32, 2 * np.pi * 5 / 32, 2 * np.pi * 1 / 32, 7 * np.pi / 64])
    rng = np.random.default_rng(2)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    t, z, y, x = torch.meshgrid(*[torch.arange(L, device=dev, dtype=torch.float64) for L in dims[::-1]],
                                indexing='ij')
    ph = torch.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = (ph[..., None, None] * torch.from_numpy(chi).to(dev))[None].contiguous()
    out = torch.empty_like(psi)
    ctx.apply_D(psi, out, 1, 0)
    want = ph[..., None, None] * torch.from_numpy(od.free_symbol(p, w['kappa']) @ chi).to(dev)
    assert float((out[0] - want).abs().max()) < 1e-12


def _residual(ctx, b, x):
    import torch
    r = torch.empty_like(b)
    ctx.apply_D(x, r, b.shape[0], 0)
    r = b - r
    return (r.reshape(b.shape[0], -1).norm(dim=1) / b.reshape(b.shape[0], -1).norm(dim=1)).cpu().numpy()


@pytest.mark.parametrize('prec', [0, 1])
def test_solve_c2(prec):
    """16^4 (eps 0.35, kappa 0.1355, blocks 4^4, N_v 16), one Z2 source, FP64
    and mixed: residual recomputed by the oracle's D."""
    import torch
    w = syn.CONFIGS['c2']
    dev = torch.device('cuda:0')
    U = syn.gauge_field(w['dims'], w['eps'], w['seed'])
    ctx = _ctx(w)
    ctx.load_gauge(torch.from_numpy(U).to(dev))
    V0 = syn.gaussian_vectors(w['dims'], w['nv'], w['seed'])
    ctx.setup(ctx.setup_params(w['nv'], prec, init_vectors=torch.from_numpy(V0).to(dev)))
    b = syn.z2_source(w['dims'], w['seed'])
    x = torch.zeros(b.shape, dtype=torch.complex128, device=dev)
    rc, info = ctx.solve(torch.from_numpy(b).to(dev), x, 1, tol=1e-10)
    assert rc == 0
    Fb = od.clover_blocks(U, w['kappa'], w['csw'])
    r = b - od.apply_D(U, Fb, x.cpu().numpy(), w['kappa'], BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_solve_c3_12rhs_mixed(c3):
    """32^3x64, 12 point sources, mixed precision, graph-captured V-cycle:
    every RHS to 1e-10 by the FP64 operator, and sampled residual sites by
    the single-site oracle."""
    import torch
    w, ctx, U, dev = c3
    ctx.setup(ctx.setup_params(w['nv'], 1, seed=3, coarse_iters=30))
    b = torch.from_numpy(syn.point_sources(w['dims'], 12)).to(dev)
    x = torch.zeros_like(b)
    rc, info = ctx.solve(b, x, 12, tol=1e-10, use_graph=1)
    assert rc == 0
    assert _residual(ctx, b, x).max() <= 1e-10
    Un, xn, bn = U.cpu().numpy(), x.cpu().numpy(), b.cpu().numpy()
    for c in _samples(w['dims'], 6, 9)[:8]:
        for r in (0, 7):
            res = bn[r, c[3], c[2], c[1], c[0]] - od.apply_D_site(Un, xn[r], c, w['kappa'], w['csw'], BC)
            assert np.abs(res).max() <= 1e-9 * np.abs(xn[r]).max()
