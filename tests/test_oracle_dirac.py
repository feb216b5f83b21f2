"""Pins of the oracle's Wilson-clover operator (Sec. 2, eq. (1) and (2))
against facts that do not come from the oracle itself."""
import numpy as np
import pytest

import synthetic as syn
from oracle import dirac as od

BC_AP = (1, 1, 1, -1)


def _rand_psi(dims, n=1, seed=7):
    return syn.gaussian_vectors(dims, n, seed, syn.STREAM_PROBE)


def test_gamma_algebra():
    g = od.GAMMA
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * np.eye(4) * (m == n))
    # eq. (2): gamma_5 = -g1 g2 g3 g4 is diag(1,1,-1,-1) in the chiral basis
    assert np.allclose(od.GAMMA5, np.diag([1, 1, -1, -1]))
    for m in range(4):
        assert np.allclose(od.GAMMA5 @ g[m], -g[m] @ od.GAMMA5)


@pytest.mark.parametrize('dims,bc', [((4, 4, 4, 4), BC_AP), ((6, 4, 2, 8), (1, -1, 1, -1))])
def test_free_field_plane_wave(dims, bc):
    """U = 1: D e^{ipx} chi = [1 - 2k sum cos p + 2ik sum gamma sin p] chi e^{ipx}."""
    kappa = 0.13
    U = syn.unit_gauge(dims)
    Fb = od.clover_blocks(U, kappa, 1.0)
    rng = np.random.default_rng(3)
    moms = od.allowed_momenta(dims, bc)
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing='ij')
    for trial in range(4):
        p = np.array([moms[mu][rng.integers(dims[mu])] for mu in range(4)])
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        psi = ph[..., None, None] * chi
        out = od.apply_D(U, Fb, psi, kappa, bc)
        want = ph[..., None, None] * (od.free_symbol(p, kappa) @ chi)
        assert np.abs(out - want).max() < 1e-13


def test_free_field_dense_spectrum():
    """Eigenvalues of the dense free D on 4^4 equal, as a multiset, the
    eigenvalues of the momentum-space symbol (each times 3 colours):
    1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p)."""
    dims = (4, 4, 4, 4)
    kappa = 0.11
    U = syn.unit_gauge(dims)
    Fb = od.clover_blocks(U, kappa, 1.0)
    D = od.dense_D(U, Fb, kappa, BC_AP, dims)
    ev = np.linalg.eigvals(D)
    moms = od.allowed_momenta(dims, BC_AP)
    want = []
    for px in moms[0]:
        for py in moms[1]:
            for pz in moms[2]:
                for pt in moms[3]:
                    p = np.array([px, py, pz, pt])
                    a = 1 - 2 * kappa * np.cos(p).sum()
                    b = 2 * kappa * np.sqrt((np.sin(p) ** 2).sum())
                    want += [a + 1j * b] * 6 + [a - 1j * b] * 6
    key = lambda z: (round(z.real, 9), round(z.imag, 9))  # noqa: E731
    a = sorted(ev, key=key)
    b = sorted(want, key=key)
    assert np.abs(np.array(a) - np.array(b)).max() < 1e-10


def test_gamma5_hermiticity():
    """eq. (2): <phi, D psi> = <gamma5 D gamma5 phi, psi> for random U."""
    dims = (4, 4, 4, 8)
    U = syn.gauge_field(dims, 0.5, 1)
    kappa, csw = 0.124, 1.3
    Fb = od.clover_blocks(U, kappa, csw)
    phi, psi = _rand_psi(dims, 2)
    lhs = np.vdot(phi, od.apply_D(U, Fb, psi, kappa, BC_AP))
    rhs = np.vdot(od.gamma5(od.apply_D(U, Fb, od.gamma5(phi), kappa, BC_AP)), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def _gauge_transform(U, om):
    """U^Om_mu(x) = Om(x) U_mu(x) Om(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        out[mu] = om @ U[mu] @ od.dagger(od.shift(om, mu, +1))
    return out


def test_gauge_covariance():
    """D[U^Om](Om psi) = Om D[U] psi, and F[U^Om](x) = Om(x) F[U](x) Om(x)^dag."""
    dims = (4, 4, 2, 6)
    U = syn.gauge_field(dims, 0.6, 2)
    om = syn.random_su3(syn.shape_of(dims), 11)
    Ug = _gauge_transform(U, om)
    kappa, csw = 0.12, 1.1
    Fb = od.clover_blocks(U, kappa, csw)
    Fbg = od.clover_blocks(Ug, kappa, csw)
    psi = _rand_psi(dims)[0]
    rot = lambda f: np.einsum('...ab,...sb->...sa', om, f)  # noqa: E731
    lhs = od.apply_D(Ug, Fbg, rot(psi), kappa, BC_AP)
    rhs = rot(od.apply_D(U, Fb, psi, kappa, BC_AP))
    assert np.abs(lhs - rhs).max() < 1e-12
    Ff = od.clover_full(U, kappa, csw)
    Ffg = od.clover_full(Ug, kappa, csw)
    big = np.einsum('st,...ab->...satb', np.eye(4), om).reshape(om.shape[:-2] + (12, 12))
    assert np.abs(Ffg - big @ Ff @ od.dagger(big)).max() < 1e-12


@pytest.mark.parametrize('dims', [(2, 2, 2, 2), (4, 2, 2, 4), (4, 4, 4, 4)])
def test_dense_assembly_matches(dims):
    """The rolled implementation against an entry-by-entry dense assembly
    (extent-2 directions: both hops reach the same neighbour and are summed)."""
    U = syn.gauge_field(dims, 0.5, 3)
    kappa, csw = 0.124, 1.0
    Fb = od.clover_blocks(U, kappa, csw)
    D = od.dense_D(U, Fb, kappa, BC_AP, dims)
    psi = _rand_psi(dims, 1, 5)[0]
    out = od.apply_D(U, Fb, psi, kappa, BC_AP)
    assert np.abs(D @ psi.reshape(-1) - out.reshape(-1)).max() < 1e-12


def test_dsap_is_block_diagonal_part():
    dims = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = syn.gauge_field(dims, 0.5, 4)
    kappa = 0.124
    Fb = od.clover_blocks(U, kappa, 1.0)
    Ds = od.dense_D(U, Fb, kappa, BC_AP, dims, block=block)
    D = od.dense_D(U, Fb, kappa, BC_AP, dims)
    # block mask from coordinates, written independently
    V = 256
    bid = np.zeros(V, int)
    for n in range(V):
        x, y, z, t = n % 4, (n // 4) % 4, (n // 16) % 4, n // 64
        bid[n] = (x // 2) + 2 * ((y // 2) + 2 * ((z // 2) + 2 * (t // 2)))
    same = (bid[:, None] == bid[None, :])
    mask = np.kron(same, np.ones((12, 12)))
    assert np.abs(Ds - D * mask).max() == 0.0
    psi = _rand_psi(dims, 1, 6)[0]
    out = od.apply_Dsap(U, Fb, psi, kappa, BC_AP, block)
    assert np.abs(Ds @ psi.reshape(-1) - out.reshape(-1)).max() < 1e-12
    # a single domain covering the lattice: D_SAP = D
    out2 = od.apply_Dsap(U, Fb, psi, kappa, BC_AP, dims)
    assert np.abs(out2 - od.apply_D(U, Fb, psi, kappa, BC_AP)).max() < 1e-14


def test_clover_properties():
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, 0.5, 5)
    kappa, csw = 0.13, 1.1
    F = od.clover_full(U, kappa, csw)
    assert np.abs(F - od.dagger(F)).max() < 1e-14
    # [F, gamma5] = 0: the off-diagonal chiral blocks vanish
    assert np.abs(F[..., :6, 6:]).max() < 1e-14 and np.abs(F[..., 6:, :6]).max() < 1e-14
    assert np.abs(F).max() > 1e-2
    # F = 0 at U = 1
    assert np.abs(od.clover_full(syn.unit_gauge(dims), kappa, csw)).max() == 0.0


def test_clover_constant_abelian_field():
    """Closed form: U_y(x) = diag(e^{iBx}, e^{-iBx}, 1), other links 1, B = 2 pi / Lx.
    Every leaf in the (x, y) plane equals diag(e^{iB}, e^{-iB}, 1), the other
    planes are trivial, so F = -c_sw kappa sin(B) sigma_xy (x) diag(1, -1, 0)."""
    dims = (6, 4, 4, 4)
    U = syn.unit_gauge(dims)
    B = 2 * np.pi / dims[0]
    x = np.arange(dims[0])
    U[1, ..., 0, 0] = np.exp(1j * B * x)
    U[1, ..., 1, 1] = np.exp(-1j * B * x)
    kappa, csw = 0.125, 1.7
    F = od.clover_full(U, kappa, csw)
    want = -csw * kappa * np.sin(B) * np.kron(od.SIGMA[0, 1], np.diag([1.0, -1.0, 0.0]))
    assert np.abs(F - want).max() < 1e-14


def test_single_site_evaluation_matches_field_oracle():
    dims = (4, 6, 2, 4)
    U = syn.gauge_field(dims, 0.5, 8)
    kappa, csw = 0.13, 1.2
    Fb = od.clover_blocks(U, kappa, csw)
    psi = _rand_psi(dims, 1, 9)[0]
    full = od.apply_D(U, Fb, psi, kappa, BC_AP)
    Ff = od.clover_full(U, kappa, csw)
    rng = np.random.default_rng(1)
    for _ in range(12):
        c = tuple(int(rng.integers(L)) for L in dims)
        assert np.abs(od.clover_site(U, c, kappa, csw) - Ff[c[3], c[2], c[1], c[0]]).max() < 1e-14
        got = od.apply_D_site(U, psi, c, kappa, csw, BC_AP)
        assert np.abs(got - full[c[3], c[2], c[1], c[0]]).max() < 1e-13
