"""Oracle: the Wilson-clover operator of Sec. 2, eq. (1), in plain NumPy FP64.

Layout (shared with the library's external ABI): a spinor field is
[..., Lt, Lz, Ly, Lx, 4 spin, 3 colour]; a gauge field is
[4 mu, Lt, Lz, Ly, Lx, 3, 3] with U_mu(x) the link x -> x+mu; the clover field
is [Lt, Lz, Ly, Lx, 2 chirality, 6, 6] (the two diagonal 6x6 blocks of the
12x12 matrix F(x) in the chiral basis, index spin_local*3 + colour).

Readings where the paper is silent (Sec. 2):
  * gamma matrices: chiral basis gamma_k = [[0, -i s_k], [i s_k, 0]] (k=1,2,3),
    gamma_4 = [[0, -1], [-1, 0]]; then gamma_5 = -g1 g2 g3 g4 = diag(1,1,-1,-1),
    matching the definition next to eq. (2);
  * F(x) (only described as a Hermitian 12x12 matrix built from links):
    F = i c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}, with
    sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], Fhat = (Q - Q^dag)/8 and Q the
    sum of the four plaquette leaves at x in the (mu, nu) plane;
  * boundary conditions ("periodic or anti-periodic"): a hop that crosses the
    lattice boundary in direction mu is multiplied by bc[mu] (+1 or -1); the
    stored links are never modified.

Pins (tests/test_oracle_dirac.py): free-field closed form (plane waves and the
dense spectrum), gamma_5-hermiticity (eq. 2), gauge covariance, an
independently written dense assembly by loops over sites, the clover's
Hermiticity / chirality / vanishing at U = 1 and a closed form for a constant
abelian field (which fixes the leaf orientation and the 1/8 and c_sw kappa
factors of the reading above; the reading itself is not fixed by the paper).
"""
import numpy as np

# ----------------------------------------------------------------------------
# Spin algebra (Sec. 2, eq. (2))
# ----------------------------------------------------------------------------
_S1 = np.array([[0, 1], [1, 0]], np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], np.complex128)
_S3 = np.array([[1, 0], [0, -1]], np.complex128)
_Z2 = np.zeros((2, 2), np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def _chiral(a):
    return np.block([[_Z2, -1j * a], [1j * a, _Z2]])


GAMMA = np.array([_chiral(_S1), _chiral(_S2), _chiral(_S3),
                  np.block([[_Z2, -_I2], [-_I2, _Z2]])])
GAMMA5 = -GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)
SIGMA = np.array([[0.5j * (GAMMA[m] @ GAMMA[n] - GAMMA[n] @ GAMMA[m]) for n in range(4)]
                  for m in range(4)])


def site_axis(mu):
    """Array axis of direction mu for arrays with two trailing internal axes."""
    return -3 - mu


def dims_of(field):
    """(Lx, Ly, Lz, Lt) of a field [..., Lt, Lz, Ly, Lx, a, b]."""
    lt, lz, ly, lx = field.shape[-6:-2]
    return (lx, ly, lz, lt)


def shift(f, mu, sign, bc=None):
    """g(x) = f(x + sign*mu) on the periodic lattice; with bc given, values
    that wrapped around the boundary are multiplied by bc[mu]."""
    ax = site_axis(mu)
    g = np.roll(f, -sign, axis=ax)
    if bc is not None and bc[mu] != 1:
        L = f.shape[ax]
        idx = [slice(None)] * f.ndim
        idx[ax] = L - 1 if sign > 0 else 0
        g[tuple(idx)] *= bc[mu]
    return g


def dagger(u):
    return np.conj(np.swapaxes(u, -1, -2))


# ----------------------------------------------------------------------------
# Clover term F(x) (Sec. 2, after eq. (1); reading in the module docstring)
# ----------------------------------------------------------------------------
def plaquette_leaves(U, mu, nu):
    """Q_{mu nu}(x): the four plaquettes in the (mu, nu) plane that touch x,
    each traversed mu-then-nu (counter-clockwise), starting and ending at x."""
    um, un = U[mu], U[nu]
    sh = lambda f, d, s: shift(f, d, s)  # noqa: E731  f(x + s d)
    l1 = um @ sh(un, mu, 1) @ dagger(sh(um, nu, 1)) @ dagger(un)
    um_m = sh(um, mu, -1)
    un_m = sh(un, mu, -1)
    l2 = un @ dagger(sh(um_m, nu, 1)) @ dagger(un_m) @ um_m
    um_mn = sh(um_m, nu, -1)
    un_mn = sh(un_m, nu, -1)
    un_n = sh(un, nu, -1)
    l3 = dagger(um_m) @ dagger(un_mn) @ um_mn @ un_n
    um_n = sh(um, nu, -1)
    l4 = dagger(un_n) @ um_n @ sh(un_n, mu, 1) @ dagger(um)
    return l1 + l2 + l3 + l4


def clover_full(U, kappa, csw):
    """F(x) as a full 12x12 matrix per site, index spin*3 + colour."""
    shp = U.shape[1:-2]
    F = np.zeros(shp + (12, 12), np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            q = plaquette_leaves(U, mu, nu)
            fhat = (q - dagger(q)) / 8.0
            F += 1j * csw * kappa * np.einsum('ab,...cd->...acbd', SIGMA[mu, nu], fhat).reshape(shp + (12, 12))
    return F


def clover_blocks(U, kappa, csw):
    """F(x) as its two chiral 6x6 diagonal blocks, [Lt,Lz,Ly,Lx,2,6,6]."""
    F = clover_full(U, kappa, csw)
    return np.stack([F[..., :6, :6], F[..., 6:, 6:]], axis=-3)


def clover_apply(Fb, psi):
    """F(x) psi(x) for the chiral-block clover field."""
    p = psi.reshape(psi.shape[:-2] + (2, 6))
    out = np.einsum('...kab,...kb->...ka', Fb, p)
    return out.reshape(psi.shape)


# ----------------------------------------------------------------------------
# The operator D of eq. (1) and its pieces
# ----------------------------------------------------------------------------
def hop(U, psi, mu, sign, kappa, bc):
    """One hopping term of eq. (1):
    sign=+1: -kappa (1 - gamma_mu) U_mu(x) psi(x+mu)
    sign=-1: -kappa (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)."""
    if sign > 0:
        nb = shift(psi, mu, +1, bc)
        t = np.einsum('...ab,...sb->...sa', U[mu], nb)
        proj = ONE4 - GAMMA[mu]
    else:
        nb = shift(psi, mu, -1, bc)
        ub = shift(U[mu], mu, -1)
        t = np.einsum('...ba,...sb->...sa', np.conj(ub), nb)
        proj = ONE4 + GAMMA[mu]
    return -kappa * np.einsum('st,...tc->...sc', proj, t)


def apply_D(U, Fb, psi, kappa, bc):
    """out = D psi, eq. (1): (1 + F(x)) psi(x) - kappa sum_mu [...]."""
    out = psi + clover_apply(Fb, psi)
    for mu in range(4):
        out += hop(U, psi, mu, +1, kappa, bc)
        out += hop(U, psi, mu, -1, kappa, bc)
    return out


def crossing_mask(dims, block, mu, sign):
    """1 on sites whose hop in direction sign*mu leaves the site's domain
    (Sec. 3, SAP paragraph: domains of block extent), 0 elsewhere.  A
    direction with a single domain never crosses.  Shaped to broadcast over
    [..., Lt, Lz, Ly, Lx, 4, 3]."""
    L, b = dims[mu], block[mu]
    c = np.arange(L)
    if L == b:
        m = np.zeros(L)
    elif sign > 0:
        m = (c % b == b - 1).astype(float)
    else:
        m = (c % b == 0).astype(float)
    shp = [1, 1, 1, 1, 1, 1]
    shp[3 - mu] = L
    return m.reshape(shp)


def apply_Dsap(U, Fb, psi, kappa, bc, block):
    """D_SAP: eq. (1) with every hop between distinct domains turned off
    (Sec. 3, SAP paragraph)."""
    dims = dims_of(psi)
    out = psi + clover_apply(Fb, psi)
    for mu in range(4):
        for s in (+1, -1):
            out += (1.0 - crossing_mask(dims, block, mu, s)) * hop(U, psi, mu, s, kappa, bc)
    return out


def apply_hop_cross(U, psi, mu, sign, kappa, bc, block):
    """The part of D that hops from a site, in direction sign*mu, into the
    neighbouring domain (used for the off-diagonal coarse blocks, eq. (7))."""
    dims = dims_of(psi)
    return crossing_mask(dims, block, mu, sign) * hop(U, psi, mu, sign, kappa, bc)


def gamma5(psi):
    return np.einsum('st,...tc->...sc', GAMMA5, psi)


def chiral_project(psi, s):
    """P_s psi with P_{+/-} = (1 +/- gamma_5)/2 (Sec. 3 footnote); s=0 is +."""
    out = np.zeros_like(psi)
    sp = slice(0, 2) if s == 0 else slice(2, 4)
    out[..., sp, :] = psi[..., sp, :]
    return out


# ----------------------------------------------------------------------------
# Dense matrices for brute-force checks (small lattices only)
# ----------------------------------------------------------------------------
def site_index(c, dims):
    x, y, z, t = c
    lx, ly, lz, _ = dims
    return x + lx * (y + ly * (z + lz * t))


def dense_D(U, Fb, kappa, bc, dims, block=None):
    """eq. (1) assembled entry block by entry block with explicit coordinate
    arithmetic (independent of the np.roll implementation above).  With block
    given, hops between distinct domains are left out (D_SAP).  Hops that land
    on the same neighbour (extent 2) are summed, never merged."""
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    D = np.zeros((12 * V, 12 * V), np.complex128)
    Uf = U.reshape(4, V, 3, 3)
    Ff = Fb.reshape(V, 2, 6, 6)
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = [x, y, z, t]
                    n = site_index(c, dims)
                    blk = np.eye(12, dtype=np.complex128)
                    blk[:6, :6] += Ff[n, 0]
                    blk[6:, 6:] += Ff[n, 1]
                    D[12 * n:12 * n + 12, 12 * n:12 * n + 12] += blk
                    for mu in range(4):
                        L = dims[mu]
                        # forward neighbour
                        cf = list(c)
                        cf[mu] = (c[mu] + 1) % L
                        sg = bc[mu] if c[mu] == L - 1 else 1.0
                        if block is None or (cf[mu] // block[mu]) == (c[mu] // block[mu]):
                            m = site_index(cf, dims)
                            D[12 * n:12 * n + 12, 12 * m:12 * m + 12] += \
                                -kappa * sg * np.kron(ONE4 - GAMMA[mu], Uf[mu, n])
                        # backward neighbour
                        cb = list(c)
                        cb[mu] = (c[mu] - 1) % L
                        sg = bc[mu] if c[mu] == 0 else 1.0
                        if block is None or (cb[mu] // block[mu]) == (c[mu] // block[mu]):
                            m = site_index(cb, dims)
                            D[12 * n:12 * n + 12, 12 * m:12 * m + 12] += \
                                -kappa * sg * np.kron(ONE4 + GAMMA[mu], np.conj(Uf[mu, m]).T)
    return D


def free_symbol(p, kappa):
    """Momentum-space D at U = 1, F = 0: 1 - 2 kappa sum cos p + 2 i kappa sum gamma sin p
    (a 4x4 spin matrix; eq. (1) acting on a plane wave e^{i p.x})."""
    m = (1.0 - 2.0 * kappa * np.sum(np.cos(p))) * ONE4
    for mu in range(4):
        m = m + 2j * kappa * np.sin(p[mu]) * GAMMA[mu]
    return m


def allowed_momenta(dims, bc):
    """Momenta compatible with the boundary conditions: p = 2 pi n / L
    (periodic) or (2 n + 1) pi / L (antiperiodic)."""
    out = []
    for mu in range(4):
        L = dims[mu]
        n = np.arange(L)
        out.append(2 * np.pi * n / L if bc[mu] == 1 else (2 * n + 1) * np.pi / L)
    return out


# ----------------------------------------------------------------------------
# Single-site evaluation (for sampled checks on lattices too large for the
# whole-field oracle): eq. (1) and the clover term at one site, by explicit
# coordinate arithmetic on the canonical arrays.
# ----------------------------------------------------------------------------
def _at(field, c):
    """field[..., t, z, y, x, a, b] at coordinates c = (x, y, z, t)."""
    return field[..., c[3], c[2], c[1], c[0], :, :]


def _step(c, dims, mu, s):
    cc = list(c)
    cc[mu] = (c[mu] + s) % dims[mu]
    return tuple(cc)


def clover_site(U, c, kappa, csw):
    """F(x) at coordinates c as a 12x12 matrix (same reading as clover_full)."""
    dims = (U.shape[4], U.shape[3], U.shape[2], U.shape[1])
    F = np.zeros((12, 12), np.complex128)
    lk = lambda mu, x: _at(U[mu], x)  # noqa: E731
    for mu in range(4):
        for nu in range(mu + 1, 4):
            xm = _step(c, dims, mu, -1)
            xn = _step(c, dims, nu, -1)
            xmn = _step(xm, dims, nu, -1)
            q = (lk(mu, c) @ lk(nu, _step(c, dims, mu, 1)) @ dagger(lk(mu, _step(c, dims, nu, 1))) @ dagger(lk(nu, c))
                 + lk(nu, c) @ dagger(lk(mu, _step(xm, dims, nu, 1))) @ dagger(lk(nu, xm)) @ lk(mu, xm)
                 + dagger(lk(mu, xm)) @ dagger(lk(nu, xmn)) @ lk(mu, xmn) @ lk(nu, xn)
                 + dagger(lk(nu, xn)) @ lk(mu, xn) @ lk(nu, _step(xn, dims, mu, 1)) @ dagger(lk(mu, c)))
            fh = (q - dagger(q)) / 8.0
            F += 1j * csw * kappa * np.kron(SIGMA[mu, nu], fh)
    return F


def apply_D_site(U, psi, c, kappa, csw, bc):
    """(D psi)(x) at coordinates c, eq. (1); psi [Lt,Lz,Ly,Lx,4,3]."""
    dims = (U.shape[4], U.shape[3], U.shape[2], U.shape[1])
    p0 = _at(psi, c).reshape(12)
    out = p0 + clover_site(U, c, kappa, csw) @ p0
    for mu in range(4):
        xf = _step(c, dims, mu, 1)
        sf = bc[mu] if c[mu] == dims[mu] - 1 else 1.0
        out -= kappa * sf * np.kron(ONE4 - GAMMA[mu], _at(U[mu], c)) @ _at(psi, xf).reshape(12)
        xb = _step(c, dims, mu, -1)
        sb = bc[mu] if c[mu] == 0 else 1.0
        out -= kappa * sb * np.kron(ONE4 + GAMMA[mu], dagger(_at(U[mu], xb))) @ _at(psi, xb).reshape(12)
    return out.reshape(4, 3)
