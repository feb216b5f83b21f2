"""Pure-gauge SU(3) heat-bath: smooth, physically distributed gauge fields as
solver inputs.

Input generation only (no Dirac operator, no multigrid arithmetic).  It samples
the Wilson plaquette action S = beta sum_P (1 - Re tr U_P / 3) with the
Cabibbo-Marinari scheme (Phys. Lett. B 119 (1982) 387): each link is updated
in the three SU(2) subgroups of SU(3) in turn, each subgroup element drawn
from its exact conditional distribution with the Kennedy-Pendleton method
(Phys. Lett. B 156 (1985) 393).  Links of one direction and one site parity
are independent given the rest and are updated together.

Layout as in the rest of the package: U[mu][t][z][y][x][3][3], U_mu(x)
linking x to x + mu, periodic in every direction (boundary phases of the
fermions are not part of the gauge field).  The stream is
numpy.random.default_rng([seed, 7]).
"""
import numpy as np

STREAM_HEATBATH = 7
SUBGROUPS = ((0, 1), (0, 2), (1, 2))


def _shift(f, mu, s):
    """f(x + s mu) for a field shaped [t][z][y][x]..."""
    return np.roll(f, -s, axis=3 - mu)


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def staple_sum(U, mu):
    """A_mu(x) = sum over nu != mu of the two staples closing U_mu(x) into a
    plaquette, so that Re tr(U_mu(x) A_mu(x)) is the sum of Re tr U_P over
    the six plaquettes containing the link."""
    A = np.zeros_like(U[mu])
    for nu in range(4):
        if nu == mu:
            continue
        # U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        A += _shift(U[nu], mu, 1) @ _dag(_shift(U[mu], nu, 1)) @ _dag(U[nu])
        # U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        unm = _shift(U[nu], nu, -1)
        A += _dag(_shift(unm, mu, 1)) @ _dag(_shift(U[mu], nu, -1)) @ unm
    return A


def plaquette(U):
    """Average of Re tr U_P / 3 over all sites and the six planes."""
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = U[mu] @ _shift(U[nu], mu, 1) @ _dag(_shift(U[mu], nu, 1)) @ _dag(U[nu])
            s += np.trace(P, axis1=-2, axis2=-1).real.mean() / 3.0
    return s / 6.0


def kp_x0(alpha, g):
    """Draws x0 in [-1, 1] with density proportional to sqrt(1 - x0^2)
    exp(alpha x0), one per entry of alpha (> 0), by Kennedy-Pendleton:
    x0 = 1 - 2 lam^2 with lam^2 ~ Gamma(3/2, scale 1/(2 alpha)) built from one
    exponential and one squared normal deviate, accepted with probability
    sqrt(1 - lam^2)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    out = np.empty(alpha.shape)
    todo = np.ones(alpha.shape, bool)
    while todo.any():
        a = alpha[todo]
        n = a.size
        r1, r2, r3, r4 = (1.0 - g.random(n) for _ in range(4))  # (0, 1]
        lam2 = -(np.log(r1) + np.cos(2.0 * np.pi * r2) ** 2 * np.log(r3)) / (2.0 * a)
        ok = r4 * r4 <= 1.0 - lam2
        idx = np.flatnonzero(todo)
        out[idx[ok]] = 1.0 - 2.0 * lam2[ok]
        todo[idx[ok]] = False
    return out


def _su2_from(q):
    """2x2 matrices q0 + i q.sigma from quaternion components [..., 4]."""
    q0, q1, q2, q3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    m = np.empty(q.shape[:-1] + (2, 2), np.complex128)
    m[..., 0, 0] = q0 + 1j * q3
    m[..., 0, 1] = q2 + 1j * q1
    m[..., 1, 0] = -q2 + 1j * q1
    m[..., 1, 1] = q0 - 1j * q3
    return m


def su2_heatbath(w, beta, g):
    """For 2x2 blocks w (the subgroup block of U A), draws r in SU(2) with
    density proportional to exp((beta / 3) Re tr(r w)) under the Haar measure.
    Re tr(r w) only sees the quaternion part k v of w (v in SU(2), k >= 0):
    with x = r v it is 2 k x0, so x0 comes from the Kennedy-Pendleton draw
    with alpha = 2 beta k / 3, x's direction is uniform, and r = x v^+."""
    c = np.stack([(w[..., 0, 0] + w[..., 1, 1]).real / 2,
                  (w[..., 0, 1] + w[..., 1, 0]).imag / 2,
                  (w[..., 0, 1] - w[..., 1, 0]).real / 2,
                  (w[..., 0, 0] - w[..., 1, 1]).imag / 2], axis=-1)
    k = np.sqrt((c * c).sum(-1))
    kk = np.maximum(k, 1e-300)
    v = _su2_from(c / kk[..., None])
    x0 = kp_x0(np.maximum(2.0 * beta * k / 3.0, 1e-12), g)
    ct = 2.0 * g.random(k.shape) - 1.0
    ph = 2.0 * np.pi * g.random(k.shape)
    rr = np.sqrt(np.maximum(1.0 - x0 * x0, 0.0))
    st = np.sqrt(np.maximum(1.0 - ct * ct, 0.0))
    x = _su2_from(np.stack([x0, rr * st * np.cos(ph), rr * st * np.sin(ph), rr * ct], axis=-1))
    return x @ _dag(v)


def reunitarize(U):
    """Projects each 3x3 matrix back onto SU(3): Gram-Schmidt of rows 0 and 1,
    row 2 = conj(row 0 x row 1)."""
    a = U[..., 0, :]
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = U[..., 1, :]
    b = b - (np.conj(a) * b).sum(-1, keepdims=True) * a
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    c = np.conj(np.cross(a, b))
    return np.stack([a, b, c], axis=-2)


def parity_mask(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing='ij')
    return ((x + y + z + t) & 1).astype(bool)


def sweep(U, beta, g, odd=None):
    """One heat-bath sweep in place: for each direction and site parity, the
    three subgroup updates of every link of that class."""
    if odd is None:
        odd = parity_mask(U.shape[1:5][::-1])
    for mu in range(4):
        for par in (False, True):
            sel = odd == par
            A = staple_sum(U, mu)[sel]
            Ul = U[mu][sel]
            for (i, j) in SUBGROUPS:
                W = Ul @ A
                w = W[:, [i, j]][:, :, [i, j]]
                r = su2_heatbath(w, beta, g)
                Ul[:, [i, j], :] = r @ Ul[:, [i, j], :]
            U[mu][sel] = Ul
    U[:] = reunitarize(U)
    return U


def heatbath_field(dims, beta, sweeps, seed, start=None, record=None):
    """Gauge field after `sweeps` heat-bath sweeps at coupling beta from a
    cold start (all links 1) or from `start`; record(sweep, U) is called
    after every sweep when given."""
    g = np.random.default_rng([int(seed), STREAM_HEATBATH])
    lx, ly, lz, lt = dims
    if start is None:
        U = np.zeros((4, lt, lz, ly, lx, 3, 3), np.complex128)
        U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    else:
        U = np.array(start, dtype=np.complex128)
    odd = parity_mask(dims)
    for n in range(sweeps):
        sweep(U, beta, g, odd)
        if record is not None:
            record(n, U)
    return U
