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


# ---------------------------------------------------------------------------
# The same sampler in torch, for lattices where the host version is too slow
# (it runs on whatever device the field is on).  Same scheme, update order and
# layout; its random stream is a torch generator seeded with seed * 1000003 + 7,
# so its fields are not bit-identical to the numpy version's.
# ---------------------------------------------------------------------------
def _t_shift(f, mu, s):
    import torch
    return torch.roll(f, shifts=-s, dims=3 - mu)


def _t_dag(a):
    return a.conj().transpose(-1, -2).contiguous()


def staple_sum_torch(U, mu):
    import torch
    A = torch.zeros_like(U[mu])
    for nu in range(4):
        if nu == mu:
            continue
        A += _t_shift(U[nu], mu, 1) @ _t_dag(_t_shift(U[mu], nu, 1)) @ _t_dag(U[nu])
        unm = _t_shift(U[nu], nu, -1)
        A += _t_dag(_t_shift(unm, mu, 1)) @ _t_dag(_t_shift(U[mu], nu, -1)) @ unm
    return A


def plaquette_torch(U):
    import torch
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = U[mu] @ _t_shift(U[nu], mu, 1) @ _t_dag(_t_shift(U[mu], nu, 1)) @ _t_dag(U[nu])
            s += float(torch.diagonal(P, dim1=-2, dim2=-1).sum(-1).real.mean()) / 3.0
    return s / 6.0


def kp_x0_torch(alpha, g):
    import torch
    out = torch.empty_like(alpha)
    todo = torch.ones(alpha.shape, dtype=torch.bool, device=alpha.device)
    while bool(todo.any()):
        idx = torch.nonzero(todo).flatten()
        a = alpha[idx]
        n = a.numel()
        r1, r2, r3, r4 = (1.0 - torch.rand(n, generator=g, dtype=torch.float64, device=alpha.device)
                          for _ in range(4))
        lam2 = -(torch.log(r1) + torch.cos(2.0 * torch.pi * r2) ** 2 * torch.log(r3)) / (2.0 * a)
        ok = r4 * r4 <= 1.0 - lam2
        out[idx[ok]] = 1.0 - 2.0 * lam2[ok]
        todo[idx[ok]] = False
    return out


def _t_su2_from(q0, q1, q2, q3):
    import torch
    m = torch.empty(q0.shape + (2, 2), dtype=torch.complex128, device=q0.device)
    m[..., 0, 0] = torch.complex(q0, q3)
    m[..., 0, 1] = torch.complex(q2, q1)
    m[..., 1, 0] = torch.complex(-q2, q1)
    m[..., 1, 1] = torch.complex(q0, -q3)
    return m


def su2_heatbath_torch(w, beta, g):
    import torch
    c0 = (w[..., 0, 0] + w[..., 1, 1]).real / 2
    c1 = (w[..., 0, 1] + w[..., 1, 0]).imag / 2
    c2 = (w[..., 0, 1] - w[..., 1, 0]).real / 2
    c3 = (w[..., 0, 0] - w[..., 1, 1]).imag / 2
    k = torch.sqrt(c0 * c0 + c1 * c1 + c2 * c2 + c3 * c3)
    kk = torch.clamp(k, min=1e-300)
    v = _t_su2_from(c0 / kk, c1 / kk, c2 / kk, c3 / kk)
    x0 = kp_x0_torch(torch.clamp(2.0 * beta * k / 3.0, min=1e-12), g)
    dev = k.device
    ct = 2.0 * torch.rand(k.shape, generator=g, dtype=torch.float64, device=dev) - 1.0
    ph = 2.0 * torch.pi * torch.rand(k.shape, generator=g, dtype=torch.float64, device=dev)
    rr = torch.sqrt(torch.clamp(1.0 - x0 * x0, min=0.0))
    st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
    x = _t_su2_from(x0, rr * st * torch.cos(ph), rr * st * torch.sin(ph), rr * ct)
    return x @ _t_dag(v)


def reunitarize_torch(U):
    import torch
    a = U[..., 0, :]
    a = a / torch.linalg.vector_norm(a, dim=-1, keepdim=True)
    b = U[..., 1, :]
    b = b - (a.conj() * b).sum(-1, keepdim=True) * a
    b = b / torch.linalg.vector_norm(b, dim=-1, keepdim=True)
    c = torch.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], dim=-1).conj()
    return torch.stack([a, b, c], dim=-2)


def heatbath_field_torch(dims, beta, sweeps, seed, device, record=None):
    """As heatbath_field, in torch on `device` (cold start)."""
    import torch
    lx, ly, lz, lt = dims
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + STREAM_HEATBATH)
    U = torch.zeros((4, lt, lz, ly, lx, 3, 3), dtype=torch.complex128, device=device)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    odd = torch.from_numpy(parity_mask(dims)).to(device)
    for n in range(sweeps):
        for mu in range(4):
            for par in (False, True):
                sel = odd == par
                A = staple_sum_torch(U, mu)[sel]
                Ul = U[mu][sel]
                for (i, j) in SUBGROUPS:
                    W = Ul @ A
                    w = W[:, [i, j]][:, :, [i, j]]
                    r = su2_heatbath_torch(w, beta, g)
                    Ul[:, [i, j], :] = r @ Ul[:, [i, j], :]
                U[mu][sel] = Ul
        U = reunitarize_torch(U)
        if record is not None:
            record(n, U)
    return U
