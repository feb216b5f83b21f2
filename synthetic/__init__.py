"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds input generation only: gauge links, sources, random start
vectors and random gauge transformations.  It contains none of the solver's
arithmetic (no Dirac operator, no clover term, no multigrid step), so that the
CPU oracle and the HIP path never share code.

Conventions (also the library's external layout):
  * lattice dims are given as (Lx, Ly, Lz, Lt); arrays are shaped
    (Lt, Lz, Ly, Lx, ...) so that the flat site index is x + Lx*(y + Ly*(z + Lz*t));
  * a spinor field is complex128 [nrhs][Lt][Lz][Ly][Lx][4 spin][3 colour];
  * a gauge field is complex128 [4 mu=x,y,z,t][Lt][Lz][Ly][Lx][3][3], U_mu(x)
    linking x to x+mu, row-major.

Random streams: numpy.random.default_rng([seed, stream]) with stream
0 = gauge links, 1 = sources, 2 = setup start vectors, 3 = network init,
4 = per-seed eps draws, 5 = gauge transformations, 6 = test probes.
"""
import numpy as np

STREAM_GAUGE, STREAM_SOURCE, STREAM_SETUP, STREAM_NET, STREAM_EPS, STREAM_GT, STREAM_PROBE = range(7)


def rng(seed, stream):
    return np.random.default_rng([int(seed), int(stream)])


def shape_of(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


def volume(dims):
    return int(np.prod(dims))


def _herm_traceless(draws):
    """Traceless Hermitian 3x3 from 9 Gaussian draws per matrix:
    3 diagonal reals, then (re, im) of the upper entries (0,1), (0,2), (1,2)."""
    h = np.zeros(draws.shape[:-1] + (3, 3), np.complex128)
    for k in range(3):
        h[..., k, k] = draws[..., k]
    for n, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
        z = draws[..., 3 + 2 * n] + 1j * draws[..., 4 + 2 * n]
        h[..., a, b] = z
        h[..., b, a] = np.conj(z)
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    for k in range(3):
        h[..., k, k] -= tr
    return h


def _mm(a, b):
    """Product of two batches of 3x3 matrices stored component-major [3][3][N]."""
    return np.array([[a[i, 0] * b[0, j] + a[i, 1] * b[1, j] + a[i, 2] * b[2, j] for j in range(3)]
                     for i in range(3)])


def _expi(h, eps, chunk=1 << 16):
    """exp(i eps H) for Hermitian 3x3 H by scaling and squaring: A = i eps H
    is scaled by 2^-k (one k for the whole batch, so every matrix sees the
    same operations) until its Frobenius norm is <= 1/2, exponentiated by its
    Taylor series to order 16 (truncation below 1e-19), and squared k times.
    Unitary to rounding; det 1 when H is traceless."""
    shp = h.shape
    hf = h.reshape(-1, 3, 3)
    nrm = eps * np.sqrt((np.abs(hf) ** 2).sum(axis=(1, 2))).max() if hf.size else 0.0
    k = max(0, int(np.ceil(np.log2(nrm / 0.5)))) if nrm > 0 else 0
    out = np.empty_like(hf, dtype=np.complex128)
    for c0 in range(0, hf.shape[0], chunk):
        b = np.moveaxis((1j * eps / 2.0 ** k) * hf[c0:c0 + chunk], 0, -1)  # [3][3][n]
        n = b.shape[-1]
        eye = np.zeros((3, 3, n), np.complex128)
        for i in range(3):
            eye[i, i] = 1.0
        e = eye.copy()
        for m in range(16, 0, -1):
            e = eye + _mm(b, e) / m
        for _ in range(k):
            e = _mm(e, e)
        out[c0:c0 + chunk] = np.moveaxis(e, -1, 0)
    return out.reshape(shp)


def gauge_field(dims, eps, seed):
    """U_mu(x) = exp(i eps H), H random traceless Hermitian with Gaussian
    (sigma = 1) entries.  Draw order [mu][t][z][y][x], 9 draws per link."""
    g = rng(seed, STREAM_GAUGE)
    draws = g.standard_normal((4,) + shape_of(dims) + (9,))
    return _expi(_herm_traceless(draws), eps)


def unit_gauge(dims):
    u = np.zeros((4,) + shape_of(dims) + (3, 3), np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3(shape, seed, stream=STREAM_GT, eps=1.0):
    g = rng(seed, stream)
    draws = g.standard_normal(tuple(shape) + (9,))
    return _expi(_herm_traceless(draws), eps)


def z2_source(dims, seed, nrhs=1):
    """Each of the 12 V components real +-1 with probability 1/2 (imag 0)."""
    g = rng(seed, STREAM_SOURCE)
    bits = g.integers(0, 2, size=(nrhs,) + shape_of(dims) + (4, 3))
    return (1.0 - 2.0 * bits).astype(np.complex128)


def point_sources(dims, nrhs=12):
    """RHS k = 3*spin + colour: unit vector at the origin, spin and colour of k."""
    b = np.zeros((nrhs,) + shape_of(dims) + (4, 3), np.complex128)
    for k in range(nrhs):
        b[k, 0, 0, 0, 0, (k // 3) % 4, k % 3] = 1.0
    return b


def gaussian_vectors(dims, n, seed, stream=STREAM_SETUP):
    """n complex Gaussian fields (re, im each N(0,1))."""
    g = rng(seed, stream)
    d = g.standard_normal((n,) + shape_of(dims) + (4, 3, 2))
    return d[..., 0] + 1j * d[..., 1]


def gaussian_coarse(n_sites, dof, n, seed, stream=STREAM_PROBE):
    g = rng(seed, stream)
    d = g.standard_normal((n, n_sites, dof, 2))
    return d[..., 0] + 1j * d[..., 1]


def gaussian_clover(dims, seed, stream=STREAM_PROBE):
    """A random field of two Hermitian 6x6 blocks per site, [V][2][6][6]."""
    g = rng(seed, stream)
    d = g.standard_normal((volume(dims), 2, 6, 6, 2))
    a = d[..., 0] + 1j * d[..., 1]
    return 0.05 * (a + np.conj(np.swapaxes(a, -1, -2)))


def net_weights(C, L, seed, scale=None):
    """Start weights of the equivariant network, [L][9, C, C, 4, 4] complex:
    small Gaussian entries (re, im each N(0, scale^2)) plus, on the identity
    path d = 0, a spin-diagonal N(0, 1/C) channel mixing (stream 3)."""
    g = rng(seed, STREAM_NET)
    s = scale if scale is not None else 0.1 / np.sqrt(9 * C * 4)
    Ws = []
    for _ in range(L):
        W = s * (g.standard_normal((9, C, C, 4, 4)) + 1j * g.standard_normal((9, C, C, 4, 4)))
        W[0] += np.eye(4)[None, None] * (g.standard_normal((C, C))[..., None, None] / np.sqrt(C))
        Ws.append(W)
    return Ws


# Workload recipes (lattice, generator parameters, hierarchy) used by tests and bench.
CONFIGS = {
    'c1': dict(dims=(4, 4, 4, 4), eps=0.5, seed=1, kappa=0.124, csw=1.0, block=(2, 2, 2, 2),
               nv=8, nrhs=1, source='z2'),
    'c2': dict(dims=(16, 16, 16, 16), eps=0.35, seed=1, kappa=0.1355, csw=1.0, block=(4, 4, 4, 4),
               nv=16, nrhs=1, source='z2'),
    'c3': dict(dims=(32, 32, 32, 64), eps=0.3, seed=1, kappa=0.1365, csw=1.1, block=(4, 4, 4, 8),
               nv=32, nrhs=12, source='point'),
}


# ----------------------------------------------------------------------------
# Device-side generation for large lattices (same recipe, evaluated with torch
# on the GPU; agrees with the NumPy arrays above to rounding).  Used where a
# 32^3x64-sized input would take minutes on the host.
# ----------------------------------------------------------------------------
def gauge_field_torch(dims, eps, seed, device, chunk=1 << 22):
    """gauge_field() with the same Gaussian draws and the same scaling and
    squaring Taylor evaluation, carried out in complex128 on `device`."""
    import torch
    g = rng(seed, STREAM_GAUGE)
    draws = g.standard_normal((4,) + shape_of(dims) + (9,))
    h = _herm_traceless(draws).reshape(-1, 3, 3)
    del draws
    nrm = eps * np.sqrt((np.abs(h) ** 2).sum(axis=(1, 2))).max()
    k = max(0, int(np.ceil(np.log2(nrm / 0.5)))) if nrm > 0 else 0
    out = torch.empty((h.shape[0], 3, 3), dtype=torch.complex128, device=device)
    eye = torch.eye(3, dtype=torch.complex128, device=device)
    for c0 in range(0, h.shape[0], chunk):
        b = torch.from_numpy(h[c0:c0 + chunk]).to(device) * (1j * eps / 2.0 ** k)
        e = eye.expand_as(b).clone()
        for m in range(16, 0, -1):
            e = eye + torch.matmul(b, e) / m
        for _ in range(k):
            e = torch.matmul(e, e)
        out[c0:c0 + chunk] = e
    return out.reshape((4,) + shape_of(dims) + (3, 3))


def gaussian_vectors_torch(dims, n, seed, device):
    """n complex Gaussian fields drawn on the device from a seeded torch
    generator (deterministic for a given seed and device type)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 1000003 + STREAM_SETUP)
    shp = (n,) + shape_of(dims) + (4, 3)
    re = torch.randn(shp, generator=gen, dtype=torch.float64, device=device)
    im = torch.randn(shp, generator=gen, dtype=torch.float64, device=device)
    return torch.complex(re, im)
