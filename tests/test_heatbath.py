"""The heat-bath gauge generator (input generation for the smooth-field
workload), pinned to closed forms: the Kennedy-Pendleton draw against the
Bessel-function moments of its target density, the SU(2) subgroup update
against the same moment of Re tr(r w), the staple sum against the plaquette
it must reproduce, and the plaquette at strong coupling against the leading
terms of the strong-coupling expansion."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import iv

import synthetic as syn
from synthetic import heatbath as hb


@pytest.mark.parametrize('alpha', [0.5, 2.0, 8.0])
def test_kp_sampler_mean_matches_bessel_ratio(alpha):
    # density sqrt(1 - x^2) exp(alpha x) on [-1, 1] has mean I_2(alpha) / I_1(alpha)
    g = np.random.default_rng(11)
    x = hb.kp_x0(np.full(200000, alpha), g)
    assert x.min() >= -1 and x.max() <= 1
    err = x.std() / np.sqrt(x.size)
    assert abs(x.mean() - iv(2, alpha) / iv(1, alpha)) < 5 * err


def test_kp_sampler_distribution():
    alpha = 3.0
    g = np.random.default_rng(12)
    x = np.sort(hb.kp_x0(np.full(50000, alpha), g))
    f = lambda t: np.sqrt(1 - t * t) * np.exp(alpha * t)
    norm = integrate.quad(f, -1, 1)[0]
    grid = np.linspace(-1, 1, 201)
    cdf = np.array([integrate.quad(f, -1, t)[0] for t in grid]) / norm
    emp = np.searchsorted(x, grid, side='right') / x.size
    # Kolmogorov-Smirnov distance, 1.95 / sqrt(n) is the 0.1% level
    assert np.abs(emp - cdf).max() < 1.95 / np.sqrt(x.size)


def test_su2_update_moment_and_group():
    g = np.random.default_rng(13)
    beta = 4.0
    w = g.normal(size=(2, 2)) + 1j * g.normal(size=(2, 2))
    W = np.broadcast_to(w, (100000, 2, 2))
    r = hb.su2_heatbath(W, beta, g)
    assert np.abs(r @ np.conj(np.swapaxes(r, -1, -2)) - np.eye(2)).max() < 1e-13
    assert np.abs(np.linalg.det(r) - 1).max() < 1e-13
    # quaternion part of w: k = sqrt(sum c_b^2) with c_b = Re tr(e_b^+ w) / 2,
    # e = (1, i sigma_1, i sigma_2, i sigma_3), computed from the Pauli matrices
    sig = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    e = [sig[0]] + [1j * s for s in sig[1:]]
    k = np.sqrt(sum((np.trace(np.conj(b.T) @ w).real / 2) ** 2 for b in e))
    alpha = 2 * beta * k / 3
    val = np.trace(r @ w, axis1=-2, axis2=-1).real
    want = 2 * k * iv(2, alpha) / iv(1, alpha)
    assert abs(val.mean() - want) < 5 * val.std() / np.sqrt(val.size)


def test_staple_sum_reproduces_plaquettes():
    dims = (4, 4, 2, 6)
    U = syn.gauge_field(dims, 0.8, 3)
    tot = sum(np.trace(U[mu] @ hb.staple_sum(U, mu), axis1=-2, axis2=-1).real.sum() for mu in range(4))
    # every plaquette has four links: sum over links = 4 x sum over plaquettes
    assert tot == pytest.approx(4 * 3 * 6 * syn.volume(dims) * hb.plaquette(U), rel=1e-12)


def test_links_stay_su3():
    U = hb.heatbath_field((4, 4, 4, 4), 5.7, 3, 2)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-12


def test_strong_coupling_plaquette():
    # <Re tr U_P / 3> = beta / 18 + beta^2 / 216 + O(beta^3) for SU(3)
    beta = 0.5
    ps = []
    hb.heatbath_field((4, 4, 4, 4), beta, 60, 5, record=lambda n, U: ps.append(hb.plaquette(U)))
    p = np.mean(ps[10:])
    assert abs(p - (beta / 18 + beta ** 2 / 216)) < 0.003


# ---------------------------------------------------------------- the torch version (run here on the CPU)
def test_torch_kp_sampler_mean():
    import torch
    g = torch.Generator()
    g.manual_seed(21)
    alpha = 2.0
    x = hb.kp_x0_torch(torch.full((400000,), alpha, dtype=torch.float64), g)
    err = float(x.std()) / np.sqrt(x.numel())
    assert abs(float(x.mean()) - iv(2, alpha) / iv(1, alpha)) < 5 * err


def test_torch_su2_update_moment():
    import torch
    g = torch.Generator()
    g.manual_seed(22)
    beta = 4.0
    w = np.random.default_rng(23).normal(size=(2, 2)) + 1j * np.random.default_rng(24).normal(size=(2, 2))
    r = hb.su2_heatbath_torch(torch.from_numpy(w).expand(100000, 2, 2).contiguous(), beta, g).numpy()
    assert np.abs(np.linalg.det(r) - 1).max() < 1e-13
    sig = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    e = [sig[0]] + [1j * s for s in sig[1:]]
    k = np.sqrt(sum((np.trace(np.conj(b.T) @ w).real / 2) ** 2 for b in e))
    alpha = 2 * beta * k / 3
    val = np.trace(r @ w, axis1=-2, axis2=-1).real
    assert abs(val.mean() - 2 * k * iv(2, alpha) / iv(1, alpha)) < 5 * val.std() / np.sqrt(val.size)


def test_torch_staples_and_plaquette_match_numpy():
    import torch
    dims = (4, 4, 2, 6)
    U = syn.gauge_field(dims, 0.8, 3)
    Ut = torch.from_numpy(U)
    assert hb.plaquette_torch(Ut) == pytest.approx(hb.plaquette(U), rel=1e-13)
    for mu in range(4):
        assert np.abs(hb.staple_sum_torch(Ut, mu).numpy() - hb.staple_sum(U, mu)).max() < 1e-12
    R = hb.reunitarize_torch(Ut * 1.001).numpy()
    assert np.abs(R - hb.reunitarize(U * 1.001)).max() < 1e-13


def test_torch_strong_coupling_plaquette_and_group():
    beta = 0.5
    ps = []
    U = hb.heatbath_field_torch((4, 4, 4, 4), beta, 40, 5, 'cpu', record=lambda n, U: ps.append(hb.plaquette_torch(U)))
    assert abs(np.mean(ps[10:]) - (beta / 18 + beta ** 2 / 216)) < 0.004
    u = U.numpy()
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-12
