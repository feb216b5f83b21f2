"""Pins of the oracle's equivariant network: adjointness of the transport,
gauge equivariance, invariances of the subspace loss, and the hand-derived
backward against central finite differences."""
import numpy as np

import synthetic as syn
from oracle import amg, dirac as od, net

BC = (1, 1, 1, -1)
DIMS = (4, 4, 4, 4)
BLOCK = (2, 2, 2, 2)


def _U():
    return syn.gauge_field(DIMS, 0.5, 3)


def test_transport_adjoint():
    U = _U()
    a, b = syn.gaussian_vectors(DIMS, 2, 9)
    for d in range(9):
        lhs = np.vdot(a, net.transport(U, b, d, BC))
        rhs = np.vdot(net.transport(U, a, net.opposite(d), BC), b)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_equivariance():
    U = _U()
    om = syn.random_su3(syn.shape_of(DIMS), 4)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = om @ U[mu] @ od.dagger(od.shift(om, mu, +1))
    Ws = syn.net_weights(3, 2, 1, scale=0.2)
    r = syn.gaussian_vectors(DIMS, 3, 5)
    rot = lambda f: np.einsum('...ab,...sb->...sa', om, f)  # noqa: E731
    out = net.forward(U, Ws, r, BC)[-1]
    outg = net.forward(Ug, Ws, rot(r), BC)[-1]
    assert np.abs(outg - rot(out)).max() < 1e-12 * np.abs(out).max()


def test_loss_invariances():
    A = syn.gaussian_vectors(DIMS, 3, 6)
    Q = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 3, 7), DIMS, BLOCK)
    l0, _ = net.subspace_loss(A, Q, DIMS, BLOCK)
    assert 0.0 < l0 < 1.0
    # invertible mixing of the output channels does not change span(A)
    M = np.array([[1.0, 0.3, 0], [0.2j, 1.1, 0.4], [0, 0.5, 0.9 - 0.1j]])
    l1, _ = net.subspace_loss(np.einsum('ij,j...->i...', M, A), Q, DIMS, BLOCK)
    assert abs(l1 - l0) < 1e-12
    # a unitary change of the teacher basis does not change the loss
    Uq, _ = np.linalg.qr(np.array([[1, 2j, 0], [0.5, 1, 1], [0, 1j, 2]]))
    l2, _ = net.subspace_loss(A, np.einsum('ij,j...->i...', Uq, Q), DIMS, BLOCK)
    assert abs(l2 - l0) < 1e-12
    # teacher inside span(A): zero loss
    l3, _ = net.subspace_loss(A, amg.block_orthonormalize(A, DIMS, BLOCK), DIMS, BLOCK)
    assert abs(l3) < 1e-12


def test_backward_matches_finite_differences():
    U = _U()
    C = 2
    Ws = syn.net_weights(C, 2, 2, scale=0.3)
    r = syn.gaussian_vectors(DIMS, C, 8)
    Q = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, C, 10), DIMS, BLOCK)

    def L(Ws_):
        return net.subspace_loss(net.forward(U, Ws_, r, BC)[-1], Q, DIMS, BLOCK)[0]

    acts = net.forward(U, Ws, r, BC)
    _, g = net.subspace_loss(acts[-1], Q, DIMS, BLOCK)
    gWs, _ = net.backward(U, Ws, acts, g, BC)
    rng = np.random.default_rng(0)
    h = 1e-6
    for trial in range(6):
        l = trial % 2
        idx = tuple(rng.integers(s) for s in Ws[l].shape)
        for unit in (1.0, 1j):
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l][idx] += h * unit
            Wm[l][idx] -= h * unit
            fd = (L(Wp) - L(Wm)) / (2 * h)
            an = 2 * (gWs[l][idx].real if unit == 1.0 else gWs[l][idx].imag)
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)


def test_adam_reduces_loss():
    U = _U()
    C = 2
    Ws = syn.net_weights(C, 2, 3, scale=0.3)
    r = syn.gaussian_vectors(DIMS, C, 11)
    Q = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, C, 12), DIMS, BLOCK)
    opt = net.Adam(lr=2e-2)
    losses = []
    for _ in range(15):
        acts = net.forward(U, Ws, r, BC)
        l, g = net.subspace_loss(acts[-1], Q, DIMS, BLOCK)
        losses.append(l)
        gWs, _ = net.backward(U, Ws, acts, g, BC)
        Ws = opt.step(Ws, gWs)
    assert losses[-1] < losses[0]


def test_adam_matches_hand_computed_iterates():
    """Adam as Kingma and Ba define it (Algorithm 1; beta1 0.9, beta2 0.999,
    eps 1e-8) on one complex weight, whose real and imaginary parts see the
    real gradient sequences (1, -1, 1) and (1, 2, 2).  Bias-corrected
    moments, worked out by hand from the recursions m_t = b1 m_{t-1} +
    (1 - b1) g_t, v_t = b2 v_{t-1} + (1 - b2) g_t^2:
      (1, -1, 1): m_hat = 1, -(1 - b1)/(1 + b1) = -1/19,
                  (b1^2 - b1 + 1)/(1 + b1 + b1^2) = 91/271; v_hat = 1 always;
      (1, 2, 2):  m_hat = 1, (b1 + 2)/(1 + b1) = 29/19,
                  (b1^2 + 2 b1 + 2)/(1 + b1 + b1^2) = 461/271;
                  v_hat = 1, (b2 + 4)/(1 + b2) = 4.999/1.999,
                  (b2^2 + 4 b2 + 4)/(1 + b2 + b2^2) = 8.994001/2.997001.
    Each step moves a part by -lr m_hat / (sqrt(v_hat) + eps).  A wrong
    beta1 changes the first sequence's steps, a wrong beta2 the second's."""
    lr, eps = 0.01, 1e-8
    re_g, im_g = (1.0, -1.0, 1.0), (1.0, 2.0, 2.0)
    mh_re = (1.0, -1.0 / 19.0, 91.0 / 271.0)
    mh_im = (1.0, 29.0 / 19.0, 461.0 / 271.0)
    vh_im = (1.0, 4.999 / 1.999, 8.994001 / 2.997001)
    W = [np.array([0.3 + 0.7j])]
    want = W[0].copy()
    opt = net.Adam(lr=lr)
    for t in range(3):
        # the oracle's gradients are dL/d conj(W): the real gradient of a part is twice its part
        W = opt.step(W, [np.array([0.5 * re_g[t] + 0.5j * im_g[t]])])
        want = want - lr * (mh_re[t] / (1.0 + eps) + 1j * mh_im[t] / (np.sqrt(vh_im[t]) + eps))
        assert abs(W[0][0] - want[0]) < 1e-15, t
