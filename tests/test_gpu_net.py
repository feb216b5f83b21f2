"""GPU parity of the equivariant network (FP32 kernels vs the FP64 oracle):
forward, loss, gradient, one Adam step; network-initialised setup."""
import numpy as np
import pytest

import synthetic as syn
from oracle import amg, net
from gpu_common import Problem, rel, BC_AP

pytestmark = pytest.mark.gpu
C = 16


@pytest.fixture(scope='module')
def setup():
    prob = Problem((4, 4, 4, 8), (2, 2, 2, 2), eps=0.4, seed=5, kappa=0.124, csw=1.0)
    Ws = syn.net_weights(C, 2, 7, scale=0.05)
    r = syn.gaussian_vectors(prob.dims, C, 8)
    Q = amg.block_orthonormalize(syn.gaussian_vectors(prob.dims, C, 9), prob.dims, prob.block)
    wflat = np.ascontiguousarray(np.stack(Ws).astype(np.complex64))
    prob.ctx.net_init(prob.T(wflat), 2, C)
    return prob, Ws, r, Q


def test_net_forward(setup):
    prob, Ws, r, Q = setup
    out = prob.zeros(r.shape)
    prob.ctx.net_forward(prob.T(r), out)
    want = net.forward(prob.U, Ws, r, BC_AP)[-1]
    assert rel(prob.N(out), want) < 2e-5


def test_net_gradient(setup):
    prob, Ws, r, Q = setup
    import torch
    g = torch.zeros((2, 9, C, C, 4, 4), dtype=torch.complex64, device=prob.dev)
    loss = prob.ctx.net_gradient(prob.T(r), prob.T(Q), g)
    acts = net.forward(prob.U, Ws, r, BC_AP)
    l_o, gA = net.subspace_loss(acts[-1], Q, prob.dims, prob.block)
    gWs, _ = net.backward(prob.U, Ws, acts, gA, BC_AP)
    assert abs(loss - l_o) < 1e-5
    assert rel(g.cpu().numpy(), np.stack(gWs)) < 1e-3


def test_net_adam_step(setup):
    prob, Ws, r, Q = setup
    import torch
    loss = prob.ctx.net_train_step(prob.T(r), prob.T(Q), 1e-3)
    acts = net.forward(prob.U, Ws, r, BC_AP)
    _, gA = net.subspace_loss(acts[-1], Q, prob.dims, prob.block)
    gWs, _ = net.backward(prob.U, Ws, acts, gA, BC_AP)
    W1 = net.Adam(lr=1e-3).step(Ws, gWs)
    got = torch.zeros((2, 9, C, C, 4, 4), dtype=torch.complex64, device=prob.dev)
    prob.ctx.net_get_weights(got)
    # the first Adam step moves each real and imaginary part by
    # lr * g / (|g| + eps) ~ lr * sign(g); compare it where the gradient part is
    # well above eps and above the FP32 gradient's rounding (elsewhere the step
    # depends on the sign of a rounding error)
    upd_g = got.cpu().numpy() - np.stack(Ws)
    upd_o = np.stack(W1) - np.stack(Ws)
    go = np.stack(gWs)
    for part in (np.real, np.imag):
        m = np.abs(part(go)) > 1e-3 * np.abs(go).max()
        assert m.sum() > 0.1 * m.size
        assert np.abs(part(upd_g) - part(upd_o))[m].max() < 1e-5
    assert np.isfinite(loss)
    # restore the weights for the other tests
    prob.ctx.net_init(prob.T(np.ascontiguousarray(np.stack(Ws).astype(np.complex64))), 2, C)


def test_net_initialised_setup_and_solve(setup):
    prob, Ws, r, Q = setup
    from paper_2111_05012_amd import PREC_MIXED
    p = prob.ctx.setup_params(C, PREC_MIXED, init_vectors=prob.T(r), n_adapt=1, init_net=1)
    prob.ctx.setup(p)
    b = syn.z2_source(prob.dims, 3)
    x = prob.zeros(b.shape)
    rc, info = prob.ctx.solve(prob.T(b), x, 1, tol=1e-10)
    assert rc == 0
    xg = prob.N(x)
    assert np.linalg.norm(b - prob.op.D(xg)) / np.linalg.norm(b) <= 1e-10
