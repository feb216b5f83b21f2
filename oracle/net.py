"""Oracle: the gauge-equivariant network that proposes initial test vectors
(learned replacement of setup step (0-a), Sec. 3), in plain NumPy FP64.

The paper does not contain this network; its definition is the reading used
by the library:
  * input: the gauge field U and C random fields r_i (a covariant vector field
    cannot be built from U alone);
  * L linear parallel-transport convolution layers, C -> C channels:
      psi'_o(x) = sum_i sum_{d=0..8} W[d, o, i] (T_d psi_i)(x),
    T_0 = 1, T_{+mu} psi(x) = U_mu(x) psi(x+mu), T_{-mu} psi(x) =
    U_mu(x-mu)^dag psi(x-mu) (hops across the boundary carry bc[mu]), W[d,o,i]
    a complex 4x4 spin matrix; no bias and no nonlinearity (both would break
    covariance);
  * loss per block X and chirality s: with A the network output restricted
    to (X, s) (K x C) and Q the teacher's orthonormal basis there,
      L_{X,s} = 1 - tr(Q^dag P_A Q) / C,  P_A = A (A^dag A)^-1 A^dag,
    the fraction of the teacher subspace outside span(A); L = mean over (X, s);
  * gradients are Wirtinger derivatives dL/d conj(.) (for a real loss,
    dL = 2 Re sum conj(g) dz); Adam on the real and imaginary parts.

Pins (tests/test_oracle_net.py): transport adjointness (T_d^dag = T_{-d});
gauge equivariance net(U^Om, Om r) = Om net(U, r); loss invariant under a
change of basis of the output and of the teacher, 0 when the teacher lies in
span(A); the backward against central finite differences of the loss;
Adam against iterates worked out by hand for gradient sequences that separate
beta1 and beta2.
"""
import numpy as np

from . import amg, dirac

NDIR = 9


def transport(U, psi, d, bc):
    """T_d psi for psi [..., Lt,Lz,Ly,Lx,4,3]; d = 0 identity, 1+mu forward, 5+mu backward."""
    if d == 0:
        return psi
    mu = (d - 1) % 4
    if d <= 4:
        return np.einsum('...ab,...sb->...sa', U[mu], dirac.shift(psi, mu, +1, bc))
    ub = dirac.shift(U[mu], mu, -1)
    return np.einsum('...ba,...sb->...sa', np.conj(ub), dirac.shift(psi, mu, -1, bc))


def opposite(d):
    return 0 if d == 0 else (d + 4 if d <= 4 else d - 4)


def layer_forward(U, W, psi, bc):
    """W [9, Cout, Cin, 4, 4]; psi [Cin, ...field] -> [Cout, ...field]."""
    out = None
    for d in range(NDIR):
        t = np.einsum('oist,i...tc->o...sc', W[d], transport(U, psi, d, bc))
        out = t if out is None else out + t
    return out


def forward(U, Ws, r, bc):
    """Returns the list of activations [r, psi_1, ..., psi_L]."""
    acts = [r]
    for W in Ws:
        acts.append(layer_forward(U, W, acts[-1], bc))
    return acts


def layer_backward(U, W, psi_in, g_out, bc):
    """Given g_out = dL/d conj(psi_out), return (dL/d conj(W), dL/d conj(psi_in))."""
    gW = np.zeros_like(W)
    g_in = np.zeros_like(psi_in)
    for d in range(NDIR):
        t = transport(U, psi_in, d, bc)
        gW[d] = np.einsum('oxsc,ixtc->oist', g_out.reshape(g_out.shape[0], -1, 4, 3),
                          np.conj(t).reshape(t.shape[0], -1, 4, 3))
        # T_d^dag = T_{-d}; W^dag acts on the spin index
        mixed = np.einsum('oits,o...sc->i...tc', np.conj(np.swapaxes(W[d], -1, -2)), g_out)
        g_in += transport(U, mixed, opposite(d), bc)
    return gW, g_in


def backward(U, Ws, acts, g_last, bc):
    gWs = [None] * len(Ws)
    g = g_last
    for l in range(len(Ws) - 1, -1, -1):
        gWs[l], g = layer_backward(U, Ws[l], acts[l], g, bc)
    return gWs, g


def subspace_loss(A, Q, dims, block):
    """Loss and dL/d conj(A) for network output A and teacher basis Q (both
    [C, ...field]); per block and chirality, L = 1 - tr(Q^dag P_A Q)/C, mean
    over the 2 N_X (block, chirality) pairs."""
    C = A.shape[0]
    Ab = amg.to_blocks(A, dims, block)  # [C, X, 2, K]
    Qb = amg.to_blocks(Q, dims, block)
    nX = Ab.shape[1]
    G = np.einsum('ixsk,jxsk->xsij', np.conj(Ab), Ab)  # A^dag A
    B = np.einsum('ixsk,jxsk->xsij', np.conj(Ab), Qb)  # A^dag Q
    Gi = np.linalg.inv(G)
    f = np.einsum('xsij,xsjk,xsik->xs', Gi, B, np.conj(B)).real  # tr(G^-1 B B^dag)
    loss = np.mean(1.0 - f / C)
    # dL/d conj(A) = -(Q B^dag G^-1 - A G^-1 B B^dag G^-1) / (C * 2 nX)
    M1 = np.einsum('xsji,xsjk->xsik', np.conj(B), Gi)            # B^dag G^-1   [j->rows of Q]
    M2 = np.einsum('xsij,xsjk,xslk,xslm->xsim', Gi, B, np.conj(B), Gi)  # G^-1 B B^dag G^-1
    gb = -(np.einsum('jxsk,xsji->ixsk', Qb, M1) - np.einsum('jxsk,xsji->ixsk', Ab, M2)) / (C * 2 * nX)
    return loss, amg.from_blocks(gb, dims, block)


class Adam:
    """Adam (Kingma and Ba) on the real and imaginary parts of complex
    parameters: the real gradient of Re z and Im z is 2 dL/d conj(z)."""

    def __init__(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = self.v = None

    def step(self, Ws, gWs):
        self.t += 1
        if self.m is None:
            self.m = [np.zeros(W.shape + (2,)) for W in Ws]
            self.v = [np.zeros(W.shape + (2,)) for W in Ws]
        out = []
        for k, (W, g) in enumerate(zip(Ws, gWs)):
            gr = np.stack([2 * g.real, 2 * g.imag], axis=-1)
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * gr
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * gr ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            upd = self.lr * mh / (np.sqrt(vh) + self.eps)
            out.append(W - (upd[..., 0] + 1j * upd[..., 1]))
        return out
