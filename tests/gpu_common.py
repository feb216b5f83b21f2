"""Shared helpers of the GPU tests: a problem (gauge field, oracle operator)
and a library context on cuda:0, built from the same seeded inputs."""
import numpy as np

import synthetic as syn
from oracle import amg, dirac as od

BC_AP = (1, 1, 1, -1)


class Problem:
    def __init__(self, dims, block, eps=0.5, seed=1, kappa=0.124, csw=1.0, bc=BC_AP, U=None):
        import torch
        from paper_2111_05012_amd import Context
        self.dims, self.block, self.bc = tuple(dims), tuple(block), tuple(bc)
        self.kappa, self.csw = kappa, csw
        self.U = syn.gauge_field(dims, eps, seed) if U is None else U
        self.Fb = od.clover_blocks(self.U, kappa, csw)
        self.op = amg.FineOp(self.U, self.Fb, kappa, bc, block)
        self.dev = torch.device('cuda:0')
        self.ctx = Context(dims, block, bc, kappa, csw)
        self.ctx.load_gauge(self.T(self.U))

    def T(self, a):
        import torch
        return torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)

    def zeros(self, shape):
        import torch
        return torch.zeros(shape, dtype=torch.complex128, device=self.dev)

    @staticmethod
    def N(t):
        return t.cpu().numpy()


def rel(a, b):
    """max-norm error relative to the max-norm of the reference."""
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)
