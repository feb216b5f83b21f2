"""48^3x96 three-level solve (the largest workload): runs in a module of
its own, after the 32^3x64 context of the other full-size tests is closed,
so that the whole device memory is available."""
import gc

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


def _residual(ctx, b, x):
    """per-RHS ||b - D x|| / ||b|| with the library's FP64 operator"""
    import torch
    r = torch.empty_like(b)
    ctx.apply_D(x, r, b.shape[0], 0)
    r = b - r
    return (torch.linalg.vector_norm(r.reshape(b.shape[0], -1), dim=1) /
            torch.linalg.vector_norm(b.reshape(b.shape[0], -1), dim=1)).cpu().numpy()


def test_three_level_c5_12rhs():
    """48^3x96 (eps 0.28, kappa 0.1368, c_sw 1.1): three levels (blocks 4^4
    with N_v 24, then 2^4 with N_v 32), 12 point sources in chunks of 2,
    mixed precision; every RHS to 1e-10 by the FP64 operator (chunks of 2 keep the
    FP64 Krylov basis within memory)."""
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    dims, block = (48, 48, 48, 96), (4, 4, 4, 4)
    dev = torch.device('cuda:0')
    U = syn.gauge_field_torch(dims, 0.28, 1, dev)
    from paper_2111_05012_amd import Context
    ctx = Context(dims, block, BC, 0.1368, 1.1)
    try:
        ctx.load_gauge(U)
        del U
        torch.cuda.empty_cache()
        ctx.setup(ctx.setup_params(24, 1, seed=5, coarse_iters=30, nlevels=3, block1=(2, 2, 2, 2), nv1=32,
                                   mr1_iters=4, seed1=6))
        b = torch.from_numpy(syn.point_sources(dims, 12)).to(dev)
        x = torch.zeros_like(b)
        rc, info = ctx.solve(b, x, 12, tol=1e-10, rhs_chunk=2)
        print('c5 three-level: iters', list(info.iters[:12]), 'vcycles', info.vcycles, 't_solve %.2f s' % info.t_solve,
              flush=True)
        assert rc == 0
        res = []
        for k in range(0, 12, 4):
            res.append(_residual(ctx, b[k:k + 4].contiguous(), x[k:k + 4].contiguous()))
        assert np.concatenate(res).max() <= 1e-10
    finally:
        ctx.close()
