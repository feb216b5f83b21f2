#!/usr/bin/env python
"""AMG time-to-solution benchmark on one MI355X.

One step = the whole hot path on one batch: load the gauge field (clover
build), the mixed-precision adaptive setup, and the FGMRES(16) solve of all
right-hand sides to a relative residual of 1e-10 (recomputed with the FP64
operator).  Default workload: 32^3x64, eps 0.3, kappa 0.1365, c_sw 1.1, 12 unit
point sources (one per spin-colour at the origin), 2-level AMG with blocks
4^3x8 and N_v = 32, SAP(4 sweeps, MR 6) smoother, coarse BiCGStab.

Printed as one JSON line: time-to-solution in seconds (lower is better), the
roofline of the dominant kernel class, the fine Dslash HBM bandwidth, the
plain FP64 AMG on the same GPU for comparison, and the CPU oracle baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6

# roofline of each kernel class: what bounds it, and its work unit for the
# counter-based traffic (profiles/pmc_traffic.json, per unit of work)
CLASS_BOUND = {'sap_half': 'alu32', 'sap_cross': 'hbm', 'coarse_mv': 'alu32', 'dslash64': 'hbm', 'dslash32': 'hbm',
               'restrict': 'hbm', 'prolong': 'hbm', 'coarse_build': 'alu32', 'ortho': 'hbm'}
CLASS_SOURCES = {'sap_half': ['fine.hip', 'wc_dirac.h', 'wc_common.h'],
                 'dslash64': ['fine.hip', 'wc_dirac.h', 'wc_common.h']}

WORKLOADS = {
    'c3': dict(dims=(32, 32, 32, 64), eps=0.3, seed=1, kappa=0.1365, csw=1.1, block=(4, 4, 4, 8), nv=32,
               nrhs=12, source='point'),
    'c2': dict(dims=(16, 16, 16, 16), eps=0.35, seed=1, kappa=0.1355, csw=1.0, block=(4, 4, 4, 4), nv=16,
               nrhs=1, source='z2'),
    # a pure-gauge heat-bath field (Wilson action, beta 6.0, 60 sweeps from a
    # cold start) instead of random links: smooth, physically distributed
    # gauge fields as a stand-in for the paper's ensembles
    'hb16': dict(dims=(16, 16, 16, 16), gauge=('heatbath', 6.0, 60), seed=1, kappa=0.1345, csw=1.769,
                 block=(4, 4, 4, 4), nv=16, nrhs=12, source='point'),
}
SETUP = dict(n_init=3, n_adapt=3, sap_sweeps=4, mr_iters=6, coarse_iters=30, coarse_tol=0.1)


def log(*a):
    print('[bench]', *a, file=sys.stderr, flush=True)


def gauge_numpy(w, dims):
    """The workload's gauge field on the host (random links of spread eps, or
    a heat-bath field), at lattice dims."""
    import synthetic as syn
    if 'gauge' not in w:
        return syn.gauge_field(dims, w['eps'], w['seed'])
    from synthetic import heatbath as hb
    kind, beta, sweeps = w['gauge']

    def progress(n, U):
        if (n + 1) % 10 == 0:
            log('heat-bath %s beta %g: sweep %d of %d, plaquette %.5f' % ('x'.join(map(str, dims)), beta, n + 1,
                                                                        sweeps, hb.plaquette(U)))
    return hb.heatbath_field(dims, beta, sweeps, w['seed'], record=progress)


def gauge_desc(w):
    if 'gauge' in w:
        return 'heat-bath gauge field (Wilson action, beta %g, %d sweeps)' % (w['gauge'][1], w['gauge'][2])
    return 'eps %g' % w['eps']


def make_inputs(w, dev):
    import torch
    import synthetic as syn
    dims = w['dims']
    if 'gauge' in w:
        U = torch.from_numpy(gauge_numpy(w, dims)).to(dev)
    else:
        U = syn.gauge_field_torch(dims, w['eps'], w['seed'], dev)
    if w['source'] == 'point':
        b = torch.from_numpy(syn.point_sources(dims, w['nrhs'])).to(dev)
    else:
        b = torch.from_numpy(syn.z2_source(dims, w['seed'], w['nrhs'])).to(dev)
    V0 = syn.gaussian_vectors_torch(dims, w['nv'], w['seed'], dev)
    return U, b, V0


def run_step(ctx, U, b, x, V0, w, prec, rhs_chunk=0, nrhs=None):
    """load gauge + setup + solve; returns (setup_s, solve_s, info, rc)."""
    import torch
    nrhs = nrhs or w['nrhs']
    t0 = time.perf_counter()
    ctx.load_gauge(U)
    prm = ctx.setup_params(w['nv'], prec, init_vectors=V0, **SETUP)
    ctx.setup(prm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, info = ctx.solve(b, x, nrhs, restart=16, tol=1e-10, max_iters=2000, rhs_chunk=rhs_chunk, use_graph=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1, info, rc


CLASSES = ['dslash64', 'dslash32', 'sap_half', 'sap_cross', 'restrict', 'prolong', 'coarse_solve', 'coarse_mv',
           'coarse_build', 'ortho']
LEAVES = ['dslash64', 'dslash32', 'sap_half', 'sap_cross', 'restrict', 'prolong', 'coarse_mv', 'coarse_build', 'ortho']


def source_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, 'paper_2111_05012_amd', 'csrc', f), 'rb') as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(cls, units_per_launch):
    """HBM bytes per launch of a kernel class from the committed counter runs
    (FETCH_SIZE + WRITE_SIZE, calibrated by a 1 GiB copy), or None when there
    are none or the kernel's sources changed since they were taken."""
    try:
        with open(os.path.join(ROOT, 'profiles', 'pmc_traffic.json')) as f:
            t = json.load(f)['kernels'][cls]
    except (OSError, KeyError, ValueError):
        return None
    if cls not in CLASS_SOURCES or t.get('source_sha') != source_sha(CLASS_SOURCES[cls]):
        return None
    if 'fetch_per_unit' not in t:
        return None
    return (t['fetch_per_unit'] + t['write_per_unit']) * units_per_launch


def kernel_profile(ctx, U, b, x, V0, w, prec):
    ctx.kernel_timing(1)
    s, v, info, rc = run_step(ctx, U, b, x, V0, w, prec)
    st = {k: ctx.kernel_stats(k) for k in CLASSES}
    ctx.kernel_timing(0)
    return st, s + v


def dslash_bandwidth(ctx, w, dev, reps=20):
    """fine FP64 D, 1 RHS, on the loaded gauge field: average event-timed
    kernel duration and algorithmic GB/s (1536 B/site: spinor in/out 192+192,
    4 links 576, clover 576)."""
    import torch
    import synthetic as syn
    V = syn.volume(w['dims'])
    psi = torch.randn((1,) + syn.shape_of(w['dims']) + (4, 3), dtype=torch.complex128, device=dev)
    out = torch.empty_like(psi)
    ctx.apply_D(psi, out, 1, 0)
    ctx.kernel_timing(1)
    for _ in range(reps):
        ctx.apply_D(psi, out, 1, 0)
    st = ctx.kernel_stats('dslash64')
    ctx.kernel_timing(0)
    ms = st['ms'] / st['count']
    return dict(ms_per_launch=ms, bytes_per_launch=1536.0 * V, gbs=1536.0 * V / (ms * 1e-3) / 1e9,
                bytes_per_site=1536, launches=st['count'])


def cpu_baseline(w, units, gpu_iters):
    """The FP64 NumPy oracle timed on the host: per-unit costs of each class
    measured on a sample lattice with the workload's parameters, scaled
    linearly in volume to the workload, times the units of work the GPU run
    did (from the kernel profile).  Returns the extrapolated oracle
    time-to-solution in seconds."""
    import numpy as np
    import synthetic as syn
    from oracle import amg, dirac as od
    dims_s = (8, 8, 8, 16) if w['dims'] == (32, 32, 32, 64) else (8, 8, 8, 8)
    blk = w['block']
    Vs = syn.volume(dims_s)
    scale = syn.volume(w['dims']) / Vs
    bc = (1, 1, 1, -1)
    t_wall0, t_cpu0 = time.perf_counter(), time.process_time()
    U = gauge_numpy(w, dims_s)
    Fb = od.clover_blocks(U, w['kappa'], w['csw'])
    op = amg.FineOp(U, Fb, w['kappa'], bc, blk)
    nv = w['nv']
    psi = syn.gaussian_vectors(dims_s, 1, 3)

    def timeit(f, n=1):
        t = time.perf_counter()
        for _ in range(n):
            f()
        return (time.perf_counter() - t) / n

    cost = {}
    cost['dslash'] = timeit(lambda: op.D(psi), 3)
    cost['sap'] = timeit(lambda: amg.sap(op, psi, SETUP['sap_sweeps'], SETUP['mr_iters']))
    V = amg.block_orthonormalize(syn.gaussian_vectors(dims_s, nv, 5), dims_s, blk)
    cost['ortho'] = timeit(lambda: amg.block_orthonormalize(V, dims_s, blk))
    cost['restrict'] = timeit(lambda: amg.restrict(V, psi, dims_s, blk), 3)
    xc = amg.restrict(V, psi, dims_s, blk)
    cost['prolong'] = timeit(lambda: amg.prolong(V, xc, dims_s, blk), 3)
    # the coarse operator build costs 2 nv applications of D-sized operators
    # plus restrictions of nv vectors: timed at nv/4 and scaled by 4^2
    nvb = max(nv // 4, 1)
    Vb = V[:nvb]
    cost['coarse_build'] = timeit(lambda: amg.coarse_operator(op, Vb)) * (nv / nvb) ** 2
    Dc = amg.coarse_operator(op, Vb)
    cd = amg.coarse_dims(dims_s, blk)
    Dc_full = np.zeros(Dc.shape[:2] + (2 * nv, 2 * nv), complex)
    Dc_full[:, :, :2 * nvb, :2 * nvb] = Dc
    xcv = syn.gaussian_coarse(Dc.shape[0], 2 * nv, 1, 7)[0]
    cost['coarse_mv'] = timeit(lambda: amg.coarse_apply(Dc_full, xcv, cd), 3)
    wall = time.perf_counter() - t_wall0
    cpu = time.process_time() - t_cpu0
    est = 0.0
    parts = {}
    for cls, key in (('dslash64', 'dslash'), ('dslash32', 'dslash'), ('restrict', 'restrict'),
                     ('prolong', 'prolong'), ('coarse_mv', 'coarse_mv')):
        parts[cls] = units[cls]['units'] * cost[key] * scale
    # one oracle SAP application = 2 * sweeps half-sweeps
    parts['sap_half'] = units['sap_half']['units'] * cost['sap'] / (2 * SETUP['sap_sweeps']) * scale
    parts['coarse_build'] = units['coarse_build']['units'] * cost['coarse_build'] * scale
    parts['ortho'] = units['ortho']['units'] * cost['ortho'] * scale
    est = sum(parts.values())
    return dict(value=est, unit='s', cores=max(1, round(cpu / wall)), kind='oracle',
                sample=('FP64 NumPy oracle per-unit costs (D, SAP(4,6), restrict, prolong with N_v=%d, '
                        'coarse 9-point matvec, block orthonormalisation, coarse-operator build timed at '
                        'N_v=%d and scaled by (%d/%d)^2) measured on an %s lattice with the workload\'s '
                        'blocks and parameters (%.1f s wall), scaled linearly by volume (x%.0f) and '
                        'multiplied by the units of work of the GPU run; extrapolated, not a full oracle solve'
                        % (nv, nvb, nv, nvb, 'x'.join(map(str, dims_s)), wall, scale)),
                parts={k: round(v, 2) for k, v in parts.items()})


def profile_kernels(ctx, U, b, x, V0, w, dev):
    """Kernel-only program for counter collection.  A warm-up pass (the
    autotuner's trial launches, workspace allocation), then a plain copy of
    1 GiB three times (reads 1 GiB, writes 1 GiB: the scale of FETCH_SIZE /
    WRITE_SIZE, and the marker after which dispatches count), then the
    measured pass: the mixed setup, the fine FP64 D (1 RHS) five times, two
    SAP applications and two V-cycles on all RHS."""
    import torch
    from paper_2111_05012_amd import PREC_FP64, PREC_MIXED
    prm = ctx.setup_params(w['nv'], PREC_MIXED, init_vectors=V0, **SETUP)
    psi = b[:1].contiguous()
    out = torch.empty_like(psi)
    xs = torch.empty_like(b)

    def one_pass(nd):
        ctx.load_gauge(U)
        ctx.setup(prm)
        for _ in range(nd):
            ctx.apply_D(psi, out, 1, PREC_FP64)
        for _ in range(2):
            ctx.sap(b, xs, w['nrhs'], SETUP['sap_sweeps'], SETUP['mr_iters'], PREC_MIXED)
        for _ in range(2):
            ctx.vcycle(b, xs, w['nrhs'])
        torch.cuda.synchronize()

    one_pass(1)
    log('profile-kernels warm-up done')
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    one_pass(5)
    log('profile-kernels done')


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=2)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--workload', default='c3', choices=sorted(WORKLOADS))
    ap.add_argument('--plain-rhs', type=int, default=1, help='RHS solved by the plain FP64 comparison (0: skip)')
    ap.add_argument('--plain-batched', type=int, default=1,
                    help='also time the FP64 AMG with all RHS batched (separates the batching and precision gains)')
    ap.add_argument('--no-cpu', action='store_true')
    ap.add_argument('--paper-solvers', action='store_true',
                    help="also time the paper's flexible BiCGStab with the mixed V-cycle and the comparison "
                         'solver (flexible BiCGStab preconditioned by an FP32 BiCGStab) on the same system')
    ap.add_argument('--profile-kernels', action='store_true',
                    help='short kernel-only run for hardware counters: a 1 GiB copy, then D, SAP, V-cycle')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py: this build runs on one GPU only (--gpus %d requested); the multi-GPU path is a '
              'design in DESIGN.md, not implemented' % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2111_05012_amd import Context, PREC_FP64, PREC_MIXED

    w = WORKLOADS[args.workload]
    dev = torch.device('cuda:0')
    log('generating inputs', w['dims'])
    U, b, V0 = make_inputs(w, dev)
    x = torch.zeros_like(b)
    ctx = Context(w['dims'], w['block'], (1, 1, 1, -1), w['kappa'], w['csw'])
    if args.profile_kernels:
        profile_kernels(ctx, U, b, x, V0, w, dev)
        return

    for k in range(args.warmup):
        s, v, info, rc = run_step(ctx, U, b, x, V0, w, PREC_MIXED)
        log('warmup %d: setup %.3f s solve %.3f s iters %s' % (k, s, v, list(info.iters[:w['nrhs']])))
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        s, v, info, rc = run_step(ctx, U, b, x, V0, w, PREC_MIXED)
        times.append((s, v))
        log('step %d: setup %.3f s solve %.3f s' % (k, s, v))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tts = (t1 - t0) / args.steps
    iters = list(info.iters[:w['nrhs']])
    relres = max(info.relres[:w['nrhs']])
    converged = rc == 0
    log('TTS %.3f s, outer iters %s, max relres %.2e' % (tts, iters, relres))

    # kernel-class profile of one more (untimed) step
    prof, prof_s = kernel_profile(ctx, U, b, x, V0, w, PREC_MIXED)
    leaf_ms = {k: prof[k]['ms'] for k in LEAVES if prof[k]['bytes'] or prof[k]['flops']}
    dom = max(leaf_ms, key=leaf_ms.get)
    d = prof[dom]
    kernels = {}
    for k in CLASSES:
        p = prof[k]
        if p['count'] == 0:
            continue
        kernels[k] = dict(ms=round(p['ms'], 3), launches=p['count'],
                          gbs=round(p['bytes'] / (p['ms'] * 1e-3) / 1e9, 1) if p['bytes'] else None,
                          tflops=round(p['flops'] / (p['ms'] * 1e-3) / 1e12, 2) if p['flops'] else None,
                          share=round(p['ms'] / (prof_s * 1e3), 3))
    nl = max(d['count'], 1)
    V = 1
    for L in w['dims']:
        V *= L
    # units of the class per launch: RHS x sites (half the lattice for a SAP half-sweep)
    units = d['units'] / nl * (V / 2 if dom in ('sap_half', 'sap_cross') else V)
    traffic = counter_traffic(dom, units)
    if CLASS_BOUND.get(dom, 'hbm') == 'hbm':
        achieved = d['bytes'] / (d['ms'] * 1e-3) / 1e9
        roof = dict(kernel=dom, bound='hbm', achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit='GB/s',
                    frac=round(achieved / HBM_PEAK_GBS, 4))
    else:
        achieved = d['flops'] / (d['ms'] * 1e-3) / 1e12
        roof = dict(kernel=dom, bound='alu', achieved=round(achieved, 2), peak=FP32_PEAK_TFLOPS, unit='TFLOP/s',
                    frac=round(achieved / FP32_PEAK_TFLOPS, 4))
    roof.update(traffic=round(traffic) if traffic else None, ms_per_launch=round(d['ms'] / nl, 4),
                bytes_per_launch=d['bytes'] / nl, flops_per_launch=d['flops'] / nl,
                traffic_note='HBM bytes per launch from FETCH_SIZE + WRITE_SIZE (profiles/pmc_traffic.json, '
                             'scaled by a 1 GiB copy); null when the kernel changed since the counters were taken')
    dsl = dslash_bandwidth(ctx, w, dev)
    log('dslash fp64: %.3f ms, %.0f GB/s' % (dsl['ms_per_launch'], dsl['gbs']))

    plain = None
    if args.plain_rhs > 0:
        nr = min(args.plain_rhs, w['nrhs'])
        bp = b[:nr].contiguous()
        xp = torch.zeros_like(bp)
        sp, vp, infop, rcp = run_step(ctx, U, bp, xp, V0, w, PREC_FP64, rhs_chunk=1, nrhs=nr)
        per = vp / nr
        plain = dict(setup_s=round(sp, 3), solve_s_per_rhs=round(per, 3), rhs_measured=nr,
                     tts_s=round(sp + per * w['nrhs'], 3),
                     tts_note='setup + %d x measured per-RHS solve (one RHS at a time, FP64 everywhere)'
                              % w['nrhs'], iters=list(infop.iters[:nr]),
                     relres_max=max(infop.relres[:nr]))
        log('plain fp64: setup %.3f s, solve/rhs %.3f s' % (sp, per))
    plain_b = None
    if args.plain_batched and w['nrhs'] > 1:
        xb = torch.zeros_like(b)
        sb, vb, infob, rcb = run_step(ctx, U, b, xb, V0, w, PREC_FP64)
        plain_b = dict(setup_s=round(sb, 3), solve_s=round(vb, 3), tts_s=round(sb + vb, 3),
                       iters=list(infob.iters[:w['nrhs']]), relres_max=max(infob.relres[:w['nrhs']]),
                       converged=rcb == 0, note='FP64 everywhere, all %d RHS batched' % w['nrhs'])
        log('plain fp64 batched: setup %.3f s, solve %.3f s' % (sb, vb))

    paper = None
    if args.paper_solvers:
        from paper_2111_05012_amd import PC_AMG, PC_BICG32
        paper = {}
        # the paper's outer solver with the multigrid preconditioner (setup as in the step)
        ctx.load_gauge(U)
        ctx.setup(ctx.setup_params(w['nv'], PREC_MIXED, init_vectors=V0, **SETUP))
        for name, pc, kw in (('fbicgstab_amg', PC_AMG, {}),
                             ('mbicgs', PC_BICG32, dict(inner_iters=50, inner_tol=0.1))):
            xq = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rcq, infq = ctx.solve_bicgstab(b, xq, w['nrhs'], tol=1e-10, max_iters=500, precond=pc, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            paper[name] = dict(solve_s=round(dt, 3), iters=list(infq.iters[:w['nrhs']]),
                               precond_applications=infq.vcycles, relres_max=max(infq.relres[:w['nrhs']]),
                               converged=rcq == 0)
            log('%s: solve %.3f s, outer iterations %s' % (name, dt, list(infq.iters[:w['nrhs']])))
        paper['note'] = ("Sec. 2 flexible BiCGStab, all RHS batched, FP64 outer; fbicgstab_amg: M = mixed V-cycle "
                         "(solve only, the setup is the step's); mbicgs: M = FP32 stabilised BiCGStab on D "
                         "(50 iterations or 0.1 relative residual), no setup")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, prof, iters)
        log('cpu baseline (extrapolated) %.1f s' % cpu['value'])

    res = dict(
        metric='AMG time-to-solution @ rel.res 1e-10 vs plain FP64 AMG; fine Dslash HBM GB/s',
        value=round(tts, 4), unit='s', n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(tts * 1e3, 2), higher_is_better=False, scaling='weak', vs_baseline=None,
        dtype='f32', data='synthetic',
        config=dict(workload='%s Wilson-clover AMG solve: %s lattice, %s, kappa %g, c_sw %g, %d %s sources, '
                             'blocks %s, N_v %d, SAP(4,6), mixed precision (FP16 links/vectors, FP32 inner, '
                             'FP64 FGMRES(16)), tol 1e-10'
                             % (args.workload, 'x'.join(map(str, w['dims'])), gauge_desc(w), w['kappa'], w['csw'],
                                w['nrhs'], w['source'], 'x'.join(map(str, w['block'])), w['nv']),
                    global_batch=w['nrhs'], parallelism='single GPU'),
        setup_s=round(sum(t[0] for t in times) / len(times), 4),
        solve_s=round(sum(t[1] for t in times) / len(times), 4),
        outer_iters=iters, relres_max=relres, converged=converged,
        roofline=roof, dslash_fp64=dsl, kernels=kernels, plain_fp64=plain, plain_fp64_batched=plain_b,
        speedup_vs_plain=round(plain['tts_s'] / tts, 2) if plain else None,
        speedup_vs_plain_batched=round(plain_b['tts_s'] / tts, 2) if plain_b else None,
        autotune=ctx.autotune_info(),
        paper_solvers=paper,
        cpu_baseline=cpu)
    print(json.dumps(res), flush=True)


if __name__ == '__main__':
    main()
