"""Pins of the oracle's multigrid pieces (Sec. 3) against dense linear
algebra, library routines and exact special cases."""
import numpy as np
import pytest

import synthetic as syn
from oracle import amg, dirac as od

BC_AP = (1, 1, 1, -1)
DIMS = (4, 4, 4, 4)
BLOCK = (2, 2, 2, 2)


@pytest.fixture(scope='module')
def small():
    U = syn.gauge_field(DIMS, 0.5, 1)
    kappa, csw = 0.124, 1.0
    Fb = od.clover_blocks(U, kappa, csw)
    op = amg.FineOp(U, Fb, kappa, BC_AP, BLOCK)
    D = od.dense_D(U, Fb, kappa, BC_AP, DIMS)
    return op, D


def _colour_index(dims, block):
    col = np.broadcast_to(amg.domain_colour(dims, block), syn.shape_of(dims) + (4, 3))
    return col.reshape(-1)


def test_block_roundtrip():
    v = syn.gaussian_vectors((4, 2, 6, 4), 3, 1)
    b = amg.to_blocks(v, (4, 2, 6, 4), (2, 2, 3, 2))
    assert b.shape == (3, 2 * 1 * 2 * 2, 2, 6 * 24)
    assert np.array_equal(amg.from_blocks(b, (4, 2, 6, 4), (2, 2, 3, 2)), v)


def test_mr_step_is_minimal_residual(small):
    """One MR step minimises ||b - alpha A b|| over alpha in every domain, so
    the new residual is orthogonal to A b domain by domain; the residual
    norm never grows, and r = b - D_SAP x is kept exactly."""
    op, _ = small
    b = syn.gaussian_vectors(DIMS, 1, 3)[0]
    x1, r1 = amg.mr_domains(op, b, 1)
    Ab = op.Dsap(b)
    ortho = amg.domain_sums(np.conj(Ab) * r1, DIMS, BLOCK)
    assert np.abs(ortho).max() < 1e-12
    prev = amg.domain_sums(np.abs(b) ** 2, DIMS, BLOCK).real
    for k in range(1, 7):
        x, r = amg.mr_domains(op, b, k)
        now = amg.domain_sums(np.abs(r) ** 2, DIMS, BLOCK).real
        assert np.all(now <= prev * (1 + 1e-13))
        prev = now
        assert np.abs(r - (b - op.Dsap(x))).max() < 1e-12
    # A = c 1 (kappa = 0, no clover): MR is exact after one step
    U = syn.unit_gauge(DIMS)
    op0 = amg.FineOp(U, np.zeros(syn.shape_of(DIMS) + (2, 6, 6), complex), 0.0, BC_AP, BLOCK)
    x, r = amg.mr_domains(op0, b, 1)
    assert np.abs(r).max() < 1e-14 and np.abs(x - b).max() < 1e-14


def test_sap_is_red_black_block_gauss_seidel(small):
    """With exact block solves, the SAP listing is multiplicative Schwarz on
    the two colours: e <- (1 - S_o D)(1 - S_e D) e with S_c the inverse of
    D restricted to the colour-c domains, written here from dense matrices."""
    op, D = small
    n = D.shape[0]
    col = _colour_index(DIMS, BLOCK)
    S = []
    for c in (0, 1):
        idx = np.where(col == c)[0]
        Sc = np.zeros((n, n), complex)
        Sc[np.ix_(idx, idx)] = np.linalg.inv(D[np.ix_(idx, idx)])
        S.append(Sc)
    E = (np.eye(n) - S[1] @ D) @ (np.eye(n) - S[0] @ D)
    b = syn.gaussian_vectors(DIMS, 1, 4)[0]
    Dinv_b = np.linalg.solve(D, b.reshape(-1))
    sweeps = 3
    want = Dinv_b - np.linalg.matrix_power(E, sweeps) @ Dinv_b

    Ds = od.dense_D(op.U, op.Fb, op.kappa, BC_AP, DIMS, block=BLOCK)

    def exact_block(rc):
        return np.linalg.solve(Ds, rc.reshape(-1)).reshape(rc.shape)

    got = amg.sap(op, b, sweeps, block_solver=exact_block)
    assert np.abs(got.reshape(-1) - want).max() < 1e-11 * np.abs(want).max()


def test_sap_converges_for_small_kappa():
    U = syn.gauge_field(DIMS, 0.5, 2)
    kappa = 0.06
    Fb = od.clover_blocks(U, kappa, 1.0)
    op = amg.FineOp(U, Fb, kappa, BC_AP, BLOCK)
    b = syn.gaussian_vectors(DIMS, 1, 5)[0]
    x = amg.sap(op, b, sweeps=12, mr_iters=12)
    res = np.linalg.norm(b - op.D(x)) / np.linalg.norm(b)
    assert res < 1e-8


def _dense_P(V, dims, block):
    nv = V.shape[0]
    nX = amg.n_blocks(dims, block)
    cols = []
    for X in range(nX):
        for k in range(2 * nv):
            e = np.zeros((nX, 2 * nv), complex)
            e[X, k] = 1.0
            cols.append(amg.prolong(V, e, dims, block).reshape(-1))
    return np.array(cols).T


def test_orthonormalisation_matches_library_qr():
    V = syn.gaussian_vectors(DIMS, 6, 8)
    Q = amg.block_orthonormalize(V, DIMS, BLOCK)
    Vb = amg.to_blocks(V, DIMS, BLOCK)
    Qb = amg.to_blocks(Q, DIMS, BLOCK)
    for X in (0, 5, 15):
        for s in (0, 1):
            A = Vb[:, X, s, :].T
            q, r = np.linalg.qr(A)
            q = q * (np.diag(r) / np.abs(np.diag(r)))
            assert np.abs(Qb[:, X, s, :].T - q).max() < 1e-13
    P = _dense_P(Q, DIMS, BLOCK)
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-13


def test_restrict_prolong_identities():
    V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 4, 9), DIMS, BLOCK)
    P = _dense_P(V, DIMS, BLOCK)
    x = syn.gaussian_vectors(DIMS, 2, 10)
    xc = amg.restrict(V, x, DIMS, BLOCK)
    assert np.abs(xc.reshape(2, -1) - (P.conj().T @ x.reshape(2, -1).T).T).max() < 1e-13
    yc = syn.gaussian_coarse(16, 8, 1, 3)[0]
    assert np.abs(amg.restrict(V, amg.prolong(V, yc, DIMS, BLOCK), DIMS, BLOCK) - yc).max() < 1e-13
    PR = P @ P.conj().T
    assert np.abs(PR @ PR - PR).max() < 1e-13 and np.abs(PR - PR.conj().T).max() < 1e-14


@pytest.mark.parametrize('block', [(2, 2, 2, 2), (2, 4, 2, 2)])
def test_coarse_operator_is_galerkin(small, block):
    """eq. (7): Dc = P^dag D P, checked against dense brute force, including a
    direction with a single block (no crossing) and extent-2 coarse
    directions (forward and backward blocks reach the same neighbour)."""
    op0, D = small
    op = amg.FineOp(op0.U, op0.Fb, op0.kappa, BC_AP, block)
    V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 3, 12), DIMS, block)
    Dc = amg.coarse_operator(op, V)
    cd = amg.coarse_dims(DIMS, block)
    P = _dense_P(V, DIMS, block)
    M = amg.coarse_dense(Dc, cd)
    assert np.abs(M - P.conj().T @ D @ P).max() < 1e-13
    xc = syn.gaussian_coarse(M.shape[0] // 6, 6, 1, 4)[0]
    assert np.abs(amg.coarse_apply(Dc, xc, cd).reshape(-1) - M @ xc.reshape(-1)).max() < 1e-13
    # coarse gamma_5-hermiticity: Gamma Dc Gamma = Dc^dag, Gamma = diag(1_Nv, -1_Nv)
    G = np.kron(np.eye(M.shape[0] // 6), np.diag([1, 1, 1, -1, -1, -1]))
    assert np.abs(G @ M @ G - M.conj().T).max() < 1e-13


def test_full_basis_coarse_correction_is_exact(small):
    """N_v = 6|X|: P is unitary, so P Dc^-1 P^dag = D^-1 (the coarse step of
    the V-cycle alone solves the system)."""
    op, D = small
    V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 96, 13), DIMS, BLOCK)
    mg = amg.TwoLevel(op, V, sap_sweeps=0, coarse='exact')
    b = syn.gaussian_vectors(DIMS, 1, 14)
    x = mg.vcycle(b)
    want = np.linalg.solve(D, b.reshape(-1))
    assert np.abs(x.reshape(-1) - want).max() < 1e-11 * np.abs(want).max()


def test_bicgstab_converges_to_dense_solution(small):
    op, _ = small
    V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 4, 15), DIMS, BLOCK)
    Dc = amg.coarse_operator(op, V)
    cd = amg.coarse_dims(DIMS, BLOCK)
    M = amg.coarse_dense(Dc, cd)
    b = syn.gaussian_coarse(16, 8, 1, 5)[0]
    x, its = amg.bicgstab(lambda z: amg.coarse_apply(Dc, z[None], cd)[0], b, 200, 1e-13)
    want = np.linalg.solve(M, b.reshape(-1))
    assert its < 200
    assert np.abs(x.reshape(-1) - want).max() < 1e-10 * np.abs(want).max()
    # a non-normal test matrix where the omega stabilisation engages
    rng = np.random.default_rng(0)
    A = np.eye(60) * 2 + np.diag(rng.standard_normal(59) * 3, 1) + 0.3j * rng.standard_normal((60, 60))
    bb = rng.standard_normal(60) + 0j
    x, its = amg.bicgstab(lambda z: A @ z, bb, 500, 1e-12)
    assert np.linalg.norm(A @ x - bb) <= 1e-11 * np.linalg.norm(bb)


@pytest.mark.parametrize('smoothing', ['post', 'pre', 'both'])
def test_vcycle_error_propagator(small, smoothing):
    """With an exact coarse solve and exact block solves in SAP (both linear),
    the preconditioner's error propagator 1 - M D is the product of the
    Richardson steps' (1 - S D) for the smoother and (1 - P Dc^-1 P^dag D)
    for the coarse grid, in the order of the cycle (post: coarse grid first;
    pre: smoother first; both: smoother, coarse grid, smoother), built here
    from dense matrices."""
    op, D = small
    n = D.shape[0]
    V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 4, 16), DIMS, BLOCK)
    mg = amg.TwoLevel(op, V, sap_sweeps=2, coarse='exact', smoothing=smoothing)
    Ds = od.dense_D(op.U, op.Fb, op.kappa, BC_AP, DIMS, block=BLOCK)
    mg.smoother = lambda r: amg.sap(op, r, 2, block_solver=lambda rc: np.linalg.solve(
        Ds, rc.reshape(-1)).reshape(rc.shape))
    col = _colour_index(DIMS, BLOCK)
    Sc = []
    for c in (0, 1):
        idx = np.where(col == c)[0]
        S = np.zeros((n, n), complex)
        S[np.ix_(idx, idx)] = np.linalg.inv(D[np.ix_(idx, idx)])
        Sc.append(S)
    Esap = np.linalg.matrix_power((np.eye(n) - Sc[1] @ D) @ (np.eye(n) - Sc[0] @ D), 2)
    P = _dense_P(V, DIMS, BLOCK)
    Cc = P @ np.linalg.inv(P.conj().T @ D @ P) @ P.conj().T
    Ec = np.eye(n) - Cc @ D
    E = {'post': Esap @ Ec, 'pre': Ec @ Esap, 'both': Esap @ Ec @ Esap}[smoothing]
    v = syn.gaussian_vectors(DIMS, 1, 17)
    Mv = mg.vcycle(v).reshape(-1)
    want = (np.eye(n) - E) @ np.linalg.solve(D, v.reshape(-1))
    assert np.abs(Mv - want).max() < 1e-10 * np.abs(want).max()


def test_fgmres_is_gmres_without_preconditioner(small):
    """With M = 1 and no restart, the k-th FGMRES iterate minimises
    ||b - D y|| over the Krylov space span{b, Db, ..., D^{k-1} b}."""
    op, D = small
    b = syn.z2_source(DIMS, 1)[0]
    for k in (3, 7):
        x, its, _ = amg.fgmres(op.D, lambda v: v, b, tol=0.0, restart=50, max_iters=k)
        assert its == k
        Kr = [b.reshape(-1)]
        for _ in range(k - 1):
            Kr.append(D @ Kr[-1])
        Q, _ = np.linalg.qr(np.array(Kr).T)
        y, *_ = np.linalg.lstsq(D @ Q, b.reshape(-1), rcond=None)
        best = np.linalg.norm(b.reshape(-1) - D @ Q @ y)
        got = np.linalg.norm(b.reshape(-1) - D @ x.reshape(-1))
        assert abs(got - best) < 1e-9 * best


def test_two_level_solve_matches_dense_lu(small):
    """Config-1-like: setup then AMG-preconditioned FGMRES(16) to 1e-10; the
    solution agrees with dense LU; the paper's flexible BiCGStab as well."""
    op, D = small
    V0 = syn.gaussian_vectors(DIMS, 8, 1)
    mg = amg.setup(op, V0, n_init=3, n_adapt=3, coarse_iters=50, coarse_tol=0.1)
    P = _dense_P(mg.V, DIMS, BLOCK)
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-12
    b = syn.z2_source(DIMS, 1)[0]
    want = np.linalg.solve(D, b.reshape(-1))
    x, its, res = amg.fgmres(op.D, mg.vcycle, b, tol=1e-10, restart=16)
    assert res <= 1e-10
    cond = np.linalg.cond(D)
    assert np.linalg.norm(x.reshape(-1) - want) <= cond * 1e-10 * np.linalg.norm(want)
    _, its_plain, _ = amg.fgmres(op.D, lambda v: v, b, tol=1e-10, restart=16)
    assert its < its_plain
    x2, _, res2 = amg.flexible_bicgstab(op.D, mg.vcycle, b, tol=1e-10)
    assert res2 <= 1e-10


def test_level1_pieces_are_galerkin(small):
    """Level 1 of a three-level hierarchy: the coarse chirality Gamma commutes
    with nothing but is respected by the construction, R1 P1 = 1, and
    Dc2 = P1^dag Dc P1 by dense brute force, including extent-2 directions."""
    op, D = small
    V = amg.block_orthonormalize(syn.gaussian_vectors(DIMS, 3, 31), DIMS, BLOCK)
    Dc = amg.coarse_operator(op, V)
    cd = amg.coarse_dims(DIMS, BLOCK)  # 2^4 coarse sites, n = 6
    cop = amg.CoarseOp(Dc, cd, (1, 1, 2, 2))
    W = syn.gaussian_coarse(16, 6, 2, 32)
    W = amg.coarse_block_orthonormalize(W, cd, cop.block)
    nX2 = amg.n_blocks(cd, cop.block)
    cols = []
    for X in range(nX2):
        for k in range(4):
            e = np.zeros((nX2, 4), complex)
            e[X, k] = 1
            cols.append(amg.coarse_prolong(W, e, cd, cop.block).reshape(-1))
    P1 = np.array(cols).T
    assert np.abs(P1.conj().T @ P1 - np.eye(P1.shape[1])).max() < 1e-13
    M = amg.coarse_dense(Dc, cd)
    Dc2 = amg.coarse_coarse_operator(cop, W)
    M2 = amg.coarse_dense(Dc2, amg.coarse_dims(cd, cop.block))
    assert np.abs(M2 - P1.conj().T @ M @ P1).max() < 1e-13
    # the in-block part is the block diagonal of the dense coarse matrix
    x = syn.gaussian_coarse(16, 6, 1, 33)[0]
    bid = np.array([amg.coarse_to_blocks(np.eye(16 * 6)[i].reshape(16, 6), cd, cop.block).nonzero()[0][0]
                    for i in range(96)])
    mask = bid[:, None] == bid[None, :]
    assert np.abs(cop.Dsap(x).reshape(-1) - (M * mask) @ x.reshape(-1)).max() < 1e-13


def test_mr_global_minimises_residual():
    rng = np.random.default_rng(4)
    A = np.eye(30) * 3 + 0.4 * (rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30)))
    b = rng.standard_normal(30) + 0j
    x1 = amg.mr_global(lambda z: A @ z, b, 1)
    r1 = b - A @ x1
    assert abs(np.vdot(A @ b, r1)) < 1e-12 * np.linalg.norm(b) ** 2
    prev = np.linalg.norm(b)
    for k in range(1, 8):
        r = np.linalg.norm(b - A @ amg.mr_global(lambda z: A @ z, b, k))
        assert r <= prev * (1 + 1e-13)
        prev = r


def test_three_level_solve_matches_dense_lu(small):
    """Three levels on 4^4: level 0 blocks 2^4 (coarse 2^4, N_v 4), level 1
    blocks 1x1x2x2 (level-2 lattice 2x2x1x1, N_v 4); FGMRES(16) to 1e-10
    agrees with dense LU; with an exact level-2 solve and the level-1 cycle,
    the preconditioner still reduces the iteration count versus M = 1."""
    op, D = small
    V0 = syn.gaussian_vectors(DIMS, 4, 41)
    mg = amg.setup(op, V0, n_init=3, n_adapt=1, coarse_iters=50, coarse_tol=0.1)
    cop = amg.CoarseOp(mg.Dc, mg.cdims, (1, 1, 2, 2))
    W0 = syn.gaussian_coarse(16, 8, 4, 42)
    lv1 = amg.setup_level1(cop, W0, n_init=2, n_adapt=1)
    three = amg.ThreeLevel(op, mg.V, lv1)
    b = syn.z2_source(DIMS, 1)[0]
    x, its, res = amg.fgmres(op.D, three.vcycle, b, tol=1e-10, restart=16)
    assert res <= 1e-10
    want = np.linalg.solve(D, b.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - want) <= np.linalg.cond(D) * 1e-10 * np.linalg.norm(want)
    _, its_plain, _ = amg.fgmres(op.D, lambda v: v, b, tol=1e-10, restart=16)
    assert its < its_plain


# ---------------------------------------------------------------- the omega stabilisation of step (1b)
def _first_step(A, b):
    """alpha, s and t of the first BiCGStab step from x = 0 (p = r = r~ = b)."""
    v = A @ b
    alpha = np.vdot(b, b) / np.vdot(b, v)
    s = b - alpha * v
    return alpha, s, A @ s


def _rotations(n2, cos_t):
    c, d = cos_t, np.sqrt(1 - cos_t ** 2)
    return np.kron(np.eye(n2), np.array([[c, -d], [d, c]])).astype(complex)


@pytest.mark.parametrize('case', ['rot50', 'rot90pct', 'nonnormal'])
def test_bicgstab_omega_stabilisation_residual_ratio(case):
    """After one step from x = 0 the residual is s - omega t.  With the
    minimising omega = <t,s>/<t,t> its squared norm relative to ||s||^2 is
    1 - rho^2, rho = |cos(t, s)|.  Sleijpen and van der Vorst enlarge omega
    by stab/rho whenever rho < stab = 0.7, which makes the ratio
    1 - 2 (0.7 rho) + 0.7^2 = 1.49 - 1.4 rho.  Both branches are checked, and
    that the enlarged one differs from the plain one."""
    rng = np.random.default_rng(5)
    if case == 'rot50':
        A, b = _rotations(20, 0.5), rng.standard_normal(40) + 0j  # rho = 0.5 exactly
    elif case == 'rot90pct':
        A, b = _rotations(20, 0.9), rng.standard_normal(40) + 0j  # rho = 0.9: no enlargement
    else:
        A = (np.diag(np.exp(2j * np.pi * rng.random(50))) + 0.2 * np.diag(rng.standard_normal(49), 1)
             + 0.05 * (rng.standard_normal((50, 50)) + 1j * rng.standard_normal((50, 50))))
        b = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    _, s, t = _first_step(A, b)
    rho = abs(np.vdot(t, s)) / (np.linalg.norm(t) * np.linalg.norm(s))
    x1, its = amg.bicgstab(lambda z: A @ z, b, 1)
    assert its == 1
    ratio = np.linalg.norm(b - A @ x1) ** 2 / np.linalg.norm(s) ** 2
    if case == 'rot50':
        assert abs(rho - 0.5) < 1e-12
    if case == 'rot90pct':
        assert abs(rho - 0.9) < 1e-12
        assert abs(ratio - (1 - rho ** 2)) < 1e-12
    else:
        assert rho < 0.7  # the stabilisation engages
        assert abs(ratio - (1.49 - 1.4 * rho)) < 1e-12
        assert abs(ratio - (1 - rho ** 2)) > 1e-3


def test_bicgstab_stops_when_t_is_orthogonal_to_s():
    """<t, s> = 0 with t != 0: the minimising omega is 0 and the enlarged one
    undefined (0 * 0.7 / 0); the next beta would divide by omega.  The
    solver keeps x + alpha p and stops instead of producing a NaN.  The
    operator is a stub returning chosen vectors: v = (1, 1) for p = b =
    (1, 0) gives alpha = 1 and s = (0, -1); t = (1, 0) is orthogonal to s."""
    calls = []

    def stub(z):
        calls.append(z.copy())
        return np.array([1.0 + 0j, 1.0]) if len(calls) == 1 else np.array([1.0 + 0j, 0.0])

    b = np.array([1.0 + 0j, 0.0])
    x, its = amg.bicgstab(stub, b, 5)
    assert len(calls) == 2 and its == 1
    assert np.all(np.isfinite(x)) and np.abs(x - b).max() == 0.0


# ---------------------------------------------------------------- setup (0-a), (0-b) as dense algebra
def _block_qr(V, dims, block):
    """Per block X and chirality s, the QR factorisation of the columns
    P_s v_i restricted to X in the order i = 1..N_v, with a positive real R
    diagonal (numpy's Householder QR, signs fixed)."""
    Vb = amg.to_blocks(V, dims, block)
    out = np.empty_like(Vb)
    for X in range(Vb.shape[1]):
        for s in (0, 1):
            q, r = np.linalg.qr(Vb[:, X, s, :].T)
            out[:, X, s, :] = (q * (np.diag(r) / np.abs(np.diag(r)))).T
    return amg.from_blocks(out, dims, block)


def test_setup_equals_dense_construction(small):
    """With exact SAP block solves and an exact coarse solve every step of the
    setup is linear algebra that can be written with dense matrices:
      (0-a) SAP = (1 - E_sap) D^-1 with E_sap = [(1 - S_o D)(1 - S_e D)]^n
            (red-black block Gauss-Seidel, S_c the inverse of D on the
            colour-c domains), applied n_init times to V0, then a blockwise QR;
      (0-b) M = (1 - E_sap (1 - P (P^dag D P)^-1 P^dag D)) D^-1 (coarse grid
            then smoother) applied to every vector, then the blockwise QR,
            n_adapt times, P rebuilt from the new vectors each time.
    The oracle's setup must give the same vectors."""
    op, D = small
    n = D.shape[0]
    sweeps, n_init, n_adapt, nv = 2, 2, 2, 4
    col = _colour_index(DIMS, BLOCK)
    S = []
    for c in (0, 1):
        idx = np.where(col == c)[0]
        Sc = np.zeros((n, n), complex)
        Sc[np.ix_(idx, idx)] = np.linalg.inv(D[np.ix_(idx, idx)])
        S.append(Sc)
    I = np.eye(n)
    Esap = np.linalg.matrix_power((I - S[1] @ D) @ (I - S[0] @ D), sweeps)
    Dinv = np.linalg.inv(D)
    Msap = (I - Esap) @ Dinv
    V0 = syn.gaussian_vectors(DIMS, nv, 61)
    shp = V0.shape
    W = V0.reshape(nv, n).T
    for _ in range(n_init):
        W = Msap @ W
    V = _block_qr(W.T.reshape(shp), DIMS, BLOCK)
    for _ in range(n_adapt):
        P = _dense_P(V, DIMS, BLOCK)
        Ec = I - P @ np.linalg.solve(P.conj().T @ D @ P, P.conj().T @ D)
        M = (I - Esap @ Ec) @ Dinv
        V = _block_qr((M @ V.reshape(nv, n).T).T.reshape(shp), DIMS, BLOCK)

    Ds_inv = np.linalg.inv(od.dense_D(op.U, op.Fb, op.kappa, BC_AP, DIMS, block=BLOCK))

    def exact_block(rc):
        return (Ds_inv @ rc.reshape(-1, n).T).T.reshape(rc.shape)

    mg = amg.setup(op, V0, n_init=n_init, n_adapt=n_adapt, sap_sweeps=sweeps, coarse='exact',
                   block_solver=exact_block)
    assert np.abs(mg.V - V).max() < 1e-9 * np.abs(V).max()


# ---------------------------------------------------------------- even-odd block solve
def test_eo_schur_complement_matches_dense(small):
    """The even-odd block solve's first MR step, in closed form: with one
    iteration x_e = alpha c_e, alpha = <S c, c>/<S c, S c> per domain, where
    S and c = b_e - H_eo A_o^-1 b_o are built here from the dense D_SAP by
    parity blocks and a dense inverse of A_o."""
    op, _ = small
    Ds = od.dense_D(op.U, op.Fb, op.kappa, BC_AP, DIMS, block=BLOCK)
    par = np.broadcast_to(amg.site_parity(DIMS), syn.shape_of(DIMS) + (4, 3)).reshape(-1)
    e, o = np.where(par == 0)[0], np.where(par == 1)[0]
    S = Ds[np.ix_(e, e)] - Ds[np.ix_(e, o)] @ np.linalg.solve(Ds[np.ix_(o, o)], Ds[np.ix_(o, e)])
    b = syn.gaussian_vectors(DIMS, 1, 31)[0]
    bf = b.reshape(-1)
    c = bf[e] - Ds[np.ix_(e, o)] @ np.linalg.solve(Ds[np.ix_(o, o)], bf[o])
    Sc = S @ c
    # per-domain alpha from the dense vectors
    blk = amg.to_blocks(np.arange(bf.size).reshape(b.shape), DIMS, BLOCK)  # flat index per (X, s, k)
    xe = np.zeros(bf.size, complex)
    pos = {int(i): j for j, i in enumerate(e)}
    for X in range(blk.shape[0]):
        idx = [pos[int(i)] for i in blk[X].reshape(-1) if int(i) in pos]
        a = np.vdot(Sc[idx], c[idx]) / np.vdot(Sc[idx], Sc[idx])
        xe[e[idx]] = a * c[idx]
    xo = np.zeros(bf.size, complex)
    xo[o] = np.linalg.solve(Ds[np.ix_(o, o)], bf[o] - Ds[np.ix_(o, e)] @ xe[e])
    x1, r1 = amg.eo_mr_domains(op, b, 1)
    assert np.abs(x1.reshape(-1) - (xe + xo)).max() < 1e-12
    # the odd sites' residual vanishes (exact A_o^-1)
    assert np.abs(r1.reshape(-1)[o]).max() < 1e-12
    assert np.abs(r1 - (b - op.Dsap(x1))).max() == 0


def test_eo_block_solve_converges_to_dense_block_inverse(small):
    """Many even-odd MR iterations solve the block system: x -> D_SAP^-1 b."""
    op, _ = small
    Ds = od.dense_D(op.U, op.Fb, op.kappa, BC_AP, DIMS, block=BLOCK)
    b = syn.gaussian_vectors(DIMS, 1, 32)[0]
    want = np.linalg.solve(Ds, b.reshape(-1))
    x, r = amg.eo_mr_domains(op, b, 60)
    assert np.linalg.norm(x.reshape(-1) - want) / np.linalg.norm(want) < 1e-10
    # and it converges faster per iteration than plain MR on D_SAP
    xe6, re6 = amg.eo_mr_domains(op, b, 6)
    xm6, rm6 = amg.mr_domains(op, b, 6)
    assert np.linalg.norm(re6) < np.linalg.norm(rm6)


def test_eo_sap_with_exact_block_solves_is_block_gauss_seidel(small):
    """SAP with the even-odd block solve iterated to convergence equals SAP
    with exact block solves (the dense red-black block Gauss-Seidel)."""
    op, _ = small
    b = syn.gaussian_vectors(DIMS, 1, 33)[0]
    Ds_inv = np.linalg.inv(od.dense_D(op.U, op.Fb, op.kappa, BC_AP, DIMS, block=BLOCK))
    exact = amg.sap(op, b, 2, block_solver=lambda r: (Ds_inv @ r.reshape(-1)).reshape(r.shape))
    eo = amg.sap(op, b, 2, block_solver=lambda r: amg.eo_mr_domains(op, r, 80)[0])
    assert np.abs(eo - exact).max() / np.abs(exact).max() < 1e-10
