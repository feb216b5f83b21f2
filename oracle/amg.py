"""Oracle: the multigrid method of Sec. 3 in plain NumPy FP64.

Objects and the passages they follow:
  * minimal-residual block solve (SAP paragraph: "MINRES" with a fixed number
    of iterations; read as MR because D_SAP is not Hermitian), and as a
    variant the same MR on the even-odd Schur complement of each domain;
  * SAP with fixed iterations (the SAP listing of Sec. 3): domains = the
    multigrid blocks, even/odd domain colour = parity of the sum of the block
    coordinates, even colour first;
  * block orthonormalisation <I|J> = delta_IJ over I = (X, s, i) (Sec. 3,
    construction of the coarse grid operator), by modified Gram-Schmidt
    applied twice in the order i = 1..N_nv;
  * restriction eq. (5), prolongation eq. (6), coarse operator eq. (7);
  * coarse solve: BiCGStab with the Sleijpen-van der Vorst stabilisation of
    omega (step (1b));
  * the preconditioner M = (1) coarse refinement then (2) SAP smoother
    (numerical steps (1)-(2));
  * setup (0-a) and (0-b);
  * outer solver: flexible GMRES(m) in FP64 (right preconditioning, classical
    Gram-Schmidt applied twice); the paper's own outer solver, flexible
    BiCGStab (Sec. 3 listing), is also given.

Coarse vector layout: [..., X, 2 N_v] with X the coarse site index
X_x + N_x (X_y + N_y (X_z + N_z X_t)) and internal index s*N_v + i (s = 0 for
P_+ = spins {0, 1}, s = 1 for P_- = spins {2, 3}).  The coarse operator is
stored as 9 blocks per coarse site, Dc[X, d, n, m] = <X,n| D |X+e_d, m> with
d = 0 (self), 1+mu (forward mu), 5+mu (backward mu); hops that reach the same
neighbour block (extent 2) stay in separate blocks and are summed on use.

Pins (tests/test_oracle_amg.py): MR's one-step optimality and monotone
residual; the even-odd variant's Schur complement against the dense one, its
zero odd-site residual and its convergence to the dense block solve; SAP with exact block solves equal to the dense red-black block
Gauss-Seidel iteration, and its convergence to D^-1 b; orthonormality, span
and agreement with a sign-fixed library QR; R P = 1, P R an orthogonal
projector, Dc = P^dag D P by dense brute force, coarse gamma_5-hermiticity,
exactness of the coarse correction with a full local basis; BiCGStab
converging to the dense solve, its first step's residual reduction
1.49 - 1.4 |cos(t, s)| when the omega enlargement engages (1 - cos^2 when it
does not), and its stop at <t, s> = 0; the V-cycle's error propagator against
its dense product form; the whole setup (0-a)/(0-b), with exact block and
coarse solves, against the same steps written as dense matrix products and
blockwise QR; FGMRES against dense LU and, with M = 1, against the
minimal-residual property of GMRES over the dense Krylov space.
"""
import numpy as np

from . import dirac

NDIR = 9


# ----------------------------------------------------------------------------
# Block geometry
# ----------------------------------------------------------------------------
def coarse_dims(dims, block):
    for mu in range(4):
        if dims[mu] % block[mu]:
            raise ValueError('block does not divide the lattice')
    return tuple(dims[mu] // block[mu] for mu in range(4))


def n_blocks(dims, block):
    return int(np.prod(coarse_dims(dims, block)))


def to_blocks(v, dims, block):
    """[..., Lt,Lz,Ly,Lx,4,3] -> [..., X, s, k]: per block X and chirality s the
    6|X| components, ordered (site in block t,z,y,x; spin in chirality; colour)."""
    lead = v.shape[:-6]
    nx, ny, nz, nt = coarse_dims(dims, block)
    bx, by, bz, bt = block
    L = len(lead)
    a = v.reshape(lead + (nt, bt, nz, bz, ny, by, nx, bx, 2, 2, 3))
    perm = list(range(L)) + [L + i for i in (0, 2, 4, 6, 8, 1, 3, 5, 7, 9, 10)]
    a = a.transpose(perm)
    return a.reshape(lead + (nt * nz * ny * nx, 2, 6 * bx * by * bz * bt))


def from_blocks(b, dims, block):
    lead = b.shape[:-3]
    nx, ny, nz, nt = coarse_dims(dims, block)
    bx, by, bz, bt = block
    L = len(lead)
    a = b.reshape(lead + (nt, nz, ny, nx, 2, bt, bz, by, bx, 2, 3))
    # current order: nt nz ny nx s bt bz by bx sl c -> nt bt nz bz ny by nx bx s sl c
    perm = list(range(L)) + [L + i for i in (0, 5, 1, 6, 2, 7, 3, 8, 4, 9, 10)]
    a = a.transpose(perm)
    lx, ly, lz, lt = dims
    return a.reshape(lead + (lt, lz, ly, lx, 4, 3))


def domain_colour(dims, block):
    """Per-site colour (0 even, 1 odd) of its domain: parity of the sum of the
    block coordinates.  Shaped [Lt,Lz,Ly,Lx,1,1]."""
    cs = []
    for mu in range(4):
        c = np.arange(dims[mu]) // block[mu]
        shp = [1, 1, 1, 1]
        shp[3 - mu] = dims[mu]
        cs.append(c.reshape(shp))
    col = (cs[0] + cs[1] + cs[2] + cs[3]) % 2
    return col[..., None, None]


def check_sap_geometry(dims, block):
    cd = coarse_dims(dims, block)
    if any(c % 2 for c in cd):
        raise ValueError('SAP colouring needs an even number of domains per direction')


def domain_sums(f, dims, block):
    """Sum of f over each domain: [..., Lt,Lz,Ly,Lx,4,3] -> [..., nt,1,nz,1,ny,1,nx,1,1,1]."""
    lead = f.shape[:-6]
    nx, ny, nz, nt = coarse_dims(dims, block)
    bx, by, bz, bt = block
    a = f.reshape(lead + (nt, bt, nz, bz, ny, by, nx, bx, 12))
    L = len(lead)
    return a.sum(axis=(L + 1, L + 3, L + 5, L + 7, L + 8), keepdims=True)


def _per_domain(f, d, dims, block):
    """Multiply field f by per-domain scalars d (from domain_sums)."""
    lead = f.shape[:-6]
    nx, ny, nz, nt = coarse_dims(dims, block)
    bx, by, bz, bt = block
    a = f.reshape(lead + (nt, bt, nz, bz, ny, by, nx, bx, 12))
    return (a * d).reshape(f.shape)


# ----------------------------------------------------------------------------
# Fine operator bundle
# ----------------------------------------------------------------------------
class FineOp:
    """The operator of eq. (1) with its domain decomposition."""

    def __init__(self, U, Fb, kappa, bc, block):
        self.U, self.Fb, self.kappa, self.bc = U, Fb, kappa, tuple(bc)
        self.block = tuple(block)
        self.dims = (U.shape[4], U.shape[3], U.shape[2], U.shape[1])

    def D(self, psi):
        return dirac.apply_D(self.U, self.Fb, psi, self.kappa, self.bc)

    def Dsap(self, psi):
        return dirac.apply_Dsap(self.U, self.Fb, psi, self.kappa, self.bc, self.block)

    def hop_cross(self, psi, mu, sign):
        return dirac.apply_hop_cross(self.U, psi, mu, sign, self.kappa, self.bc, self.block)


# ----------------------------------------------------------------------------
# SAP smoother (Sec. 3, SAP paragraph and listing)
# ----------------------------------------------------------------------------
def mr_domains(op, b, iters):
    """Minimal-residual iterations on D_SAP, independently in every domain,
    from x = 0:  p = A r;  alpha = <p, r> / <p, p>;  x += alpha r;  r -= alpha p,
    with the inner products taken over each domain.  Returns (x, r)."""
    x = np.zeros_like(b)
    r = b.copy()
    for _ in range(iters):
        p = op.Dsap(r)
        pr = domain_sums(np.conj(p) * r, op.dims, op.block)
        pp = domain_sums(np.abs(p) ** 2, op.dims, op.block).real
        alpha = np.where(pp > 0, pr / np.where(pp > 0, pp, 1.0), 0.0)
        x = x + _per_domain(r, alpha, op.dims, op.block)
        r = r - _per_domain(p, alpha, op.dims, op.block)
    return x, r


def site_parity(dims):
    """Per-site parity (x + y + z + t) mod 2, shaped [Lt,Lz,Ly,Lx,1,1]."""
    cs = []
    for mu in range(4):
        shp = [1, 1, 1, 1]
        shp[3 - mu] = dims[mu]
        cs.append(np.arange(dims[mu]).reshape(shp))
    return ((cs[0] + cs[1] + cs[2] + cs[3]) % 2)[..., None, None]


def clover_inverse(Fb):
    """Per-site inverse of the site-local part 1 + F(x), as its two chiral
    6x6 blocks (like the clover field)."""
    return np.linalg.inv(np.eye(6) + Fb)


def eo_mr_domains(op, b, iters, Ainv=None):
    """Even-odd preconditioned MR block solve on every domain (the smoother
    variant of the SAP block solve).  In a domain, D_SAP splits by site
    parity into [[A_e, H_eo], [H_oe, A_o]] with A = 1 + F (site-local) and H
    the in-domain hops.  With the Schur complement S = A_e - H_eo A_o^-1 H_oe
    on the even sites:
        c_e = b_e - H_eo A_o^-1 b_o,
        x_e = MR(iters) on S x_e = c_e from 0 (domain inner products over
              the even sites),
        x_o = A_o^-1 (b_o - H_oe x_e).
    Ainv: the per-site blocks used for A^-1 (default: the exact inverse).
    Returns (x, r) with r = b - D_SAP x, the block solve's true residual."""
    dims, block = op.dims, op.block
    if Ainv is None:
        Ainv = clover_inverse(op.Fb)
    odd = site_parity(dims) == 1

    def ev(f):
        return np.where(odd, 0.0, f)

    def od(f):
        return np.where(odd, f, 0.0)

    def A(f):
        return f + dirac.clover_apply(op.Fb, f)

    def Ai(f):
        return dirac.clover_apply(Ainv, f)

    def H(f):
        return op.Dsap(f) - A(f)

    def S(v):
        return ev(A(v)) - ev(H(od(Ai(od(H(v))))))

    c = ev(b) - ev(H(od(Ai(od(b)))))
    xe = np.zeros_like(b)
    r = c
    for _ in range(iters):
        p = S(r)
        pr = domain_sums(np.conj(p) * r, dims, block)
        pp = domain_sums(np.abs(p) ** 2, dims, block).real
        alpha = np.where(pp > 0, pr / np.where(pp > 0, pp, 1.0), 0.0)
        xe = xe + _per_domain(r, alpha, dims, block)
        r = r - _per_domain(p, alpha, dims, block)
    xo = od(Ai(od(b) - od(H(xe))))
    x = xe + xo
    return x, b - op.Dsap(x)


def sap(op, b, sweeps=4, mr_iters=6, block_solver=None):
    """SAP with fixed iterations, as the listing: x = 0, r = b; for each sweep:
    x += M_e r; r = b - D x; x += M_o r; r = b - D x.  M_{e/o} is the block
    solve on the domains of one colour (MR with mr_iters iterations, or the
    given block_solver(r_restricted) -> x)."""
    check_sap_geometry(op.dims, op.block)
    col = domain_colour(op.dims, op.block)
    x = np.zeros_like(b)
    r = b.copy()
    for _ in range(sweeps):
        for c in (0, 1):
            rc = np.where(col == c, r, 0.0)
            if block_solver is None:
                dx, _ = mr_domains(op, rc, mr_iters)
            else:
                dx = block_solver(rc)
            x = x + np.where(col == c, dx, 0.0)
            r = b - op.D(x)
    return x


# ----------------------------------------------------------------------------
# Test-vector basis, restriction, prolongation (eqs. (5), (6))
# ----------------------------------------------------------------------------
def block_orthonormalize(V, dims, block, passes=2):
    """Orthonormalise, for every block X and chirality s separately, the
    vectors P_s v_i restricted to X, in the order i = 1..N_v (modified
    Gram-Schmidt, repeated `passes` times).  V: [Nv, Lt,Lz,Ly,Lx,4,3]."""
    Vb = to_blocks(V, dims, block).copy()
    nv = Vb.shape[0]
    for _ in range(passes):
        for i in range(nv):
            for k in range(i):
                c = np.sum(np.conj(Vb[k]) * Vb[i], axis=-1)
                Vb[i] -= c[..., None] * Vb[k]
            nrm = np.sqrt(np.sum(np.abs(Vb[i]) ** 2, axis=-1))
            Vb[i] /= nrm[..., None]
    return from_blocks(Vb, dims, block)


def restrict(V, x, dims, block):
    """eq. (5): x_c(X, s, i) = <X, s, i | x>.  x: [..., fine] -> [..., X, 2Nv]."""
    Vb = to_blocks(V, dims, block)
    xb = to_blocks(x, dims, block)
    xc = np.einsum('ixsk,...xsk->...xsi', np.conj(Vb), xb)
    return xc.reshape(xc.shape[:-2] + (2 * V.shape[0],))


def prolong(V, xc, dims, block):
    """eq. (6): x'(y) = sum_I x_c(I) |I>(y)."""
    nv = V.shape[0]
    Vb = to_blocks(V, dims, block)
    c = xc.reshape(xc.shape[:-1] + (2, nv))
    xb = np.einsum('ixsk,...xsi->...xsk', Vb, c)
    return from_blocks(xb, dims, block)


# ----------------------------------------------------------------------------
# Coarse operator (eq. (7)) and its application
# ----------------------------------------------------------------------------
def coarse_operator(op, V):
    """Dc[X, d, (s,i), (s',j)] = <X,s,i| D |X+e_d, s',j>, built from D_SAP
    (self block) and the domain-crossing hops (8 neighbour blocks) applied to
    the vectors P_{s'} v_j and restricted."""
    nv = V.shape[0]
    nX = n_blocks(op.dims, op.block)
    n = 2 * nv
    Dc = np.zeros((nX, NDIR, n, n), np.complex128)
    for sp in (0, 1):
        W = dirac.chiral_project(V, sp)
        cols = slice(sp * nv, (sp + 1) * nv)
        Y = op.Dsap(W)
        Dc[:, 0, :, cols] = np.transpose(restrict(V, Y, op.dims, op.block), (1, 2, 0))
        for mu in range(4):
            for sign, d in ((+1, 1 + mu), (-1, 5 + mu)):
                Y = op.hop_cross(W, mu, sign)
                Dc[:, d, :, cols] = np.transpose(restrict(V, Y, op.dims, op.block), (1, 2, 0))
    return Dc


def coarse_shift(xc, cdims, mu, sign):
    """g(X) = xc(X + sign e_mu) on the periodic coarse lattice; xc [..., X, n]."""
    lead = xc.shape[:-2]
    nx, ny, nz, nt = cdims
    a = xc.reshape(lead + (nt, nz, ny, nx, xc.shape[-1]))
    a = np.roll(a, -sign, axis=-2 - mu)
    return a.reshape(xc.shape)


def coarse_apply(Dc, xc, cdims):
    """y(X) = sum_d Dc(X, X+e_d) x(X+e_d)."""
    y = np.einsum('xnm,...xm->...xn', Dc[:, 0], xc)
    for mu in range(4):
        for sign, d in ((+1, 1 + mu), (-1, 5 + mu)):
            y = y + np.einsum('xnm,...xm->...xn', Dc[:, d], coarse_shift(xc, cdims, mu, sign))
    return y


def coarse_dense(Dc, cdims):
    """The coarse operator as one dense matrix (small lattices only)."""
    nX, _, n, _ = Dc.shape
    M = np.zeros((nX * n, nX * n), np.complex128)
    nx, ny, nz, nt = cdims
    for X in range(nX):
        c = [X % nx, (X // nx) % ny, (X // (nx * ny)) % nz, X // (nx * ny * nz)]
        M[X * n:(X + 1) * n, X * n:(X + 1) * n] += Dc[X, 0]
        for mu in range(4):
            for sign, d in ((+1, 1 + mu), (-1, 5 + mu)):
                cc = list(c)
                cc[mu] = (c[mu] + sign) % cdims[mu]
                Y = cc[0] + nx * (cc[1] + ny * (cc[2] + nz * cc[3]))
                M[X * n:(X + 1) * n, Y * n:(Y + 1) * n] += Dc[X, d]
    return M


# ----------------------------------------------------------------------------
# Coarse solve (step (1b)): BiCGStab with the stabilised omega
# ----------------------------------------------------------------------------
def bicgstab(apply_A, b, iters, tol=0.0, stab=0.7):
    """BiCGStab from x = 0 for one right-hand side, at most `iters`
    iterations, stopping once ||r|| <= tol ||b||.  The omega of each step is
    enlarged to omega * stab / |cos(t, s)| whenever |cos(t, s)| < stab
    (Sleijpen and van der Vorst's stabilisation).  Stops, keeping its current
    iterate, on a zero denominator (<r~, r>, <r~, v>, <t, t> or <t, s>).
    Returns (x, iterations done)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.sqrt(np.vdot(b, b).real)
    if bn == 0:
        return x, 0
    rt = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    done = 0
    for it in range(iters):
        rho = np.vdot(rt, r)
        if rho == 0:
            break
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        rv = np.vdot(rt, v)
        if rv == 0:
            break
        alpha = rho / rv
        s = r - alpha * v
        t = apply_A(s)
        ts = np.vdot(t, s)
        tt = np.vdot(t, t).real
        ss = np.vdot(s, s).real
        if tt == 0 or ts == 0:
            # t = 0, or t orthogonal to s: omega = <t,s>/<t,t> is 0 and the
            # stabilised omega would be 0 * stab / 0; the next beta divides by
            # omega, so this is a breakdown: keep x + alpha p and stop
            x = x + alpha * p
            done = it + 1
            break
        omega = ts / tt
        cosang = abs(ts) / np.sqrt(tt * ss) if ss > 0 else 1.0
        if cosang < stab:
            omega = omega * stab / cosang
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        done = it + 1
        if np.sqrt(np.vdot(r, r).real) <= tol * bn:
            break
    return x, done


# ----------------------------------------------------------------------------
# Two-level hierarchy, V-cycle, setup
# ----------------------------------------------------------------------------
class TwoLevel:
    """Fine operator + test vectors + coarse operator + preconditioner
    parameters.  coarse='bicgstab' uses the stabilised BiCGStab with
    (coarse_iters, coarse_tol); coarse='exact' a dense solve (for pins)."""

    def __init__(self, op, V, sap_sweeps=4, mr_iters=6, coarse_iters=50, coarse_tol=0.1,
                 coarse='bicgstab', smoothing='post', block_solver=None):
        self.op, self.V = op, V
        self.block_solver = block_solver
        assert smoothing in ('post', 'pre', 'both')
        self.smoothing = smoothing
        self.sap_sweeps, self.mr_iters = sap_sweeps, mr_iters
        self.coarse_iters, self.coarse_tol, self.coarse = coarse_iters, coarse_tol, coarse
        self.cdims = coarse_dims(op.dims, op.block)
        self.Dc = coarse_operator(op, V)
        self._lu = None

    def R(self, x):
        return restrict(self.V, x, self.op.dims, self.op.block)

    def P(self, xc):
        return prolong(self.V, xc, self.op.dims, self.op.block)

    def Dc_apply(self, xc):
        return coarse_apply(self.Dc, xc, self.cdims)

    def coarse_solve(self, bc):
        """Solve Dc x = b for every right-hand side (bc: [..., X, n])."""
        shp = bc.shape
        flat = bc.reshape((-1,) + shp[-2:])
        if self.coarse == 'exact':
            if self._lu is None:
                self._lu = coarse_dense(self.Dc, self.cdims)
            sol = np.linalg.solve(self._lu, flat.reshape(flat.shape[0], -1).T).T
            return sol.reshape(shp)
        out = np.zeros_like(flat)
        for k in range(flat.shape[0]):
            out[k], _ = bicgstab(lambda z: self.Dc_apply(z), flat[k],
                                 self.coarse_iters, self.coarse_tol)
        return out.reshape(shp)

    def smoother(self, r):
        if self.sap_sweeps == 0:
            return np.zeros_like(r)
        return sap(self.op, r, self.sap_sweeps, self.mr_iters, self.block_solver)

    def coarse_correction(self, r):
        """M_1 r: (1a) restrict, (1b) coarse solve, (1c) prolong."""
        return self.P(self.coarse_solve(self.R(r)))

    def vcycle(self, v):
        """M v as Richardson steps x <- x + M_i (v - D x) from x = 0 (Sec. 3).
        'post' (the paper's choice): the coarse-grid step M_1, then the SAP
        smoother M_2; 'pre': M_2 first, then M_1; 'both': M_2, M_1, M_2 (the
        smoother before and after the coarse solve, which Sec. 3 allows)."""
        steps = {'post': (self.coarse_correction, self.smoother),
                 'pre': (self.smoother, self.coarse_correction),
                 'both': (self.smoother, self.coarse_correction, self.smoother)}[self.smoothing]
        x = steps[0](v)
        for M in steps[1:]:
            x = x + M(v - self.op.D(x))
        return x


def setup(op, V0, n_init=3, n_adapt=3, sap_sweeps=4, mr_iters=6, coarse_iters=50,
          coarse_tol=0.1, smoothing='post', coarse='bicgstab', block_solver=None):
    """Setup stage (0): (0-a) SAP applied n_init times to the random start
    vectors as an approximate D^-1, block orthonormalisation, coarse operator;
    (0-b) n_adapt times: every vector replaced by M v with the current
    preconditioner, then re-orthonormalised and the coarse operator rebuilt.
    coarse and block_solver select the coarse solve and the SAP block solve
    as in TwoLevel and sap (default: stabilised BiCGStab and MR)."""
    V = V0.copy()
    for _ in range(n_init):
        V = sap(op, V, sap_sweeps, mr_iters, block_solver)
    V = block_orthonormalize(V, op.dims, op.block)
    kw = dict(smoothing=smoothing, coarse=coarse, block_solver=block_solver)
    mg = TwoLevel(op, V, sap_sweeps, mr_iters, coarse_iters, coarse_tol, **kw)
    for _ in range(n_adapt):
        V = mg.vcycle(V)
        V = block_orthonormalize(V, op.dims, op.block)
        mg = TwoLevel(op, V, sap_sweeps, mr_iters, coarse_iters, coarse_tol, **kw)
    return mg


# ----------------------------------------------------------------------------
# Outer solvers
# ----------------------------------------------------------------------------
def fgmres(apply_D, apply_M, b, tol=1e-10, restart=16, max_iters=1000):
    """Flexible GMRES(restart) from x = 0 with right preconditioning and
    classical Gram-Schmidt applied twice, for one right-hand side.  At every
    restart the residual is recomputed as b - D x.  Returns (x, iterations,
    true relative residual)."""
    shp = b.shape
    bf = b.reshape(-1)
    bn = np.linalg.norm(bf)
    x = np.zeros_like(bf)
    if bn == 0:
        return x.reshape(shp), 0, 0.0
    r = bf.copy()
    its = 0
    while True:
        beta = np.linalg.norm(r)
        if beta <= tol * bn or its >= max_iters:
            break
        m = restart
        Vk = np.zeros((m + 1, bf.size), np.complex128)
        Zk = np.zeros((m, bf.size), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        Vk[0] = r / beta
        k = 0
        for j in range(m):
            Zk[j] = apply_M(Vk[j].reshape(shp)).reshape(-1)
            w = apply_D(Zk[j].reshape(shp)).reshape(-1)
            h = Vk[:j + 1].conj() @ w
            w = w - Vk[:j + 1].T @ h
            h2 = Vk[:j + 1].conj() @ w
            w = w - Vk[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0:
                Vk[j + 1] = w / hn
            # Givens rotations: c real, s complex, [c s; -conj(s) c]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            elif abs(a) == 0:
                cs[j], sn[j] = 0.0, np.conj(bb) / abs(bb)
            else:
                cs[j], sn[j] = abs(a) / den, (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) <= tol * bn or hn == 0 or its >= max_iters:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Zk[:k].T @ y
        r = bf - apply_D(x.reshape(shp)).reshape(-1)
    return x.reshape(shp), its, np.linalg.norm(r) / bn


def flexible_bicgstab(apply_D, apply_M, b, tol=1e-10, max_iters=1000):
    """BiCGStab with flexible preconditioning (Sec. 3 listing, Vogel 2007),
    x0 = 0, shadow vector r~ = r0, with the two break points of the listing.
    The garbled last line of the listing is taken as
    p <- r_{i+1} + beta (p_i - omega_i D M p_i)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.sqrt(np.vdot(b, b).real)
    rt = r.copy()
    p = r.copy()
    its = 0
    while its < max_iters:
        Mp = apply_M(p)
        DMp = apply_D(Mp)
        rr = np.vdot(rt, r)
        alpha = rr / np.vdot(rt, DMp)
        x = x + alpha * Mp
        s = r - alpha * DMp
        its += 1
        if np.sqrt(np.vdot(s, s).real) <= tol * bn:
            break
        Ms = apply_M(s)
        t = apply_D(Ms)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + omega * Ms
        r = s - omega * t
        if np.sqrt(np.vdot(r, r).real) <= tol * bn:
            break
        beta = (alpha / omega) * np.vdot(rt, r) / rr
        p = r + beta * (p - omega * DMp)
    res = b - apply_D(x)
    return x, its, np.sqrt(np.vdot(res, res).real) / bn


# ----------------------------------------------------------------------------
# Multi-level extension (Sec. 3: "a multi-level implementation is
# straightforward").  The level-1 operator is the 9-point block stencil Dc on
# the coarse lattice with n = 2 N_v dof per site; its chirality is
# Gamma = diag(1_{N_v}, -1_{N_v}) (the coarse image of gamma_5), so the two
# halves of the dof play the role of the spins {0,1} / {2,3}.  Level-1 blocks
# aggregate coarse sites exactly as level-0 blocks aggregate fine sites.
# Reading (the paper gives no details): the level-1 smoother is `mr1_iters`
# global minimal-residual iterations on Dc, the level-1 cycle is a V-cycle, and
# the coarsest solve is the stabilised BiCGStab.
# ----------------------------------------------------------------------------
def coarse_to_blocks(v, cdims, block):
    """[..., X (cdims), n] -> [..., X2, s, k]: per level-1 block X2 and half s
    the (n/2)|X2| components, ordered (site in block t,z,y,x; dof in half)."""
    lead = v.shape[:-2]
    n = v.shape[-1]
    nx, ny, nz, nt = coarse_dims(cdims, block)
    bx, by, bz, bt = block
    L = len(lead)
    a = v.reshape(lead + (nt, bt, nz, bz, ny, by, nx, bx, 2, n // 2))
    perm = list(range(L)) + [L + i for i in (0, 2, 4, 6, 8, 1, 3, 5, 7, 9)]
    a = a.transpose(perm)
    return a.reshape(lead + (nt * nz * ny * nx, 2, (n // 2) * bx * by * bz * bt))


def coarse_from_blocks(b, cdims, block, n):
    lead = b.shape[:-3]
    nx, ny, nz, nt = coarse_dims(cdims, block)
    bx, by, bz, bt = block
    L = len(lead)
    a = b.reshape(lead + (nt, nz, ny, nx, 2, bt, bz, by, bx, n // 2))
    perm = list(range(L)) + [L + i for i in (0, 5, 1, 6, 2, 7, 3, 8, 4, 9)]
    a = a.transpose(perm)
    return a.reshape(lead + (int(np.prod(cdims)), n))


class CoarseOp:
    """The level-1 operator (block stencil Dc on cdims) with a level-1 block
    decomposition; provides the same interface as FineOp on coarse vectors
    [..., X, n]."""

    def __init__(self, Dc, cdims, block):
        self.Dc, self.cdims, self.block = Dc, tuple(cdims), tuple(block)
        self.n = Dc.shape[-1]

    def D(self, x):
        return coarse_apply(self.Dc, x, self.cdims)

    def _cross(self, mu, sign):
        """per-site mask (1 where the hop sign*mu leaves the level-1 block)."""
        L, b = self.cdims[mu], self.block[mu]
        c = np.arange(L)
        if L == b:
            m = np.zeros(L)
        elif sign > 0:
            m = (c % b == b - 1).astype(float)
        else:
            m = (c % b == 0).astype(float)
        shp = [1, 1, 1, 1]
        shp[3 - mu] = L
        full = np.broadcast_to(m.reshape(shp), tuple(self.cdims[::-1]))
        return full.reshape(-1, 1)

    def hop(self, x, mu, sign):
        d = 1 + mu if sign > 0 else 5 + mu
        return np.einsum('xnm,...xm->...xn', self.Dc[:, d], coarse_shift(x, self.cdims, mu, sign))

    def Dsap(self, x):
        y = np.einsum('xnm,...xm->...xn', self.Dc[:, 0], x)
        for mu in range(4):
            for sign in (+1, -1):
                y = y + (1.0 - self._cross(mu, sign)) * self.hop(x, mu, sign)
        return y

    def hop_cross(self, x, mu, sign):
        return self._cross(mu, sign) * self.hop(x, mu, sign)


def coarse_chiral_project(x, s):
    n = x.shape[-1]
    out = np.zeros_like(x)
    sl = slice(0, n // 2) if s == 0 else slice(n // 2, n)
    out[..., sl] = x[..., sl]
    return out


def coarse_block_orthonormalize(W, cdims, block, passes=2):
    """<I|J> = delta_IJ on level 1, per level-1 block and half, order k = 1..N."""
    n = W.shape[-1]
    Wb = coarse_to_blocks(W, cdims, block).copy()
    for _ in range(passes):
        for i in range(Wb.shape[0]):
            for k in range(i):
                c = np.sum(np.conj(Wb[k]) * Wb[i], axis=-1)
                Wb[i] -= c[..., None] * Wb[k]
            Wb[i] /= np.sqrt(np.sum(np.abs(Wb[i]) ** 2, axis=-1))[..., None]
    return coarse_from_blocks(Wb, cdims, block, n)


def coarse_restrict(W, x, cdims, block):
    Wb = coarse_to_blocks(W, cdims, block)
    xb = coarse_to_blocks(x, cdims, block)
    xc = np.einsum('ixsk,...xsk->...xsi', np.conj(Wb), xb)
    return xc.reshape(xc.shape[:-2] + (2 * W.shape[0],))


def coarse_prolong(W, xc, cdims, block):
    nv = W.shape[0]
    Wb = coarse_to_blocks(W, cdims, block)
    c = xc.reshape(xc.shape[:-1] + (2, nv))
    return coarse_from_blocks(np.einsum('ixsk,...xsi->...xsk', Wb, c), cdims, block, W.shape[-1])


def coarse_coarse_operator(cop, W):
    """Dc2[X2, d, (s,k), (s',l)] = <X2,s,k| Dc |X2+e_d, s',l>, by the same
    9-term construction as the level-0 coarse operator."""
    nv = W.shape[0]
    nX = n_blocks(cop.cdims, cop.block)
    n = 2 * nv
    Dc2 = np.zeros((nX, NDIR, n, n), np.complex128)
    for sp in (0, 1):
        Wp = coarse_chiral_project(W, sp)
        cols = slice(sp * nv, (sp + 1) * nv)
        Dc2[:, 0, :, cols] = np.transpose(coarse_restrict(W, cop.Dsap(Wp), cop.cdims, cop.block), (1, 2, 0))
        for mu in range(4):
            for sign, d in ((+1, 1 + mu), (-1, 5 + mu)):
                Y = cop.hop_cross(Wp, mu, sign)
                Dc2[:, d, :, cols] = np.transpose(coarse_restrict(W, Y, cop.cdims, cop.block), (1, 2, 0))
    return Dc2


def mr_global(apply_A, b, iters):
    """Minimal-residual iterations on the whole vector from x = 0 (level-1
    smoother): p = A r; alpha = <p,r>/<p,p>; x += alpha r; r -= alpha p."""
    x = np.zeros_like(b)
    r = b.copy()
    for _ in range(iters):
        p = apply_A(r)
        pp = np.vdot(p, p).real
        if pp == 0:
            break
        alpha = np.vdot(p, r) / pp
        x = x + alpha * r
        r = r - alpha * p
    return x


class Level1:
    """Level-1 (coarse) hierarchy: operator Dc on cdims, level-1 test vectors
    W, level-2 operator Dc2, and the level-1 V-cycle used as the coarse solve
    of level 0: x = P1 BiCGStab(Dc2, R1 b); x += MR(b - Dc x)."""

    def __init__(self, cop, W, mr1_iters=4, coarse_iters=50, coarse_tol=0.1):
        self.cop, self.W = cop, W
        self.mr1_iters, self.coarse_iters, self.coarse_tol = mr1_iters, coarse_iters, coarse_tol
        self.cdims2 = coarse_dims(cop.cdims, cop.block)
        self.Dc2 = coarse_coarse_operator(cop, W)

    def vcycle(self, b):
        shp = b.shape
        flat = b.reshape((-1,) + shp[-2:])
        out = np.zeros_like(flat)
        for k in range(flat.shape[0]):
            bc2 = coarse_restrict(self.W, flat[k], self.cop.cdims, self.cop.block)
            xc2, _ = bicgstab(lambda z: coarse_apply(self.Dc2, z, self.cdims2), bc2, self.coarse_iters,
                              self.coarse_tol)
            x = coarse_prolong(self.W, xc2, self.cop.cdims, self.cop.block)
            r = flat[k] - self.cop.D(x)
            out[k] = x + mr_global(self.cop.D, r, self.mr1_iters)
        return out.reshape(shp)


def setup_level1(cop, W0, n_init=3, n_adapt=3, mr1_iters=4, coarse_iters=50, coarse_tol=0.1, init_mr_iters=8):
    """Setup of level 1, as (0-a)/(0-b) one level down: MR (init_mr_iters
    iterations, as the approximate inverse) applied n_init times to the start
    vectors, orthonormalisation per level-1 block and half, Dc2; then n_adapt
    passes replacing every vector by the level-1 V-cycle applied to it."""
    W = W0.copy()
    for _ in range(n_init):
        W = np.array([mr_global(cop.D, w, init_mr_iters) for w in W])
    W = coarse_block_orthonormalize(W, cop.cdims, cop.block)
    lv = Level1(cop, W, mr1_iters, coarse_iters, coarse_tol)
    for _ in range(n_adapt):
        W = lv.vcycle(W)
        W = coarse_block_orthonormalize(W, cop.cdims, cop.block)
        lv = Level1(cop, W, mr1_iters, coarse_iters, coarse_tol)
    return lv


class ThreeLevel(TwoLevel):
    """Level 0 with a level-1 V-cycle as its coarse solve."""

    def __init__(self, op, V, lv1, sap_sweeps=4, mr_iters=6, smoothing='post'):
        self.op, self.V = op, V
        self.sap_sweeps, self.mr_iters = sap_sweeps, mr_iters
        self.smoothing = smoothing
        self.block_solver = None
        self.cdims = coarse_dims(op.dims, op.block)
        self.Dc = coarse_operator(op, V)
        self.lv1 = lv1
        self.coarse = 'level1'

    def coarse_solve(self, bc):
        return self.lv1.vcycle(bc)
