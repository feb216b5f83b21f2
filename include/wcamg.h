/*
 * wcamg.h -- C ABI of libwcamg, an algebraic multigrid (AMG) solver for the
 * Wilson-clover Dirac equation D x = b on one AMD MI355X (gfx950).
 *
 * The operator is eq. (1) of Kanamori, Ishikawa, Matsufuru, arXiv:2111.05012
 * (Sec. 2):
 *   D psi(x) = (1 + F(x)) psi(x)
 *              - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                             + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * and the solver is the paper's multigrid preconditioner (Sec. 3: setup
 * (0-a)/(0-b), restriction eq. (5), coarse solve of eq. (4) with the coarse
 * operator eq. (7), prolongation eq. (6), SAP smoother) inside an outer
 * flexible GMRES in FP64.
 *
 * Conventions (fixed by this ABI):
 *  - Lattice extents dims = {Lx, Ly, Lz, Lt}; canonical site index
 *    x + Lx*(y + Ly*(z + Lz*t)).
 *  - Spinor fields: complex128 [nrhs][V][4 spin][3 colour] (interleaved re, im).
 *  - Gauge fields:  complex128 [4 mu = x,y,z,t][V][3][3], U_mu(x) links x to
 *    x+mu, row-major.  Boundary phases are NOT folded into U.
 *  - Clover fields: complex128 [V][2][6][6]: the two diagonal 6x6 blocks of
 *    the 12x12 matrix F(x) in the chiral basis (block b holds spins 2b, 2b+1;
 *    index spin_in_block*3 + colour).  F excludes the identity.
 *  - Gamma matrices, chiral basis: gamma_k = [[0, -i s_k], [i s_k, 0]]
 *    (k = 1,2,3 with Pauli matrices s_k), gamma_4 = [[0, -1], [-1, 0]], so
 *    gamma_5 = -gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1) (eq. (2)).
 *  - Clover term: F = i c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu},
 *    sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], Fhat = (Q - Q^dag)/8 with Q the
 *    four plaquette leaves at x in the (mu, nu) plane.
 *  - Multigrid blocks (= SAP domains, Sec. 3) of extents block[4] divide dims.
 *    Coarse vectors: complex128 [nrhs][NC][2 nv], NC = prod(dims/block) coarse
 *    sites ordered like fine sites, internal index s*nv + i (s = 0: spins 0,1;
 *    s = 1: spins 2,3).  Coarse operator: complex128 [NC][9][2nv][2nv],
 *    Dc[X][d][n][m] = <X, n| D |X + e_d, m>, d = 0 self, 1 + mu forward,
 *    5 + mu backward neighbour.
 *
 * Pointers: "where" selects WCAMG_DEVICE (device memory, read/written in
 * order on the context's stream, asynchronously) or WCAMG_HOST (host memory,
 * the call is synchronous).  The caller owns every buffer it passes; the
 * library keeps no caller pointer after a call returns (device reads of a
 * device input may still be in flight on the stream).  The library owns its
 * internal copies (gauge, clover, test vectors, coarse operators,
 * workspaces), all freed by wcamg_destroy.
 *
 * Errors: every int function returns WCAMG_OK (0), a negative error code or
 * a positive warning; no C++ exception crosses the ABI.  The message of the
 * last failure is returned by wcamg_last_error.  A context is not
 * thread-safe: use one context per host thread / stream.
 */
#ifndef WCAMG_H
#define WCAMG_H

#ifdef __cplusplus
extern "C" {
#endif

#define WCAMG_OK 0
#define WCAMG_NOT_CONVERGED 1 /* solve: some right-hand side missed the tolerance */
#define WCAMG_EINVAL (-1)     /* invalid argument (checked before any device call) */
#define WCAMG_ENOMEM (-2)     /* device allocation failed */
#define WCAMG_EHIP (-3)       /* HIP runtime error */
#define WCAMG_ESTATE (-4)     /* call out of order (e.g. no gauge field, no setup) */
#define WCAMG_ENUMERIC (-5)   /* NaN/Inf or breakdown detected */

#define WCAMG_DEVICE 0
#define WCAMG_HOST 1

#define WCAMG_PREC_FP64 0  /* everything in FP64 */
#define WCAMG_PREC_MIXED 1 /* FP16 hop matrices -kappa U, clover and test vectors, FP32 arithmetic,
                              FP64 outer solver */

typedef struct wcamg_ctx wcamg_ctx;

typedef struct {
  int dims[4];  /* Lx, Ly, Lz, Lt: each even and >= 2 */
  int block[4]; /* multigrid block = SAP domain extents; must divide dims */
  int bc[4];    /* +1 periodic, -1 antiperiodic, per direction */
  double kappa; /* hopping parameter of eq. (1) */
  double csw;   /* clover coefficient */
} wcamg_lattice;

/* Create a context on the current HIP device.  hip_stream: a hipStream_t to
 * issue all work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL
 * for a library-owned stream.  Validates the lattice (EINVAL) before touching
 * the device. */
int wcamg_create(wcamg_ctx** out, const wcamg_lattice* lat, void* hip_stream);
/* Free everything the context owns.  NULL is accepted. */
void wcamg_destroy(wcamg_ctx* ctx);
/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char* wcamg_last_error(const wcamg_ctx* ctx);
/* Synchronise the context's stream. */
int wcamg_sync(wcamg_ctx* ctx);

/* Load the gauge field U (canonical layout), convert it to the internal
 * blocked layout in FP64 and FP16, and build the clover term F (Sec. 2).
 * Invalidates any previous setup. */
int wcamg_load_gauge(wcamg_ctx* ctx, const void* U, int where);
/* Override the clover term with F (canonical clover layout; Hermitian blocks
 * expected, only the upper triangles and real diagonals are read). */
int wcamg_load_clover(wcamg_ctx* ctx, const void* F, int where);
/* Copy the FP64 clover term out (canonical clover layout). */
int wcamg_get_clover(wcamg_ctx* ctx, void* F, int where);

/* out = D in for nrhs spinor fields, eq. (1).  prec = WCAMG_PREC_FP64
 * (FP64 throughout) or WCAMG_PREC_MIXED (FP32 arithmetic on FP32-rounded
 * input, with the hop matrices -kappa U_mu and the clover term F stored in
 * FP16, each rounded once from FP64).  in and out must not alias. */
int wcamg_apply_D(wcamg_ctx* ctx, const void* in, void* out, int nrhs, int prec, int where);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): out = D in
 * exactly as wcamg_apply_D with device pointers (canonical layout, complex128
 * [nrhs][V][4][3]), but its two staging fields in the internal layout are
 * taken from a fixed scratch area of WCAMG_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on (from the loading of its code object
 * until the process ends), instead of the context's workspaces.  Limit:
 * 2 * nrhs * 12 * V * (16 bytes in FP64, 8 in WCAMG_PREC_MIXED), each field
 * rounded up to 256 bytes, must not exceed WCAMG_NOALLOC_SCRATCH_BYTES
 * (EINVAL before any device work otherwise; e.g. 16^4 sites: 2 right-hand
 * sides in FP64, 5 in mixed precision).  The call allocates nothing and
 * runs no autotuning: the launch variant is the one already tuned for this
 * shape, else the default one.  Stream-ordered and asynchronous on the
 * context's stream.  Every call on one GPU shares that GPU's scratch area
 * (whatever the context): calls that overlap on one GPU, from different
 * streams or host threads, race and must be ordered by the caller. */
#define WCAMG_NOALLOC_SCRATCH_BYTES (64 << 20)
int wcamg_apply_D_noalloc(wcamg_ctx* ctx, const void* in, void* out, int nrhs, int prec);
/* out = D_SAP in: eq. (1) with every hop between distinct blocks removed
 * (Sec. 3, SAP paragraph). */
int wcamg_apply_Dsap(wcamg_ctx* ctx, const void* in, void* out, int nrhs, int prec, int where);
/* x = SAP(b): the Schwarz alternating procedure with fixed iterations
 * (Sec. 3 listing): x = 0, r = b; per sweep, even then odd domains
 * (colour = parity of the sum of block coordinates) get x += M r with M
 * the block solve, and r = b - D x.  Needs an even number of blocks per
 * direction (EINVAL).  block_solve:
 *   WCAMG_BLOCK_MR: mr_iters minimal-residual iterations on D_SAP of the
 *     domain from 0 (the paper's choice);
 *   WCAMG_BLOCK_EO_MR: the even-odd preconditioned variant (mixed precision,
 *     even block extents): with A = 1 + F and H the in-domain hops split by
 *     site parity, mr_iters MR iterations on the Schur complement
 *     S = A_e - H_eo A_o^-1 H_oe for c_e = b_e - H_eo A_o^-1 b_o, then
 *     x_o = A_o^-1 (b_o - H_oe x_e), with A_o^-1 stored in FP16 as
 *     (1 + F)^-1 - 1. */
#define WCAMG_BLOCK_MR 0
#define WCAMG_BLOCK_EO_MR 1
int wcamg_sap(wcamg_ctx* ctx, const void* b, void* x, int nrhs, int sweeps, int mr_iters, int block_solve, int prec,
              int where);

typedef struct {
  int nv;            /* test vectors N_v (<= 64) */
  int n_init;        /* (0-a): SAP applications to the start vectors */
  int n_adapt;       /* (0-b): adaptive refinement passes */
  int sap_sweeps;    /* SAP sweeps n (paper: 4) */
  int mr_iters;      /* MR iterations per block solve (paper: 6) */
  int coarse_iters;  /* coarse BiCGStab: maximum iterations */
  double coarse_tol; /* coarse BiCGStab: relative residual tolerance */
  int prec;          /* WCAMG_PREC_FP64 or WCAMG_PREC_MIXED */
  const void* init_vectors; /* nv start vectors (canonical spinor layout), or NULL: complex
                               Gaussian vectors from the library's counter-based generator (seed) */
  int init_where;    /* WCAMG_DEVICE or WCAMG_HOST for init_vectors */
  /* three-level hierarchy (nlevels = 3): level 1 aggregates block1 coarse
   * sites; its smoother is mr1_iters global minimal-residual iterations on
   * the level-1 operator, its coarse solve the BiCGStab above on the level-2
   * operator.  Level-1 setup: (0-a) init_mr1_iters MR iterations applied
   * n_init times to the start vectors, (0-b) n_adapt level-1 V-cycles. */
  int nlevels;       /* 2 (default when 0) or 3 */
  int block1[4];     /* level-1 blocks on the coarse lattice */
  int nv1;           /* level-1 test vectors */
  int mr1_iters;
  int init_mr1_iters;
  const void* init_vectors1; /* nv1 level-1 start vectors, complex128 [nv1][NC][2nv] (device), or
                                NULL: drawn by the library's counter-based generator from seed1 */
  unsigned long long seed1;
  /* learned start: when nonzero, step (0-a) is replaced by the network of
   * wcamg_net_init applied to init_vectors (nv must equal its channels). */
  int init_net;
  unsigned long long seed; /* start vectors when init_vectors is NULL */
  /* Position of the SAP smoother in the V-cycle (Sec. 3 allows it before,
   * after, or before and after the coarse solve); each step is a Richardson
   * step x <- x + M_i (b - D x) from x = 0:
   * WCAMG_SMOOTH_POST (0, the paper's choice): coarse grid, then smoother;
   * WCAMG_SMOOTH_PRE (1): smoother, then coarse grid;
   * WCAMG_SMOOTH_BOTH (2): smoother, coarse grid, smoother. */
  int smoothing;
  /* SAP block solve: 0 = WCAMG_BLOCK_MR (default), 1 = WCAMG_BLOCK_EO_MR
   * (the even-odd preconditioned variant of wcamg_sap; mixed precision). */
  int sap_eo;
  /* Test vectors per batch in the setup's SAP and V-cycle applications
   * (0: all nv at once).  The vectors are independent there, so the result
   * does not depend on it; smaller batches shrink four of the setup's
   * workspaces (SAP residual and corrections, V-cycle fields) from nv to
   * vec_chunk spinor fields, at some cost in speed. */
  int vec_chunk;
} wcamg_setup_params;
#define WCAMG_SMOOTH_POST 0
#define WCAMG_SMOOTH_PRE 1
#define WCAMG_SMOOTH_BOTH 2

/* Setup stage (0) of Sec. 3: (0-a) SAP applied n_init times to the start
 * vectors, block orthonormalisation (<I|J> = delta_IJ), coarse operator
 * eq. (7); (0-b) n_adapt times: every vector replaced by M v (the V-cycle
 * with the current hierarchy), re-orthonormalised, coarse operator rebuilt.
 * Synchronous. */
int wcamg_setup(wcamg_ctx* ctx, const wcamg_setup_params* p);

/* Install nv test vectors as given (canonical spinor layout; the caller
 * orthonormalises them), with the preconditioner parameters of p (its
 * init_vectors / n_init / n_adapt are ignored), and build the coarse
 * operator.  Component test hook. */
int wcamg_set_test_vectors(wcamg_ctx* ctx, const void* V, const wcamg_setup_params* p, int where);
/* Copy the stored test vectors out (canonical spinor layout, nv fields). */
int wcamg_get_test_vectors(wcamg_ctx* ctx, void* V, int where);
/* Block-orthonormalise nv fields (canonical layout) per block and
 * chirality in the order i = 1..nv, positive real diagonal (CholQR2). */
int wcamg_orthonormalize(wcamg_ctx* ctx, const void* in, void* out, int nv, int prec, int where);
/* eq. (5): out[r][X][s nv + i] = <X, s, i | in_r>, with the stored vectors. */
int wcamg_restrict(wcamg_ctx* ctx, const void* in, void* out, int nrhs, int where);
/* eq. (6): out_r = sum_I in[r][I] |I>. */
int wcamg_prolong(wcamg_ctx* ctx, const void* in, void* out, int nrhs, int where);
/* Copy a coarse operator out: level 1 = Dc (complex128 [NC][9][2nv][2nv],
 * see above), level 2 = the level-2 operator of a three-level hierarchy
 * (complex128 [NC2][9][2nv1][2nv1], same conventions one level down). */
int wcamg_get_coarse_op(wcamg_ctx* ctx, int level, void* Dc, int where);
/* Three-level hook: install nv1 level-1 test vectors as given (complex128
 * [nv1][NC][2nv]; the caller orthonormalises them per level-1 block and
 * half) on a hierarchy created with nlevels = 3, and build the level-2
 * operator. */
int wcamg_set_level1_vectors(wcamg_ctx* ctx, const void* W, int where);
/* Copy the level-1 test vectors out (complex128 [nv1][NC][2nv]). */
int wcamg_get_level1_vectors(wcamg_ctx* ctx, void* W, int where);
/* Replace the coarse operator of a level (1: Dc of eq. (7); 2: the level-2
 * operator of a three-level hierarchy) by Dc (the canonical coarse-operator
 * layout, complex128), converted to the hierarchy's coarse precision
 * (complex64 with round to nearest even in mixed precision).  Component test
 * hook: the coarse matvec, the coarse solve and the V-cycle then use it; the
 * level-2 operator is not rebuilt from a replaced level 1, and the next
 * setup or set_test_vectors builds both anew.  ESTATE without a hierarchy
 * (or without level 2 when level = 2). */
int wcamg_set_coarse_op(wcamg_ctx* ctx, int level, const void* Dc, int where);
/* out = D_c in on coarse vectors of a level (1 or 2, as above): the 9-point
 * block stencil y(X) = sum_d D_c(X, X + e_d) x(X + e_d) of eq. (7);
 * complex128 [nrhs][NC][2nv] (level 2: [nrhs][NC2][2nv1]). */
int wcamg_apply_coarse(wcamg_ctx* ctx, int level, const void* in, void* out, int nrhs, int where);
/* x = coarse solve of D_c x = b on a level (1 or 2): BiCGStab from x = 0 with
 * the stabilised omega (Sec. 3 step (1b)), at most iters iterations,
 * stopping per right-hand side at ||r|| <= tol ||b||; in mixed precision in
 * FP32 on the complex64 operator. */
int wcamg_coarse_solve(wcamg_ctx* ctx, int level, const void* b, void* x, int nrhs, int iters, double tol,
                       int where);
/* out = M in: one application of the multigrid preconditioner, Sec. 3
 * steps (1a)-(1c) then (2). */
int wcamg_vcycle(wcamg_ctx* ctx, const void* in, void* out, int nrhs, int where);

typedef struct {
  int restart;   /* FGMRES restart length m (1..32) */
  double tol;    /* relative residual ||b - D x|| / ||b|| per right-hand side */
  int max_iters; /* total Arnoldi steps per right-hand side */
  int rhs_chunk; /* right-hand sides per batch (0: all) */
  int use_graph; /* capture the V-cycle in a HIP graph and replay it */
  int phase_times; /* nonzero: time the solve's phases (the info's t_precond ... t_outer) with HIP
                      events; the V-cycles then run without graphs */
  int ortho;       /* orthogonalisation of the Arnoldi vectors: 0 = classical Gram-Schmidt twice
                      with the second pass delayed into the next step (two sweeps over the basis
                      per step; the last Hessenberg column of a cycle keeps its first-pass
                      values), 1 = classical Gram-Schmidt twice (three sweeps per step);
                      other values: WCAMG_EINVAL */
} wcamg_solve_params;

#define WCAMG_MAX_RHS 64
typedef struct {
  int iters[WCAMG_MAX_RHS];        /* outer iterations per right-hand side */
  double relres[WCAMG_MAX_RHS];    /* final ||b - D x|| / ||b||, recomputed with FP64 D */
  int converged[WCAMG_MAX_RHS];
  int vcycles;                     /* preconditioner applications (batched) */
  double t_solve;                  /* seconds, wall clock of the whole solve */
  /* Seconds per phase of the solve, in the split of the paper's Table 1
   * (Sec. 5), measured with HIP events on the context's stream when the
   * solve parameters ask for phase_times, else 0.  t_precond: every
   * application of the preconditioner M; within it t_coarse: the coarse
   * solves (step (1b); with three levels, the whole level-1 cycle),
   * t_smoother: the SAP smoother (step (2)), t_rp: restriction and
   * prolongation (steps (1a), (1c)), t_prec_other: the rest of M (the
   * residual with D before the smoother, conversions); t_outer = t_solve -
   * t_precond: the outer solver (FP64 D, orthogonalisation, host work). */
  double t_precond, t_coarse, t_smoother, t_rp, t_prec_other, t_outer;
} wcamg_solve_info;

/* Solve D x = b for nrhs right-hand sides (canonical layout, DEVICE
 * pointers b and x; synchronous) with flexible
 * GMRES(restart) in FP64, right-preconditioned by the multigrid V-cycle,
 * from x = 0.  Returns WCAMG_NOT_CONVERGED if some right-hand side missed
 * tol within max_iters (info filled either way). */
int wcamg_solve(wcamg_ctx* ctx, const void* b, void* x, int nrhs, const wcamg_solve_params* p,
                wcamg_solve_info* info);

/* The paper's own outer solver (Sec. 3, "BiCGStab algorithm with flexible
 * preconditioning", after Vogel 2007) in FP64, from x = 0, with the shadow
 * vector r~ = b and the listing's last line read as
 * p <- r + beta (p - omega D M p).  The preconditioner M is
 *   WCAMG_PC_AMG:    the multigrid V-cycle (Sec. 3; needs wcamg_setup), or
 *   WCAMG_PC_BICG32: the comparison solver's preconditioner (Sec. 5,
 *                    "MBiCGs"): a BiCGStab on D in FP32 arithmetic (FP32
 *                    links, clover and spinors) with the omega
 *                    stabilisation of the coarse solve, from 0, stopping at
 *                    inner_tol relative residual or inner_iters iterations.
 * Each iteration applies M twice.  The listing's first break point (after
 * s) is taken at the end of that iteration instead: the omega step it skips
 * is then a correction of the order of the tolerance.  Right-hand sides are
 * batched as in wcamg_solve (b, x: DEVICE pointers, canonical layout;
 * synchronous); info->iters counts outer iterations and info->vcycles the
 * batched applications of M. */
#define WCAMG_PC_AMG 0
#define WCAMG_PC_BICG32 1
typedef struct {
  double tol;        /* relative residual ||b - D x|| / ||b|| per right-hand side */
  int max_iters;     /* outer iterations per right-hand side */
  int rhs_chunk;     /* right-hand sides per batch (0: all) */
  int precond;       /* WCAMG_PC_AMG or WCAMG_PC_BICG32 */
  int inner_iters;   /* WCAMG_PC_BICG32: iterations of the inner solve (>= 1) */
  double inner_tol;  /* WCAMG_PC_BICG32: relative residual of the inner solve */
  int phase_times;   /* as in wcamg_solve_params (WCAMG_PC_AMG splits t_precond) */
} wcamg_bicg_params;
int wcamg_solve_bicgstab(wcamg_ctx* ctx, const void* b, void* x, int nrhs, const wcamg_bicg_params* p,
                         wcamg_solve_info* info);

/* Gauge-equivariant network proposing initial test vectors (replaces setup
 * step (0-a) when wcamg_setup_params.init_net is set).  Layers
 *   psi'_o(x) = sum_i sum_{d=0..8} W[d][o][i] (T_d psi_i)(x),
 * T_0 = 1, T_{+mu} psi(x) = U_mu(x) psi(x+mu), T_{-mu} psi(x) =
 * U_mu(x-mu)^dag psi(x-mu) (boundary hops carry bc), W[d][o][i] a complex
 * 4x4 spin matrix; no bias or nonlinearity (gauge covariant).  Weights:
 * complex64 [layers][9][C][C][4][4]; C = 16.  Inputs r and outputs: C
 * spinor fields (canonical layout, complex128).  The loss against a teacher
 * basis Q (C fields, orthonormal per block and chirality) is the mean over
 * blocks and chiralities of 1 - tr(Q^dag P_A Q)/C, P_A the projector on the
 * span of the output A there. */
int wcamg_net_init(wcamg_ctx* ctx, int layers, int channels, const void* weights, int where);
int wcamg_net_get_weights(wcamg_ctx* ctx, void* weights, int where);
int wcamg_net_forward(wcamg_ctx* ctx, const void* r, void* out, int where);
/* Loss and its gradient dL/d conj(W) (complex64, weight layout; grad may be
 * NULL) for inputs r and teacher basis Q on the loaded gauge field. */
int wcamg_net_gradient(wcamg_ctx* ctx, const void* r, const void* teacher, double* loss, void* grad, int where);
/* One training step: loss, gradient, then Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) with learning rate lr on the real and imaginary parts. */
int wcamg_net_train_step(wcamg_ctx* ctx, const void* r, const void* teacher, double lr, double* loss, int where);

/* Launch-variant autotuner (on by default): the first time a kernel is
 * launched for a new key (kernel, shapes, precision, GPU architecture) each
 * candidate variant (Dslash workgroup size or tiling, coarse-matvec right-hand
 * sides per thread or matrix cores, restriction and prolongation kernel,
 * coarse-operator contraction) is timed with HIP events on the real operands
 * and the fastest is kept.  Variants compute the same quantities in the same
 * precision; results may differ by rounding (summation order).  cache_path
 * (or the environment variable WCAMG_AUTOTUNE_CACHE at create time) names a
 * flat JSON file {"key": variant}: its entries are merged into the table now
 * (they override known keys), the merged table is written back at once and
 * again after each newly tuned key; NULL keeps the current file. */
int wcamg_autotune(wcamg_ctx* ctx, int enable, const char* cache_path);
/* Time spent tuning (ms, not part of any solve), keys tuned by this context
 * and keys known (tuned or loaded). Pointers may be NULL. */
int wcamg_autotune_info(wcamg_ctx* ctx, double* tune_ms, int* keys_tuned, int* keys_known);

/* Per-kernel-class timing with HIP events on the context stream, for
 * roofline measurements: enable (1) / disable (0, also clears nothing).
 * When enabled, the work of each class is bracketed by events: "dslash64",
 * "dslash32" (one launch of the fine operator), "sap_half" (one SAP
 * half-sweep launch: the domain solves), "sap_cross" (the crossing-hop
 * correction launched before a mixed half-sweep), "restrict", "prolong", "coarse_mv",
 * "coarse_solve" (one whole coarse BiCGStab), "coarse_build" (one coarse
 * operator construction), "ortho" (one block orthonormalisation), "gs" (the
 * classical Gram-Schmidt of one FGMRES Arnoldi step, both passes).  Classes
 * nest ("coarse_mv" launches inside "coarse_solve" are recorded in both),
 * except that nothing inside "coarse_build" or "ortho" is recorded
 * separately.  Graph replay is disabled while timing is on. */
int wcamg_kernel_timing(wcamg_ctx* ctx, int enable);
/* Accumulated time (ms), launch count, algorithmic bytes and flops (the
 * compulsory traffic / arithmetic of the work, 0 when not defined for the
 * class) and right-hand-side units of a class since timing was enabled.
 * bytes, flops, units may be NULL. */
int wcamg_kernel_stats(wcamg_ctx* ctx, const char* name, double* total_ms, int* count, double* bytes,
                       double* flops, double* units);

#ifdef __cplusplus
}
#endif
#endif /* WCAMG_H */
