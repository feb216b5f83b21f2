// Host-side launchers of the libwcamg kernels (internal interface between
// the solver orchestration and the HIP kernels).
#pragma once
#include "wc_common.h"

namespace wc {

// Storage type of a complex field.
enum CT { C128 = 0, C64 = 1, C32H = 2 };  // double2, float2, half2_t
inline size_t ct_size(int t) { return t == C128 ? 16 : (t == C64 ? 8 : 4); }

inline int round8(int n) { return ((n + 7) / 8) * 8; }

// ---------------------------------------------------------------- layout
// canonical complex128 [nrhs][V][4][3]  <->  internal [nrhs][12][V] (blocked site order)
void launch_pack_spinor(const Geo& g, const double2* canon, void* out, int out_t, size_t out_rs, int nrhs,
                        hipStream_t st);
void launch_unpack_spinor(const Geo& g, const void* in, int in_t, size_t in_rs, double2* canon, int nrhs,
                          hipStream_t st);
// canonical complex128 [4][V][3][3] -> internal [4][9][V] in FP64 and FP16
// U64 = U; U16 = FP16 rounding of h U (h = -kappa: the hop matrices)
void launch_pack_gauge(const Geo& g, const double2* canon, double2* U64, half2_t* U16, double h, hipStream_t st);
// clover F(x) from the FP64 links: packed Hermitian chiral blocks [36 pairs][V] in FP64 and FP16.
// sigma: the chiral 2x2 blocks of sigma_{mu nu}, [6 planes][2 chiralities][2][2] complex (re, im).
void launch_clover_build(const Geo& g, const double2* U64, double kappa, double csw, const double* sigma,
                         double2* C64, half2_t* C16, hipStream_t st);
// canonical clover complex128 [V][2][6][6] <-> packed
// M16 = FP16 of (1 + F)^-1 - 1 per site and chirality block (packed like the clover)
void launch_clover_inverse(const Geo& g, const double2* C64, half2_t* M16, hipStream_t st);
void launch_pack_clover(const Geo& g, const double2* canon, double2* C64, half2_t* C16, hipStream_t st);
void launch_unpack_clover(const Geo& g, const double2* C64, double2* canon, hipStream_t st);

// ---------------------------------------------------------------- Dslash family
enum { OP_D = 0, OP_DSAP = 1, OP_HOP = 2 };
struct DslashArgs {
  Geo g;
  int op = OP_D;      // OP_D: full eq.(1); OP_DSAP: in-block hops only; OP_HOP: one crossing hop
  int hopdir = 0;     // OP_HOP: 0..3 = +mu, 4..7 = -mu
  int chir = -1;      // >= 0: input projected on chirality chir (spins 2chir, 2chir+1)
  int nrhs = 1;
  const void* in = nullptr;
  int in_t = C128;
  size_t in_rs = 0;
  void* out = nullptr;
  int out_t = C128;
  size_t out_rs = 0;
  const void* b = nullptr;  // non-null: out = b - D in  (b has out's type and stride)
  const void* U = nullptr;
  const void* C = nullptr;
  int fields16 = 0;  // 0: FP64 links/clover, 1: FP16
  int fields32 = 0;  // 1: FP32 links/clover (with compute32)
  int compute32 = 0; // 0: FP64 arithmetic, 1: FP32
  double kappa = 0;
  int block_size = 256;  // threads per workgroup (64 .. 512, autotuned); -1: colour-split variant,
                         // -2: LDS-staged tiles, -3: LDS-staged tiles with the backward hops
                         // handed over as half-spinors, -10 - NR: NR right-hand sides per thread
                         // (NR = 2, 4; all OP_D only)
};
void launch_dslash(const DslashArgs& a, hipStream_t st);
// t-slices per tile of the LDS-staged operator, 0 when it does not apply
int dslash_lds_slices(const Geo& g);

// ---------------------------------------------------------------- SAP smoother
struct SapArgs {
  Geo g;
  int nrhs = 1, sweeps = 4, mr = 6;
  int mixed = 0;  // 0: FP64 everything; 1: FP32 spinors and arithmetic, FP16 hop matrices/clover
  double kappa = 0;
  const void* b = nullptr;      // source
  void* x = nullptr;            // solution (output)
  const void* xinit = nullptr;  // optional: x starts from xinit instead of 0 (x = xinit + SAP(b))
  void* r = nullptr;            // workspace residual
  // workspace: the last block corrections (FP64 path, even-odd variant), or
  // (mixed path) the spin-projected corrections on the domain faces,
  // [rhs][block][6][sap_face_slots] complex64 with per-rhs stride fs
  void* delta = nullptr;
  size_t rs = 0;                // per-rhs stride of all spinor fields
  size_t fs = 0;                // per-rhs stride of the face buffer (mixed path)
  const void* U = nullptr;
  const void* C = nullptr;
  const void* FL = nullptr;     // face hop matrices (launch_face_links), mixed path
  // even-odd preconditioned block solve (mixed precision only): M holds the
  // FP16 (1 + F)^-1 - 1 (launch_clover_inverse)
  int eo = 0;
  const void* M = nullptr;
};
// Faces of a domain (multigrid block), in the order (mu, side): side 0 is
// the face at local coordinate 0, side 1 at B_mu - 1; face mu has Vb / B_mu
// sites, indexed lexicographically by the other three local coordinates.
// sap_face_slots = sum over mu of 2 Vb / B_mu.
int sap_face_slots(const Geo& g);
// FL[block][face][9][face site]: the FP16 hop matrix (-kappa U, times the
// boundary sign of the hop) of the hop that leaves the block through that
// face site: U_mu(y) for side 1, U_mu(y - mu) for side 0.  Built from the
// FP16 links after every gauge load; nblk * 9 * sap_face_slots elements.
void launch_face_links(const Geo& g, const void* U16, void* FL, hipStream_t st);
// one half-sweep (colour col of sweep `sweep`) of the SAP listing.  Mixed
// precision: launch_sap_cross (the crossing-hop correction of the residual,
// when sap_needs_cross) must precede launch_sap_half on the same stream.
bool sap_needs_cross(const SapArgs& a, int sweep, int col);
void launch_sap_cross(const SapArgs& a, int sweep, int col, hipStream_t st);
void launch_sap_half(const SapArgs& a, int sweep, int col, hipStream_t st);
int sap_lds_bytes(const Geo& g, int mixed);  // FP64 path
int sap_dom_lds_bytes(const Geo& g);          // mixed path

// ---------------------------------------------------------------- coarse level
struct CGeo {
  int N[4];
  int sN[4];
  int NC;
};
inline CGeo make_cgeo(const int* n) {
  CGeo c;
  for (int m = 0; m < 4; ++m) c.N[m] = n[m];
  c.sN[0] = 1;
  for (int m = 1; m < 4; ++m) c.sN[m] = c.sN[m - 1] * n[m - 1];
  c.NC = n[0] * n[1] * n[2] * n[3];
  return c;
}

// restriction eq.(5): out[r][X][s*nv+i] = sum_{y in X, a in s} conj(V_i(y,a)) in_r(y,a)
// V: [nv][12][V] of type v_t; in: [nrhs][12][V] (in_rs); out element (r, X, n) at
// r*out_rs + X*out_xs + n.  acc64: accumulate in FP64.
// tile: sites per LDS tile (0: largest that fits 48 KiB; else a power of two dividing Vb);
// RESTRICT_MFMA64: FP64 matrix-core path (FP64 output, equal FP64 or FP32 operands,
// nv, nrhs <= 32); RESTRICT_MFMA32: FP32 matrix-core path (FP16 vectors, FP32 or
// FP16 input, FP32 output, nv, nrhs <= 32)
// RESTRICT_MFMA32D: as RESTRICT_MFMA32 with register operands (no LDS staging),
// block volume divisible by 32
constexpr int RESTRICT_MFMA64 = -64;
constexpr int RESTRICT_MFMA32 = -32;
constexpr int RESTRICT_MFMA32D = -33;
void launch_restrict(const Geo& g, int nv, int nrhs, const void* V, int v_t, const void* in, int in_t,
                     size_t in_rs, void* out, int out_t, size_t out_rs, size_t out_xs, int acc64,
                     hipStream_t st, int tile = 0);
// prolongation eq.(6): out_r(y,a) (+)= sum_i V_i(y,a) xc[r][X(y)][s(a)*nv+i]
// variant: 0 the default kernel for the types; PROLONG_MFMA32 the FP32 matrix-core
// path (FP16 or FP32 vectors, FP32 coefficients and output, nv, nrhs <= 32)
constexpr int PROLONG_MFMA32 = -32;
void launch_prolong(const Geo& g, int nv, int nrhs, const void* V, int v_t, const void* xc, int xc_t,
                    size_t xc_rs, size_t xc_xs, void* out, int out_t, size_t out_rs, int accumulate,
                    int compute32, hipStream_t st, int variant = 0);
// coarse 9-point stencil: y[r][X] = sum_d Dc[X][d] x[r][X+e_d]   (or y = b - Dc x)
// Dc stored [X][d][m][n] (column-major blocks), vectors [nrhs][NC][N]
// variant: right-hand sides per thread (0: automatic; else 1, 4, 8, 12 or 16), or
// COARSE_MV_MFMA (complex64, 2 nv <= 64, nrhs <= 32: matrix cores) or
// COARSE_MV_MFMA16 (the same for nrhs <= 16, real and imaginary parts in one
// 32-column operand).
// active (optional): per-rhs flags at active[r * astride]; rhs with a zero flag are skipped.
constexpr int COARSE_MV_MFMA = -1;
constexpr int COARSE_MV_MFMA16 = -2;
void launch_coarse_mv(const CGeo& cg, int N, const void* Dc, const void* x, void* y, const void* b, int nrhs,
                      size_t rs, int prec32, hipStream_t st, int variant = 0, const int* active = nullptr,
                      int astride = 0);
// coarse operator eq.(7) from the stored test vectors V [nv][12][V] (mixed: FP16 V,
// links, clover; FP32 arithmetic; complex64 Dc) into Dc [X][9][m][n].
// variant (mixed only): 0 vector-ALU contraction, 1 matrix-core contraction (nv <= 32),
// which needs a workspace `part` of coarse_build_chunks(g) * nblk * (2 nv)^2 complex64
// backward blocks [X][5 + mu] of a coarse operator from the forward ones by
// coarse gamma_5-hermiticity (the build computes d = 0..4 only)
void launch_coarse_mirror(const CGeo& cg, int nv, void* Dc, int prec32, hipStream_t st);
void launch_coarse_build(const Geo& g, int nv, double kappa, const void* V, const void* U, const void* C, void* Dc,
                         int mixed, hipStream_t st, int variant = 0, void* part = nullptr);
int coarse_build_chunks(const Geo& g);
// level-1 aggregation (multi-level): coarse vectors [rhs][X1][n1], level-1
// test vectors W [nw][X1][n1], level-1 blocks b1, level-2 vectors [rhs][X2][2nw]
void launch_l1_restrict(const CGeo& c1, const int* b1, int n1, int nw, int nrhs, const void* W, int w_t,
                        const void* x, int x_t, size_t x_rs, void* out, int out_t, size_t out_rs, size_t out_xs,
                        hipStream_t st);
void launch_l1_prolong(const CGeo& c1, const int* b1, int n1, int nw, int nrhs, const void* W, int w_t,
                       const void* xc, int xc_t, size_t xc_rs, size_t xc_xs, void* out, int out_t, size_t out_rs,
                       hipStream_t st);
void launch_l1_build(const CGeo& c1, const int* b1, int n1, int nw, const void* Dc1, const void* W, void* Dc2,
                     int prec32, hipStream_t st);
// Cholesky-based coefficients for block orthonormalisation: given the Gram
// matrices G[j][X][s*nv+i] = <v_i, v_j>_{X,s} (FP64), write
// coef[j][X][s*nv+i] = (L^{-H})_{ij} with G = L L^H.  Returns nonzero via
// *bad (device int) when a pivot is not positive.
void launch_cholesky_coef(int nblk, int nv, const double2* G, size_t g_rs, void* coef, int coef_t,
                          size_t coef_rs, int* bad, hipStream_t st);

// ---------------------------------------------------------------- vector kernels
void launch_convert(const void* in, int in_t, void* out, int out_t, size_t n, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);

// per-rhs reductions: for r < nrhs over vectors of n complex numbers (stride rs):
// result[r*nd + k] for k < nd dots (a_k, b_k) -- see blas.hip for the sets
int reduce_nwg(size_t n);
// partial sums of up to 3 inner products <a_k, b_k> per rhs: part[r][wg][k] (complex)
// active (optional): per-rhs flags at active[r * astride]; inactive rhs write zero partials
void launch_dots_partial(int nd, const void* const* a, const void* const* b, int t, size_t n, size_t rs,
                         int nrhs, double2* part, hipStream_t st, const int* active = nullptr, int astride = 0);

// BiCGStab on device-resident per-rhs scalars (coarse solve)
struct BicgScal {
  double2 rho, rho_old, alpha, omega, beta;  // complex scalars
  double bnorm2, rnorm2, tol2;
  int active, iters, final_step, pad;
};
void launch_bicg_init(const void* b, void* x, void* r, void* rt, void* p, void* v, int t, size_t n, size_t rs,
                      int nrhs, double tol, double2* part, BicgScal* sc, hipStream_t st);
// x (FP64) += alpha mp + omega ms for the active right-hand sides; mp, ms of type zt (C128 or C64)
void launch_fbicg_x(double2* x, const void* mp, const void* ms, int zt, size_t n, size_t rs, int nrhs,
                    const BicgScal* sc, hipStream_t st);
void launch_bicg_p(void* p, const void* r, const void* v, int t, size_t n, size_t rs, int nrhs,
                   const BicgScal* sc, hipStream_t st);
void launch_bicg_alpha(const void* rt, const void* v, int t, size_t n, size_t rs, int nrhs, double2* part,
                       BicgScal* sc, hipStream_t st);
void launch_bicg_s(void* s, const void* r, const void* v, int t, size_t n, size_t rs, int nrhs,
                   const BicgScal* sc, hipStream_t st);
void launch_bicg_omega(const void* tt, const void* s, int t, size_t n, size_t rs, int nrhs, double2* part,
                       BicgScal* sc, double stab, hipStream_t st);
// x += alpha p + omega s (skipped when x is null); r = s - omega t; rho, |r|^2
void launch_bicg_xr(void* x, void* r, const void* p, const void* s, const void* tt, const void* rt, int t,
                    size_t n, size_t rs, int nrhs, double2* part, BicgScal* sc, hipStream_t st);

// FGMRES helpers (FP64 basis)
// One Gram-Schmidt sweep over a chunk of nq basis vectors Q_k = Q + k*vs
// (nq <= GS_CHUNK) of every right-hand side (offset r*rs, n complex numbers
// each), the new Arnoldi vector w and, in the two-vector modes, the pending
// vector p.  Coefficient arrays are [k][nrhs]; in the two-vector modes index
// nq is the coefficient of p.  Dot products conj(u) v are summed per
// right-hand side in a fixed order and written to h1/h2 ([k][nrhs], chunk
// offset applied by the caller), h1p/h2p ([nrhs]) and norm2 ([nrhs], skipped
// when null).  part holds nrhs * reduce_nwg(n) * (2 GS_CHUNK + 3) partial sums.
//   GS_DOT:       h1[k] = Q_k^H w                                 (nq >= 1)
//   GS_AXPY_DOT:  w -= sum_k c1[k] Q_k, then h1[k] = Q_k^H w       (nq >= 1)
//   GS_AXPY_NORM: w -= sum_k c1[k] Q_k, then norm2 = |w|^2         (nq >= 1)
//   GS_DOT2:      h1[k] = Q_k^H w, h2[k] = Q_k^H p, h1p = p^H w, h2p = p^H p,
//                 ww = w^H w (when not null)
//   GS_COMB2:     p <- c1[nq] p + sum_k c1[k] Q_k (stored if write_p),
//                 w <- w - c2[nq] p - sum_k c2[k] Q_k (old p), then norm2 = |w|^2;
//                 with vin set, also vin = vscale[r] * w (FP32, [rhs][n] at offset r*rs)
enum GsMode { GS_DOT = 0, GS_AXPY_DOT = 1, GS_AXPY_NORM = 2, GS_DOT2 = 3, GS_COMB2 = 4 };
constexpr int GS_CHUNK = 16;
struct GsArgs {
  const double2* Q = nullptr;
  size_t vs = 0;
  int nq = 0;
  double2* p = nullptr;
  double2* w = nullptr;
  const double2* c1 = nullptr;
  const double2* c2 = nullptr;
  int write_p = 0;
  size_t n = 0, rs = 0;
  int nrhs = 0;
  double2* part = nullptr;
  double2 *h1 = nullptr, *h2 = nullptr, *h1p = nullptr, *h2p = nullptr;
  double* norm2 = nullptr;
  double* ww = nullptr;
  float2* vin = nullptr;
  const double* vscale = nullptr;
};
void launch_gs(int mode, const GsArgs& a, hipStream_t st);
// out[r] = w[r] * scale[r]; optional FP32 copy out32
void launch_scale(const double2* w, const double* scale, double2* out, float2* out32, size_t n, size_t rs, int nrhs,
                  hipStream_t st);
// x[r] += sum_k y[k][r] Z_k[r]   (Z of type z_t)
void launch_update_x(double2* x, const void* Z, int z_t, size_t zs, int nk, const double2* y, size_t n, size_t rs,
                     int nrhs, hipStream_t st);
// norm2[r] = ||v[r]||^2
void launch_norm2(const void* v, int t, size_t n, size_t rs, int nrhs, double2* part, double* norm2,
                  hipStream_t st);

// global MR steps on coarse vectors: alpha[r] = <p,r>/<p,p>; x += alpha r, r -= alpha p
void launch_mr_alpha(const void* p, const void* r, int t, size_t n, size_t rs, int nrhs, double2* part,
                     double2* alpha, hipStream_t st);
void launch_mr_update(void* x, void* r, const void* p, const double2* alpha, int t, size_t n, size_t rs, int nrhs,
                      hipStream_t st);
// n complex Gaussian numbers (re, im each N(0,1)) from a counter-based generator
void launch_gauss(void* out, int t, size_t n, unsigned long long seed, hipStream_t st);

// equivariant network (net.hip): C = net_channels() channels, fields [C][12][V] FP32
int net_channels();
void launch_ptc(const Geo& g, const float2* W, const float2* in, float2* out, const double2* U, int adjoint,
                hipStream_t st);
int ptc_wgrad_nwg(const Geo& g);
void launch_ptc_wgrad(const Geo& g, const float2* gout, const float2* in, const double2* U, float2* part,
                      float2* grad, hipStream_t st);
void launch_net_loss_coef(int nblk, const double2* G, const double2* B, size_t rs, double scale, float2* coefQ,
                          float2* coefA, double* lpart, hipStream_t st);
void launch_adam(float2* w, const float2* grad, float2* m, float2* v, size_t n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t st);

}  // namespace wc
