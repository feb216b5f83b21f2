// Fine-level kernels: layout conversion, clover construction, the
// Wilson-clover operator of eq. (1) (full, domain-decomposed D_SAP and single
// domain-crossing hops) and the SAP smoother (Sec. 3) with minimal-residual
// block solves.
//
// Internal layouts (blocked site order, block-major planes, see wc_common.h):
//   spinor  [rhs][blk][12 = spin*3 + colour][Vb]          complex (double2 / float2)
//   links   [blk][36 = mu*9 + row*3 + col][Vb]           complex (double2: U;
//           half2: the hop matrices -kappa U, the form the FP32 kernels use)
//   clover  [blk][36 pairs][Vb]: per chirality b (pairs 18b..18b+17) the
//           Hermitian 6x6 block as 6 real diagonal entries (pairs 0..2)
//           followed by the 15 upper entries (i<j, row-major) as complex
//           numbers.
#include "wc_dirac.h"
#include "wc_kernels.h"

namespace wc {

// Logical (tile, right-hand-side group) of a workgroup in a 1-D grid of
// round8(ntile * ng) workgroups, the groups fastest: the groups of one tile
// are consecutive on one XCD, so the tile's links and clover are read from
// memory once and then from that XCD's L2.  False for the padding workgroups.
__device__ __forceinline__ bool tile_rhs(int ntile, int ng, int& tile, int& rg) {
  const int n = ntile * ng;
  const int L = xcd_remap(blockIdx.x, n);
  if (L >= n) return false;
  tile = L / ng;
  rg = L - tile * ng;
  return true;
}

// ---------------------------------------------------------------------------
// Layout conversion
// ---------------------------------------------------------------------------
__device__ __forceinline__ int blocked_index(const Geo& g, int cs) {
  int x = cs % g.L[0];
  int r = cs / g.L[0];
  int y = r % g.L[1];
  r /= g.L[1];
  int z = r % g.L[2];
  int t = r / g.L[2];
  int c[4] = {x, y, z, t};
  int blk = 0, loc = 0;
#pragma unroll
  for (int m = 3; m >= 0; --m) {
    blk = blk * g.NB[m] + c[m] / g.B[m];
    loc = loc * g.B[m] + c[m] % g.B[m];
  }
  return blk * g.Vb + loc;
}

template <class TO>
__global__ __launch_bounds__(256) void k_pack_spinor(Geo g, const double2* __restrict__ canon, TO* __restrict__ out,
                                                     size_t out_rs) {
  int cs = blockIdx.x * 256 + threadIdx.x;
  if (cs >= g.V) return;
  int r = blockIdx.y;
  int s = blocked_index(g, cs);
  const double2* src = canon + ((size_t)r * g.V + cs) * 12;
  TO* dst = out + r * out_rs;
  const size_t fb = fbase(g, 12, s);
#pragma unroll
  for (int a = 0; a < 12; ++a) st(dst, (size_t)a * g.Vb + fb, ld<double>(src, a));
}

template <class TI>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geo g, const TI* __restrict__ in, size_t in_rs,
                                                       double2* __restrict__ canon) {
  int cs = blockIdx.x * 256 + threadIdx.x;
  if (cs >= g.V) return;
  int r = blockIdx.y;
  int s = blocked_index(g, cs);
  double2* dst = canon + ((size_t)r * g.V + cs) * 12;
  const TI* src = in + r * in_rs;
  const size_t fb = fbase(g, 12, s);
#pragma unroll
  for (int a = 0; a < 12; ++a) st(dst, a, ld<double>(src, (size_t)a * g.Vb + fb));
}

// U64 = U; U16 = the hop matrices h U in FP16 (h = -kappa: one rounding of the
// FP64 product), the form in which the mixed-precision kernels apply them
__global__ __launch_bounds__(256) void k_pack_gauge(Geo g, const double2* __restrict__ canon,
                                                    double2* __restrict__ U64, half2_t* __restrict__ U16, double h) {
  int cs = blockIdx.x * 256 + threadIdx.x;
  if (cs >= g.V) return;
  int mu = blockIdx.y;
  int s = blocked_index(g, cs);
  const double2* src = canon + ((size_t)mu * g.V + cs) * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double2 v = src[e];
    size_t o = (size_t)(mu * 9 + e) * g.Vb + fbase(g, 36, s);
    U64[o] = v;
    st(U16, o, cplx<double>{h * v.x, h * v.y});
  }
}

// pack a full Hermitian 6x6 chiral block pair (canonical [2][6][6]) into 36 pairs
__device__ __forceinline__ void clover_pack_site(const double2 (&f)[2][6][6], int ps, size_t base, double2* C64,
                                                 half2_t* C16) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    double d[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] = f[b][i][i].x;
    double2 pr[18];
    pr[0] = make_double2(d[0], d[1]);
    pr[1] = make_double2(d[2], d[3]);
    pr[2] = make_double2(d[4], d[5]);
    int k = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j) pr[k++] = f[b][i][j];
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      size_t o = (size_t)(18 * b + q) * ps + base;
      C64[o] = pr[q];
      if (C16) st(C16, o, cplx<double>{pr[q].x, pr[q].y});
    }
  }
}

__global__ __launch_bounds__(256) void k_pack_clover(Geo g, const double2* __restrict__ canon,
                                                     double2* __restrict__ C64, half2_t* __restrict__ C16) {
  int cs = blockIdx.x * 256 + threadIdx.x;
  if (cs >= g.V) return;
  int s = blocked_index(g, cs);
  double2 f[2][6][6];
  const double2* src = canon + (size_t)cs * 72;
  for (int b = 0; b < 2; ++b)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) f[b][i][j] = src[(b * 6 + i) * 6 + j];
  clover_pack_site(f, g.Vb, fbase(g, 36, s), C64, C16);
}

__global__ __launch_bounds__(256) void k_unpack_clover(Geo g, const double2* __restrict__ C64,
                                                       double2* __restrict__ canon) {
  int cs = blockIdx.x * 256 + threadIdx.x;
  if (cs >= g.V) return;
  int s = blocked_index(g, cs);
  double2* dst = canon + (size_t)cs * 72;
  for (int b = 0; b < 2; ++b) {
    double2 pr[18];
    for (int q = 0; q < 18; ++q) pr[q] = C64[(size_t)(18 * b + q) * g.Vb + fbase(g, 36, s)];
    double d[6] = {pr[0].x, pr[0].y, pr[1].x, pr[1].y, pr[2].x, pr[2].y};
    int k = 3;
    for (int i = 0; i < 6; ++i) {
      dst[(b * 6 + i) * 6 + i] = make_double2(d[i], 0.0);
      for (int j = i + 1; j < 6; ++j) {
        double2 u = pr[k++];
        dst[(b * 6 + i) * 6 + j] = u;
        dst[(b * 6 + j) * 6 + i] = make_double2(u.x, -u.y);
      }
    }
  }
}

// M(x) = (1 + F(x))^-1 - 1 per chirality block, from the packed FP64 clover,
// in the packed clover format, FP16 (one rounding of the FP64 result): the
// site-local inverse of the even-odd preconditioned domain solve.  Gauss-
// Jordan elimination with partial pivoting in FP64, one thread per (site,
// chirality block).
__global__ __launch_bounds__(256) void k_clover_inverse(Geo g, const double2* __restrict__ C64,
                                                        half2_t* __restrict__ M16) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)2 * g.V) return;
  const int s = (int)(e >> 1), bb = (int)(e & 1);
  const size_t base = fbase(g, 36, s);
  double2 pr[18];
  for (int q = 0; q < 18; ++q) pr[q] = C64[(size_t)(18 * bb + q) * g.Vb + base];
  cplx<double> a[6][12];  // [A | 1]
  const double d[6] = {pr[0].x, pr[0].y, pr[1].x, pr[1].y, pr[2].x, pr[2].y};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 12; ++j) a[i][j] = {0, 0};
  int k = 3;
  for (int i = 0; i < 6; ++i) {
    a[i][i] = {1.0 + d[i], 0};
    a[i][6 + i] = {1.0, 0};
    for (int j = i + 1; j < 6; ++j) {
      const double2 u = pr[k++];
      a[i][j] = {u.x, u.y};
      a[j][i] = {u.x, -u.y};
    }
  }
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    double best = a[col][col].x * a[col][col].x + a[col][col].y * a[col][col].y;
    for (int i = col + 1; i < 6; ++i) {
      const double m2 = a[i][col].x * a[i][col].x + a[i][col].y * a[i][col].y;
      if (m2 > best) {
        best = m2;
        piv = i;
      }
    }
    if (piv != col)
      for (int j = 0; j < 12; ++j) {
        const cplx<double> t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
    const cplx<double> pv = a[col][col];
    const double n2 = pv.x * pv.x + pv.y * pv.y;
    const cplx<double> inv = {pv.x / n2, -pv.y / n2};
    for (int j = 0; j < 12; ++j) a[col][j] = inv * a[col][j];
    for (int i = 0; i < 6; ++i) {
      if (i == col) continue;
      const cplx<double> f = a[i][col];
      for (int j = 0; j < 12; ++j) a[i][j] = a[i][j] - f * a[col][j];
    }
  }
  // the inverse of a Hermitian matrix is Hermitian: pack its diagonal (real)
  // and upper triangle, minus the identity
  double2 out[18];
  out[0] = make_double2(a[0][6].x - 1.0, a[1][7].x - 1.0);
  out[1] = make_double2(a[2][8].x - 1.0, a[3][9].x - 1.0);
  out[2] = make_double2(a[4][10].x - 1.0, a[5][11].x - 1.0);
  k = 3;
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j) out[k++] = make_double2(a[i][6 + j].x, a[i][6 + j].y);
  for (int q = 0; q < 18; ++q)
    st(M16, (size_t)(18 * bb + q) * g.Vb + base, cplx<double>{out[q].x, out[q].y});
}

void launch_clover_inverse(const Geo& g, const double2* C64, half2_t* M16, hipStream_t st) {
  const size_t n = (size_t)2 * g.V;
  k_clover_inverse<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(g, C64, M16);
}

// ---------------------------------------------------------------------------
// Clover construction: F(x) = i c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x),
// Fhat = (Q - Q^dag) / 8, Q = sum of the four plaquette leaves at x in the
// (mu, nu) plane (each traversed mu then nu).  FP64, once per gauge field.
// ---------------------------------------------------------------------------
struct Su3 {
  cplx<double> a[9];
};
__device__ __forceinline__ Su3 su3_load(const Geo& g, const double2* U, int mu, int s) {
  Su3 m;
  const size_t fb = fbase(g, 36, s);
  for (int e = 0; e < 9; ++e) m.a[e] = ld<double>(U, (size_t)(mu * 9 + e) * g.Vb + fb);
  return m;
}
__device__ __forceinline__ Su3 su3_mul(const Su3& x, const Su3& y) {
  Su3 z;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> acc = {0, 0};
      for (int k = 0; k < 3; ++k) cmac(acc, x.a[i * 3 + k], y.a[k * 3 + j]);
      z.a[i * 3 + j] = acc;
    }
  return z;
}
__device__ __forceinline__ Su3 su3_dag(const Su3& x) {
  Su3 z;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) z.a[i * 3 + j] = cj(x.a[j * 3 + i]);
  return z;
}

// site index of x + da*e_a + db*e_b (da, db in {-1, 0, 1}) on the periodic lattice
__device__ __forceinline__ int shifted(const Geo& g, int s, int a, int da, int b, int db) {
  int sign;
  bool inb;
  if (da != 0) {
    SiteCoord c = decompose(g, s);
    s = da > 0 ? neighbour<true>(g, s, c, a, sign, inb) : neighbour<false>(g, s, c, a, sign, inb);
  }
  if (db != 0) {
    SiteCoord c = decompose(g, s);
    s = db > 0 ? neighbour<true>(g, s, c, b, sign, inb) : neighbour<false>(g, s, c, b, sign, inb);
  }
  return s;
}

struct SigmaTab {
  double v[6][2][2][2][2];  // [plane][chirality][row][col][re/im]
};

__global__ __launch_bounds__(128) void k_clover_build(Geo g, const double2* __restrict__ U, double kappa,
                                                      double csw, SigmaTab sig, double2* __restrict__ C64,
                                                      half2_t* __restrict__ C16) {
  int s = blockIdx.x * 128 + threadIdx.x;
  if (s >= g.V) return;
  double2 f[2][6][6];
  for (int b = 0; b < 2; ++b)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) f[b][i][j] = make_double2(0.0, 0.0);
  int plane = 0;
  for (int mu = 0; mu < 4; ++mu) {
    for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
      // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
      Su3 l1 = su3_mul(su3_mul(su3_load(g, U, mu, s), su3_load(g, U, nu, shifted(g, s, mu, 1, nu, 0))),
                       su3_mul(su3_dag(su3_load(g, U, mu, shifted(g, s, nu, 1, mu, 0))),
                               su3_dag(su3_load(g, U, nu, s))));
      // leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
      int xm = shifted(g, s, mu, -1, nu, 0);
      Su3 l2 = su3_mul(su3_mul(su3_load(g, U, nu, s), su3_dag(su3_load(g, U, mu, shifted(g, s, mu, -1, nu, 1)))),
                       su3_mul(su3_dag(su3_load(g, U, nu, xm)), su3_load(g, U, mu, xm)));
      // leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
      int xmn = shifted(g, s, mu, -1, nu, -1);
      int xn = shifted(g, s, nu, -1, mu, 0);
      Su3 l3 = su3_mul(su3_mul(su3_dag(su3_load(g, U, mu, xm)), su3_dag(su3_load(g, U, nu, xmn))),
                       su3_mul(su3_load(g, U, mu, xmn), su3_load(g, U, nu, xn)));
      // leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
      Su3 l4 = su3_mul(su3_mul(su3_dag(su3_load(g, U, nu, xn)), su3_load(g, U, mu, xn)),
                       su3_mul(su3_load(g, U, nu, shifted(g, s, mu, 1, nu, -1)), su3_dag(su3_load(g, U, mu, s))));
      Su3 fh;
      for (int e = 0; e < 9; ++e) {
        int i = e / 3, j = e % 3;
        cplx<double> q = l1.a[e] + l2.a[e] + l3.a[e] + l4.a[e];
        cplx<double> qt = l1.a[j * 3 + i] + l2.a[j * 3 + i] + l3.a[j * 3 + i] + l4.a[j * 3 + i];
        fh.a[e] = 0.125 * (q - cj(qt));
      }
      // F_b[(s1,c1),(s2,c2)] += i csw kappa sigma_b[s1][s2] Fhat[c1][c2]
      for (int b = 0; b < 2; ++b)
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s2 = 0; s2 < 2; ++s2) {
            cplx<double> sg = {sig.v[plane][b][s1][s2][0], sig.v[plane][b][s1][s2][1]};
            cplx<double> fac = cplx<double>{0.0, csw * kappa} * sg;
            for (int c1 = 0; c1 < 3; ++c1)
              for (int c2 = 0; c2 < 3; ++c2) {
                cplx<double> add = fac * fh.a[c1 * 3 + c2];
                double2& e = f[b][s1 * 3 + c1][s2 * 3 + c2];
                e.x += add.x;
                e.y += add.y;
              }
          }
    }
  }
  clover_pack_site(f, g.Vb, fbase(g, 36, s), C64, C16);
}

// ---------------------------------------------------------------------------
// Dslash family
// ---------------------------------------------------------------------------
template <class R, class TI, class TO, class TL, class TC, int OP>
__global__ __launch_bounds__(512) void k_dslash(Geo g, const TI* __restrict__ in, size_t in_rs, TO* __restrict__ out,
                                                size_t out_rs, const TO* __restrict__ b, const TL* __restrict__ U,
                                                const TC* __restrict__ C, R kappa, int hopdir, int chir, int ng) {
  const int bs = blockDim.x;
  int ntile = (g.V + bs - 1) / bs;
  int tile, r;
  if (!tile_rhs(ntile, ng, tile, r)) return;
  int s = tile * bs + threadIdx.x;
  if (s >= g.V) return;
  const TI* inr = in + r * in_rs;
  SiteCoord c = decompose(g, s);
  const int ps = g.Vb;
  const size_t fb12 = fbase_b(g, 12, s, c.blk), fb36 = fbase_b(g, 36, s, c.blk);
  cplx<R> acc[12];
  cplx<R> psi[12];
  cplx<R> u[9];
  const int a0 = chir == 1 ? 6 : 0, a1 = chir == 0 ? 6 : 12;  // components kept by the chirality projection
  if (OP != OP_HOP) {
    ld_spinor<R>(inr, ps, fb12, psi);
#pragma unroll
    for (int a = 0; a < 12; ++a)
      if (a < a0 || a >= a1) psi[a] = {0, 0};
#pragma unroll
    for (int a = 0; a < 12; ++a) acc[a] = psi[a];
    clover_acc<R>(C, ps, fb36, psi, acc);
  } else {
#pragma unroll
    for (int a = 0; a < 12; ++a) acc[a] = {0, 0};
  }
  // one hop at a time (not unrolled): keeps a single neighbour spinor live
#pragma unroll 1
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fw = dir < 4;
    if (OP == OP_HOP && dir != hopdir) continue;
    int sign, nblk;
    bool inb;
    int nb = fw ? neighbour<true>(g, s, c, mu, sign, inb, nblk) : neighbour<false>(g, s, c, mu, sign, inb, nblk);
    if (OP == OP_DSAP && !inb) continue;
    if (OP == OP_HOP && inb) continue;
    ld_spinor<R>(inr, ps, fbase_b(g, 12, nb, nblk), psi);
#pragma unroll
    for (int a = 0; a < 12; ++a)
      if (a < a0 || a >= a1) psi[a] = {0, 0};
    R coef = -kappa * (R)sign;
    if (fw) {
      ld_link<R>(U, ps, mu, fb36, u);
      hop_any<true>(mu, psi, u, coef, acc);
    } else {
      ld_link<R>(U, ps, mu, fbase_b(g, 36, nb, nblk), u);
      hop_any<false>(mu, psi, u, coef, acc);
    }
  }
  TO* outr = out + r * out_rs;
  if (b) {
    const TO* br = b + r * out_rs;
#pragma unroll
    for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, ld<R>(br, (size_t)a * ps + fb12) - acc[a]);
  } else {
#pragma unroll
    for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, acc[a]);
  }
}

// One hop for a single colour row: with w the link row (forward: U[r][.],
// backward: conj(U[.][r]) = row r of U^dag), acc[spin] += coef * row r of
// (1 -/+ gamma_mu) W psi.
template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_row_acc(const cplx<R> (&psi)[12], const cplx<R> (&w)[3], R coef,
                                            cplx<R> (&acc)[4]) {
  using P = Proj<MU>;
  constexpr int T0 = FWD ? P::t0 : (P::t0 ^ 2);
  constexpr int T1 = FWD ? P::t1 : (P::t1 ^ 2);
  constexpr int S0 = FWD ? P::s0 : (P::s0 ^ 2);
  constexpr int S1 = FWD ? P::s1 : (P::s1 ^ 2);
  cplx<R> g0 = {0, 0}, g1 = {0, 0};
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    cplx<R> h0 = psi[cc] + unit<T0>(psi[(2 + P::pi0) * 3 + cc]);
    cplx<R> h1 = psi[3 + cc] + unit<T1>(psi[(2 + P::pi1) * 3 + cc]);
    if (FWD) {
      cmac(g0, w[cc], h0);
      cmac(g1, w[cc], h1);
    } else {
      cjmac(g0, w[cc], h0);
      cjmac(g1, w[cc], h1);
    }
  }
  g0 = coef * g0;
  g1 = coef * g1;
  acc[0] = acc[0] + g0;
  acc[1] = acc[1] + g1;
  acc[2] = acc[2] + unit<S0>(P::pi0 == 0 ? g0 : g1);
  acc[3] = acc[3] + unit<S1>(P::pi1 == 0 ? g0 : g1);
}

// Colour-split variant of the full operator: three wavefronts share a tile
// of 64 sites, wavefront r computing the colour-r row of the result for all 4
// spins.  Each thread reads the whole neighbour spinor (shared through the
// caches with the other two rows) but only row r of each link, and holds a
// quarter of the accumulators, for higher occupancy.
template <class R, class TI, class TO, class TL, class TC>
__global__ __launch_bounds__(192) void k_dslash_cs(Geo g, const TI* __restrict__ in, size_t in_rs,
                                                   TO* __restrict__ out, size_t out_rs, const TO* __restrict__ b,
                                                   const TL* __restrict__ U, const TC* __restrict__ C, R kappa,
                                                   int ng) {
  const int ntile = (g.V + 63) >> 6;
  int tile, rh;
  if (!tile_rhs(ntile, ng, tile, rh)) return;
  const int r = threadIdx.x >> 6;  // colour row of this wavefront
  const int s = tile * 64 + (threadIdx.x & 63);
  if (s >= g.V) return;
  const TI* inr = in + rh * in_rs;
  SiteCoord c = decompose(g, s);
  const int ps = g.Vb;
  const size_t fb12 = fbase_b(g, 12, s, c.blk), fb36 = fbase_b(g, 36, s, c.blk);
  cplx<R> psi[12];
  cplx<R> acc[4];
  ld_spinor<R>(inr, ps, fb12, psi);
  // (1 + F) psi, row r of each spin: F row (b, sl*3 + r) of chiral block b
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) acc[sp] = psi[sp * 3 + r];
#pragma unroll
  for (int bq = 0; bq < 2; ++bq) {
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int i = sl * 3 + r;  // row inside the 6x6 block
      cplx<R> a = {0, 0};
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        cplx<R> f;
        if (i == j) {
          cplx<R> dp = ld<R>(C, (size_t)(18 * bq + i / 2) * ps + fb36);
          f = {(i & 1) ? dp.y : dp.x, (R)0};
        } else {
          int lo = i < j ? i : j, hi = i < j ? j : i;
          int k = 3 + lo * 5 - lo * (lo - 1) / 2 + (hi - lo - 1);  // index of (lo, hi) among the 15 upper entries
          cplx<R> u = ld<R>(C, (size_t)(18 * bq + k) * ps + fb36);
          f = i < j ? u : cj(u);
        }
        cmac(a, f, psi[6 * bq + j]);
      }
      acc[2 * bq + sl] = acc[2 * bq + sl] + a;
    }
  }
#pragma unroll 1
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fw = dir < 4;
    int sign, nblk;
    bool inb;
    int nb = fw ? neighbour<true>(g, s, c, mu, sign, inb, nblk) : neighbour<false>(g, s, c, mu, sign, inb, nblk);
    ld_spinor<R>(inr, ps, fbase_b(g, 12, nb, nblk), psi);
    const size_t nb36 = fbase_b(g, 36, nb, nblk);
    cplx<R> u[3];  // row r of U_mu(x) (forward) or column r of U_mu(x-mu) (backward: row r of U^dag, conjugated)
#pragma unroll
    for (int e = 0; e < 3; ++e)
      u[e] = fw ? ld<R>(U, (size_t)(mu * 9 + r * 3 + e) * ps + fb36) : ld<R>(U, (size_t)(mu * 9 + e * 3 + r) * ps + nb36);
    const R coef = -kappa * (R)sign;
    switch (dir) {
      case 0: hop_row_acc<0, true>(psi, u, coef, acc); break;
      case 1: hop_row_acc<1, true>(psi, u, coef, acc); break;
      case 2: hop_row_acc<2, true>(psi, u, coef, acc); break;
      case 3: hop_row_acc<3, true>(psi, u, coef, acc); break;
      case 4: hop_row_acc<0, false>(psi, u, coef, acc); break;
      case 5: hop_row_acc<1, false>(psi, u, coef, acc); break;
      case 6: hop_row_acc<2, false>(psi, u, coef, acc); break;
      default: hop_row_acc<3, false>(psi, u, coef, acc); break;
    }
  }
  TO* outr = out + rh * out_rs;
  if (b) {
    const TO* br = b + rh * out_rs;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      size_t o = (size_t)(sp * 3 + r) * ps + fb12;
      st(outr, o, ld<R>(br, o) - acc[sp]);
    }
  } else {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) st(outr, (size_t)(sp * 3 + r) * ps + fb12, acc[sp]);
  }
}

// Multi-RHS variant of the full operator: a thread applies D at one site to
// NR right-hand sides, so that the site's clover block and each link are
// loaded once and used NR times (grid.y = right-hand-side groups).
template <class R, class TI, class TO, class TL, class TC, int NR>
__global__ __launch_bounds__(256) void k_dslash_nr(Geo g, int nrhs, const TI* __restrict__ in, size_t in_rs,
                                                   TO* __restrict__ out, size_t out_rs, const TO* __restrict__ b,
                                                   const TL* __restrict__ U, const TC* __restrict__ C, R kappa) {
  const int ntile = (g.V + 255) >> 8;
  int tile, rg;
  if (!tile_rhs(ntile, (nrhs + NR - 1) / NR, tile, rg)) return;
  const int s = tile * 256 + threadIdx.x;
  if (s >= g.V) return;
  const int r0 = rg * NR;
  const SiteCoord c = decompose(g, s);
  const int ps = g.Vb;
  const size_t fb12 = fbase_b(g, 12, s, c.blk), fb36 = fbase_b(g, 36, s, c.blk);
  cplx<R> acc[NR][12], psi[12], u[9];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (r0 + q < nrhs) {
      ld_spinor<R>(in + (size_t)(r0 + q) * in_rs, ps, fb12, psi);
#pragma unroll
      for (int a = 0; a < 12; ++a) acc[q][a] = psi[a];
      clover_acc<R>(C, ps, fb36, psi, acc[q]);
    }
  }
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const int mu = k >> 1;
    const bool fw = (k & 1) == 0;
    int sign, nblk;
    bool inb;
    const int nb = fw ? neighbour<true>(g, s, c, mu, sign, inb, nblk) : neighbour<false>(g, s, c, mu, sign, inb, nblk);
    const size_t nb12 = fbase_b(g, 12, nb, nblk);
    ld_link<R>(U, ps, mu, fw ? fb36 : fbase_b(g, 36, nb, nblk), u);
    const R coef = -kappa * (R)sign;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      if (r0 + q < nrhs) {
        ld_spinor<R>(in + (size_t)(r0 + q) * in_rs, ps, nb12, psi);
        if (fw)
          hop_any<true>(mu, psi, u, coef, acc[q]);
        else
          hop_any<false>(mu, psi, u, coef, acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (r0 + q < nrhs) {
      TO* outr = out + (size_t)(r0 + q) * out_rs;
      if (b) {
        const TO* br = b + (size_t)(r0 + q) * out_rs;
#pragma unroll
        for (int a = 0; a < 12; ++a)
          st(outr, (size_t)a * ps + fb12, ld<R>(br, (size_t)a * ps + fb12) - acc[q][a]);
      } else {
#pragma unroll
        for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, acc[q][a]);
      }
    }
  }
}

// LDS-staged variant of the full operator.  A workgroup takes one tile: a
// slab of tt consecutive t-slices of one block (TS = B0 B1 B2 tt sites, one
// thread per site).  The tile's input spinors are staged in LDS once, so every
// hop to a neighbour inside the tile reads LDS; hops leaving the tile read
// memory.  The forward and backward hop of each direction are taken back to
// back, so that the backward link U_mu(x - mu), the forward link of another
// site of the tile, is read while that line is still in the caches.
template <class R, class TI, class TO, class TL, class TC>
__global__ __launch_bounds__(256) void k_dslash_lds(Geo g, int tt, const TI* __restrict__ in, size_t in_rs,
                                                    TO* __restrict__ out, size_t out_rs, const TO* __restrict__ b,
                                                    const TL* __restrict__ U, const TC* __restrict__ C, R kappa,
                                                    int ng) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* sp = (cplx<R>*)smem;  // [12][TS]
  const int TS = blockDim.x;
  const int per_blk = g.B[3] / tt;
  const int ntile = g.nblk * per_blk;
  int tile, rh;
  if (!tile_rhs(ntile, ng, tile, rh)) return;  // whole workgroup: no barrier is left waiting
  const int blk = tile / per_blk, tb = tile - blk * per_blk;
  const int loc0 = tb * TS;
  const int l = threadIdx.x;
  const int s = blk * g.Vb + loc0 + l;
  const TI* inr = in + rh * in_rs;
  const SiteCoord c = decompose(g, s);
  const int ps = g.Vb;
  const size_t fb12 = fbase_b(g, 12, s, blk), fb36 = fbase_b(g, 36, s, blk);
  const int t_lo = tb * tt, t_hi = t_lo + tt;
  cplx<R> acc[12], psi[12], u[9];
  ld_spinor<R>(inr, ps, fb12, psi);
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    sp[a * TS + l] = psi[a];
    acc[a] = psi[a];
  }
  clover_acc<R>(C, ps, fb36, psi, acc);
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const int mu = k >> 1;
    const bool fw = (k & 1) == 0;
    int sign, nblk;
    bool inb;
    const int nb = fw ? neighbour<true>(g, s, c, mu, sign, inb, nblk) : neighbour<false>(g, s, c, mu, sign, inb, nblk);
    bool intile = inb;
    if (mu == 3) intile = inb && (fw ? c.lc[3] + 1 < t_hi : c.lc[3] - 1 >= t_lo);
    if (intile) {
      const int nl = nb - blk * g.Vb - loc0;
#pragma unroll
      for (int a = 0; a < 12; ++a) psi[a] = sp[a * TS + nl];
    } else {
      ld_spinor<R>(inr, ps, fbase_b(g, 12, nb, nblk), psi);
    }
    const R coef = -kappa * (R)sign;
    if (fw) {
      ld_link<R>(U, ps, mu, fb36, u);
      hop_any<true>(mu, psi, u, coef, acc);
    } else {
      ld_link<R>(U, ps, mu, fbase_b(g, 36, nb, nblk), u);
      hop_any<false>(mu, psi, u, coef, acc);
    }
  }
  TO* outr = out + rh * out_rs;
  if (b) {
    const TO* br = b + rh * out_rs;
#pragma unroll
    for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, ld<R>(br, (size_t)a * ps + fb12) - acc[a]);
  } else {
#pragma unroll
    for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, acc[a]);
  }
}

// Half-spinor exchange variant of the full operator.  Tiles as in
// k_dslash_lds (a t-slab of one block, one thread per site, the tile's input
// spinors in LDS).  For each direction mu a thread loads only its own link
// U_mu(x): it takes its forward hop, and it computes the projected backward
// hop -kappa sign (1 + gamma_mu) U_mu(x)^dag psi(x) that the site x + mu
// receives, handing it over through LDS as a half-spinor (6 complex).  A site
// whose x - mu lies outside the tile takes that hop itself from memory.  Every
// link of the tile is read once.
template <class R, class TI, class TO, class TL, class TC>
__global__ __launch_bounds__(256) void k_dslash_hx(Geo g, int tt, const TI* __restrict__ in, size_t in_rs,
                                                   TO* __restrict__ out, size_t out_rs, const TO* __restrict__ b,
                                                   const TL* __restrict__ U, const TC* __restrict__ C, R kappa,
                                                    int ng) {
  extern __shared__ __align__(16) char smem[];
  const int TS = blockDim.x;
  cplx<R>* sp = (cplx<R>*)smem;  // [12][TS] input spinors of the tile
  cplx<R>* hx = sp + 12 * TS;     // [6][TS] backward half-spinors by receiving site
  const int per_blk = g.B[3] / tt;
  const int ntile = g.nblk * per_blk;
  int tile, rh;
  if (!tile_rhs(ntile, ng, tile, rh)) return;  // whole workgroup: no barrier is left waiting
  const int blk = tile / per_blk, tb = tile - blk * per_blk;
  const int loc0 = tb * TS;
  const int l = threadIdx.x;
  const int s = blk * g.Vb + loc0 + l;
  const TI* inr = in + rh * in_rs;
  const SiteCoord c = decompose(g, s);
  const int ps = g.Vb;
  const size_t fb12 = fbase_b(g, 12, s, blk), fb36 = fbase_b(g, 36, s, blk);
  const int t_lo = tb * tt, t_hi = t_lo + tt;
  cplx<R> acc[12];
  {
    cplx<R> psi[12];
    ld_spinor<R>(inr, ps, fb12, psi);
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      sp[a * TS + l] = psi[a];
      acc[a] = psi[a];
    }
    clover_acc<R>(C, ps, fb36, psi, acc);
  }
  __syncthreads();
  cplx<R> psi[12], u[9], g0[3], g1[3];
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    int sign, nblk;
    bool inb;
    const int nbf = neighbour<true>(g, s, c, mu, sign, inb, nblk);
    const bool fin = inb && (mu != 3 || c.lc[3] + 1 < t_hi);
    const R coef = -kappa * (R)sign;
    ld_link<R>(U, ps, mu, fb36, u);
    // the backward hop that x + mu receives from x, handed over through LDS
    if (fin) {
#pragma unroll
      for (int a = 0; a < 12; ++a) psi[a] = sp[a * TS + l];
      hop_half_any<false>(mu, psi, u, coef, g0, g1);
      const int nl = nbf - blk * g.Vb - loc0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        hx[q * TS + nl] = g0[q];
        hx[(3 + q) * TS + nl] = g1[q];
      }
#pragma unroll
      for (int a = 0; a < 12; ++a) psi[a] = sp[a * TS + nl];
    } else {
      ld_spinor<R>(inr, ps, fbase_b(g, 12, nbf, nblk), psi);
    }
    // the forward hop x -> x + mu
    hop_any<true>(mu, psi, u, coef, acc);
    __syncthreads();
    // the backward hop x - mu -> x
    const int nbb = neighbour<false>(g, s, c, mu, sign, inb, nblk);
    const bool bin = inb && (mu != 3 || c.lc[3] - 1 >= t_lo);
    if (bin) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        g0[q] = hx[q * TS + l];
        g1[q] = hx[(3 + q) * TS + l];
      }
      hop_recon_any<false>(mu, g0, g1, acc);
    } else {
      ld_spinor<R>(inr, ps, fbase_b(g, 12, nbb, nblk), psi);
      ld_link<R>(U, ps, mu, fbase_b(g, 36, nbb, nblk), u);
      hop_any<false>(mu, psi, u, -kappa * (R)sign, acc);
    }
    __syncthreads();  // hx is rewritten by the next direction
  }
  TO* outr = out + rh * out_rs;
  if (b) {
    const TO* br = b + rh * out_rs;
#pragma unroll
    for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, ld<R>(br, (size_t)a * ps + fb12) - acc[a]);
  } else {
#pragma unroll
    for (int a = 0; a < 12; ++a) st(outr, (size_t)a * ps + fb12, acc[a]);
  }
}

// t-slices per tile of the LDS-staged operator (tile <= 256 sites), 0 if the
// block's x-y-z cross-section alone exceeds 256 sites
int dslash_lds_slices(const Geo& g) {
  const int bxyz = g.B[0] * g.B[1] * g.B[2];
  if (bxyz > 256) return 0;
  int tt = 1;
  for (int d = 1; d <= g.B[3]; ++d)
    if (g.B[3] % d == 0 && bxyz * d <= 256) tt = d;
  return tt;
}

template <class R, class TI, class TO, class TL, class TC>
static void dslash_dispatch(const DslashArgs& a, hipStream_t st) {
  if ((a.block_size == -12 || a.block_size == -14) && a.op == OP_D) {
    const int NR = -a.block_size - 10;
    const int nt = (a.g.V + 255) / 256;
    dim3 grid(round8(nt * ((a.nrhs + NR - 1) / NR)));
    auto go = [&](auto kern) {
      kern<<<grid, 256, 0, st>>>(a.g, a.nrhs, (const TI*)a.in, a.in_rs, (TO*)a.out, a.out_rs, (const TO*)a.b,
                                 (const TL*)a.U, (const TC*)a.C, (R)a.kappa);
    };
    if (NR == 2)
      go(k_dslash_nr<R, TI, TO, TL, TC, 2>);
    else if (NR == 4)
      go(k_dslash_nr<R, TI, TO, TL, TC, 4>);
    else
      throw std::runtime_error("launch_dslash: unsupported right-hand sides per thread");
    return;
  }
  if ((a.block_size == -2 || a.block_size == -3) && a.op == OP_D) {
    const int tt = dslash_lds_slices(a.g);
    if (tt < 1) throw std::runtime_error("launch_dslash: no LDS tile for this block shape");
    const int TS = a.g.B[0] * a.g.B[1] * a.g.B[2] * tt;
    const int ntile = a.g.nblk * (a.g.B[3] / tt);
    const dim3 grid(round8(ntile * a.nrhs));
    if (a.block_size == -2)
      k_dslash_lds<R, TI, TO, TL, TC><<<grid, TS, (size_t)12 * TS * sizeof(cplx<R>), st>>>(
          a.g, tt, (const TI*)a.in, a.in_rs, (TO*)a.out, a.out_rs, (const TO*)a.b, (const TL*)a.U, (const TC*)a.C,
          (R)a.kappa, a.nrhs);
    else
      k_dslash_hx<R, TI, TO, TL, TC><<<grid, TS, (size_t)18 * TS * sizeof(cplx<R>), st>>>(
          a.g, tt, (const TI*)a.in, a.in_rs, (TO*)a.out, a.out_rs, (const TO*)a.b, (const TL*)a.U, (const TC*)a.C,
          (R)a.kappa, a.nrhs);
    return;
  }
  if (a.block_size < 0 && a.op == OP_D) {
    int nt = (a.g.V + 63) / 64;
    k_dslash_cs<R, TI, TO, TL, TC><<<dim3(round8(nt * a.nrhs)), 192, 0, st>>>(
        a.g, (const TI*)a.in, a.in_rs, (TO*)a.out, a.out_rs, (const TO*)a.b, (const TL*)a.U, (const TC*)a.C,
        (R)a.kappa, a.nrhs);
    return;
  }
  const int bs = a.block_size > 0 ? a.block_size : 256;
  int ntile = (a.g.V + bs - 1) / bs;
  dim3 grid(round8(ntile * a.nrhs));
  const TI* in = (const TI*)a.in;
  TO* out = (TO*)a.out;
  const TO* b = (const TO*)a.b;
  const TL* U = (const TL*)a.U;
  const TC* C = (const TC*)a.C;
  R kappa = (R)a.kappa;
  switch (a.op) {
    case OP_D:
      k_dslash<R, TI, TO, TL, TC, OP_D><<<grid, bs, 0, st>>>(a.g, in, a.in_rs, out, a.out_rs, b, U, C, kappa, 0,
                                                              a.chir, a.nrhs);
      break;
    case OP_DSAP:
      k_dslash<R, TI, TO, TL, TC, OP_DSAP><<<grid, bs, 0, st>>>(a.g, in, a.in_rs, out, a.out_rs, b, U, C, kappa,
                                                                 0, a.chir, a.nrhs);
      break;
    default:
      k_dslash<R, TI, TO, TL, TC, OP_HOP><<<grid, bs, 0, st>>>(a.g, in, a.in_rs, out, a.out_rs, b, U, C, kappa,
                                                                a.hopdir, a.chir, a.nrhs);
      break;
  }
}

void launch_dslash(const DslashArgs& a, hipStream_t st) {
  if (!a.fields16 && !a.compute32) {
    if (a.in_t == C128 && a.out_t == C128)
      return dslash_dispatch<double, double2, double2, double2, double2>(a, st);
    if (a.in_t == C64 && a.out_t == C128)
      return dslash_dispatch<double, float2, double2, double2, double2>(a, st);
  }
  if (a.fields32 && a.compute32) {
    if (a.in_t == C64 && a.out_t == C64) return dslash_dispatch<float, float2, float2, float2, float2>(a, st);
  }
  if (a.fields16 && a.compute32) {
    if (a.in_t == C64 && a.out_t == C64) return dslash_dispatch<float, float2, float2, half2_t, half2_t>(a, st);
    if (a.in_t == C32H && a.out_t == C64) return dslash_dispatch<float, half2_t, float2, half2_t, half2_t>(a, st);
  }
  throw std::runtime_error("launch_dslash: unsupported precision combination");
}

// ---------------------------------------------------------------------------
// SAP smoother.  One workgroup per domain of the active colour and right-hand
// side, one thread per site.  Each half-sweep:
//   1. r_X = (first visit ? b_X : r_X) + kappa * (domain-crossing hops of the
//      other colour's latest correction delta)  -- i.e. r -= D delta restricted
//      to this domain, which equals r = b - D x there (neighbouring domains all
//      have the other colour);
//   2. MR(mr) on D_SAP restricted to the domain from 0 (residual through LDS);
//   3. x_X += correction, r_X = MR residual, delta_X = correction.
// ---------------------------------------------------------------------------
enum { SAP_FIRST = 1, SAP_DELTA = 2, SAP_NO_R = 4, SAP_NO_DELTA = 8, SAP_R_IN = 16 };

template <class R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One DPP move of a float (lanes that the row mask leaves out, or whose
// source lies outside the row, read 0).
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, true));
}

// Sum over the wavefront, valid in lane 63 only: an inclusive scan within
// each row of 16 lanes (row_shr 1, 2, 4, 8), then row 0's total into row 1
// and row 2's into row 3 (row_bcast:15), then rows 0+1 into rows 2 and 3
// (row_bcast:31).  Six dependent VALU steps, where a butterfly of lane
// shuffles makes six round trips through the LDS crossbar.
__device__ __forceinline__ float wave_sum_hi(float v) {
  v += dpp_mov<0x111>(v);
  v += dpp_mov<0x112>(v);
  v += dpp_mov<0x114>(v);
  v += dpp_mov<0x118>(v);
  v += dpp_mov<0x142, 0xa>(v);
  v += dpp_mov<0x143, 0xc>(v);
  return v;
}

template <class R, class TS, class TL, class TC>
__global__ __launch_bounds__(512) void k_sap_half(Geo g, int colour, int flags, int mr, R kappa,
                                                   const TS* __restrict__ b, TS* __restrict__ r, TS* __restrict__ x,
                                                   TS* __restrict__ delta, const TS* __restrict__ xinit, size_t rs,
                                                   const TL* __restrict__ U, const TC* __restrict__ C) {
  extern __shared__ __align__(16) char smem[];
  const int Vb = g.Vb;
  cplx<R>* lds = (cplx<R>*)smem;  // [12][Vb]
  R* red = (R*)(lds + 12 * Vb);   // [nwaves][3]
  // the k-th domain of this colour
  const int half = g.NB[0] >> 1;
  int k = blockIdx.x;
  int row = k / half, j = k - row * half;
  int by = row % g.NB[1];
  int rz = row / g.NB[1];
  int bz = rz % g.NB[2];
  int bt = rz / g.NB[2];
  int bx = 2 * j + ((colour + by + bz + bt) & 1);
  int blk = bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
  const int l = threadIdx.x;
  const bool act = l < Vb;
  const int s = blk * Vb + (act ? l : 0);
  const size_t off = blockIdx.y * rs;
  const int nw = (blockDim.x + 63) >> 6;
  SiteCoord c = decompose(g, s);
  const size_t fb12 = fbase_b(g, 12, s, blk), fb36 = fbase_b(g, 36, s, blk);

  cplx<R> rho[12], xm[12], p[12], psi[12], u[9];
  if (act) {
    ld_spinor<R>((flags & SAP_FIRST) ? b + off : r + off, Vb, fb12, rho);
    if (flags & SAP_DELTA) {
#pragma unroll 1
      for (int mu = 0; mu < 4; ++mu) {
        int sign, nblk;
        bool inb;
        int nb = neighbour<true>(g, s, c, mu, sign, inb, nblk);
        if (!inb) {
          ld_spinor<R>(delta + off, Vb, fbase_b(g, 12, nb, nblk), psi);
          ld_link<R>(U, Vb, mu, fb36, u);
          hop_any<true>(mu, psi, u, kappa * (R)sign, rho);
        }
        nb = neighbour<false>(g, s, c, mu, sign, inb, nblk);
        if (!inb) {
          ld_spinor<R>(delta + off, Vb, fbase_b(g, 12, nb, nblk), psi);
          ld_link<R>(U, Vb, mu, fbase_b(g, 36, nb, nblk), u);
          hop_any<false>(mu, psi, u, kappa * (R)sign, rho);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 12; ++a) xm[a] = {0, 0};

  for (int it = 0; it < mr; ++it) {
    if (act) {
#pragma unroll
      for (int a = 0; a < 12; ++a) lds[a * Vb + l] = rho[a];
    }
    __syncthreads();
    R pr_re = 0, pr_im = 0, pp = 0;
    if (act) {
#pragma unroll
      for (int a = 0; a < 12; ++a) p[a] = rho[a];
      clover_acc<R>(C, Vb, fb36, rho, p);
#pragma unroll 1
      for (int mu = 0; mu < 4; ++mu) {
        int sign;
        bool inb;
        int nb = neighbour<true>(g, s, c, mu, sign, inb);
        if (inb) {
          int nl = nb - blk * Vb;
#pragma unroll
          for (int a = 0; a < 12; ++a) psi[a] = lds[a * Vb + nl];
          ld_link<R>(U, Vb, mu, fb36, u);
          hop_any<true>(mu, psi, u, -kappa * (R)sign, p);
        }
        nb = neighbour<false>(g, s, c, mu, sign, inb);
        if (inb) {
          int nl = nb - blk * Vb;
#pragma unroll
          for (int a = 0; a < 12; ++a) psi[a] = lds[a * Vb + nl];
          ld_link<R>(U, Vb, mu, fb36 + (nl - l), u);  // same block: the neighbour's planes are nl - l further
          hop_any<false>(mu, psi, u, -kappa * (R)sign, p);
        }
      }
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        pr_re += p[a].x * rho[a].x + p[a].y * rho[a].y;
        pr_im += p[a].x * rho[a].y - p[a].y * rho[a].x;
        pp += p[a].x * p[a].x + p[a].y * p[a].y;
      }
    }
    pr_re = wave_sum(pr_re);
    pr_im = wave_sum(pr_im);
    pp = wave_sum(pp);
    if ((l & 63) == 0) {
      red[(l >> 6) * 3 + 0] = pr_re;
      red[(l >> 6) * 3 + 1] = pr_im;
      red[(l >> 6) * 3 + 2] = pp;
    }
    __syncthreads();
    R sre = 0, sim = 0, spp = 0;
    for (int w = 0; w < nw; ++w) {
      sre += red[w * 3 + 0];
      sim += red[w * 3 + 1];
      spp += red[w * 3 + 2];
    }
    cplx<R> alpha = {0, 0};
    if (spp > 0) alpha = {sre / spp, sim / spp};
    if (act) {
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        xm[a] = xm[a] + alpha * rho[a];
        rho[a] = rho[a] - alpha * p[a];
      }
    }
  }
  if (act) {
    TS* xr = x + off;
    TS* rr = r + off;
    TS* dr = delta + off;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      size_t o = (size_t)a * Vb + fb12;
      cplx<R> x0 = {0, 0};
      if (!(flags & SAP_FIRST)) x0 = ld<R>(xr, o);
      else if (xinit) x0 = ld<R>(xinit + off, o);
      st(xr, o, x0 + xm[a]);
      st(rr, o, rho[a]);
      st(dr, o, xm[a]);
    }
  }
}

// Mixed-precision SAP half-sweep: one workgroup per domain of the active
// colour for ALL right-hand sides.  The domain's FP16 hop matrices are staged
// in LDS and its clover in registers once; the MR block solves of the
// right-hand sides then run in turn with the residual exchanged through LDS.
// Links of hops that leave the domain are not needed by D_SAP; the
// crossing-hop correction of the residual runs before, in k_sap_cross_face
// (from the spin projections that the other colour's domain solves wrote on
// their faces) or, for the even-odd block solve, in k_sap_cross (from its
// whole corrections).
__device__ __forceinline__ cplx<float> h2f(half2_t v) { return {(float)v.x, (float)v.y}; }

template <bool FWD>
__device__ __forceinline__ void hop_h(int mu, const cplx<float> (&psi)[12], const half2_t* u16, float coef,
                                      cplx<float> (&acc)[12]) {
  cplx<float> u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = h2f(u16[e]);
  hop_any<FWD>(mu, psi, u, coef, acc);
}

// The crossing-hop correction of a mixed-precision SAP half-sweep from whole
// block corrections (the even-odd block solve's hand-over; the default path
// uses k_sap_cross_face), as a kernel of its own ahead of the domain solves:
// for every site x of the
// active colour's domains and every right-hand side,
//   r(x) = src(x) - sum_{hops x -> y leaving the domain} sign H delta(y)
// with H the hop's FP16 matrix -kappa U (or its adjoint) spin-projected
// (r = b - D x restricted to the active colour, updated with the other
// colour's last block corrections delta).  src is b on a colour's first visit
// (every site is then written), else r itself (sites without a crossing hop
// are left alone).  One thread per (site, right-hand side): memory-bound
// work at full occupancy, where inside the domain solve's single workgroup
// per CU the dependent global loads of the hops stood exposed.
__global__ __launch_bounds__(256) void k_sap_cross(Geo g, int colour, int first,
                                                   const float2* __restrict__ b, float2* __restrict__ r,
                                                   const float2* __restrict__ delta, size_t rs,
                                                   const half2_t* __restrict__ U) {
  const int Vb = g.Vb;
  const size_t nsite = (size_t)(g.nblk >> 1) * Vb;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nsite) return;
  const int k = (int)(e / Vb), loc = (int)(e - (size_t)k * Vb);
  const int half = g.NB[0] >> 1;
  const int row = k / half, j = k - row * half;
  const int by = row % g.NB[1];
  const int rz = row / g.NB[1];
  const int bz = rz % g.NB[2];
  const int bt = rz / g.NB[2];
  const int bx = 2 * j + ((colour + by + bz + bt) & 1);
  const int blk = bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
  const int s = blk * Vb + loc;
  const SiteCoord c = decompose(g, s);
  // right-hand sides outermost (blockIdx.y): consecutive workgroups are
  // neighbouring domains, which share the lines of their faces in the L2
  const size_t off = (size_t)blockIdx.y * rs;
  const size_t fb12 = fbase_b(g, 12, s, blk), fb36 = fbase_b(g, 36, s, blk);
  const float2* src = (first ? b : r) + off;
  cplx<float> acc[12], psi[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) acc[a] = {0, 0};
  bool any = false;
#pragma unroll 1
  for (int d = 0; d < 8; ++d) {
    int sign, nblk;
    bool inb;
    const int mu = d & 3;
    const int nb = d < 4 ? neighbour<true>(g, s, c, mu, sign, inb, nblk) : neighbour<false>(g, s, c, mu, sign, inb, nblk);
    if (inb) continue;
    any = true;
    ld_spinor<float>(delta + off, Vb, fbase_b(g, 12, nb, nblk), psi);
    const size_t lb = d < 4 ? fb36 : fbase_b(g, 36, nb, nblk);
    half2_t ub[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) ub[q] = U[(size_t)(mu * 9 + q) * Vb + lb];
    if (d < 4)
      hop_h<true>(mu, psi, ub, -(float)sign, acc);
    else
      hop_h<false>(mu, psi, ub, -(float)sign, acc);
  }
  if (!any && !first) return;
  float2* dst = r + off;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const size_t o = (size_t)a * Vb + fb12;
    st(dst, o, ld<float>(src, o) + acc[a]);
  }
}

// Zero slots after the Vb sites of each residual component in the domain
// kernel's LDS exchange buffer (64 keeps paired LDS offsets in 512-byte units).
constexpr int SAP_DOM_PAD = 64;

// Face bookkeeping of a domain: faces in the order (mu, side), side 0 at
// local coordinate 0, side 1 at B_mu - 1; a face site is indexed
// lexicographically by its other three local coordinates, so that the sites
// of a face, taken in site order, have consecutive indices.
__host__ __device__ __forceinline__ int face_slots(const Geo& g) {
  return 2 * (g.Vb / g.B[0] + g.Vb / g.B[1] + g.Vb / g.B[2] + g.Vb / g.B[3]);
}
__host__ __device__ __forceinline__ int face_off(const Geo& g, int mu, int side) {
  int o = 0;
  for (int m = 0; m < mu; ++m) o += 2 * (g.Vb / g.B[m]);
  return o + side * (g.Vb / g.B[mu]);
}
template <int MU>
__device__ __forceinline__ int face_index(const Geo& g, const int (&lc)[4]) {
  int f = 0, st = 1;
#pragma unroll
  for (int m = 0; m < 4; ++m)
    if (m != MU) {
      f += lc[m] * st;
      st *= g.B[m];
    }
  return f;
}

// Write the spin projections of a block correction psi for the hops that
// enter the domain through face MU: on side 0 the hops y -> y + mu of the
// sites y just outside (forward projection), on side 1 the hops y -> y - mu
// (backward projection).  Layout [block][6][FT] (this block's fw given).
template <int MU>
__device__ __forceinline__ void face_put(const Geo& g, const SiteCoord& c, int FT, const cplx<float> (&psi)[12],
                                         float2* fw) {
  const int f = face_index<MU>(g, c.lc);
  cplx<float> h0[3], h1[3];
  if (c.lc[MU] == 0) {
    hop_proj<MU, true>(psi, h0, h1);
    float2* o = fw + face_off(g, MU, 0) + f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      st(o, (size_t)q * FT, h0[q]);
      st(o, (size_t)(3 + q) * FT, h1[q]);
    }
  }
  if (c.lc[MU] == g.B[MU] - 1) {
    hop_proj<MU, false>(psi, h0, h1);
    float2* o = fw + face_off(g, MU, 1) + f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      st(o, (size_t)q * FT, h0[q]);
      st(o, (size_t)(3 + q) * FT, h1[q]);
    }
  }
}

// The crossing-hop correction from the face buffer (mixed path): for every
// site y of the active colour's domains and every right-hand side,
//   r(y) = src(y) - sum_{hops y -> x leaving the domain} W h(x)
// with h the spin projection that the neighbouring domain wrote for that
// hop (face_put) and W its FP16 hop matrix (boundary sign applied) from the
// face-ordered copy FL, U for forward hops and U^dag for backward ones.
// Sites of a face read consecutive face slots, so every load is coalesced
// and no line brings a neighbour's interior.
template <int MU>
__device__ __forceinline__ void face_get(const Geo& g, const SiteCoord& c, int FT, const float2* __restrict__ fr,
                                         const half2_t* __restrict__ FL, cplx<float> (&acc)[12], bool& any) {
  const int F = g.Vb / g.B[MU];
  const int f = face_index<MU>(g, c.lc);
#pragma unroll
  for (int side = 1; side >= 0; --side) {
    if (c.lc[MU] != (side ? g.B[MU] - 1 : 0)) continue;
    any = true;
    // the neighbouring block across this face (the block count per
    // direction is even, so it differs from this block)
    int bk = c.bk[MU] + (side ? 1 : -1);
    if (bk < 0) bk += g.NB[MU];
    if (bk >= g.NB[MU]) bk -= g.NB[MU];
    const int nblk = c.blk + (bk - c.bk[MU]) * g.sN[MU];
    // the producer's face on the opposite side
    const float2* hp = fr + (size_t)nblk * 6 * FT + face_off(g, MU, 1 - side) + f;
    cplx<float> h0[3], h1[3], u[9];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      h0[q] = ld<float>(hp, (size_t)q * FT);
      h1[q] = ld<float>(hp, (size_t)(3 + q) * FT);
    }
    const half2_t* up = FL + (size_t)c.blk * 9 * FT + (size_t)face_off(g, MU, side) * 9 + f;
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = h2f(up[(size_t)e * F]);
    cplx<float> g0[3], g1[3];
    if (side) {
      hop_mul<true>(h0, h1, u, -1.0f, g0, g1);
      hop_recon<MU, true>(g0, g1, acc);
    } else {
      hop_mul<false>(h0, h1, u, -1.0f, g0, g1);
      hop_recon<MU, false>(g0, g1, acc);
    }
  }
}

__global__ __launch_bounds__(256) void k_sap_cross_face(Geo g, int colour, int first,
                                                        const float2* __restrict__ b, float2* __restrict__ r,
                                                        const float2* __restrict__ face, size_t rs, size_t fs,
                                                        const half2_t* __restrict__ FL) {
  const int Vb = g.Vb;
  const size_t nsite = (size_t)(g.nblk >> 1) * Vb;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nsite) return;
  const int k = (int)(e / Vb), loc = (int)(e - (size_t)k * Vb);
  const int half = g.NB[0] >> 1;
  const int row = k / half, j = k - row * half;
  const int by = row % g.NB[1];
  const int rz = row / g.NB[1];
  const int bz = rz % g.NB[2];
  const int bt = rz / g.NB[2];
  const int bx = 2 * j + ((colour + by + bz + bt) & 1);
  const int blk = bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
  const int s = blk * Vb + loc;
  const SiteCoord c = decompose(g, s);
  const int FT = face_slots(g);
  const size_t off = (size_t)blockIdx.y * rs;
  const float2* fr = face + (size_t)blockIdx.y * fs;
  cplx<float> acc[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) acc[a] = {0, 0};
  bool any = false;
  face_get<0>(g, c, FT, fr, FL, acc, any);
  face_get<1>(g, c, FT, fr, FL, acc, any);
  face_get<2>(g, c, FT, fr, FL, acc, any);
  face_get<3>(g, c, FT, fr, FL, acc, any);
  if (!any && !first) return;
  const size_t fb12 = fbase_b(g, 12, s, blk);
  const float2* src = (first ? b : r) + off;
  float2* dst = r + off;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const size_t o = (size_t)a * Vb + fb12;
    st(dst, o, ld<float>(src, o) + acc[a]);
  }
}

// FL (see launch_face_links): one thread per (block, face slot).
__global__ __launch_bounds__(256) void k_face_links(Geo g, const half2_t* __restrict__ U, half2_t* __restrict__ FL) {
  const int FT = face_slots(g);
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)g.nblk * FT) return;
  const int blk = (int)(e / FT);
  int j = (int)(e - (size_t)blk * FT);
  int mu = 0, side = 0;
  while (j >= 2 * (g.Vb / g.B[mu])) {
    j -= 2 * (g.Vb / g.B[mu]);
    ++mu;
  }
  const int F = g.Vb / g.B[mu];
  side = j >= F;
  const int f = j - side * F;
  // local coordinates: the face's own coordinate, the others from f
  int lc[4], rem = f;
  for (int m = 0; m < 4; ++m) {
    if (m == mu) {
      lc[m] = side ? g.B[m] - 1 : 0;
    } else {
      lc[m] = rem % g.B[m];
      rem /= g.B[m];
    }
  }
  const int s = blk * g.Vb + lc[0] + g.B[0] * (lc[1] + g.B[1] * (lc[2] + g.B[2] * lc[3]));
  const SiteCoord c = decompose(g, s);
  int sign, nblk;
  bool inb;
  size_t base;
  if (side) {
    (void)neighbour<true>(g, s, c, mu, sign, inb, nblk);
    base = fbase_b(g, 36, s, blk);
  } else {
    const int nb = neighbour<false>(g, s, c, mu, sign, inb, nblk);
    base = fbase_b(g, 36, nb, nblk);
  }
  half2_t* o = FL + (size_t)blk * 9 * FT + (size_t)face_off(g, mu, side) * 9 + f;
  for (int q = 0; q < 9; ++q) {
    half2_t u = U[(size_t)(mu * 9 + q) * g.Vb + base];
    if (sign < 0) {
      u.x = -u.x;
      u.y = -u.y;
    }
    o[(size_t)q * F] = u;
  }
}


// VB: the domain volume when known at compile time (LDS offsets become
// immediates), 0 for any volume.
template <int VB>
__global__ __launch_bounds__(512) void k_sap_dom(Geo g, int colour, int flags, int mr, int nrhs,
                                                 const float2* __restrict__ b, float2* __restrict__ r,
                                                 float2* __restrict__ x, float2* __restrict__ face,
                                                 const float2* __restrict__ xinit, size_t rs, size_t fs,
                                                 const half2_t* __restrict__ U, const half2_t* __restrict__ C) {
  extern __shared__ __align__(16) char smem[];
  const int Vb = VB ? VB : g.Vb;
  // residual exchange [12][Vbp]: slots Vb .. Vbp-1 of every component hold
  // zeros, the neighbour of a hop that leaves the domain
  const int Vbp = Vb + SAP_DOM_PAD;
  cplx<float>* lds = (cplx<float>*)smem;
  half2_t* lu = (half2_t*)(smem + 12 * Vbp * sizeof(cplx<float>));  // [4][9][Vb] -kappa sign U_mu(x) of the domain
  float* red = (float*)(lu + 36 * Vb);                     // [nwaves][3]
  const int half = g.NB[0] >> 1;
  int k = xcd_remap(blockIdx.x, g.nblk >> 1);
  if (k >= (g.nblk >> 1)) return;
  int row = k / half, j = k - row * half;
  int by = row % g.NB[1];
  int rz = row / g.NB[1];
  int bz = rz % g.NB[2];
  int bt = rz / g.NB[2];
  int bx = 2 * j + ((colour + by + bz + bt) & 1);
  int blk = bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
  const int l = threadIdx.x;
  // with the volume known at compile time the launch has exactly Vb threads
  const bool act = VB ? true : l < Vb;
  const int s = blk * Vb + (act ? l : 0);
  const int nw = VB ? (VB + 63) / 64 : (blockDim.x + 63) >> 6;
  SiteCoord c = decompose(g, s);
  const size_t fb12 = fbase_b(g, 12, s, blk), fb36 = fbase_b(g, 36, s, blk);
  const int FT = face_slots(g);

  // per direction, held in registers for the whole launch: the slot of the
  // neighbour's residual (its local index in the domain, or the zero slot Vb
  // for a hop that leaves it; bits 0..15) and, for backward hops, the local
  // index whose stored link the hop uses (the neighbour's, or any valid one:
  // it multiplies zeros; bits 16..31).  Every hop is then computed, with no
  // branch per direction, so the loads of the next hop can be issued while
  // the current one is multiplied.
  float fsign[4];
  int ninfo[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    int sign;
    bool inb;
    int mu = d & 3;
    int nb = d < 4 ? neighbour<true>(g, s, c, mu, sign, inb) : neighbour<false>(g, s, c, mu, sign, inb);
    if (d < 4) fsign[mu] = (float)sign;
    const int nl = act ? nb - blk * Vb : 0;
    ninfo[d] = inb ? (nl | (nl << 16)) : (Vb | ((act ? l : 0) << 16));
  }
  if (l < SAP_DOM_PAD) {
#pragma unroll
    for (int a = 0; a < 12; ++a) lds[a * Vbp + Vb + l] = {0, 0};
  }
  // the domain's forward hop matrices (FP16 -kappa U_mu(x)) times the
  // boundary sign of their hop (bc of a hop x -> x + mu that crosses the
  // lattice boundary, which is also the sign of the backward hop x + mu -> x;
  // a sign change is exact in FP16), read by the site (forward hops) and by
  // its in-domain neighbours (their backward hops)
  if (act) {
#pragma unroll
    for (int q = 0; q < 36; ++q) {
      half2_t u = U[(size_t)q * Vb + fb36];
      if (fsign[q / 9] < 0) {
        u.x = -u.x;
        u.y = -u.y;
      }
      lu[(size_t)q * Vb + l] = u;
    }
  }
  __syncthreads();

  // the site's clover (FP16), held in registers for the whole launch
  half2_t cl[36];
#pragma unroll
  for (int q = 0; q < 36; ++q) cl[q] = C[(size_t)q * Vb + fb36];
  // the residual of the current right-hand side; the crossing-hop correction
  // has been applied by k_sap_cross (SAP_R_IN)
  const float2* rsrc = ((flags & SAP_FIRST) && !(flags & SAP_R_IN)) ? b : r;
  cplx<float> rho[12];
  if (act) ld_spinor<float>(rsrc, Vb, fb12, rho);
  // wait for the first residual and the clover here: inside the loop both
  // then always come from registers whose loads are complete, and no
  // instruction of an MR iteration waits for the previous right-hand side's
  // stores
#pragma unroll
  for (int a = 0; a < 12; ++a) asm volatile("" ::"v"(rho[a].x), "v"(rho[a].y));
#pragma unroll
  for (int q = 0; q < 36; ++q) asm volatile("" ::"v"(__builtin_bit_cast(uint32_t, cl[q])));
  for (int rr = 0; rr < nrhs; ++rr) {
    const size_t off = rr * rs;
    cplx<float> xm[12], p[12], psi[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) xm[a] = {0, 0};
    // The global loads that this right-hand side's end needs (its x, the
    // next one's residual) are issued now and arrive during the MR
    // iterations, which touch only LDS and registers; the stores of the
    // previous right-hand side, issued just before, drain meanwhile (a wait
    // for a load also waits for every store issued before it).
    // Both loads are unconditional (x itself stands in when there is no
    // start vector, the current residual after the last right-hand side) so
    // that every path through the loop has the same loads in flight and the
    // compiler's wait counts do not fall to the path without them.
    float2* xr = x + off;
    const bool have_x0 = !(flags & SAP_FIRST) || xinit;
    const float2* x0src = !(flags & SAP_FIRST) ? xr : (xinit ? xinit + off : xr);
    cplx<float> x0[12], nrho[12];
    if (act) {
      ld_spinor<float>(x0src, Vb, fb12, x0);
      ld_spinor<float>(rsrc + off + (rr + 1 < nrhs ? rs : 0), Vb, fb12, nrho);
    }
    for (int it = 0; it < mr; ++it) {
      if (act) {
#pragma unroll
        for (int a = 0; a < 12; ++a) lds[a * Vbp + l] = rho[a];
      }
      __syncthreads();
      float pr_re = 0, pr_im = 0, pp = 0;
      if (act) {
        // p = (1 + F) rho + in-domain hops (the stored links are the hop
        // matrices -kappa U)
#pragma unroll
        for (int a = 0; a < 12; ++a) p[a] = rho[a];
        // the clover stays FP16 in registers (36 VGPRs) and enters the
        // products as FP16 operands of mixed-precision FMAs: the empty asm
        // keeps the compiler from hoisting 72 FP32 conversions out of the
        // loop, which would hold 72 VGPRs instead
        half2_t clv[36];
#pragma unroll
        for (int q = 0; q < 36; ++q) {
          uint32_t bits = __builtin_bit_cast(uint32_t, cl[q]);
          asm volatile("" : "+v"(bits));
          clv[q] = __builtin_bit_cast(half2_t, bits);
        }
        clover_acc<float>(clv, 1, 0, rho, p);
        // unrolled: direction and projection are compile-time constants
#pragma unroll
        for (int d = 0; d < 8; ++d) {
          const int inf = ninfo[d];
          const int nl = inf & 0xffff;
          // The t-hops that leave the domain are skipped: when the sites of
          // one t-slice fill whole wavefronts (B_x B_y B_z a multiple of
          // 64), a wavefront's t-hop leaves the domain for all its lanes or
          // for none, and the skip is a branch the whole wavefront takes.
          if ((d & 3) == 3 && nl == Vb) continue;
#pragma unroll
          for (int a = 0; a < 12; ++a) psi[a] = lds[a * Vbp + nl];
          half2_t ub[9];
          const int ls = d < 4 ? l : (inf >> 16);  // U_mu(x) or U_mu(x - mu), scaled
#pragma unroll
          for (int e = 0; e < 9; ++e) ub[e] = lu[((d & 3) * 9 + e) * Vb + ls];
          if (d < 4)
            hop_h<true>(d & 3, psi, ub, 1.0f, p);
          else
            hop_h<false>(d & 3, psi, ub, 1.0f, p);
        }
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          pr_re += p[a].x * rho[a].x + p[a].y * rho[a].y;
          pr_im += p[a].x * rho[a].y - p[a].y * rho[a].x;
          pp += p[a].x * p[a].x + p[a].y * p[a].y;
        }
      }
      pr_re = wave_sum_hi(pr_re);
      pr_im = wave_sum_hi(pr_im);
      pp = wave_sum_hi(pp);
      if ((l & 63) == 63) {
        red[(l >> 6) * 3 + 0] = pr_re;
        red[(l >> 6) * 3 + 1] = pr_im;
        red[(l >> 6) * 3 + 2] = pp;
      }
      __syncthreads();
      // (unrolled when the wave count is known at compile time, so that the
      // partial sums are read with one LDS round trip, not one per wave)
      float sre = 0, sim = 0, spp = 0;
#pragma unroll
      for (int w = 0; w < nw; ++w) {
        sre += red[w * 3 + 0];
        sim += red[w * 3 + 1];
        spp += red[w * 3 + 2];
      }
      cplx<float> alpha = {0, 0};
      if (spp > 0) alpha = {sre / spp, sim / spp};
      if (act) {
        const cplx<float> malpha = {-alpha.x, -alpha.y};
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          cmac(xm[a], alpha, rho[a]);
          cmac(rho[a], malpha, p[a]);
        }
      }
    }
    if (act) {
      // the prefetched values are waited for before the first store, so
      // that no wait comes to stand behind this right-hand side's stores
#pragma unroll
      for (int a = 0; a < 12; ++a) asm volatile("" ::"v"(nrho[a].x), "v"(nrho[a].y));
      float2* rw = r + off;
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        size_t o = (size_t)a * Vb + fb12;
        st(xr, o, have_x0 ? x0[a] + xm[a] : xm[a]);
        if (!(flags & SAP_NO_R)) st(rw, o, rho[a]);
      }
      // the correction's spin projections on the domain's faces, for the
      // crossing hops of the other colour's next residual update
      if (!(flags & SAP_NO_DELTA)) {
        float2* fw = face + rr * fs + (size_t)blk * 6 * FT;
        face_put<0>(g, c, FT, xm, fw);
        face_put<1>(g, c, FT, xm, fw);
        face_put<2>(g, c, FT, xm, fw);
        face_put<3>(g, c, FT, xm, fw);
      }
#pragma unroll
      for (int a = 0; a < 12; ++a) rho[a] = nrho[a];
    }
    // No barrier before the next right-hand side: every thread has passed
    // the last iteration's reduction barrier after its last read of lds, and
    // the next write to red follows the next iteration's first barrier, which
    // no thread reaches before it has read red.
  }
}

// Even-odd preconditioned variant of the mixed domain solve.  In a domain,
// D_SAP splits by site parity into [[A_e, H_eo], [H_oe, A_o]] (A = 1 + F
// site-local, H the in-domain hops); with S = A_e - H_eo A_o^-1 H_oe on the
// even sites the block solve is
//   c_e = b_e - H_eo A_o^-1 b_o;  x_e = MR(mr) on S x_e = c_e from 0;
//   x_o = A_o^-1 (b_o - H_oe x_e),
// and its residual is c_e - S x_e on the even sites (equal to b - D_SAP x
// there) and b_o - H_oe x_e - A_o x_o on the odd ones.  A_o^-1 is applied as
// psi + M psi with M = (1 + F)^-1 - 1 stored in FP16 like the clover.  The
// threads are sorted by parity (the first Vb/2 take the even sites), so the
// phases that only one parity works in leave whole wavefronts idle instead
// of half of every wavefront.  One workgroup per domain of the active colour,
// all right-hand sides in turn; links, exchange buffer and reduction as in
// k_sap_dom (the buffer holds even-site values in even slots and odd-site
// values in odd slots, so one buffer serves both directions).
template <int VB>
__global__ __launch_bounds__(512) void k_sap_dom_eo(Geo g, int colour, int flags, int mr, int nrhs,
                                                    const float2* __restrict__ b, float2* __restrict__ r,
                                                    float2* __restrict__ x, float2* __restrict__ delta,
                                                    const float2* __restrict__ xinit, size_t rs,
                                                    const half2_t* __restrict__ U, const half2_t* __restrict__ C,
                                                    const half2_t* __restrict__ M) {
  extern __shared__ __align__(16) char smem[];
  const int Vb = VB ? VB : g.Vb;
  cplx<float>* lds = (cplx<float>*)smem;                            // [12][Vb] exchange, indexed by site
  half2_t* lu = (half2_t*)(smem + 12 * Vb * sizeof(cplx<float>));  // [4][9][Vb] -kappa sign U_mu(x)
  float* red = (float*)(lu + 36 * Vb);                              // [nwaves][3]
  const int half = g.NB[0] >> 1;
  int k = xcd_remap(blockIdx.x, g.nblk >> 1);
  if (k >= (g.nblk >> 1)) return;
  int row = k / half, j = k - row * half;
  int by = row % g.NB[1];
  int rz = row / g.NB[1];
  int bz = rz % g.NB[2];
  int bt = rz / g.NB[2];
  int bx = 2 * j + ((colour + by + bz + bt) & 1);
  int blk = bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
  const int l = threadIdx.x;
  const int hv = Vb >> 1;
  const bool act = l < Vb;
  const bool ev = l < hv;  // even-site thread (odd-site threads: hv <= l < Vb)
  // the site of thread l: the (l mod hv)-th site of its parity in the block
  // (block extents even: every x-row holds B_x / 2 sites of each parity)
  int loc = 0;
  {
    const int q = act ? (ev ? l : l - hv) : 0;
    const int hx = g.B[0] >> 1;
    const int rrow = q / hx, kx = q - rrow * hx;
    int t = rrow, rp = 0;
#pragma unroll
    for (int m = 1; m < 4; ++m) {
      rp += t % g.B[m];
      t /= g.B[m];
    }
    loc = rrow * g.B[0] + 2 * kx + ((rp + (ev ? 0 : 1)) & 1);
  }
  const int s = blk * Vb + loc;
  const int nw = VB ? (VB + 63) / 64 : (blockDim.x + 63) >> 6;
  SiteCoord c = decompose(g, s);
  const size_t fb12 = fbase_b(g, 12, s, blk), fb36 = fbase_b(g, 36, s, blk);
  float fsign[4];
  int ninfo[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    int sign;
    bool inb;
    int mu = d & 3;
    int nb = d < 4 ? neighbour<true>(g, s, c, mu, sign, inb) : neighbour<false>(g, s, c, mu, sign, inb);
    if (d < 4) fsign[mu] = (float)sign;
    ninfo[d] = inb ? ((nb - blk * Vb) | (1 << 10)) : 0;
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < 36; ++q) {
      half2_t u = U[(size_t)q * Vb + fb36];
      if (fsign[q / 9] < 0) {
        u.x = -u.x;
        u.y = -u.y;
      }
      lu[(size_t)q * Vb + loc] = u;
    }
  }
  // even sites hold their clover F, odd sites M = (1 + F)^-1 - 1
  half2_t cl[36];
  if (act) {
    const half2_t* src = ev ? C : M;
#pragma unroll
    for (int q = 0; q < 36; ++q) cl[q] = src[(size_t)q * Vb + fb36];
  }
  __syncthreads();

  // acc += coef * (sum of the in-domain hops applied to the exchange buffer)
  auto hops = [&](float coef, cplx<float>(&acc)[12]) {
    cplx<float> psi[12];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int inf = ninfo[d];
      if (inf & (1 << 10)) {
        const int nl = inf & 1023;
#pragma unroll
        for (int a = 0; a < 12; ++a) psi[a] = lds[a * Vb + nl];
        half2_t ub[9];
        const int ls = d < 4 ? loc : nl;
#pragma unroll
        for (int e = 0; e < 9; ++e) ub[e] = lu[((d & 3) * 9 + e) * Vb + ls];
        if (d < 4)
          hop_h<true>(d & 3, psi, ub, coef, acc);
        else
          hop_h<false>(d & 3, psi, ub, coef, acc);
      }
    }
  };
  // v + cl v (even: (1 + F) v; odd: (1 + F)^-1 v)
  auto site_op = [&](const cplx<float>(&v)[12], cplx<float>(&out)[12]) {
#pragma unroll
    for (int a = 0; a < 12; ++a) out[a] = v[a];
    clover_acc<float>(cl, 1, 0, v, out);
  };
  auto put = [&](const cplx<float>(&v)[12]) {
#pragma unroll
    for (int a = 0; a < 12; ++a) lds[a * Vb + loc] = v[a];
  };

  for (int rr = 0; rr < nrhs; ++rr) {
    const size_t off = rr * rs;
    // rho: even sites the Schur residual, odd sites b_o (kept to the end)
    cplx<float> rho[12], xm[12], p[12];
    if (act) ld_spinor<float>(((flags & SAP_FIRST) && !(flags & SAP_R_IN)) ? b + off : r + off, Vb, fb12, rho);
#pragma unroll
    for (int a = 0; a < 12; ++a) xm[a] = {0, 0};
    // c_e = b_e - H_eo A_o^-1 b_o
    if (act && !ev) {
      site_op(rho, p);
      put(p);
    }
    __syncthreads();
    if (ev) hops(-1.0f, rho);
    for (int it = 0; it < mr; ++it) {
      if (ev) put(rho);
      __syncthreads();
      if (act && !ev) {
        // t_o = A_o^-1 H_oe rho_e (xm, unused by odd sites until the end,
        // holds H_oe rho_e)
#pragma unroll
        for (int a = 0; a < 12; ++a) xm[a] = {-0.0f, -0.0f};
        hops(1.0f, xm);
        site_op(xm, p);
        put(p);
      }
      __syncthreads();
      float pr_re = 0, pr_im = 0, pp = 0;
      if (ev) {
        // p = S rho = A_e rho - H_eo t_o
        site_op(rho, p);
        hops(-1.0f, p);
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          pr_re += p[a].x * rho[a].x + p[a].y * rho[a].y;
          pr_im += p[a].x * rho[a].y - p[a].y * rho[a].x;
          pp += p[a].x * p[a].x + p[a].y * p[a].y;
        }
      }
      pr_re = wave_sum_hi(pr_re);
      pr_im = wave_sum_hi(pr_im);
      pp = wave_sum_hi(pp);
      if ((l & 63) == 63) {
        red[(l >> 6) * 3 + 0] = pr_re;
        red[(l >> 6) * 3 + 1] = pr_im;
        red[(l >> 6) * 3 + 2] = pp;
      }
      __syncthreads();
      // (unrolled when the wave count is known at compile time, so that the
      // partial sums are read with one LDS round trip, not one per wave)
      float sre = 0, sim = 0, spp = 0;
#pragma unroll
      for (int w = 0; w < nw; ++w) {
        sre += red[w * 3 + 0];
        sim += red[w * 3 + 1];
        spp += red[w * 3 + 2];
      }
      cplx<float> alpha = {0, 0};
      if (spp > 0) alpha = {sre / spp, sim / spp};
      if (ev) {
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          xm[a] = xm[a] + alpha * rho[a];
          rho[a] = rho[a] - alpha * p[a];
        }
      }
    }
    // x_o = A_o^-1 (b_o - H_oe x_e); odd residual b_o - H_oe x_e - A_o x_o
    if (ev) put(xm);
    __syncthreads();
    if (act && !ev) {
      hops(-1.0f, rho);  // q = b_o - H_oe x_e
      site_op(rho, xm);  // x_o = A_o^-1 q
      // residual q - A_o x_o = q - x_o - F x_o (F read once per block solve)
      cplx<float> fx[12];
#pragma unroll
      for (int a = 0; a < 12; ++a) fx[a] = {-0.0f, -0.0f};
      clover_acc<float>(C, Vb, fb36, xm, fx);
#pragma unroll
      for (int a = 0; a < 12; ++a) rho[a] = (rho[a] - xm[a]) - fx[a];
    }
    if (act) {
      float2* xr = x + off;
      float2* rw = r + off;
      float2* dw = delta + off;
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        size_t o = (size_t)a * Vb + fb12;
        cplx<float> x0 = {0, 0};
        if (!(flags & SAP_FIRST)) x0 = ld<float>(xr, o);
        else if (xinit) x0 = ld<float>(xinit + off, o);
        st(xr, o, x0 + xm[a]);
        if (!(flags & SAP_NO_R)) st(rw, o, rho[a]);
        if (!(flags & SAP_NO_DELTA)) st(dw, o, xm[a]);
      }
    }
    __syncthreads();  // the next right-hand side reuses lds
  }
}

int sap_dom_lds_bytes(const Geo& g) {
  int nthr = ((g.Vb + 63) / 64) * 64;
  return 12 * (g.Vb + SAP_DOM_PAD) * 8 + 36 * g.Vb * 4 + (nthr / 64) * 3 * 4;
}

int sap_lds_bytes(const Geo& g, int mixed) {
  int rsz = mixed ? 4 : 8;
  int nthr = ((g.Vb + 63) / 64) * 64;
  return 12 * g.Vb * 2 * rsz + (nthr / 64) * 3 * rsz;
}

template <class R, class TS, class TL, class TC>
static void sap_half_run(const SapArgs& a, int col, int flags, hipStream_t st) {
  const Geo& g = a.g;
  int nthr = ((g.Vb + 63) / 64) * 64;
  int lds = sap_lds_bytes(g, sizeof(R) == 4);
  dim3 grid(g.nblk / 2, a.nrhs);
  auto kern = k_sap_half<R, TS, TL, TC>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  kern<<<grid, nthr, lds, st>>>(g, col, flags, a.mr, (R)a.kappa, (const TS*)a.b, (TS*)a.r, (TS*)a.x,
                                (TS*)a.delta, (const TS*)a.xinit, a.rs, (const TL*)a.U, (const TC*)a.C);
}

bool sap_needs_cross(const SapArgs& a, int sweep, int col) { return a.mixed && (sweep > 0 || col == 1); }

void launch_sap_cross(const SapArgs& a, int sweep, int col, hipStream_t st) {
  if (!sap_needs_cross(a, sweep, col)) return;
  const size_t nsite = (size_t)(a.g.nblk / 2) * a.g.Vb;
  const dim3 grid((unsigned)((nsite + 255) / 256), a.nrhs);
  if (a.eo) {
    // the even-odd block solve hands over whole corrections
    k_sap_cross<<<grid, 256, 0, st>>>(a.g, col, sweep == 0 ? 1 : 0, (const float2*)a.b, (float2*)a.r,
                                      (const float2*)a.delta, a.rs, (const half2_t*)a.U);
    return;
  }
  if (!a.FL) throw std::runtime_error("SAP: no face hop matrices");
  k_sap_cross_face<<<grid, 256, 0, st>>>(a.g, col, sweep == 0 ? 1 : 0, (const float2*)a.b, (float2*)a.r,
                                         (const float2*)a.delta, a.rs, a.fs, (const half2_t*)a.FL);
}

int sap_face_slots(const Geo& g) { return face_slots(g); }

void launch_face_links(const Geo& g, const void* U16, void* FL, hipStream_t st) {
  const size_t n = (size_t)g.nblk * face_slots(g);
  k_face_links<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(g, (const half2_t*)U16, (half2_t*)FL);
}

void launch_sap_half(const SapArgs& a, int sweep, int col, hipStream_t st) {
  int flags = (sweep == 0 ? SAP_FIRST : 0) | ((sweep > 0 || col == 1) ? SAP_DELTA : 0);
  if (!a.mixed) return sap_half_run<double, double2, double2, double2>(a, col, flags, st);
  // the last visit of a colour: its residual is never read again; the last
  // half-sweep's correction is never read either
  if (sweep == a.sweeps - 1) flags |= SAP_NO_R;
  if (sweep == a.sweeps - 1 && col == 1) flags |= SAP_NO_DELTA;
  // the crossing-hop correction has been applied by launch_sap_cross; the
  // domain solves start from r
  if (flags & SAP_DELTA) flags = (flags & ~SAP_DELTA) | SAP_R_IN;
  const Geo& g = a.g;
  int nthr = ((g.Vb + 63) / 64) * 64;
  int lds = sap_dom_lds_bytes(g);
  int ndom = g.nblk / 2;
  static bool attr_set[3] = {false, false, false};
  auto go = [&](auto kern, int id) {
    if (!attr_set[id]) {
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      attr_set[id] = true;
    }
    kern<<<round8(ndom), nthr, lds, st>>>(g, col, flags, a.mr, a.nrhs, (const float2*)a.b,
                                          (float2*)a.r, (float2*)a.x, (float2*)a.delta, (const float2*)a.xinit, a.rs,
                                          a.fs, (const half2_t*)a.U, (const half2_t*)a.C);
  };
  if (a.eo) {
    if (!a.M) throw std::runtime_error("even-odd SAP: no inverse clover field");
    if (g.B[0] % 2 || g.B[1] % 2 || g.B[2] % 2 || g.B[3] % 2)
      throw std::runtime_error("even-odd SAP: block extents must be even");
    static bool attr_eo[3] = {false, false, false};
    auto go_eo = [&](auto kern, int id) {
      if (!attr_eo[id]) {
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_eo[id] = true;
      }
      kern<<<round8(ndom), nthr, lds, st>>>(g, col, flags, a.mr, a.nrhs, (const float2*)a.b, (float2*)a.r,
                                            (float2*)a.x, (float2*)a.delta, (const float2*)a.xinit, a.rs,
                                            (const half2_t*)a.U, (const half2_t*)a.C, (const half2_t*)a.M);
    };
    if (g.Vb == 512)
      go_eo(k_sap_dom_eo<512>, 0);
    else if (g.Vb == 256)
      go_eo(k_sap_dom_eo<256>, 1);
    else
      go_eo(k_sap_dom_eo<0>, 2);
    return;
  }
  if (g.Vb == 512)
    go(k_sap_dom<512>, 0);
  else if (g.Vb == 256)
    go(k_sap_dom<256>, 1);
  else
    go(k_sap_dom<0>, 2);
}

// ---------------------------------------------------------------------------
// launchers for layout / clover kernels
// ---------------------------------------------------------------------------
void launch_pack_spinor(const Geo& g, const double2* canon, void* out, int out_t, size_t out_rs, int nrhs,
                        hipStream_t st) {
  dim3 grid((g.V + 255) / 256, nrhs);
  if (out_t == C128)
    k_pack_spinor<double2><<<grid, 256, 0, st>>>(g, canon, (double2*)out, out_rs);
  else if (out_t == C64)
    k_pack_spinor<float2><<<grid, 256, 0, st>>>(g, canon, (float2*)out, out_rs);
  else
    k_pack_spinor<half2_t><<<grid, 256, 0, st>>>(g, canon, (half2_t*)out, out_rs);
}

void launch_unpack_spinor(const Geo& g, const void* in, int in_t, size_t in_rs, double2* canon, int nrhs,
                          hipStream_t st) {
  dim3 grid((g.V + 255) / 256, nrhs);
  if (in_t == C128)
    k_unpack_spinor<double2><<<grid, 256, 0, st>>>(g, (const double2*)in, in_rs, canon);
  else if (in_t == C64)
    k_unpack_spinor<float2><<<grid, 256, 0, st>>>(g, (const float2*)in, in_rs, canon);
  else
    k_unpack_spinor<half2_t><<<grid, 256, 0, st>>>(g, (const half2_t*)in, in_rs, canon);
}

void launch_pack_gauge(const Geo& g, const double2* canon, double2* U64, half2_t* U16, double h, hipStream_t st) {
  dim3 grid((g.V + 255) / 256, 4);
  k_pack_gauge<<<grid, 256, 0, st>>>(g, canon, U64, U16, h);
}

void launch_clover_build(const Geo& g, const double2* U64, double kappa, double csw, const double* sigma,
                         double2* C64, half2_t* C16, hipStream_t st) {
  SigmaTab t;
  const double* src = sigma;
  double* dst = &t.v[0][0][0][0][0];
  for (int i = 0; i < 6 * 2 * 2 * 2 * 2; ++i) dst[i] = src[i];
  k_clover_build<<<(g.V + 127) / 128, 128, 0, st>>>(g, U64, kappa, csw, t, C64, C16);
}

void launch_pack_clover(const Geo& g, const double2* canon, double2* C64, half2_t* C16, hipStream_t st) {
  k_pack_clover<<<(g.V + 255) / 256, 256, 0, st>>>(g, canon, C64, C16);
}

void launch_unpack_clover(const Geo& g, const double2* C64, double2* canon, hipStream_t st) {
  k_unpack_clover<<<(g.V + 255) / 256, 256, 0, st>>>(g, C64, canon);
}

}  // namespace wc
