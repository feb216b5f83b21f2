// Per-site pieces of the Wilson-clover operator (eq. (1)) shared by the
// fine-level and coarse-construction kernels: spin projection / SU(3)
// multiplication of one hop, link and spinor loads, the clover block product.
#pragma once
#include "wc_common.h"

namespace wc {

// ---------------------------------------------------------------------------
// Spin projection in the chiral basis.  For a hop in direction mu the factor
// (1 -/+ gamma_mu) has rank 2: with u = spins (0,1), l = spins (2,3),
//   h_k = u_k + tau_k l_{pi(k)},   result = [h ; sigma_k h_{pi(k)}]
// where pi swaps (mu = x, y) or keeps (mu = z, t) the two spins and tau,
// sigma are units in {1, i, -1, -i}; the backward sign flips both.  Units are
// coded 0: 1, 1: i, 2: -1, 3: -i.
// ---------------------------------------------------------------------------
template <int MU>
struct Proj;
template <>
struct Proj<0> {
  static constexpr int pi0 = 1, pi1 = 0, t0 = 1, t1 = 1, s0 = 3, s1 = 3;
};
template <>
struct Proj<1> {
  static constexpr int pi0 = 1, pi1 = 0, t0 = 0, t1 = 2, s0 = 2, s1 = 0;
};
template <>
struct Proj<2> {
  static constexpr int pi0 = 0, pi1 = 1, t0 = 1, t1 = 3, s0 = 3, s1 = 1;
};
template <>
struct Proj<3> {
  static constexpr int pi0 = 0, pi1 = 1, t0 = 0, t1 = 0, s0 = 0, s1 = 0;
};

// acc += coef * (1 -/+ gamma_mu) W psi with W = U (FWD) or U^dag (backward).
template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_accum(const cplx<R> (&psi)[12], const cplx<R> (&u)[9], R coef,
                                          cplx<R> (&acc)[12]) {
  using P = Proj<MU>;
  constexpr int T0 = FWD ? P::t0 : (P::t0 ^ 2);
  constexpr int T1 = FWD ? P::t1 : (P::t1 ^ 2);
  constexpr int S0 = FWD ? P::s0 : (P::s0 ^ 2);
  constexpr int S1 = FWD ? P::s1 : (P::s1 ^ 2);
  cplx<R> h0[3], h1[3], g0[3], g1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h0[c] = psi[c] + unit<T0>(psi[(2 + P::pi0) * 3 + c]);
    h1[c] = psi[3 + c] + unit<T1>(psi[(2 + P::pi1) * 3 + c]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    cplx<R> a = {0, 0}, b = {0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (FWD) {
        cmac(a, u[r * 3 + c], h0[c]);
        cmac(b, u[r * 3 + c], h1[c]);
      } else {
        cjmac(a, u[c * 3 + r], h0[c]);
        cjmac(b, u[c * 3 + r], h1[c]);
      }
    }
    g0[r] = coef * a;
    g1[r] = coef * b;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = acc[c] + g0[c];
    acc[3 + c] = acc[3 + c] + g1[c];
    acc[6 + c] = acc[6 + c] + unit<S0>(P::pi0 == 0 ? g0[c] : g1[c]);
    acc[9 + c] = acc[9 + c] + unit<S1>(P::pi1 == 0 ? g0[c] : g1[c]);
  }
}

// The pieces of hop_accum, for kernels that hand a hop's projected
// half-spinor to the site that receives it: the spin projection h of psi,
// g = coef * W h, and acc += the spin reconstruction of g (hop_recon).
template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_proj(const cplx<R> (&psi)[12], cplx<R> (&h0)[3], cplx<R> (&h1)[3]) {
  using P = Proj<MU>;
  constexpr int T0 = FWD ? P::t0 : (P::t0 ^ 2);
  constexpr int T1 = FWD ? P::t1 : (P::t1 ^ 2);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h0[c] = psi[c] + unit<T0>(psi[(2 + P::pi0) * 3 + c]);
    h1[c] = psi[3 + c] + unit<T1>(psi[(2 + P::pi1) * 3 + c]);
  }
}

template <bool FWD, class R>
__device__ __forceinline__ void hop_mul(const cplx<R> (&h0)[3], const cplx<R> (&h1)[3], const cplx<R> (&u)[9], R coef,
                                        cplx<R> (&g0)[3], cplx<R> (&g1)[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    cplx<R> a = {0, 0}, b = {0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (FWD) {
        cmac(a, u[r * 3 + c], h0[c]);
        cmac(b, u[r * 3 + c], h1[c]);
      } else {
        cjmac(a, u[c * 3 + r], h0[c]);
        cjmac(b, u[c * 3 + r], h1[c]);
      }
    }
    g0[r] = coef * a;
    g1[r] = coef * b;
  }
}

template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_half(const cplx<R> (&psi)[12], const cplx<R> (&u)[9], R coef, cplx<R> (&g0)[3],
                                         cplx<R> (&g1)[3]) {
  cplx<R> h0[3], h1[3];
  hop_proj<MU, FWD>(psi, h0, h1);
  hop_mul<FWD>(h0, h1, u, coef, g0, g1);
}

template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_recon(const cplx<R> (&g0)[3], const cplx<R> (&g1)[3], cplx<R> (&acc)[12]) {
  using P = Proj<MU>;
  constexpr int S0 = FWD ? P::s0 : (P::s0 ^ 2);
  constexpr int S1 = FWD ? P::s1 : (P::s1 ^ 2);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = acc[c] + g0[c];
    acc[3 + c] = acc[3 + c] + g1[c];
    acc[6 + c] = acc[6 + c] + unit<S0>(P::pi0 == 0 ? g0[c] : g1[c]);
    acc[9 + c] = acc[9 + c] + unit<S1>(P::pi1 == 0 ? g0[c] : g1[c]);
  }
}

template <bool FWD, class R>
__device__ __forceinline__ void hop_half_any(int mu, const cplx<R> (&psi)[12], const cplx<R> (&u)[9], R coef,
                                             cplx<R> (&g0)[3], cplx<R> (&g1)[3]) {
  switch (mu) {
    case 0: hop_half<0, FWD>(psi, u, coef, g0, g1); break;
    case 1: hop_half<1, FWD>(psi, u, coef, g0, g1); break;
    case 2: hop_half<2, FWD>(psi, u, coef, g0, g1); break;
    default: hop_half<3, FWD>(psi, u, coef, g0, g1); break;
  }
}

template <bool FWD, class R>
__device__ __forceinline__ void hop_recon_any(int mu, const cplx<R> (&g0)[3], const cplx<R> (&g1)[3],
                                              cplx<R> (&acc)[12]) {
  switch (mu) {
    case 0: hop_recon<0, FWD>(g0, g1, acc); break;
    case 1: hop_recon<1, FWD>(g0, g1, acc); break;
    case 2: hop_recon<2, FWD>(g0, g1, acc); break;
    default: hop_recon<3, FWD>(g0, g1, acc); break;
  }
}

template <bool FWD, class R>
__device__ __forceinline__ void hop_any(int mu, const cplx<R> (&psi)[12], const cplx<R> (&u)[9], R coef,
                                        cplx<R> (&acc)[12]) {
  switch (mu) {
    case 0: hop_accum<0, FWD>(psi, u, coef, acc); break;
    case 1: hop_accum<1, FWD>(psi, u, coef, acc); break;
    case 2: hop_accum<2, FWD>(psi, u, coef, acc); break;
    default: hop_accum<3, FWD>(psi, u, coef, acc); break;
  }
}

// Site-field loads: `base` is the offset of the site's plane 0 (fbase) and
// `ps` the plane stride (Vb) of the block-major layout.
template <class R, class TL>
__device__ __forceinline__ void ld_link(const TL* __restrict__ U, int ps, int mu, size_t base, cplx<R> (&u)[9]) {
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = ld<R>(U, (size_t)(mu * 9 + e) * ps + base);
}

template <class R, class TS>
__device__ __forceinline__ void ld_spinor(const TS* __restrict__ p, int ps, size_t base, cplx<R> (&psi)[12]) {
#pragma unroll
  for (int a = 0; a < 12; ++a) psi[a] = ld<R>(p, (size_t)a * ps + base);
}

// acc += F(x) psi for the packed clover field (plane stride ps, site base).
template <class R, class TC>
__device__ __forceinline__ void clover_acc(const TC* __restrict__ C, int ps, size_t base, const cplx<R> (&psi)[12],
                                           cplx<R> (&acc)[12]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    cplx<R> p[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) p[k] = ld<R>(C, (size_t)(18 * b + k) * ps + base);
    R d[6] = {p[0].x, p[0].y, p[1].x, p[1].y, p[2].x, p[2].y};
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[6 * b + i] = acc[6 * b + i] + d[i] * psi[6 * b + i];
    int k = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
      for (int j = i + 1; j < 6; ++j) {
        cmac(acc[6 * b + i], p[k], psi[6 * b + j]);
        cjmac(acc[6 * b + j], p[k], psi[6 * b + i]);
        ++k;
      }
    }
  }
}

}  // namespace wc
