// Coarse-level kernels: restriction eq. (5), prolongation eq. (6), the
// coarse 9-point block stencil of eq. (7) and the per-block Cholesky factor
// used to orthonormalise the test vectors (<I|J> = delta_IJ, Sec. 3).
//
// Test vectors are stored like spinor fields, [nv][blk][12][Vb] (blocked site
// order, block-major planes), so that block X's part of one vector is one
// contiguous range of 12 Vb elements.
// Coarse vectors are [rhs][X][N] with N = 2 nv and n = s*nv + i.  The coarse
// operator is stored [X][d][m][n] (each 2nv x 2nv block column-major) with
// d = 0 self, 1+mu forward, 5+mu backward neighbour.
#include <stdexcept>

#include "wc_dirac.h"
#include "wc_kernels.h"

namespace wc {

// matrix-core accumulator types
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));


// ---------------------------------------------------------------------------
// Restriction.  One workgroup per block X.  Thread t owns the outputs
// (s, i, rhs group of RB); tiles of TS sites of V and of the input are staged
// in LDS (V in its storage type, the input in the accumulation type).
// ---------------------------------------------------------------------------
template <class RA, class TV, class TI, class TO, int RB>
__global__ __launch_bounds__(256) void k_restrict(Geo g, int nv, int nrhs, int TS, const TV* __restrict__ V,
                                                  const TI* __restrict__ in, size_t in_rs, TO* __restrict__ out,
                                                  size_t out_rs, size_t out_xs) {
  extern __shared__ __align__(16) char smem[];
  TV* sv = (TV*)smem;                                                           // [TS][nv][12]
  cplx<RA>* si = (cplx<RA>*)(smem + (((size_t)TS * nv * 12 * sizeof(TV) + 15) & ~(size_t)15));  // [TS][nrhs][12]
  const int X = blockIdx.x;
  const int t = threadIdx.x;
  const int nrg = (nrhs + RB - 1) / RB;
  const int nout = 2 * nv * nrg;
  const int sc = t / (nv * nrg);
  const int rem = t - sc * nv * nrg;
  const int i = rem / nrg;
  const int rg = rem - i * nrg;
  const int V_ = g.V;
  const size_t base = (size_t)X * 12 * g.Vb;  // plane 0 of block X
  cplx<RA> acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = {0, 0};

  for (int s0 = 0; s0 < g.Vb; s0 += TS) {
    for (int e = t; e < TS * nv * 12; e += 256) {
      int st_ = e % TS;
      int row = e / TS;  // i*12 + a
      int ii = row / 12, a = row - ii * 12;
      sv[(st_ * nv + ii) * 12 + a] = V[(size_t)ii * 12 * V_ + base + (size_t)a * g.Vb + s0 + st_];
    }
    for (int e = t; e < TS * nrhs * 12; e += 256) {
      int st_ = e % TS;
      int row = e / TS;  // r*12 + a
      int r = row / 12, a = row - r * 12;
      si[(st_ * nrhs + r) * 12 + a] = ld<RA>(in, r * in_rs + (size_t)a * g.Vb + base + s0 + st_);
    }
    __syncthreads();
    if (t < nout) {
      for (int st_ = 0; st_ < TS; ++st_) {
#pragma unroll
        for (int a6 = 0; a6 < 6; ++a6) {
          int a = 6 * sc + a6;
          cplx<RA> vv = ld<RA>(sv, (size_t)(st_ * nv + i) * 12 + a);
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            int r = rg * RB + q;
            if (r < nrhs) cjmac(acc[q], vv, si[(st_ * nrhs + r) * 12 + a]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (t < nout) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      int r = rg * RB + q;
      if (r < nrhs) st(out, r * out_rs + X * out_xs + sc * nv + i, acc[q]);
    }
  }
}

template <class RA, class TV, class TI, class TO, int RB>
static void restrict_run(const Geo& g, int nv, int nrhs, const void* V, const void* in, size_t in_rs, void* out,
                         size_t out_rs, size_t out_xs, hipStream_t st, int tile) {
  int nrg = (nrhs + RB - 1) / RB;
  if (2 * nv * nrg > 256) throw std::runtime_error("restrict: too many outputs per block");
  // largest power-of-two tile (dividing Vb) with LDS <= 48 KiB
  int TS = 1;
  auto bytes = [&](int ts) {
    return (((size_t)ts * nv * 12 * sizeof(TV) + 15) & ~(size_t)15) + (size_t)ts * nrhs * 12 * sizeof(cplx<RA>);
  };
  while (TS * 2 <= 32 && g.Vb % (TS * 2) == 0 && bytes(TS * 2) <= 48 * 1024) TS *= 2;
  if (tile > 0 && tile < TS && g.Vb % tile == 0) TS = tile;
  k_restrict<RA, TV, TI, TO, RB><<<g.nblk, 256, bytes(TS), st>>>(g, nv, nrhs, TS, (const TV*)V, (const TI*)in,
                                                                in_rs, (TO*)out, out_rs, out_xs);
}

template <class RA, class TV, class TI, class TO>
static void restrict_rb(const Geo& g, int nv, int nrhs, const void* V, const void* in, size_t in_rs, void* out,
                        size_t out_rs, size_t out_xs, hipStream_t st, int tile) {
  // choose the rhs group so that 2 nv ceil(nrhs/RB) <= 256
  int need = (2 * nv * nrhs + 255) / 256;
  if (need <= 1)
    restrict_run<RA, TV, TI, TO, 1>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  else if (need <= 2)
    restrict_run<RA, TV, TI, TO, 2>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  else if (need <= 4)
    restrict_run<RA, TV, TI, TO, 4>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  else if (need <= 8)
    restrict_run<RA, TV, TI, TO, 8>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  else
    restrict_run<RA, TV, TI, TO, 16>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
}

// Matrix-core restriction with FP64 products and sums (the Gram matrices of
// the orthonormalisation, and the FP64 restriction), nv <= 32, nrhs <= 32:
//   out[r][X][s nv + i] = sum_{y in X, a in s} conj(v_i(y)_a) x_r(y)_a.
// One workgroup per (block, chirality); wave w owns the 16x16 output tile
// (rows i in 16 (w & 1) .., columns r in 16 (w >> 1) ..) as real and
// imaginary accumulators of v_mfma_f64_16x16x4f64 (A: lane l holds row
// l % 16 of k-slice l / 16; B: column l % 16 of k-slice l / 16; accumulator q
// of lane l is element (l / 16 + 4 q, l % 16)).  k runs over (component of
// the chirality, site) in stages of 32 sites staged in LDS.

template <class TI>
__global__ __launch_bounds__(256) void k_restrict_mf64(Geo g, int nv, int nrhs, const TI* __restrict__ V,
                                                       const TI* __restrict__ in, size_t in_rs,
                                                       double2* __restrict__ out, size_t out_rs, size_t out_xs) {
  constexpr int KC = 32;
  __shared__ double2 sv[KC][33], sx[KC][33];
  const int nlog = g.nblk * 2;
  const int lg = xcd_remap(blockIdx.x, nlog);
  if (lg >= nlog) return;
  const int X = lg >> 1, s = lg & 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int it = w & 1, rt = w >> 1;
  // the Gram matrix V^H V (in is V): Hermitian, so V is staged once and the
  // tile (i >= 16, r < 16) is written from its mirror (i < 16, r >= 16)
  const bool gram = (const void*)in == (const void*)V && nrhs == nv && in_rs == (size_t)12 * g.V;
  const bool skip = gram && it == 1 && rt == 0;
  f64x4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  const size_t base = (size_t)X * 12 * g.Vb;  // plane 0 of block X
  for (int a6 = 0; a6 < 6; ++a6) {
    const size_t pl = base + (size_t)(6 * s + a6) * g.Vb;
    for (int l0 = 0; l0 < g.Vb; l0 += KC) {
      // stage KC sites of component a for every vector and right-hand side:
      // a wavefront reads KC consecutive sites of one plane
      for (int e = t; e < 32 * KC; e += 256) {
        const int c = e / KC, kk = e - c * KC;
        const int loc = l0 + kk;
        cplx<double> v = {0, 0}, x = {0, 0};
        if (loc < g.Vb) {
          if (c < nv) v = ld<double>(V, (size_t)c * 12 * g.V + pl + loc);
          if (c < nrhs && !gram) x = ld<double>(in, (size_t)c * in_rs + pl + loc);
        }
        sv[kk][c] = make_double2(v.x, v.y);
        if (!gram) sx[kk][c] = make_double2(x.x, x.y);
      }
      __syncthreads();
      const double2(*sb)[33] = gram ? sv : sx;
#pragma unroll 4
      for (int kk = 0; kk < KC && !skip; kk += 4) {
        const int k = kk + (lane >> 4);
        const double2 va = sv[k][16 * it + (lane & 15)];
        const double2 xb = sb[k][16 * rt + (lane & 15)];
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(va.x, xb.x, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(va.y, xb.y, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(va.x, xb.y, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(-va.y, xb.x, im, 0, 0, 0);
      }
      __syncthreads();
    }
  }
  if (skip) return;
  const int r = 16 * rt + (lane & 15);
  const bool mirror = gram && it == 0 && rt == 1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 16 * it + (lane >> 4) + 4 * q;
    if (i < nv && r < nrhs) out[(size_t)r * out_rs + (size_t)X * out_xs + s * nv + i] = make_double2(re[q], im[q]);
    if (mirror && r < nv && i < nrhs)
      out[(size_t)i * out_rs + (size_t)X * out_xs + s * nv + r] = make_double2(re[q], -im[q]);
  }
}

// Matrix-core restriction in FP32 (the mixed-precision V-cycle: FP16 or FP32
// vectors and inputs, FP32 products and sums), nv <= 32, nrhs <= 32:
//   out[r][X][s nv + i] = sum_{y in X, a in s} conj(v_i(y)_a) x_r(y)_a.
// With x = xr + i xi stacked as the columns of B = [xr | xi] (2 nrhs columns,
// one or two tiles of 32), T_r = vr^T B and T_i = vi^T B give
//   Re out = T_r[:, r] + T_i[:, nrhs + r],  Im out = T_r[:, nrhs + r] - T_i[:, r]
// (two real products per k-pair instead of four).  One workgroup per (block,
// chirality); KC sites of one component plane are staged in LDS at a time
// (coalesced along the sites), the four wavefronts take every fourth k-pair
// of a stage with v_mfma_f32_32x32x2f32 (A: lane l holds row i = l % 32 of
// k-slice l / 32; B: column l % 32 of k-slice l / 32; accumulator q of lane l
// is element (8 (q / 4) + 4 (l / 32) + q % 4, l % 32)), and their partial
// tiles are summed in LDS at the end in a fixed order.
template <class TV, class TI>
__global__ __launch_bounds__(256) void k_restrict_mf32(Geo g, int nv, int nrhs, const TV* __restrict__ V,
                                                       const TI* __restrict__ in, size_t in_rs,
                                                       float2* __restrict__ out, size_t out_rs, size_t out_xs) {
  constexpr int KC = 64;
  extern __shared__ __align__(16) float lds_r[];
  float(*svr)[33] = (float(*)[33])lds_r;                  // [KC][33] Re v_i, i < 32
  float(*svi)[33] = (float(*)[33])(lds_r + KC * 33);      // [KC][33] Im v_i
  float(*sb)[65] = (float(*)[65])(lds_r + 2 * KC * 33);   // [KC][65] columns xr | xi | 0
  const int nlog = g.nblk * 2;
  const int lg = xcd_remap(blockIdx.x, nlog);
  if (lg >= nlog) return;
  const int X = lg >> 1, s = lg & 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nct = 2 * nrhs > 32 ? 2 : 1;
  f32x16 tr0, ti0, tr1, ti1;
#pragma unroll
  for (int q = 0; q < 16; ++q) tr0[q] = ti0[q] = tr1[q] = ti1[q] = 0.f;
  const size_t base = (size_t)X * 12 * g.Vb;
  for (int e = t; e < KC * 65; e += 256) (&sb[0][0])[e] = 0.f;  // columns >= 2 nrhs stay zero
  for (int e = t; e < 2 * KC * 33; e += 256) lds_r[e] = 0.f;     // vectors i >= nv stay zero
  __syncthreads();
  // stages (component a6, sites l0 .. l0 + KC - 1); the global loads of the
  // next stage are issued before the products of the current one
  const int nl = (g.Vb + KC - 1) / KC, nst = 6 * nl;
  constexpr int PV = 32 * KC / 256, PX = 32 * KC / 256;  // loads per thread (nv, nrhs <= 32)
  cplx<float> pv[PV], px[PX];
  auto fetch = [&](int st_) {
    const int a6 = st_ / nl, l0 = (st_ - a6 * nl) * KC;
    const size_t pl = base + (size_t)(6 * s + a6) * g.Vb;
#pragma unroll
    for (int m = 0; m < PV; ++m) {
      const int e = t + 256 * m, c = e / KC, loc = l0 + (e - c * KC);
      pv[m] = (c < nv && loc < g.Vb) ? ld<float>(V, (size_t)c * 12 * g.V + pl + loc) : cplx<float>{0, 0};
    }
#pragma unroll
    for (int m = 0; m < PX; ++m) {
      const int e = t + 256 * m, c = e / KC, loc = l0 + (e - c * KC);
      px[m] = (c < nrhs && loc < g.Vb) ? ld<float>(in, (size_t)c * in_rs + pl + loc) : cplx<float>{0, 0};
    }
  };
  fetch(0);
  for (int st_ = 0; st_ < nst; ++st_) {
#pragma unroll
    for (int m = 0; m < PV; ++m) {
      const int e = t + 256 * m, c = e / KC, kk = e - c * KC;
      if (c < nv) {
        svr[kk][c] = pv[m].x;
        svi[kk][c] = pv[m].y;
      }
    }
#pragma unroll
    for (int m = 0; m < PX; ++m) {
      const int e = t + 256 * m, c = e / KC, kk = e - c * KC;
      if (c < nrhs) {
        sb[kk][c] = px[m].x;
        sb[kk][nrhs + c] = px[m].y;
      }
    }
    __syncthreads();
    if (st_ + 1 < nst) fetch(st_ + 1);
#pragma unroll 2
    for (int kp = w; kp < KC / 2; kp += 4) {
      const int k = 2 * kp + (lane >> 5), c = lane & 31;
      const float ar = svr[k][c], ai = svi[k][c];
      const float b0 = sb[k][c];
      tr0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b0, tr0, 0, 0, 0);
      ti0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b0, ti0, 0, 0, 0);
      if (nct == 2) {
        const float b1 = sb[k][32 + c];
        tr1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1, tr1, 0, 0, 0);
        ti1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b1, ti1, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // partial tiles of the four wavefronts: red[w][m][row][col], m = (T_r, T_i)
  // for columns 0..31 and, with two column tiles, 32..63
  float* red = lds_r;
  const int ncol = 32 * nct;
  const size_t wstride = (size_t)2 * 32 * ncol;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3), col = lane & 31;
    red[w * wstride + (0 * 32 + row) * ncol + col] = tr0[q];
    red[w * wstride + (1 * 32 + row) * ncol + col] = ti0[q];
    if (nct == 2) {
      red[w * wstride + (0 * 32 + row) * ncol + 32 + col] = tr1[q];
      red[w * wstride + (1 * 32 + row) * ncol + 32 + col] = ti1[q];
    }
  }
  __syncthreads();
  for (int e = t; e < nv * nrhs; e += 256) {
    const int i = e / nrhs, r = e - i * nrhs;
    float re = 0.f, im = 0.f;
    for (int ww = 0; ww < 4; ++ww) {
      const float* R = red + ww * wstride;
      re += R[(0 * 32 + i) * ncol + r] + R[(1 * 32 + i) * ncol + nrhs + r];
      im += R[(0 * 32 + i) * ncol + nrhs + r] - R[(1 * 32 + i) * ncol + r];
    }
    out[(size_t)r * out_rs + (size_t)X * out_xs + s * nv + i] = make_float2(re, im);
  }
}

// Register-operand variant of k_restrict_mf32 for Vb a multiple of 32: no
// staging.  The k index of the products is (component, site) as before but
// assigned so that every lane walks consecutive sites: for component a and
// wavefront w, lane half h takes sites w Vb / 4 + h Vb / 8 + j at step j, and
// loads 4 consecutive sites of its vector (16 bytes) or right-hand side per
// load.  Lane l supplies A = v_{l % 32} and B = column l % 32 of [xr | xi].
// The four wavefronts' partial tiles are summed in LDS in a fixed order.
template <class TI>
__global__ __launch_bounds__(256) void k_restrict_mf32d(Geo g, int nv, int nrhs, const half2_t* __restrict__ V,
                                                        const TI* __restrict__ in, size_t in_rs,
                                                        float2* __restrict__ out, size_t out_rs, size_t out_xs) {
  extern __shared__ __align__(16) float lds_d[];
  const int nlog = g.nblk * 2;
  const int lg = xcd_remap(blockIdx.x, nlog);
  if (lg >= nlog) return;
  const int X = lg >> 1, s = lg & 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int c = lane & 31, h = lane >> 5;
  const int nct = 2 * nrhs > 32 ? 2 : 1;
  const int q8 = g.Vb >> 3;  // sites per lane half and wavefront
  const bool va = c < nv;
  // column c (and 32 + c) of B: real (c < nrhs) or imaginary part of rhs c mod nrhs
  const int r0 = c < nrhs ? c : c - nrhs, r1 = 32 + c < 2 * nrhs ? 32 + c - nrhs : 0;
  const bool b0ok = c < 2 * nrhs, b0im = c >= nrhs;
  const bool b1ok = 32 + c < 2 * nrhs;
  f32x16 tr0, ti0, tr1, ti1;
#pragma unroll
  for (int q = 0; q < 16; ++q) tr0[q] = ti0[q] = tr1[q] = ti1[q] = 0.f;
  const size_t base = (size_t)X * 12 * g.Vb;
  const int site0 = w * 2 * q8 + h * q8;
  for (int a6 = 0; a6 < 6; ++a6) {
    const size_t pl = base + (size_t)(6 * s + a6) * g.Vb + site0;
    const half2_t* vp = V + (size_t)(va ? c : 0) * 12 * g.V + pl;
    const TI* ip0 = in + (size_t)r0 * in_rs + pl;
    const TI* ip1 = in + (size_t)r1 * in_rs + pl;
    for (int j = 0; j < q8; j += 4) {
      half2_t v4[4];
      const uint4 raw = *(const uint4*)(vp + j);  // 16-byte aligned: Vb % 32 == 0
      __builtin_memcpy(v4, &raw, sizeof(raw));
      cplx<float> x0[4], x1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x0[u] = b0ok ? ld<float>(ip0, j + u) : cplx<float>{0, 0};
        x1[u] = (nct == 2 && b1ok) ? ld<float>(ip1, j + u) : cplx<float>{0, 0};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float ar = va ? (float)v4[u].x : 0.f, ai = va ? (float)v4[u].y : 0.f;
        const float b0 = b0im ? x0[u].y : x0[u].x;
        tr0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b0, tr0, 0, 0, 0);
        ti0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b0, ti0, 0, 0, 0);
        if (nct == 2) {
          const float b1 = x1[u].y;  // columns 32.. are imaginary parts
          tr1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1, tr1, 0, 0, 0);
          ti1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b1, ti1, 0, 0, 0);
        }
      }
    }
  }
  float* red = lds_d;
  const int ncol = 32 * nct;
  const size_t wstride = (size_t)2 * 32 * ncol;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = 8 * (q >> 2) + 4 * h + (q & 3);
    red[w * wstride + (0 * 32 + row) * ncol + c] = tr0[q];
    red[w * wstride + (1 * 32 + row) * ncol + c] = ti0[q];
    if (nct == 2) {
      red[w * wstride + (0 * 32 + row) * ncol + 32 + c] = tr1[q];
      red[w * wstride + (1 * 32 + row) * ncol + 32 + c] = ti1[q];
    }
  }
  __syncthreads();
  for (int e = t; e < nv * nrhs; e += 256) {
    const int i = e / nrhs, r = e - i * nrhs;
    float re = 0.f, im = 0.f;
    for (int ww = 0; ww < 4; ++ww) {
      const float* R = red + ww * wstride;
      re += R[(0 * 32 + i) * ncol + r] + R[(1 * 32 + i) * ncol + nrhs + r];
      im += R[(0 * 32 + i) * ncol + nrhs + r] - R[(1 * 32 + i) * ncol + r];
    }
    out[(size_t)r * out_rs + (size_t)X * out_xs + s * nv + i] = make_float2(re, im);
  }
}

int restrict_mf32_lds_bytes(int nrhs) {
  const int staging = (2 * 64 * 33 + 64 * 65) * 4;
  const int reduce = 4 * 2 * 32 * (2 * nrhs > 32 ? 64 : 32) * 4;
  return staging > reduce ? staging : reduce;
}

void launch_restrict(const Geo& g, int nv, int nrhs, const void* V, int v_t, const void* in, int in_t,
                     size_t in_rs, void* out, int out_t, size_t out_rs, size_t out_xs, int acc64,
                     hipStream_t st, int tile) {
  if (tile == RESTRICT_MFMA64) {
    if (nv > 32 || nrhs > 32 || out_t != C128 || v_t != in_t || (v_t != C128 && v_t != C64))
      throw std::runtime_error("launch_restrict: the FP64 matrix-core path needs FP64 output, equal FP64 or FP32 "
                               "operand types and nv, nrhs <= 32");
    const dim3 grid(round8(g.nblk * 2));
    if (v_t == C128)
      k_restrict_mf64<double2><<<grid, 256, 0, st>>>(g, nv, nrhs, (const double2*)V, (const double2*)in, in_rs,
                                                     (double2*)out, out_rs, out_xs);
    else
      k_restrict_mf64<float2><<<grid, 256, 0, st>>>(g, nv, nrhs, (const float2*)V, (const float2*)in, in_rs,
                                                    (double2*)out, out_rs, out_xs);
    return;
  }
  if (tile == RESTRICT_MFMA32D) {
    if (nv > 32 || nrhs > 32 || out_t != C64 || acc64 || v_t != C32H || (in_t != C64 && in_t != C32H) ||
        g.Vb % 32 != 0)
      throw std::runtime_error("launch_restrict: the register-operand matrix-core path needs FP16 vectors, FP32 or "
                               "FP16 inputs, FP32 output, nv, nrhs <= 32 and a block volume divisible by 32");
    const dim3 grid(round8(g.nblk * 2));
    const int lds = 4 * 2 * 32 * (2 * nrhs > 32 ? 64 : 32) * 4;
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)k_restrict_mf32d<float2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                64 * 1024);
      (void)hipFuncSetAttribute((const void*)k_restrict_mf32d<half2_t>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                64 * 1024);
      attr = true;
    }
    if (in_t == C64)
      k_restrict_mf32d<float2><<<grid, 256, lds, st>>>(g, nv, nrhs, (const half2_t*)V, (const float2*)in, in_rs,
                                                       (float2*)out, out_rs, out_xs);
    else
      k_restrict_mf32d<half2_t><<<grid, 256, lds, st>>>(g, nv, nrhs, (const half2_t*)V, (const half2_t*)in, in_rs,
                                                        (float2*)out, out_rs, out_xs);
    return;
  }
  if (tile == RESTRICT_MFMA32) {
    if (nv > 32 || nrhs > 32 || out_t != C64 || acc64 || v_t != C32H || (in_t != C64 && in_t != C32H))
      throw std::runtime_error("launch_restrict: the FP32 matrix-core path needs FP16 vectors, FP32 or FP16 inputs, "
                               "FP32 output and nv, nrhs <= 32");
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)k_restrict_mf32<half2_t, float2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
      (void)hipFuncSetAttribute((const void*)k_restrict_mf32<half2_t, half2_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
      attr = true;
    }
    const dim3 grid(round8(g.nblk * 2));
    const int lds = restrict_mf32_lds_bytes(nrhs);
    if (in_t == C64)
      k_restrict_mf32<half2_t, float2><<<grid, 256, lds, st>>>(g, nv, nrhs, (const half2_t*)V, (const float2*)in,
                                                               in_rs, (float2*)out, out_rs, out_xs);
    else
      k_restrict_mf32<half2_t, half2_t><<<grid, 256, lds, st>>>(g, nv, nrhs, (const half2_t*)V, (const half2_t*)in,
                                                                in_rs, (float2*)out, out_rs, out_xs);
    return;
  }
  if (v_t == C128 && in_t == C128 && out_t == C128)
    return restrict_rb<double, double2, double2, double2>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  if (v_t == C32H && in_t == C64 && out_t == C64 && !acc64)
    return restrict_rb<float, half2_t, float2, float2>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  if (v_t == C32H && in_t == C32H && out_t == C64 && !acc64)
    return restrict_rb<float, half2_t, half2_t, float2>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  if (v_t == C64 && in_t == C64 && out_t == C128 && acc64)
    return restrict_rb<double, float2, float2, double2>(g, nv, nrhs, V, in, in_rs, out, out_rs, out_xs, st, tile);
  throw std::runtime_error("launch_restrict: unsupported type combination");
}

// ---------------------------------------------------------------------------
// Prolongation.  One thread per (colour, site) (a wavefront holds one colour
// and consecutive sites); accumulators for the 4 spins x RB right-hand sides.
// ---------------------------------------------------------------------------
template <class R, class TV, class TC, class TO, int RB>
__global__ __launch_bounds__(256) void k_prolong(Geo g, int nv, int nrhs, const TV* __restrict__ V,
                                                 const TC* __restrict__ xc, size_t xc_rs, size_t xc_xs,
                                                 TO* __restrict__ out, size_t out_rs, int accumulate) {
  const int V_ = g.V;
  int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 3 * V_) return;
  int col = t / V_;
  int s = t - col * V_;
  int X = s / g.Vb;
  const size_t fb = fbase_b(g, 12, s, X);
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    cplx<R> acc[4][RB];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int q = 0; q < RB; ++q) acc[sp][q] = {0, 0};
    for (int i = 0; i < nv; ++i) {
      cplx<R> v[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) v[sp] = ld<R>(V, (size_t)i * 12 * V_ + (size_t)(sp * 3 + col) * g.Vb + fb);
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        int r = r0 + q;
        if (r < nrhs) {
          cplx<R> c0 = ld<R>(xc, r * xc_rs + X * xc_xs + i);
          cplx<R> c1 = ld<R>(xc, r * xc_rs + X * xc_xs + nv + i);
          cmac(acc[0][q], v[0], c0);
          cmac(acc[1][q], v[1], c0);
          cmac(acc[2][q], v[2], c1);
          cmac(acc[3][q], v[3], c1);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      int r = r0 + q;
      if (r < nrhs) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
          size_t o = r * out_rs + (size_t)(sp * 3 + col) * g.Vb + fb;
          cplx<R> val = acc[sp][q];
          if (accumulate) val = val + ld<R>(out, o);
          st(out, o, val);
        }
      }
    }
  }
}

template <class R, class TV, class TC, class TO>
static void prolong_run(const Geo& g, int nv, int nrhs, const void* V, const void* xc, size_t xc_rs, size_t xc_xs,
                        void* out, size_t out_rs, int accumulate, hipStream_t st) {
  int nb = (3 * g.V + 255) / 256;
  auto go = [&](auto rbtag) {
    constexpr int RB = decltype(rbtag)::value;
    k_prolong<R, TV, TC, TO, RB><<<nb, 256, 0, st>>>(g, nv, nrhs, (const TV*)V, (const TC*)xc, xc_rs, xc_xs,
                                                     (TO*)out, out_rs, accumulate);
  };
  if (nrhs <= 1)
    go(std::integral_constant<int, 1>());
  else if (nrhs <= 4)
    go(std::integral_constant<int, 4>());
  else if (nrhs <= 8)
    go(std::integral_constant<int, 8>());
  else if (nrhs <= 12)
    go(std::integral_constant<int, 12>());
  else
    go(std::integral_constant<int, 16>());
}

// Matrix-core prolongation for FP32 or FP16 vectors and FP32 coefficients
// (the update V' = V coef of the orthonormalisation; the mixed V-cycle's
// prolongation), FP32 products and sums, nv <= 32, nrhs <= 32:
//   out_r(y, a) (+)= sum_i V_i(y, a) xc[r][X(y)][s(a) nv + i].
// Computed transposed, out^T[r][k] = sum_i xc[i][r] V_i[k], so that a
// wavefront's results for one right-hand side are 32 consecutive sites.  One
// workgroup per (block, chirality); each wavefront takes tiles of 32 sites of
// one component plane; v_mfma_f32_32x32x2f32 with A = coefficients (lane l:
// row r = l % 32, i-slice l / 32) and B = vectors (lane l: i-slice l / 32,
// site l % 32); accumulator q of lane l is (r = 8 (q / 4) + 4 (l / 32) + q % 4,
// site l % 32).
template <class TV>
__global__ __launch_bounds__(256) void k_prolong_mf(Geo g, int nv, int nrhs, const TV* __restrict__ V,
                                                    const float2* __restrict__ xc, size_t xc_rs, size_t xc_xs,
                                                    float2* __restrict__ out, size_t out_rs, int accumulate) {
  const int nlog = g.nblk * 2;
  const int lg = xcd_remap(blockIdx.x, nlog);
  if (lg >= nlog) return;
  const int X = lg >> 1, s = lg & 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int lr = lane & 31, lh = lane >> 5;
  // coefficients of this lane for the 16 i-steps: xc[r = lr][X][s nv + i], i = 2 step + lh
  float cr[16], ci[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = 2 * q + lh;
    cplx<float> c = {0, 0};
    if (i < nv && lr < nrhs) c = ld<float>(xc, (size_t)lr * xc_rs + (size_t)X * xc_xs + s * nv + i);
    cr[q] = c.x;
    ci[q] = c.y;
  }
  const int nst = (g.Vb + 31) / 32;  // site tiles per component plane
  const size_t base = (size_t)X * 12 * g.Vb;
  // tiles of 32 sites of one component plane, every fourth to this wavefront;
  // the vectors of the next tile are loaded before the products of this one
  const int ntl = 6 * nst;
  TV vb[16], vn[16];
  auto fetch = [&](int tl, TV (&dst)[16]) {
    const int a = 6 * s + tl / nst;
    const int loc = (tl % nst) * 32 + lr;
    const size_t o = base + (size_t)a * g.Vb + (loc < g.Vb ? loc : 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = 2 * q + lh;
      dst[q] = V[(size_t)(i < nv ? i : 0) * 12 * g.V + o];
    }
  };
  if (w < ntl) fetch(w, vb);
  for (int tl = w; tl < ntl; tl += 4) {
    if (tl + 4 < ntl) fetch(tl + 4, vn);
    const int a = 6 * s + tl / nst;
    const int loc = (tl % nst) * 32 + lr;
    const bool in = loc < g.Vb;
    const size_t o = base + (size_t)a * g.Vb + (in ? loc : 0);
    f32x16 re, im;
#pragma unroll
    for (int q = 0; q < 16; ++q) re[q] = im[q] = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = 2 * q + lh;
      cplx<float> v = {0, 0};
      if (in && i < nv) v = ld<float>(vb, q);
      re = __builtin_amdgcn_mfma_f32_32x32x2f32(cr[q], v.x, re, 0, 0, 0);
      re = __builtin_amdgcn_mfma_f32_32x32x2f32(-ci[q], v.y, re, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_32x32x2f32(cr[q], v.y, im, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_32x32x2f32(ci[q], v.x, im, 0, 0, 0);
    }
    if (in) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int r = 8 * (q >> 2) + 4 * lh + (q & 3);
        if (r < nrhs) {
          const size_t oo = (size_t)r * out_rs + o;
          cplx<float> val = {re[q], im[q]};
          if (accumulate) val = val + ld<float>(out, oo);
          st(out, oo, val);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) vb[q] = vn[q];
  }
}

void launch_prolong(const Geo& g, int nv, int nrhs, const void* V, int v_t, const void* xc, int xc_t, size_t xc_rs,
                    size_t xc_xs, void* out, int out_t, size_t out_rs, int accumulate, int compute32,
                    hipStream_t st, int variant) {
  if (variant == PROLONG_MFMA32) {
    if (!compute32 || (v_t != C32H && v_t != C64) || xc_t != C64 || out_t != C64 || nv > 32 || nrhs > 32)
      throw std::runtime_error("launch_prolong: the matrix-core path needs FP32 arithmetic, FP16 or FP32 vectors, "
                               "FP32 coefficients and output, nv, nrhs <= 32");
    if (v_t == C32H)
      k_prolong_mf<half2_t><<<round8(g.nblk * 2), 256, 0, st>>>(g, nv, nrhs, (const half2_t*)V, (const float2*)xc,
                                                                xc_rs, xc_xs, (float2*)out, out_rs, accumulate);
    else
      k_prolong_mf<float2><<<round8(g.nblk * 2), 256, 0, st>>>(g, nv, nrhs, (const float2*)V, (const float2*)xc,
                                                               xc_rs, xc_xs, (float2*)out, out_rs, accumulate);
    return;
  }
  if (!compute32 && v_t == C128 && xc_t == C128 && out_t == C128)
    return prolong_run<double, double2, double2, double2>(g, nv, nrhs, V, xc, xc_rs, xc_xs, out, out_rs,
                                                          accumulate, st);
  if (compute32 && v_t == C32H && xc_t == C64 && out_t == C64)
    return prolong_run<float, half2_t, float2, float2>(g, nv, nrhs, V, xc, xc_rs, xc_xs, out, out_rs, accumulate,
                                                       st);
  if (compute32 && v_t == C64 && xc_t == C64 && out_t == C64) {
    if (nv <= 32 && nrhs <= 32) {
      k_prolong_mf<float2><<<round8(g.nblk * 2), 256, 0, st>>>(g, nv, nrhs, (const float2*)V, (const float2*)xc,
                                                               xc_rs, xc_xs, (float2*)out, out_rs, accumulate);
      return;
    }
    return prolong_run<float, float2, float2, float2>(g, nv, nrhs, V, xc, xc_rs, xc_xs, out, out_rs, accumulate,
                                                      st);
  }
  if (!compute32 && v_t == C64 && xc_t == C128 && out_t == C64)
    return prolong_run<double, float2, double2, float2>(g, nv, nrhs, V, xc, xc_rs, xc_xs, out, out_rs, accumulate,
                                                        st);
  throw std::runtime_error("launch_prolong: unsupported type combination");
}

// ---------------------------------------------------------------------------
// Coarse 9-point block stencil.  One thread per (coarse site X, row n); the
// NR right-hand sides of a launch row share each loaded matrix element.
// ---------------------------------------------------------------------------
template <class R, class TC, class TX, int NR>
__global__ __launch_bounds__(256) void k_coarse_mv(CGeo cg, int N, const TC* __restrict__ Dc,
                                                   const TX* __restrict__ x, TX* __restrict__ y,
                                                   const TX* __restrict__ b, size_t rs, int nrhs,
                                                   const int* __restrict__ active, int astride) {
  int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= cg.NC * N) return;
  int X = t / N, n = t - X * N;
  int r0 = blockIdx.y * NR;
  // right-hand sides whose Krylov solve has stopped are skipped (their y is not used)
  unsigned live = 0;
#pragma unroll
  for (int q = 0; q < NR; ++q)
    if (r0 + q < nrhs && (!active || active[(size_t)(r0 + q) * astride])) live |= 1u << q;
  if (!live) return;
  int c[4];
  {
    int q = X;
    for (int m = 0; m < 3; ++m) {
      c[m] = q % cg.N[m];
      q /= cg.N[m];
    }
    c[3] = q;
  }
  cplx<R> acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = {0, 0};
  for (int d = 0; d < 9; ++d) {
    int Y = X;
    if (d > 0) {
      int mu = (d - 1) & 3;
      int step = d <= 4 ? 1 : -1;
      int cc = c[mu] + step;
      if (cc == cg.N[mu]) cc = 0;
      if (cc < 0) cc = cg.N[mu] - 1;
      Y = X + (cc - c[mu]) * cg.sN[mu];
    }
    const TC* B = Dc + ((size_t)(X * 9 + d) * N) * N + n;
    const TX* xy = x + (size_t)Y * N;
    for (int m = 0; m < N; ++m) {
      cplx<R> bb = ld<R>(B, (size_t)m * N);
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (live & (1u << q)) cmac(acc[q], bb, ld<R>(xy, (r0 + q) * rs + m));
    }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    int r = r0 + q;
    if (live & (1u << q)) {
      size_t o = r * rs + (size_t)X * N + n;
      if (b)
        st(y, o, ld<R>(b, o) - acc[q]);
      else
        st(y, o, acc[q]);
    }
  }
}

// Matrix-core coarse stencil (complex64, 2 nv <= 64, nrhs <= 32).  One
// workgroup per coarse site X; wave w computes the rows 32 (w & 1) .. of the
// real (w < 2) or imaginary (w >= 2) part of y[.][X] for all right-hand sides
// with v_mfma_f32_32x32x2f32: A = the stencil block (lane l: row l % 32 of
// column-slice l / 32), B = the neighbour's vectors staged in LDS (lane l:
// slice l / 32, right-hand side l % 32).  The results pass through LDS so that
// each right-hand side's 2 nv entries are written contiguously.  Registers
// are capped for two waves per SIMD (the double-buffered operands would
// otherwise leave one).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_coarse_mv_mf(
    CGeo cg, int N, const float2* __restrict__ Dc, const float2* __restrict__ x, float2* __restrict__ y,
    const float2* __restrict__ b, size_t rs, int nrhs, const int* __restrict__ active, int astride) {
  __shared__ float2 sx[64][33];    // [m][r]
  __shared__ float sy[2][32][65];  // [re, im][r][n]
  const int X = xcd_remap(blockIdx.x, cg.NC);
  if (X >= cg.NC) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // nothing to do once every right-hand side has stopped (same decision in all threads)
  bool any = active == nullptr;
  for (int r = 0; r < nrhs && !any; ++r) any = active[(size_t)r * astride] != 0;
  if (!any) return;
  int c[4];
  {
    int q = X;
    for (int m = 0; m < 3; ++m) {
      c[m] = q % cg.N[m];
      q /= cg.N[m];
    }
    c[3] = q;
  }
  const int nt = w & 1, part = w >> 1;
  const int n = 32 * nt + (lane & 31);
  f32x16 acc;
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.f;
  // the stencil block of the next direction is loaded while the current one
  // is contracted (all 32 loads of a block in flight at once)
  auto load_block = [&](int d, float2(&dst)[32]) {
    const float2* B = Dc + (size_t)(X * 9 + d) * N * N;
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const int m = 2 * s + (lane >> 5);
      dst[s] = (m < N && n < N) ? B[(size_t)m * N + n] : make_float2(0.f, 0.f);
    }
  };
  // likewise the neighbour's vectors: thread t holds entries t + 256 q of the
  // [r][m] tile in registers until they are staged in LDS
  auto load_x = [&](int d, float2(&dst)[8]) {
    int Y = X;
    if (d > 0) {
      const int mu = (d - 1) & 3;
      int cc = c[mu] + (d <= 4 ? 1 : -1);
      if (cc == cg.N[mu]) cc = 0;
      if (cc < 0) cc = cg.N[mu] - 1;
      Y = X + (cc - c[mu]) * cg.sN[mu];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q, r = e >> 6, m = e & 63;
      dst[q] = (r < nrhs && m < N) ? x[(size_t)r * rs + (size_t)Y * N + m] : make_float2(0.f, 0.f);
    }
  };
  float2 av[32], an[32], xr[8];
  load_block(0, av);
  load_x(0, xr);
  for (int d = 0; d < 9; ++d) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      sx[e & 63][e >> 6] = xr[q];
    }
    __syncthreads();
    if (d < 8) {
      load_block(d + 1, an);
      load_x(d + 1, xr);
    }
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const float2 xb = sx[2 * s + (lane >> 5)][lane & 31];
      if (part == 0) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s].x, xb.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(-av[s].y, xb.y, acc, 0, 0, 0);
      } else {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s].x, xb.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s].y, xb.x, acc, 0, 0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 32; ++s) av[s] = an[s];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) sy[part][lane & 31][32 * nt + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3)] = acc[q];
  __syncthreads();
  for (int e = t; e < 32 * 64; e += 256) {
    const int r = e >> 6, nn = e & 63;
    if (r < nrhs && nn < N && (!active || active[(size_t)r * astride])) {
      const size_t o = (size_t)r * rs + (size_t)X * N + nn;
      float2 v = make_float2(sy[0][r][nn], sy[1][r][nn]);
      if (b) v = make_float2(b[o].x - v.x, b[o].y - v.y);
      y[o] = v;
    }
  }
}

// Matrix-core coarse stencil for nrhs <= 16.  The real and imaginary parts
// share one 32-column B operand and one accumulator: with A = Re of the
// stencil block, column c < 16 holds Re x of right-hand side c and column
// 16 + c its Im x; with A = Im of the block, column c holds -Im x and column
// 16 + c Re x.  Column c then accumulates Re y and column 16 + c Im y: two
// products per k-slice give both parts, half the matrix-core work of the
// 32-wide kernel when there are at most 16 right-hand sides.  Wave w owns rows
// 32 (w & 1) .. + 31 and the k (= m) half w >> 1; the halves are summed in a
// fixed order through LDS.  As in k_coarse_mv_mf, the next direction's block
// and neighbour vectors are loaded while the current one is contracted.
__global__ __launch_bounds__(256) void k_coarse_mv_mf16(CGeo cg, int N, const float2* __restrict__ Dc,
                                                        const float2* __restrict__ x, float2* __restrict__ y,
                                                        const float2* __restrict__ b, size_t rs, int nrhs,
                                                        const int* __restrict__ active, int astride) {
  __shared__ float2 sx[64][17];    // [m][r]
  __shared__ float sy[2][32][65];  // [k half][column][n]
  const int X = xcd_remap(blockIdx.x, cg.NC);
  if (X >= cg.NC) return;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  bool any = active == nullptr;
  for (int r = 0; r < nrhs && !any; ++r) any = active[(size_t)r * astride] != 0;
  if (!any) return;
  int c[4];
  {
    int q = X;
    for (int m = 0; m < 3; ++m) {
      c[m] = q % cg.N[m];
      q /= cg.N[m];
    }
    c[3] = q;
  }
  const int nt = w & 1, kh = w >> 1;
  const int n = 32 * nt + (lane & 31);
  const int col = lane & 31, rr = col & 15;
  const bool lo = col < 16;
  f32x16 acc;
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.f;
  auto load_block = [&](int d, float2(&dst)[16]) {
    const float2* B = Dc + (size_t)(X * 9 + d) * N * N;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int m = 32 * kh + 2 * s + (lane >> 5);
      dst[s] = (m < N && n < N) ? B[(size_t)m * N + n] : make_float2(0.f, 0.f);
    }
  };
  // thread t stages entries t + 256 q (q < 4) of the [r][m] tile, r < 16
  auto load_x = [&](int d, float2(&dst)[4]) {
    int Y = X;
    if (d > 0) {
      const int mu = (d - 1) & 3;
      int cc = c[mu] + (d <= 4 ? 1 : -1);
      if (cc == cg.N[mu]) cc = 0;
      if (cc < 0) cc = cg.N[mu] - 1;
      Y = X + (cc - c[mu]) * cg.sN[mu];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q, r = e >> 6, m = e & 63;
      dst[q] = (r < nrhs && m < N) ? x[(size_t)r * rs + (size_t)Y * N + m] : make_float2(0.f, 0.f);
    }
  };
  float2 av[16], an[16], xr[4];
  load_block(0, av);
  load_x(0, xr);
  for (int d = 0; d < 9; ++d) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      sx[e & 63][e >> 6] = xr[q];
    }
    __syncthreads();
    if (d < 8) {
      load_block(d + 1, an);
      load_x(d + 1, xr);
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const float2 xv = sx[32 * kh + 2 * s + (lane >> 5)][rr];
      const float b1 = lo ? xv.x : xv.y, b2 = lo ? -xv.y : xv.x;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s].x, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s].y, b2, acc, 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) av[s] = an[s];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q)
    sy[kh][col][32 * nt + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3)] = acc[q];
  __syncthreads();
  for (int e = t; e < 16 * 64; e += 256) {
    const int r = e >> 6, nn = e & 63;
    if (r < nrhs && nn < N && (!active || active[(size_t)r * astride])) {
      const size_t o = (size_t)r * rs + (size_t)X * N + nn;
      float2 v = make_float2(sy[0][r][nn] + sy[1][r][nn], sy[0][16 + r][nn] + sy[1][16 + r][nn]);
      if (b) v = make_float2(b[o].x - v.x, b[o].y - v.y);
      y[o] = v;
    }
  }
}

template <class R, class TC, class TX>
static void coarse_mv_run(const CGeo& cg, int N, const void* Dc, const void* x, void* y, const void* b, int nrhs,
                          size_t rs, hipStream_t st, int variant, const int* active, int astride) {
  int nb = (cg.NC * N + 255) / 256;
  auto go = [&](auto tag) {
    constexpr int NR = decltype(tag)::value;
    dim3 grid(nb, (nrhs + NR - 1) / NR);
    k_coarse_mv<R, TC, TX, NR><<<grid, 256, 0, st>>>(cg, N, (const TC*)Dc, (const TX*)x, (TX*)y, (const TX*)b, rs,
                                                     nrhs, active, astride);
  };
  int nr = variant > 0 ? variant : (nrhs == 1 ? 1 : nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : nrhs <= 12 ? 12 : 16);
  if (nr == 1)
    go(std::integral_constant<int, 1>());
  else if (nr <= 4)
    go(std::integral_constant<int, 4>());
  else if (nr <= 8)
    go(std::integral_constant<int, 8>());
  else if (nr <= 12)
    go(std::integral_constant<int, 12>());
  else
    go(std::integral_constant<int, 16>());
}

void launch_coarse_mv(const CGeo& cg, int N, const void* Dc, const void* x, void* y, const void* b, int nrhs,
                      size_t rs, int prec32, hipStream_t st, int variant, const int* active, int astride) {
  if (variant == COARSE_MV_MFMA) {
    if (!prec32 || N > 64 || nrhs > 32)
      throw std::runtime_error("coarse matvec: the matrix-core path needs complex64, 2 nv <= 64 and nrhs <= 32");
    k_coarse_mv_mf<<<round8(cg.NC), 256, 0, st>>>(cg, N, (const float2*)Dc, (const float2*)x, (float2*)y,
                                                 (const float2*)b, rs, nrhs, active, astride);
    return;
  }
  if (variant == COARSE_MV_MFMA16) {
    if (!prec32 || N > 64 || nrhs > 16)
      throw std::runtime_error("coarse matvec: the 16-wide matrix-core path needs complex64, 2 nv <= 64 and nrhs <= 16");
    k_coarse_mv_mf16<<<round8(cg.NC), 256, 0, st>>>(cg, N, (const float2*)Dc, (const float2*)x, (float2*)y,
                                                   (const float2*)b, rs, nrhs, active, astride);
    return;
  }
  if (prec32)
    coarse_mv_run<float, float2, float2>(cg, N, Dc, x, y, b, nrhs, rs, st, variant, active, astride);
  else
    coarse_mv_run<double, double2, double2>(cg, N, Dc, x, y, b, nrhs, rs, st, variant, active, astride);
}

// ---------------------------------------------------------------------------
// Coarse operator eq. (7), fused.  One workgroup per (block X, direction d,
// source chirality sp).  For d = 0 the in-block operator D_SAP is applied to
// P_sp v_j on every site of X; for d = 1..8 only the sites of X whose hop in
// direction d leaves the block contribute, through that single hop.  For a
// tile of sites the results g_j(y) and the vectors v_i(y) are staged in LDS
// and contracted:
//   Dc[X][d][(sp, j)][(s, i)] = sum_y sum_{a in s} conj(v_i(y)_a) g_j(y)_a.
// Thread t owns row n = t % N and the columns of group t / N.
// ---------------------------------------------------------------------------
template <class R, class TV, class TL, class TC, class TO, int CPG>
__global__ __launch_bounds__(256) void k_coarse_build(Geo g, int nv, R kappa, const TV* __restrict__ V,
                                                      const TL* __restrict__ U, const TC* __restrict__ C,
                                                      TO* __restrict__ Dc) {
  extern __shared__ __align__(16) char smem[];
  const int N = 2 * nv;
  const int T = 256 / nv;  // sites per tile (threads t < T nv compute the vectors g)
  cplx<R>* sv = (cplx<R>*)smem;     // [T][nv][12]
  cplx<R>* sgv = sv + T * nv * 12;  // [T][nv][12]
  // one workgroup per (X, d, sp) for the self block and the 4 forward blocks
  // (k_coarse_mirror derives the backward ones), X slowest; consecutive
  // logical indices run on one XCD, so the 10 workgroups of a block share
  // that XCD's L2
  const int nlog = g.nblk * 10;
  const int lg = xcd_remap(blockIdx.x, nlog);
  if (lg >= nlog) return;
  const int X = lg / 10, d = (lg % 10) >> 1, sp = lg & 1;
  const int t = threadIdx.x;
  const int Vg = g.V;
  const int mu = (d - 1) & 3;
  const bool fwd = d <= 4;
  int nsites;
  if (d == 0)
    nsites = g.Vb;
  else
    nsites = g.NB[mu] == 1 ? 0 : g.Vb / g.B[mu];
  const int a0 = sp * 6;  // chirality sp keeps components a0 .. a0+5
  const int n = t % N, cg = t / N;
  const int si = n / nv, ii = n - si * nv;
  cplx<R> acc[CPG];
#pragma unroll
  for (int q = 0; q < CPG; ++q) acc[q] = {0, 0};

  for (int tile0 = 0; tile0 < nsites; tile0 += T) {
    if (t < T * nv) {
      const int st_ = t / nv, j = t - st_ * nv;
      const int f = tile0 + st_;
      cplx<R> vj[12], gj[12];
      if (f < nsites) {
        int loc;
        if (d == 0) {
          loc = f;
        } else {
          int q = f, cc[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            if (m == mu) continue;
            cc[m] = q % g.B[m];
            q /= g.B[m];
          }
          cc[mu] = fwd ? g.B[mu] - 1 : 0;
          loc = cc[0] * g.sB[0] + cc[1] * g.sB[1] + cc[2] * g.sB[2] + cc[3] * g.sB[3];
        }
        const int sx = X * g.Vb + loc;
        const int ps = g.Vb;
        const size_t fb12 = fbase_b(g, 12, sx, X), fb36 = fbase_b(g, 36, sx, X);
        const TV* vjp = V + (size_t)j * 12 * Vg;
        ld_spinor<R>(vjp, ps, fb12, vj);
        SiteCoord c = decompose(g, sx);
        cplx<R> psi[12], u[9];
#pragma unroll
        for (int a = 0; a < 12; ++a) gj[a] = {0, 0};
        if (d == 0) {
#pragma unroll
          for (int a = 0; a < 12; ++a) psi[a] = (a >= a0 && a < a0 + 6) ? vj[a] : cplx<R>{0, 0};
#pragma unroll
          for (int a = 0; a < 12; ++a) gj[a] = psi[a];
          clover_acc<R>(C, ps, fb36, psi, gj);
#pragma unroll 1
          for (int dir = 0; dir < 8; ++dir) {
            const int m = dir & 3;
            int sign;
            bool inb;
            int nb = dir < 4 ? neighbour<true>(g, sx, c, m, sign, inb) : neighbour<false>(g, sx, c, m, sign, inb);
            if (!inb) continue;
            ld_spinor<R>(vjp, ps, fbase_b(g, 12, nb, X), psi);
#pragma unroll
            for (int a = 0; a < 12; ++a)
              if (a < a0 || a >= a0 + 6) psi[a] = {0, 0};
            if (dir < 4) {
              ld_link<R>(U, ps, m, fb36, u);
              hop_any<true>(m, psi, u, -kappa * (R)sign, gj);
            } else {
              ld_link<R>(U, ps, m, fbase_b(g, 36, nb, X), u);
              hop_any<false>(m, psi, u, -kappa * (R)sign, gj);
            }
          }
        } else {
          int sign, nblk;
          bool inb;
          int nb = fwd ? neighbour<true>(g, sx, c, mu, sign, inb, nblk)
                       : neighbour<false>(g, sx, c, mu, sign, inb, nblk);
          ld_spinor<R>(vjp, ps, fbase_b(g, 12, nb, nblk), psi);
#pragma unroll
          for (int a = 0; a < 12; ++a)
            if (a < a0 || a >= a0 + 6) psi[a] = {0, 0};
          if (fwd) {
            ld_link<R>(U, ps, mu, fb36, u);
            hop_any<true>(mu, psi, u, -kappa * (R)sign, gj);
          } else {
            ld_link<R>(U, ps, mu, fbase_b(g, 36, nb, nblk), u);
            hop_any<false>(mu, psi, u, -kappa * (R)sign, gj);
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < 12; ++a) vj[a] = gj[a] = {0, 0};
      }
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        sv[(st_ * nv + j) * 12 + a] = vj[a];
        sgv[(st_ * nv + j) * 12 + a] = gj[a];
      }
    }
    __syncthreads();
    if (cg * CPG < nv) {
      const int tl = min(T, nsites - tile0);
      for (int st_ = 0; st_ < tl; ++st_) {
#pragma unroll
        for (int a6 = 0; a6 < 6; ++a6) {
          const int a = 6 * si + a6;
          cplx<R> vv = sv[(st_ * nv + ii) * 12 + a];
#pragma unroll
          for (int q = 0; q < CPG; ++q) {
            const int j = cg * CPG + q;
            if (j < nv) cjmac(acc[q], vv, sgv[(st_ * nv + j) * 12 + a]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (t < N * (256 / N)) {
#pragma unroll
    for (int q = 0; q < CPG; ++q) {
      const int j = cg * CPG + q;
      if (cg * CPG < nv && j < nv) st(Dc, ((size_t)(X * 9 + d) * N + (sp * nv + j)) * N + n, acc[q]);
    }
  }
}

// Matrix-core variant of the fused build (FP16 vectors and fields, FP32
// arithmetic, nv <= 32).  The vectors g_j of a tile are formed as above; the
// contraction then runs on MFMA.  For target chirality s the block
//   C_s[i][j] = sum_k conj(v_i(k)) g_j(k),
// k over the tile's sites and the 6 components of chirality s, is a real
// 32x32 product pair: Re C = vr^T gr + vi^T gi and Im C = vr^T gi - vi^T gr.
// Wave w computes (s = w / 2, real part for even w, imaginary for odd w)
// with v_mfma_f32_32x32x2f32 (A: lane l holds row l % 32 of k-slice l / 32;
// B: column l % 32 of k-slice l / 32; accumulator v of lane l is element
// (8 (v / 4) + 4 (l / 32) + v % 4, l % 32)).  Indices i, j >= nv are padding
// held at zero in LDS.

// Work units per block X: the in-block part (d = 0) split into nch chunks of
// site tiles, then the 4 forward crossing directions d (k_coarse_mirror
// derives the backward blocks).  A unit forms g_j for both
// source chiralities sp from one set of vector and link loads and contracts
// all four (s, sp) blocks.  All units of a block are consecutive logical
// indices on one XCD, so that few blocks are in flight per XCD and their
// vectors stay in its L2.  A d = 0 chunk writes its partial block to
// part[X][chunk][(sp, j)][(s, i)]; the partials are summed in chunk order by
// k_coarse_build_sum (deterministic).
template <int T>
__global__ __launch_bounds__(256) void k_coarse_build_mf(Geo g, int nv, float kappa, const half2_t* __restrict__ V,
                                                         const half2_t* __restrict__ U,
                                                         const half2_t* __restrict__ C, float2* __restrict__ Dc,
                                                         int nch, int tpc, float2* __restrict__ part) {
  constexpr int K = T * 6;  // k per tile and chirality
  // svr/svi[s][k][i]: v_i; sgr/sgi[sp][s][k][j]: g_j of source chirality sp
  __shared__ float svr[2][K][32], svi[2][K][32], sgr[2][2][K][32], sgi[2][2][K][32];
  const int N = 2 * nv;
  const int nu = nch + 4;
  const int nlog = g.nblk * nu;
  const int lg = xcd_remap(blockIdx.x, nlog);
  if (lg >= nlog) return;
  const int X = lg / nu, u = lg - X * nu;
  const int d = u < nch ? 0 : 1 + (u - nch);
  const int chunk = u < nch ? u : 0;
  const int t = threadIdx.x;
  const int Vg = g.V;
  const int mu = (d - 1) & 3;
  const bool fwd = d <= 4;
  int nsites;
  if (d == 0)
    nsites = g.Vb;
  else
    nsites = g.NB[mu] == 1 ? 0 : g.Vb / g.B[mu];
  for (int e = t; e < 2 * K * 32; e += 256) {
    (&svr[0][0][0])[e] = 0.f;
    (&svi[0][0][0])[e] = 0.f;
  }
  for (int e = t; e < 4 * K * 32; e += 256) {
    (&sgr[0][0][0][0])[e] = 0.f;
    (&sgi[0][0][0][0])[e] = 0.f;
  }
  const int w = t >> 6, lane = t & 63;
  const int ws = w >> 1, part_ = w & 1;
  f32x16 acc[2];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[0][q] = acc[1][q] = 0.f;
  __syncthreads();

  const int tbeg = d == 0 ? chunk * tpc * T : 0;
  const int tend = d == 0 ? min(nsites, (chunk + 1) * tpc * T) : nsites;
  for (int tile0 = tbeg; tile0 < tend; tile0 += T) {
    if (t < T * nv) {
      const int j = t / T, st_ = t - j * T;  // lanes run over sites: coalesced vector loads
      const int f = tile0 + st_;
      cplx<float> vj[12], g0[12], g1[12];  // g0 / g1: source chirality 0 / 1
      if (f < tend) {
        int loc;
        if (d == 0) {
          loc = f;
        } else {
          int q = f, cc[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            if (m == mu) continue;
            cc[m] = q % g.B[m];
            q /= g.B[m];
          }
          cc[mu] = fwd ? g.B[mu] - 1 : 0;
          loc = cc[0] * g.sB[0] + cc[1] * g.sB[1] + cc[2] * g.sB[2] + cc[3] * g.sB[3];
        }
        const int sx = X * g.Vb + loc;
        const int ps = g.Vb;
        const size_t fb12 = fbase_b(g, 12, sx, X), fb36 = fbase_b(g, 36, sx, X);
        const half2_t* vjp = V + (size_t)j * 12 * Vg;
        ld_spinor<float>(vjp, ps, fb12, vj);
        SiteCoord c = decompose(g, sx);
        cplx<float> psi[12], p0[12], p1[12], u[9];
#pragma unroll
        for (int a = 0; a < 12; ++a) g0[a] = g1[a] = {0, 0};
        if (d == 0) {
          // the clover term is block diagonal in chirality: one application
          // of (1 + F) to v_j, split by rows, serves both sp
#pragma unroll
          for (int a = 0; a < 12; ++a) psi[a] = vj[a];
          clover_acc<float>(C, ps, fb36, vj, psi);
#pragma unroll
          for (int a = 0; a < 12; ++a) {
            g0[a] = a < 6 ? psi[a] : cplx<float>{0, 0};
            g1[a] = a < 6 ? cplx<float>{0, 0} : psi[a];
          }
          // both hops of direction m are loaded before either is applied
          // (more loads in flight); a neighbour outside the block reads this
          // site instead and enters with coefficient zero
#pragma unroll 1
          for (int m = 0; m < 4; ++m) {
            int sf, sb;
            bool inf, inbk;
            const int nf = neighbour<true>(g, sx, c, m, sf, inf);
            const int nk = neighbour<false>(g, sx, c, m, sb, inbk);
            const int nf_ = inf ? nf : sx, nk_ = inbk ? nk : sx;
            cplx<float> pk[12], uk[9];
            ld_spinor<float>(vjp, ps, fbase_b(g, 12, nf_, X), psi);
            ld_link<float>(U, ps, m, fb36, u);
            ld_spinor<float>(vjp, ps, fbase_b(g, 12, nk_, X), pk);
            ld_link<float>(U, ps, m, fbase_b(g, 36, nk_, X), uk);
            const float cf = inf ? -kappa * (float)sf : 0.f, ck = inbk ? -kappa * (float)sb : 0.f;
#pragma unroll
            for (int a = 0; a < 12; ++a) {
              p0[a] = a < 6 ? psi[a] : cplx<float>{0, 0};
              p1[a] = a < 6 ? cplx<float>{0, 0} : psi[a];
            }
            hop_any<true>(m, p0, u, cf, g0);
            hop_any<true>(m, p1, u, cf, g1);
#pragma unroll
            for (int a = 0; a < 12; ++a) {
              p0[a] = a < 6 ? pk[a] : cplx<float>{0, 0};
              p1[a] = a < 6 ? cplx<float>{0, 0} : pk[a];
            }
            hop_any<false>(m, p0, uk, ck, g0);
            hop_any<false>(m, p1, uk, ck, g1);
          }
        } else {
          int sign, nblk;
          bool inb;
          int nb = fwd ? neighbour<true>(g, sx, c, mu, sign, inb, nblk)
                       : neighbour<false>(g, sx, c, mu, sign, inb, nblk);
          ld_spinor<float>(vjp, ps, fbase_b(g, 12, nb, nblk), psi);
#pragma unroll
          for (int a = 0; a < 12; ++a) {
            p0[a] = a < 6 ? psi[a] : cplx<float>{0, 0};
            p1[a] = a < 6 ? cplx<float>{0, 0} : psi[a];
          }
          if (fwd) {
            ld_link<float>(U, ps, mu, fb36, u);
            hop_any<true>(mu, p0, u, -kappa * (float)sign, g0);
            hop_any<true>(mu, p1, u, -kappa * (float)sign, g1);
          } else {
            ld_link<float>(U, ps, mu, fbase_b(g, 36, nb, nblk), u);
            hop_any<false>(mu, p0, u, -kappa * (float)sign, g0);
            hop_any<false>(mu, p1, u, -kappa * (float)sign, g1);
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < 12; ++a) vj[a] = g0[a] = g1[a] = {0, 0};
      }
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        const int s = a / 6, k = st_ * 6 + (a % 6);
        svr[s][k][j] = vj[a].x;
        svi[s][k][j] = vj[a].y;
        sgr[0][s][k][j] = g0[a].x;
        sgi[0][s][k][j] = g0[a].y;
        sgr[1][s][k][j] = g1[a].x;
        sgi[1][s][k][j] = g1[a].y;
      }
    }
    __syncthreads();
    // tiles past nsites hold zeros (written above), so every k-slice is summed
    const int r = lane & 31, kh = lane >> 5;
#pragma unroll 2
    for (int kk = 0; kk < K; kk += 2) {
      const int k = kk + kh;
      const float ar = svr[ws][k][r], ai = svi[ws][k][r];
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        const float br = sgr[sp][ws][k][r], bi = sgi[sp][ws][k][r];
        if (part_ == 0) {
          acc[sp] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, acc[sp], 0, 0, 0);
          acc[sp] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, acc[sp], 0, 0, 0);
        } else {
          acc[sp] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, acc[sp], 0, 0, 0);
          acc[sp] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, br, acc[sp], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // D element (i, j): column (sp, j), row (s, i) of the column-major block
  // (d = 0: of this chunk's partial block)
  float* out = d == 0 ? (float*)part : (float*)Dc;
  const size_t blk0 = d == 0 ? (size_t)X * nch + chunk : (size_t)X * 9 + d;
  const int j = lane & 31;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
      if (i < nv && j < nv) out[2 * ((blk0 * N + (sp * nv + j)) * N + (ws * nv + i)) + part_] = acc[sp][q];
    }
  }
}

// Dc[X][0] = sum over chunks of the partial in-block blocks, in chunk order
__global__ __launch_bounds__(256) void k_coarse_build_sum(int nblk, int N, int nch, const float2* __restrict__ part,
                                                          float2* __restrict__ Dc) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nn = (size_t)N * N;
  if (e >= (size_t)nblk * nn) return;
  const size_t X = e / nn, r = e - X * nn;
  float2 s = make_float2(0.f, 0.f);
  for (int c = 0; c < nch; ++c) {
    const float2 v = part[(X * nch + c) * nn + r];
    s.x += v.x;
    s.y += v.y;
  }
  Dc[X * 9 * nn + r] = s;
}

template <class R, class TV, class TL, class TC, class TO>
static void coarse_build_run(const Geo& g, int nv, double kappa, const void* V, const void* U, const void* C,
                             void* Dc, hipStream_t st) {
  const int N = 2 * nv;
  if (N > 256) throw std::runtime_error("coarse build: 2 nv must be <= 256");
  const int ncg = 256 / N;
  const int cpg = (nv + ncg - 1) / ncg;
  const size_t lds = 2 * (size_t)(256 / nv) * nv * 12 * sizeof(cplx<R>);
  dim3 grid(round8(g.nblk * 10));
  auto go = [&](auto tag) {
    constexpr int CPG = decltype(tag)::value;
    auto kern = k_coarse_build<R, TV, TL, TC, TO, CPG>;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    kern<<<grid, 256, lds, st>>>(g, nv, (R)kappa, (const TV*)V, (const TL*)U, (const TC*)C, (TO*)Dc);
  };
  if (cpg <= 1)
    go(std::integral_constant<int, 1>());
  else if (cpg <= 2)
    go(std::integral_constant<int, 2>());
  else if (cpg <= 4)
    go(std::integral_constant<int, 4>());
  else if (cpg <= 8)
    go(std::integral_constant<int, 8>());
  else
    go(std::integral_constant<int, 16>());
}

int coarse_build_chunks(const Geo& g) {
  const int ntile = (g.Vb + 7) / 8;  // 8-site tiles
  return (ntile + 7) / 8;            // 8 tiles per chunk
}

void launch_coarse_build(const Geo& g, int nv, double kappa, const void* V, const void* U, const void* C, void* Dc,
                         int mixed, hipStream_t st, int variant, void* part) {
  if (mixed && variant == 1) {
    if (nv > 32) throw std::runtime_error("coarse build: the matrix-core variant needs nv <= 32");
    if (!part) throw std::runtime_error("coarse build: the matrix-core variant needs its partial-sum workspace");
    constexpr int T = 8;  // 256 threads cover T * nv <= 256 (site, vector) pairs
    const int tpc = 8;    // tiles per in-block chunk (64 sites)
    const int nch = coarse_build_chunks(g);
    const int N = 2 * nv;
    k_coarse_build_mf<T><<<dim3(round8(g.nblk * (nch + 4))), 256, 0, st>>>(
        g, nv, (float)kappa, (const half2_t*)V, (const half2_t*)U, (const half2_t*)C, (float2*)Dc, nch, tpc,
        (float2*)part);
    const size_t ne = (size_t)g.nblk * N * N;
    k_coarse_build_sum<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(g.nblk, N, nch, (const float2*)part,
                                                                     (float2*)Dc);
  } else if (mixed) {
    coarse_build_run<float, half2_t, half2_t, half2_t, float2>(g, nv, kappa, V, U, C, Dc, st);
  } else {
    coarse_build_run<double, double2, double2, double2, double2>(g, nv, kappa, V, U, C, Dc, st);
  }
  launch_coarse_mirror(make_cgeo(g.NB), nv, Dc, mixed, st);
}

// Backward blocks of the coarse operator from the forward ones.  The
// backward hop in direction mu is the gamma_5-conjugated adjoint of the
// forward hop of the neighbour (eq. (2)), and the basis vectors P_s v_i are
// gamma_5 eigenvectors with eigenvalue +-1 (s = 0: +1), so with
// Gamma = diag(1, ..., 1 (s = 0), -1, ..., -1 (s = 1)) eq. (7) gives
//   Dc(X, X - mu) = Gamma Dc(X - mu, X)^dag Gamma.
// In the stored layout (block d of X at [X][d][m][n] = <X, n| D |X + e_d, m>)
//   [X][5 + mu][m][n] = g(n) g(m) conj([Y][1 + mu][n][m]),  Y = X - e_mu,
// g(k) = +1 for k < nv, -1 otherwise.  One 32x32 tile of an output block per
// workgroup, transposed through LDS so that reads and writes are coalesced.
template <class T>
__global__ __launch_bounds__(256) void k_coarse_mirror(CGeo cg, int nv, T* __restrict__ Dc) {
  __shared__ T tile[32][33];
  const int N = 2 * nv;
  const int nt = (N + 31) / 32;
  int q = blockIdx.x;
  const int tn = q % nt;
  q /= nt;
  const int tm = q % nt;
  q /= nt;
  const int mu = q & 3;
  const int X = q >> 2;
  if (X >= cg.NC) return;
  int r = X, c[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    c[m] = r % cg.N[m];
    r /= cg.N[m];
  }
  const int cm = c[mu] == 0 ? cg.N[mu] - 1 : c[mu] - 1;
  const int Y = X + (cm - c[mu]) * cg.sN[mu];
  const T* src = Dc + ((size_t)Y * 9 + 1 + mu) * N * N;
  T* dst = Dc + ((size_t)X * 9 + 5 + mu) * N * N;
  const int m0 = tm * 32, n0 = tn * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // source rows n0 + i, columns m0 + j
  for (int i = ty; i < 32; i += 8) {
    const int n = n0 + i, m = m0 + tx;
    if (n < N && m < N) tile[i][tx] = src[(size_t)n * N + m];
  }
  __syncthreads();
  // destination rows m0 + j, columns n0 + i
  for (int j = ty; j < 32; j += 8) {
    const int m = m0 + j, n = n0 + tx;
    if (n < N && m < N) {
      const T v = tile[tx][j];
      const bool neg = (n < nv) != (m < nv);
      T o;
      o.x = neg ? -v.x : v.x;
      o.y = neg ? v.y : -v.y;
      dst[(size_t)m * N + n] = o;
    }
  }
}

void launch_coarse_mirror(const CGeo& cg, int nv, void* Dc, int prec32, hipStream_t st) {
  const int nt = (2 * nv + 31) / 32;
  const unsigned nb = (unsigned)((size_t)cg.NC * 4 * nt * nt);
  if (prec32)
    k_coarse_mirror<float2><<<nb, 256, 0, st>>>(cg, nv, (float2*)Dc);
  else
    k_coarse_mirror<double2><<<nb, 256, 0, st>>>(cg, nv, (double2*)Dc);
}

// ---------------------------------------------------------------------------
// Level-1 (coarse-lattice) aggregation for multi-level hierarchies.  Vectors
// on the coarse lattice are [rhs][X1][n1] (X1 lexicographic over cg.N); a
// level-1 block X2 collects b1[0] x .. x b1[3] coarse sites; the two halves
// of the n1 = 2 nv dof are the coarse chiralities.  Level-1 test vectors W
// are [nw][X1][n1]; level-2 vectors are [rhs][X2][2 nw].
// ---------------------------------------------------------------------------
struct L1Geo {
  CGeo c1;      // level-1 lattice
  CGeo c2;      // level-2 lattice
  int b1[4];    // block extents
  int vb1;      // sites per block
};

__device__ __forceinline__ int l1_site(const L1Geo& q, int X2, int loc) {
  int c2[4], cl[4];
  int r = X2, l = loc;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    c2[m] = r % q.c2.N[m];
    r /= q.c2.N[m];
    cl[m] = l % q.b1[m];
    l /= q.b1[m];
  }
  int X1 = 0;
#pragma unroll
  for (int m = 3; m >= 0; --m) X1 = X1 * q.c1.N[m] + c2[m] * q.b1[m] + cl[m];
  return X1;
}

__device__ __forceinline__ int l1_block(const L1Geo& q, int X1) {
  int r = X1, X2 = 0, mul = 1;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int c = r % q.c1.N[m];
    r /= q.c1.N[m];
    X2 += (c / q.b1[m]) * mul;
    mul *= q.c2.N[m];
  }
  return X2;
}

// out[r][X2][s*nw + k] = sum_{X1 in X2} sum_{a in half s} conj(W_k(X1)_a) x_r(X1)_a
template <class RA, class TW, class TI, class TO>
__global__ __launch_bounds__(256) void k_l1_restrict(L1Geo q, int n1, int nw, int nrhs, const TW* __restrict__ W,
                                                     const TI* __restrict__ x, size_t x_rs, TO* __restrict__ out,
                                                     size_t out_rs, size_t out_xs) {
  size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t total = (size_t)nrhs * q.c2.NC * 2 * nw;
  if (t >= total) return;
  int k = t % nw;
  size_t u = t / nw;
  int s = u % 2;
  u /= 2;
  int X2 = u % q.c2.NC;
  int r = u / q.c2.NC;
  int h = n1 / 2;
  cplx<RA> acc = {0, 0};
  for (int loc = 0; loc < q.vb1; ++loc) {
    int X1 = l1_site(q, X2, loc);
    const TW* w = W + ((size_t)k * q.c1.NC + X1) * n1 + s * h;
    const TI* xv = x + r * x_rs + (size_t)X1 * n1 + s * h;
    for (int a = 0; a < h; ++a) cjmac(acc, ld<RA>(w, a), ld<RA>(xv, a));
  }
  st(out, r * out_rs + X2 * out_xs + s * nw + k, acc);
}

// out_r(X1)_a = sum_k W_k(X1)_a xc[r][X2(X1)][s(a) nw + k]
template <class R, class TW, class TC, class TO>
__global__ __launch_bounds__(256) void k_l1_prolong(L1Geo q, int n1, int nw, int nrhs, const TW* __restrict__ W,
                                                    const TC* __restrict__ xc, size_t xc_rs, size_t xc_xs,
                                                    TO* __restrict__ out, size_t out_rs) {
  size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t total = (size_t)nrhs * q.c1.NC * n1;
  if (t >= total) return;
  int a = t % n1;
  size_t u = t / n1;
  int X1 = u % q.c1.NC;
  int r = u / q.c1.NC;
  int X2 = l1_block(q, X1);
  int s = a >= n1 / 2;
  cplx<R> acc = {0, 0};
  const TC* c = xc + r * xc_rs + X2 * xc_xs + s * nw;
  for (int k = 0; k < nw; ++k) cmac(acc, ld<R>(W, ((size_t)k * q.c1.NC + X1) * n1 + a), ld<R>(c, k));
  st(out, r * out_rs + (size_t)X1 * n1 + a, acc);
}

void launch_l1_restrict(const CGeo& c1, const int* b1, int n1, int nw, int nrhs, const void* W, int w_t,
                        const void* x, int x_t, size_t x_rs, void* out, int out_t, size_t out_rs, size_t out_xs,
                        hipStream_t st) {
  L1Geo q;
  q.c1 = c1;
  int n2[4];
  for (int m = 0; m < 4; ++m) {
    q.b1[m] = b1[m];
    n2[m] = c1.N[m] / b1[m];
  }
  q.c2 = make_cgeo(n2);
  q.vb1 = b1[0] * b1[1] * b1[2] * b1[3];
  size_t total = (size_t)nrhs * q.c2.NC * 2 * nw;
  unsigned nb = (unsigned)((total + 255) / 256);
  if (w_t == C128 && x_t == C128 && out_t == C128)
    k_l1_restrict<double, double2, double2, double2><<<nb, 256, 0, st>>>(q, n1, nw, nrhs, (const double2*)W,
                                                                         (const double2*)x, x_rs, (double2*)out,
                                                                         out_rs, out_xs);
  else if (w_t == C64 && x_t == C64 && out_t == C64)
    k_l1_restrict<float, float2, float2, float2><<<nb, 256, 0, st>>>(q, n1, nw, nrhs, (const float2*)W,
                                                                     (const float2*)x, x_rs, (float2*)out, out_rs,
                                                                     out_xs);
  else if (w_t == C64 && x_t == C64 && out_t == C128)
    k_l1_restrict<double, float2, float2, double2><<<nb, 256, 0, st>>>(q, n1, nw, nrhs, (const float2*)W,
                                                                       (const float2*)x, x_rs, (double2*)out,
                                                                       out_rs, out_xs);
  else
    throw std::runtime_error("launch_l1_restrict: unsupported type combination");
}

void launch_l1_prolong(const CGeo& c1, const int* b1, int n1, int nw, int nrhs, const void* W, int w_t,
                       const void* xc, int xc_t, size_t xc_rs, size_t xc_xs, void* out, int out_t, size_t out_rs,
                       hipStream_t st) {
  L1Geo q;
  q.c1 = c1;
  int n2[4];
  for (int m = 0; m < 4; ++m) {
    q.b1[m] = b1[m];
    n2[m] = c1.N[m] / b1[m];
  }
  q.c2 = make_cgeo(n2);
  q.vb1 = b1[0] * b1[1] * b1[2] * b1[3];
  size_t total = (size_t)nrhs * c1.NC * n1;
  unsigned nb = (unsigned)((total + 255) / 256);
  if (w_t == C128 && xc_t == C128 && out_t == C128)
    k_l1_prolong<double, double2, double2, double2><<<nb, 256, 0, st>>>(q, n1, nw, nrhs, (const double2*)W,
                                                                        (const double2*)xc, xc_rs, xc_xs,
                                                                        (double2*)out, out_rs);
  else if (w_t == C64 && xc_t == C64 && out_t == C64)
    k_l1_prolong<float, float2, float2, float2><<<nb, 256, 0, st>>>(q, n1, nw, nrhs, (const float2*)W,
                                                                    (const float2*)xc, xc_rs, xc_xs, (float2*)out,
                                                                    out_rs);
  else
    throw std::runtime_error("launch_l1_prolong: unsupported type combination");
}

// Level-2 operator from the level-1 stencil Dc1 ([X1][9][m][n], n1 x n1) and
// the level-1 test vectors W: one workgroup per (X2, d, source half sp).  For
// every site X1 of the block (or of its face in direction d) the vectors
//   g_l(X1) = sum_{d1} Dc1[X1][d1] (P_sp W_l)(X1 + e_d1)
// (d1 over the in-block hops and the self term for d = 0, the single
// crossing hop d for d > 0) are formed in LDS and contracted with conj(W_k).
template <class R, class TC, class TW, class TO>
__global__ __launch_bounds__(256) void k_l1_build(L1Geo q, int n1, int nw, const TC* __restrict__ Dc1,
                                                  const TW* __restrict__ W, TO* __restrict__ Dc2) {
  extern __shared__ __align__(16) char smem[];
  cplx<R>* gl = (cplx<R>*)smem;  // [nw][n1]
  const int X2 = blockIdx.x, d = blockIdx.y, sp = blockIdx.z;
  const int t = threadIdx.x;
  const int h = n1 / 2, N2 = 2 * nw;
  const int mu = (d - 1) & 3;
  const bool fwd = d <= 4;
  // outputs: (row n = (s,k), column l), looped by the workgroup
  const int nout = N2 * nw;
  constexpr int MAXO = 16;
  cplx<R> acc[MAXO];
#pragma unroll
  for (int o = 0; o < MAXO; ++o) acc[o] = {0, 0};
  for (int loc = 0; loc < q.vb1; ++loc) {
    // site of the block; for d > 0 only sites on the face of direction d
    int cl[4], r = loc;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cl[m] = r % q.b1[m];
      r /= q.b1[m];
    }
    if (d > 0) {
      if (q.c2.N[mu] == 1) break;  // a single block in this direction: no crossing hop
      if (cl[mu] != (fwd ? q.b1[mu] - 1 : 0)) continue;
    }
    const int X1 = l1_site(q, X2, loc);
    int c1[4];
    {
      int rr = X1;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        c1[m] = rr % q.c1.N[m];
        rr /= q.c1.N[m];
      }
    }
    // g_l(X1)_a for (l, a) pairs
    for (int e = t; e < nw * n1; e += 256) {
      const int l = e / n1, a = e - l * n1;
      cplx<R> g = {0, 0};
      for (int d1 = 0; d1 < 9; ++d1) {
        int m1 = (d1 - 1) & 3;
        int Y = X1;
        if (d1 > 0) {
          int step = d1 <= 4 ? 1 : -1;
          int cc = c1[m1] + step;
          if (cc == q.c1.N[m1]) cc = 0;
          if (cc < 0) cc = q.c1.N[m1] - 1;
          Y = X1 + (cc - c1[m1]) * q.c1.sN[m1];
          // in-block?  (same level-1 block iff the block coordinate is unchanged)
          bool inb = (cc / q.b1[m1]) == (c1[m1] / q.b1[m1]);
          if (d == 0 && !inb) continue;
          if (d > 0 && (d1 != d || inb)) continue;
        } else if (d > 0) {
          continue;
        }
        const TC* B = Dc1 + ((size_t)(X1 * 9 + d1) * n1) * n1;  // column-major: (row a, col b) at b*n1 + a
        const TW* w = W + ((size_t)l * q.c1.NC + Y) * n1 + sp * h;
        for (int b = 0; b < h; ++b) cmac(g, ld<R>(B, (size_t)(sp * h + b) * n1 + a), ld<R>(w, b));
      }
      gl[l * n1 + a] = g;
    }
    __syncthreads();
    for (int o = 0; o < MAXO; ++o) {
      int idx = t + o * 256;
      if (idx >= nout) break;
      int n = idx % N2, l = idx / N2;
      int s = n / nw, k = n - s * nw;
      const TW* w = W + ((size_t)k * q.c1.NC + X1) * n1 + s * h;
      for (int b = 0; b < h; ++b) cjmac(acc[o], ld<R>(w, b), gl[l * n1 + s * h + b]);
    }
    __syncthreads();
  }
  for (int o = 0; o < MAXO; ++o) {
    int idx = t + o * 256;
    if (idx >= nout) break;
    int n = idx % N2, l = idx / N2;
    st(Dc2, ((size_t)(X2 * 9 + d) * N2 + (sp * nw + l)) * N2 + n, acc[o]);
  }
}

void launch_l1_build(const CGeo& c1, const int* b1, int n1, int nw, const void* Dc1, const void* W, void* Dc2,
                     int prec32, hipStream_t st) {
  L1Geo q;
  q.c1 = c1;
  int n2[4];
  for (int m = 0; m < 4; ++m) {
    q.b1[m] = b1[m];
    n2[m] = c1.N[m] / b1[m];
  }
  q.c2 = make_cgeo(n2);
  q.vb1 = b1[0] * b1[1] * b1[2] * b1[3];
  if (2 * nw * nw > 16 * 256) throw std::runtime_error("l1 build: too many outputs");
  dim3 grid(q.c2.NC, 9, 2);
  if (prec32) {
    size_t lds = (size_t)nw * n1 * sizeof(cplx<float>);
    (void)hipFuncSetAttribute((const void*)k_l1_build<float, float2, float2, float2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    k_l1_build<float, float2, float2, float2><<<grid, 256, lds, st>>>(q, n1, nw, (const float2*)Dc1,
                                                                      (const float2*)W, (float2*)Dc2);
  } else {
    size_t lds = (size_t)nw * n1 * sizeof(cplx<double>);
    (void)hipFuncSetAttribute((const void*)k_l1_build<double, double2, double2, double2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    k_l1_build<double, double2, double2, double2><<<grid, 256, lds, st>>>(q, n1, nw, (const double2*)Dc1,
                                                                          (const double2*)W, (double2*)Dc2);
  }
}

// ---------------------------------------------------------------------------
// Block orthonormalisation coefficients.  One wavefront per (block X,
// chirality s): G = L L^H by a right-looking Cholesky (lane = row), then
// M = L^{-1} by forward substitution (lane = column), coef = M^H = L^{-H}
// (upper triangular, positive real diagonal).
// ---------------------------------------------------------------------------
template <class TCo>
__global__ __launch_bounds__(64) void k_cholesky_coef(int nblk, int nv, const double2* __restrict__ G, size_t g_rs,
                                                      TCo* __restrict__ coef, size_t coef_rs, int* bad) {
  extern __shared__ __align__(16) char smem[];
  cplx<double>* A = (cplx<double>*)smem;  // [nv][nv] (row i, col k)
  cplx<double>* M = A + nv * nv;          // [nv][nv]
  const int X = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int lane = threadIdx.x;
  const size_t xs = 2 * (size_t)nv;
  // A[i][j] = <v_i, v_j> = G[j][X][s*nv+i]
  for (int e = lane; e < nv * nv; e += 64) {
    int i = e % nv, j = e / nv;
    A[i * nv + j] = ld<double>(G, j * g_rs + X * xs + s * nv + i);
  }
  __syncthreads();
  int fail = 0;
  for (int j = 0; j < nv; ++j) {
    double d = A[j * nv + j].x;
    if (!(d > 0.0)) fail = 1;
    double piv = sqrt(fmax(d, 1e-300));
    __syncthreads();
    if (lane == j) A[j * nv + j] = {piv, 0.0};
    if (lane > j && lane < nv) A[lane * nv + j] = (1.0 / piv) * A[lane * nv + j];
    __syncthreads();
    if (lane > j && lane < nv) {
      cplx<double> lij = A[lane * nv + j];
      for (int k = j + 1; k <= lane; ++k) {
        cplx<double> lkj = A[k * nv + j];
        A[lane * nv + k] = A[lane * nv + k] - lij * cj(lkj);
      }
    }
    __syncthreads();
  }
  // M = L^{-1}: column j = lane, rows i >= j
  if (lane < nv) {
    int j = lane;
    for (int i = 0; i < nv; ++i) M[i * nv + j] = {0.0, 0.0};
    M[j * nv + j] = {1.0 / A[j * nv + j].x, 0.0};
    for (int i = j + 1; i < nv; ++i) {
      cplx<double> acc = {0.0, 0.0};
      for (int k = j; k < i; ++k) cmac(acc, A[i * nv + k], M[k * nv + j]);
      M[i * nv + j] = (-1.0 / A[i * nv + i].x) * acc;
    }
  }
  __syncthreads();
  // coef[j][X][s*nv+i] = conj(M[j][i]) for i <= j
  for (int e = lane; e < nv * nv; e += 64) {
    int i = e % nv, j = e / nv;
    cplx<double> val = {0.0, 0.0};
    if (i <= j) val = cj(M[j * nv + i]);
    st(coef, j * coef_rs + X * xs + s * nv + i, val);
  }
  if (fail && lane == 0) atomicOr(bad, 1);
}

void launch_cholesky_coef(int nblk, int nv, const double2* G, size_t g_rs, void* coef, int coef_t, size_t coef_rs,
                          int* bad, hipStream_t st) {
  if (nv > 64) throw std::runtime_error("cholesky: nv > 64");
  size_t lds = 2 * (size_t)nv * nv * sizeof(double2);
  if (coef_t == C128)
    k_cholesky_coef<double2><<<2 * nblk, 64, lds, st>>>(nblk, nv, G, g_rs, (double2*)coef, coef_rs, bad);
  else
    k_cholesky_coef<float2><<<2 * nblk, 64, lds, st>>>(nblk, nv, G, g_rs, (float2*)coef, coef_rs, bad);
}

}  // namespace wc
