// Kernels of the gauge-equivariant network that proposes initial test
// vectors (learned replacement of setup step (0-a)): parallel-transport
// convolution layers psi'_o(x) = sum_i sum_d W[d][o][i] (T_d psi_i)(x) with
// T_0 = 1, T_{+mu} psi(x) = U_mu(x) psi(x+mu), T_{-mu} psi(x) =
// U_mu(x-mu)^dag psi(x-mu), their adjoint (input gradient), the weight
// gradient, the per-block coefficients of the subspace loss, and Adam.
// Channels are fields [C][blk][12][Vb] (FP32, block-major planes like every
// site field), weights [9][C][C][4][4] complex64.
#include <stdexcept>

#include "wc_dirac.h"
#include "wc_kernels.h"

namespace wc {

constexpr int NETC = 16;          // channels
constexpr int NTS = 256 / NETC;   // sites per workgroup tile

__device__ __forceinline__ int opp_dir(int d) { return d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4); }

// (T_d f)(x) for one field f ([blk][12][Vb]) at site s, FP64 links, FP32 result
__device__ __forceinline__ void transport_site(const Geo& g, const double2* __restrict__ U,
                                               const float2* __restrict__ f, int s, const SiteCoord& c, int d,
                                               cplx<float> (&out)[12]) {
  const int ps = g.Vb;
  if (d == 0) {
    ld_spinor<float>(f, ps, fbase_b(g, 12, s, c.blk), out);
    return;
  }
  const int mu = (d - 1) & 3;
  int sign, nblk;
  bool inb;
  cplx<float> psi[12], u[9];
  int nb;
  if (d <= 4) {
    nb = neighbour<true>(g, s, c, mu, sign, inb, nblk);
    ld_spinor<float>(f, ps, fbase_b(g, 12, nb, nblk), psi);
    ld_link<float>(U, ps, mu, fbase_b(g, 36, s, c.blk), u);
  } else {
    nb = neighbour<false>(g, s, c, mu, sign, inb, nblk);
    ld_spinor<float>(f, ps, fbase_b(g, 12, nb, nblk), psi);
    ld_link<float>(U, ps, mu, fbase_b(g, 36, nb, nblk), u);
  }
  const float sg = (float)sign;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      cplx<float> a = {0, 0};
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        if (d <= 4)
          cmac(a, u[r * 3 + cc], psi[sp * 3 + cc]);
        else
          cjmac(a, u[cc * 3 + r], psi[sp * 3 + cc]);
      }
      out[sp * 3 + r] = sg * a;
    }
}

// One layer (adjoint = 0): out_o = sum_d sum_i W[d][o][i] T_d in_i.
// Adjoint (input gradient, adjoint = 1): out_i = sum_d T_d sum_o W[opp d][o][i]^dag in_o,
// i.e. the same form with weights W'[d][i][o] = W[opp d][o][i]^dag.
// Workgroup = 16 sites x 16 channels; per direction each thread transports
// one channel of one site into LDS, then mixes all 16 through the 4x4 spin weights.
__global__ __launch_bounds__(256) void k_ptc(Geo g, const float2* __restrict__ W, const float2* __restrict__ in,
                                             float2* __restrict__ out, const double2* __restrict__ U, int adjoint) {
  __shared__ cplx<float> tp[NTS][NETC][12];
  __shared__ cplx<float> wd[NETC][NETC][16];
  const int t = threadIdx.x;
  const int ts = t / NETC, ch = t % NETC;
  const int V = g.V;
  const int s = blockIdx.x * NTS + ts;
  const bool act = s < V;
  const size_t fs = (size_t)12 * V;
  SiteCoord c = decompose(g, act ? s : 0);
  cplx<float> acc[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) acc[a] = {0, 0};
  for (int d = 0; d < 9; ++d) {
    // stage the 16x16 spin-matrix weights of this direction
    for (int e = t; e < NETC * NETC * 16; e += 256) {
      int st = e & 15, io = e >> 4;
      int b = io % NETC, a = io / NETC;  // wd[a][b]: output channel a, input channel b
      cplx<float> w;
      if (!adjoint) {
        w = ld<float>(W, (((size_t)d * NETC + a) * NETC + b) * 16 + st);
      } else {
        int sr = st >> 2, sc = st & 3;  // W'[d][a][b][sr][sc] = conj(W[opp d][b][a][sc][sr])
        w = cj(ld<float>(W, (((size_t)opp_dir(d) * NETC + b) * NETC + a) * 16 + sc * 4 + sr));
      }
      wd[a][b][st] = w;
    }
    cplx<float> tv[12];
    if (act)
      transport_site(g, U, in + ch * fs, s, c, d, tv);
    else
#pragma unroll
      for (int a = 0; a < 12; ++a) tv[a] = {0, 0};
#pragma unroll
    for (int a = 0; a < 12; ++a) tp[ts][ch][a] = tv[a];
    __syncthreads();
    for (int b = 0; b < NETC; ++b) {
#pragma unroll
      for (int sr = 0; sr < 4; ++sr)
#pragma unroll
        for (int sc = 0; sc < 4; ++sc) {
          cplx<float> w = wd[ch][b][sr * 4 + sc];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) cmac(acc[sr * 3 + cc], w, tp[ts][b][sc * 3 + cc]);
        }
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int a = 0; a < 12; ++a) st(out + ch * fs, (size_t)a * g.Vb + fbase_b(g, 12, s, c.blk), acc[a]);
  }
}

// Weight gradient partials: part[wg][d][o][i][sr*4+sc] =
//   sum_{x in the workgroup's tiles} sum_c gout_o(x)[sr,c] conj((T_d in_i)(x)[sc,c])
__global__ __launch_bounds__(256) void k_ptc_wgrad(Geo g, const float2* __restrict__ gout,
                                                   const float2* __restrict__ in, const double2* __restrict__ U,
                                                   float2* __restrict__ part) {
  __shared__ cplx<float> tp[NTS][NETC][12];
  __shared__ cplx<float> gp[NTS][NETC][12];
  const int t = threadIdx.x;
  const int d = blockIdx.y;
  const int ts = t / NETC, ch = t % NETC;
  const int o = t / NETC, i = t % NETC;  // output of this thread
  const int V = g.V;
  const size_t fs = (size_t)12 * V;
  cplx<float> acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = {0, 0};
  for (int t0 = blockIdx.x * NTS; t0 < V; t0 += gridDim.x * NTS) {
    const int s = t0 + ts;
    cplx<float> tv[12], gv[12];
    if (s < V) {
      SiteCoord c = decompose(g, s);
      transport_site(g, U, in + ch * fs, s, c, d, tv);
      ld_spinor<float>(gout + ch * fs, g.Vb, fbase_b(g, 12, s, c.blk), gv);
    } else {
#pragma unroll
      for (int a = 0; a < 12; ++a) tv[a] = gv[a] = {0, 0};
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      tp[ts][ch][a] = tv[a];
      gp[ts][ch][a] = gv[a];
    }
    __syncthreads();
    for (int q = 0; q < NTS; ++q) {
#pragma unroll
      for (int sr = 0; sr < 4; ++sr)
#pragma unroll
        for (int sc = 0; sc < 4; ++sc)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) cjmac(acc[sr * 4 + sc], tp[q][i][sc * 3 + cc], gp[q][o][sr * 3 + cc]);
    }
    __syncthreads();
  }
  float2* p = part + (((size_t)blockIdx.x * 9 + d) * NETC * NETC + o * NETC + i) * 16;
#pragma unroll
  for (int q = 0; q < 16; ++q) p[q] = make_float2(acc[q].x, acc[q].y);
}

// grad[e] = sum_wg part[wg][e] (fixed order), e over 9*C*C*16 entries
__global__ __launch_bounds__(256) void k_sum_parts(const float2* __restrict__ part, int nwg, size_t n,
                                                   float2* __restrict__ out) {
  size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double re = 0, im = 0;
  for (int w = 0; w < nwg; ++w) {
    float2 v = part[(size_t)w * n + e];
    re += v.x;
    im += v.y;
  }
  out[e] = make_float2((float)re, (float)im);
}

// Per (block X, chirality s), from G[j][X][s C + i] = <A_i, A_j> and
// B[j][X][s C + i] = <A_i, Q_j> (FP64): with Gi = G^{-1},
//   f = tr(Gi B B^dag), loss part 1 - f / C,
//   coefQ[j][X][s C + i] = -scale (B^dag Gi)[i][j],
//   coefA[j][X][s C + i] = +scale (Gi B B^dag Gi)[i][j],
// so that dL/d conj(A)_j = sum_i Q_i coefQ[j][i] + A_i coefA[j][i].
__global__ __launch_bounds__(64) void k_net_loss_coef(int nblk, const double2* __restrict__ G,
                                                      const double2* __restrict__ B, size_t rs, double scale,
                                                      float2* __restrict__ coefQ, float2* __restrict__ coefA,
                                                      double* __restrict__ lpart) {
  constexpr int C = NETC;
  __shared__ cplx<double> A[C][C], M[C][C], Gi[C][C], Bm[C][C], T1[C][C], T2[C][C];
  const int X = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int lane = threadIdx.x;
  const size_t xs = 2 * C;
  for (int e = lane; e < C * C; e += 64) {
    int i = e % C, j = e / C;
    A[i][j] = ld<double>(G, j * rs + X * xs + s * C + i);
    Bm[i][j] = ld<double>(B, j * rs + X * xs + s * C + i);
  }
  __syncthreads();
  // Cholesky G = L L^H (lane = row), in place in the lower triangle of A
  for (int j = 0; j < C; ++j) {
    double dj = A[j][j].x;
    double piv = sqrt(fmax(dj, 1e-300));
    __syncthreads();
    if (lane == j) A[j][j] = {piv, 0.0};
    if (lane > j && lane < C) A[lane][j] = (1.0 / piv) * A[lane][j];
    __syncthreads();
    if (lane > j && lane < C) {
      cplx<double> lij = A[lane][j];
      for (int k = j + 1; k <= lane; ++k) A[lane][k] = A[lane][k] - lij * cj(A[k][j]);
    }
    __syncthreads();
  }
  // M = L^{-1} (lane = column)
  if (lane < C) {
    int j = lane;
    for (int i = 0; i < C; ++i) M[i][j] = {0.0, 0.0};
    M[j][j] = {1.0 / A[j][j].x, 0.0};
    for (int i = j + 1; i < C; ++i) {
      cplx<double> acc = {0.0, 0.0};
      for (int k = j; k < i; ++k) cmac(acc, A[i][k], M[k][j]);
      M[i][j] = (-1.0 / A[i][i].x) * acc;
    }
  }
  __syncthreads();
  // Gi = M^H M
  for (int e = lane; e < C * C; e += 64) {
    int i = e / C, j = e % C;
    cplx<double> acc = {0, 0};
    for (int k = 0; k < C; ++k) cjmac(acc, M[k][i], M[k][j]);
    Gi[i][j] = acc;
  }
  __syncthreads();
  // T1 = B^dag Gi ; T2 = Gi B
  for (int e = lane; e < C * C; e += 64) {
    int i = e / C, j = e % C;
    cplx<double> a1 = {0, 0}, a2 = {0, 0};
    for (int k = 0; k < C; ++k) {
      cjmac(a1, Bm[k][i], Gi[k][j]);
      cmac(a2, Gi[i][k], Bm[k][j]);
    }
    T1[i][j] = a1;
    T2[i][j] = a2;
  }
  __syncthreads();
  // f = tr(Gi B B^dag) = sum_{i,k} T2[i][k] conj(B[i][k]); M2 = T2 B^dag Gi = T2 T1^... : (Gi B)(B^dag Gi)
  double fpart = 0;
  for (int e = lane; e < C * C; e += 64) {
    int i = e / C, k = e % C;
    fpart += T2[i][k].x * Bm[i][k].x + T2[i][k].y * Bm[i][k].y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fpart += __shfl_xor(fpart, o, 64);
  for (int e = lane; e < C * C; e += 64) {
    int i = e % C, j = e / C;  // coefficient for output j, input i
    cplx<double> m2 = {0, 0};
    for (int k = 0; k < C; ++k) cmac(m2, T2[i][k], T1[k][j]);
    st(coefQ, j * rs + X * xs + s * C + i, (-scale) * T1[i][j]);
    st(coefA, j * rs + X * xs + s * C + i, scale * m2);
  }
  if (lane == 0) lpart[blockIdx.x] = 1.0 - fpart / C;
}

// Adam on the real and imaginary parts: g = 2 dL/d conj(w)
__global__ __launch_bounds__(256) void k_adam(float2* __restrict__ w, const float2* __restrict__ grad,
                                              float2* __restrict__ m, float2* __restrict__ v, size_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float2 g = grad[e];
  float gr = 2.f * g.x, gi = 2.f * g.y;
  float2 mm = m[e], vv = v[e];
  mm.x = b1 * mm.x + (1.f - b1) * gr;
  mm.y = b1 * mm.y + (1.f - b1) * gi;
  vv.x = b2 * vv.x + (1.f - b2) * gr * gr;
  vv.y = b2 * vv.y + (1.f - b2) * gi * gi;
  m[e] = mm;
  v[e] = vv;
  float2 ww = w[e];
  ww.x -= lr * (mm.x / c1) / (sqrtf(vv.x / c2) + eps);
  ww.y -= lr * (mm.y / c1) / (sqrtf(vv.y / c2) + eps);
  w[e] = ww;
}

// ---------------------------------------------------------------- launchers
int net_channels() { return NETC; }

void launch_ptc(const Geo& g, const float2* W, const float2* in, float2* out, const double2* U, int adjoint,
                hipStream_t st) {
  k_ptc<<<(g.V + NTS - 1) / NTS, 256, 0, st>>>(g, W, in, out, U, adjoint);
}

int ptc_wgrad_nwg(const Geo& g) {
  int tiles = (g.V + NTS - 1) / NTS;
  return tiles < 512 ? tiles : 512;
}

void launch_ptc_wgrad(const Geo& g, const float2* gout, const float2* in, const double2* U, float2* part,
                      float2* grad, hipStream_t st) {
  int nwg = ptc_wgrad_nwg(g);
  k_ptc_wgrad<<<dim3(nwg, 9), 256, 0, st>>>(g, gout, in, U, part);
  size_t n = (size_t)9 * NETC * NETC * 16;
  k_sum_parts<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(part, nwg * 1, n, grad);
}

void launch_net_loss_coef(int nblk, const double2* G, const double2* B, size_t rs, double scale, float2* coefQ,
                          float2* coefA, double* lpart, hipStream_t st) {
  k_net_loss_coef<<<2 * nblk, 64, 0, st>>>(nblk, G, B, rs, scale, coefQ, coefA, lpart);
}

void launch_adam(float2* w, const float2* grad, float2* m, float2* v, size_t n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t st) {
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(w, grad, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace wc
