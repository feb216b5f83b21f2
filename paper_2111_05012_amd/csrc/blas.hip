// Vector kernels: precision conversion, deterministic per-rhs reductions,
// the steps of the coarse BiCGStab with device-resident scalars (so that a
// whole coarse solve can be captured in a graph), and the FP64
// Gram-Schmidt / update kernels of the outer FGMRES.
//
// Reductions are two-stage and fixed-order (per-workgroup partial sums,
// then one workgroup per right-hand side adds them in index order): results
// do not depend on scheduling.
#include <algorithm>
#include <stdexcept>
#include <utility>

#include "wc_kernels.h"

namespace wc {

constexpr int RED_THREADS = 256;

template <class R>
__device__ __forceinline__ R wsum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of K doubles per thread; result valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
  __shared__ double red[RED_THREADS / 64][K];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wsum(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0;
      for (int q = 0; q < RED_THREADS / 64; ++q) s += red[q][k];
      v[k] = s;
    }
  }
  __syncthreads();
}

int reduce_nwg(size_t n) {
  size_t w = (n + 4 * RED_THREADS - 1) / (4 * RED_THREADS);
  if (w > 512) w = 512;
  if (w < 1) w = 1;
  return (int)w;
}

// ---------------------------------------------------------------- elementwise
template <class TI, class TO>
__global__ __launch_bounds__(256) void k_convert(const TI* __restrict__ in, TO* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t stride = (size_t)gridDim.x * 256;
  for (; i < n; i += stride) st(out, i, ld<double>(in, i));
}

template <class TI>
static void convert_to(const TI* in, void* out, int out_t, size_t n, hipStream_t st) {
  int nb = (int)std::min<size_t>((n + 255) / 256, 65536);
  if (out_t == C128) k_convert<TI, double2><<<nb, 256, 0, st>>>(in, (double2*)out, n);
  else if (out_t == C64) k_convert<TI, float2><<<nb, 256, 0, st>>>(in, (float2*)out, n);
  else k_convert<TI, half2_t><<<nb, 256, 0, st>>>(in, (half2_t*)out, n);
}

void launch_convert(const void* in, int in_t, void* out, int out_t, size_t n, hipStream_t st) {
  if (n == 0) return;
  if (in_t == C128) convert_to((const double2*)in, out, out_t, n, st);
  else if (in_t == C64) convert_to((const float2*)in, out, out_t, n, st);
  else convert_to((const half2_t*)in, out, out_t, n, st);
}

__global__ __launch_bounds__(256) void k_zero(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t stride = (size_t)gridDim.x * 256;
  for (size_t k = i; k < n16; k += stride) p[k] = make_uint4(0, 0, 0, 0);
  if (i < ntail) tail[i] = 0;
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  size_t n16 = bytes / 16;
  size_t ntail = bytes - n16 * 16;
  int nb = (int)std::min<size_t>((n16 + 255) / 256 + 1, 65536);
  k_zero<<<nb, 256, 0, st>>>((uint4*)p, n16, (unsigned char*)p + n16 * 16, ntail);
}

// ---------------------------------------------------------------- inner products
// part[(r * nwg + wg) * nd + k] = partial of <a_k[r], b_k[r]>
template <class T, int ND>
__global__ __launch_bounds__(RED_THREADS) void k_dots_partial(const T* a0, const T* b0, const T* a1, const T* b1,
                                                              const T* a2, const T* b2, size_t n, size_t rs,
                                                              double2* part, const int* active, int astride) {
  const int r = blockIdx.y;
  const size_t off = r * rs;
  if (active && !active[(size_t)r * astride]) {
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < ND; ++k) part[((size_t)r * gridDim.x + blockIdx.x) * ND + k] = make_double2(0.0, 0.0);
    return;
  }
  const T* A[3] = {a0, a1, a2};
  const T* B[3] = {b0, b1, b2};
  double v[2 * ND];
#pragma unroll
  for (int k = 0; k < 2 * ND; ++k) v[k] = 0;
  for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * RED_THREADS) {
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      cplx<double> x = ld<double>(A[k] + off, i), y = ld<double>(B[k] + off, i);
      v[2 * k] += x.x * y.x + x.y * y.y;
      v[2 * k + 1] += x.x * y.y - x.y * y.x;
    }
  }
  block_sum<2 * ND>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < ND; ++k)
      part[((size_t)r * gridDim.x + blockIdx.x) * ND + k] = make_double2(v[2 * k], v[2 * k + 1]);
}

template <class T>
static void dots_partial_t(int nd, const void* const* a, const void* const* b, size_t n, size_t rs, int nrhs,
                           double2* part, hipStream_t st, const int* active, int astride) {
  dim3 grid(reduce_nwg(n), nrhs);
  const T* A[3] = {(const T*)a[0], nd > 1 ? (const T*)a[1] : nullptr, nd > 2 ? (const T*)a[2] : nullptr};
  const T* B[3] = {(const T*)b[0], nd > 1 ? (const T*)b[1] : nullptr, nd > 2 ? (const T*)b[2] : nullptr};
  if (nd == 1)
    k_dots_partial<T, 1><<<grid, RED_THREADS, 0, st>>>(A[0], B[0], A[1], B[1], A[2], B[2], n, rs, part, active,
                                                       astride);
  else if (nd == 2)
    k_dots_partial<T, 2><<<grid, RED_THREADS, 0, st>>>(A[0], B[0], A[1], B[1], A[2], B[2], n, rs, part, active,
                                                       astride);
  else
    k_dots_partial<T, 3><<<grid, RED_THREADS, 0, st>>>(A[0], B[0], A[1], B[1], A[2], B[2], n, rs, part, active,
                                                       astride);
}

void launch_dots_partial(int nd, const void* const* a, const void* const* b, int t, size_t n, size_t rs, int nrhs,
                         double2* part, hipStream_t st, const int* active, int astride) {
  if (t == C128) dots_partial_t<double2>(nd, a, b, n, rs, nrhs, part, st, active, astride);
  else if (t == C64) dots_partial_t<float2>(nd, a, b, n, rs, nrhs, part, st, active, astride);
  else throw std::runtime_error("dots: unsupported type");
}

// sum of partials for rhs r (thread 0 of a one-wavefront launch per rhs)
__device__ __forceinline__ cplx<double> sum_parts(const double2* part, int nwg, int nd, int r, int k) {
  cplx<double> s = {0, 0};
  for (int w = 0; w < nwg; ++w) {
    double2 p = part[((size_t)r * nwg + w) * nd + k];
    s.x += p.x;
    s.y += p.y;
  }
  return s;
}

__global__ void k_norm2_fin(const double2* part, int nwg, double* norm2) {
  int r = blockIdx.x;
  if (threadIdx.x == 0) norm2[r] = sum_parts(part, nwg, 1, r, 0).x;
}

void launch_norm2(const void* v, int t, size_t n, size_t rs, int nrhs, double2* part, double* norm2,
                  hipStream_t st) {
  const void* a[1] = {v};
  launch_dots_partial(1, a, a, t, n, rs, nrhs, part, st);
  k_norm2_fin<<<nrhs, 64, 0, st>>>(part, reduce_nwg(n), norm2);
}

// ---------------------------------------------------------------- BiCGStab (coarse solve)
__device__ __forceinline__ cplx<double> C(double2 a) { return {a.x, a.y}; }
__device__ __forceinline__ double2 D2(cplx<double> a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ cplx<double> cdiv(cplx<double> a, cplx<double> b) {
  double den = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den};
}

template <class T>
__global__ __launch_bounds__(RED_THREADS) void k_bicg_init(const T* b, T* x, T* r, T* rt, T* p, T* v, size_t n,
                                                           size_t rs, double2* part) {
  const int rr = blockIdx.y;
  const size_t off = rr * rs;
  double v2[1] = {0};
  for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * RED_THREADS) {
    cplx<double> bb = ld<double>(b + off, i);
    st(x + off, i, cplx<double>{0, 0});
    st(r + off, i, bb);
    st(rt + off, i, bb);
    st(p + off, i, cplx<double>{0, 0});
    st(v + off, i, cplx<double>{0, 0});
    v2[0] += bb.x * bb.x + bb.y * bb.y;
  }
  block_sum<1>(v2);
  if (threadIdx.x == 0) part[(size_t)rr * gridDim.x + blockIdx.x] = make_double2(v2[0], 0.0);
}

__global__ void k_bicg_init_fin(const double2* part, int nwg, BicgScal* sc, double tol) {
  int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  BicgScal s;
  double b2 = sum_parts(part, nwg, 1, r, 0).x;
  s.bnorm2 = b2;
  s.rnorm2 = b2;
  s.rho = make_double2(b2, 0.0);  // <rt, r> with rt = r = b
  s.rho_old = make_double2(1.0, 0.0);
  s.alpha = make_double2(1.0, 0.0);
  s.omega = make_double2(1.0, 0.0);
  s.beta = make_double2(0.0, 0.0);
  s.tol2 = tol * tol;
  s.active = b2 > 0.0 ? 1 : 0;
  s.iters = 0;
  s.final_step = 0;
  s.pad = 0;
  sc[r] = s;
}

void launch_bicg_init(const void* b, void* x, void* r, void* rt, void* p, void* v, int t, size_t n, size_t rs,
                      int nrhs, double tol, double2* part, BicgScal* sc, hipStream_t st) {
  dim3 grid(reduce_nwg(n), nrhs);
  if (t == C128)
    k_bicg_init<double2><<<grid, RED_THREADS, 0, st>>>((const double2*)b, (double2*)x, (double2*)r, (double2*)rt,
                                                       (double2*)p, (double2*)v, n, rs, part);
  else
    k_bicg_init<float2><<<grid, RED_THREADS, 0, st>>>((const float2*)b, (float2*)x, (float2*)r, (float2*)rt,
                                                      (float2*)p, (float2*)v, n, rs, part);
  k_bicg_init_fin<<<nrhs, 64, 0, st>>>(part, reduce_nwg(n), sc, tol);
}

static inline dim3 ew_grid(size_t n, int nrhs) {
  return dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096), nrhs);
}

// p = r + beta (p - omega v)
template <class T, class R>
__global__ __launch_bounds__(256) void k_bicg_p(T* p, const T* r, const T* v, size_t n, size_t rs,
                                                const BicgScal* sc) {
  const int rr = blockIdx.y;
  if (!sc[rr].active) return;
  const size_t off = rr * rs;
  cplx<R> beta = {(R)sc[rr].beta.x, (R)sc[rr].beta.y}, om = {(R)sc[rr].omega.x, (R)sc[rr].omega.y};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    cplx<R> pp = ld<R>(p + off, i), vv = ld<R>(v + off, i), r_ = ld<R>(r + off, i);
    st(p + off, i, r_ + beta * (pp - om * vv));
  }
}

void launch_bicg_p(void* p, const void* r, const void* v, int t, size_t n, size_t rs, int nrhs, const BicgScal* sc,
                   hipStream_t st) {
  if (t == C128)
    k_bicg_p<double2, double><<<ew_grid(n, nrhs), 256, 0, st>>>((double2*)p, (const double2*)r, (const double2*)v,
                                                                n, rs, sc);
  else
    k_bicg_p<float2, float><<<ew_grid(n, nrhs), 256, 0, st>>>((float2*)p, (const float2*)r, (const float2*)v, n, rs,
                                                              sc);
}

__global__ void k_bicg_alpha_fin(const double2* part, int nwg, BicgScal* sc) {
  int r = blockIdx.x;
  if (threadIdx.x != 0 || !sc[r].active) return;
  cplx<double> rv = sum_parts(part, nwg, 1, r, 0);
  if (rv.x == 0.0 && rv.y == 0.0)
    sc[r].active = 0;
  else
    sc[r].alpha = D2(cdiv(C(sc[r].rho), rv));
}

void launch_bicg_alpha(const void* rt, const void* v, int t, size_t n, size_t rs, int nrhs, double2* part,
                       BicgScal* sc, hipStream_t st) {
  const void* a[1] = {rt};
  const void* b[1] = {v};
  launch_dots_partial(1, a, b, t, n, rs, nrhs, part, st, &sc->active, sizeof(BicgScal) / sizeof(int));
  k_bicg_alpha_fin<<<nrhs, 64, 0, st>>>(part, reduce_nwg(n), sc);
}

// s = r - alpha v
template <class T, class R>
__global__ __launch_bounds__(256) void k_bicg_s(T* s, const T* r, const T* v, size_t n, size_t rs,
                                                const BicgScal* sc) {
  const int rr = blockIdx.y;
  if (!sc[rr].active) return;
  const size_t off = rr * rs;
  cplx<R> al = {(R)sc[rr].alpha.x, (R)sc[rr].alpha.y};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    st(s + off, i, ld<R>(r + off, i) - al * ld<R>(v + off, i));
}

void launch_bicg_s(void* s, const void* r, const void* v, int t, size_t n, size_t rs, int nrhs, const BicgScal* sc,
                   hipStream_t st) {
  if (t == C128)
    k_bicg_s<double2, double><<<ew_grid(n, nrhs), 256, 0, st>>>((double2*)s, (const double2*)r, (const double2*)v,
                                                                n, rs, sc);
  else
    k_bicg_s<float2, float><<<ew_grid(n, nrhs), 256, 0, st>>>((float2*)s, (const float2*)r, (const float2*)v, n, rs,
                                                              sc);
}

// omega = <t,s>/<t,t>, enlarged to omega*stab/|cos| when |cos(t,s)| < stab.
// t = 0 or <t,s> = 0 (with s != 0) is a breakdown: omega = 0 (the enlarged
// omega would be 0 * stab / 0) and this is the right-hand side's last step,
// which keeps x + alpha p.
__global__ void k_bicg_omega_fin(const double2* part, int nwg, BicgScal* sc, double stab) {
  int r = blockIdx.x;
  if (threadIdx.x != 0 || !sc[r].active) return;
  cplx<double> ts = sum_parts(part, nwg, 3, r, 0);
  double tt = sum_parts(part, nwg, 3, r, 1).x;
  double ss = sum_parts(part, nwg, 3, r, 2).x;
  if (tt == 0.0 || (ts.x == 0.0 && ts.y == 0.0)) {
    sc[r].omega = make_double2(0.0, 0.0);
    sc[r].final_step = 1;
    return;
  }
  cplx<double> om = {ts.x / tt, ts.y / tt};
  double cosang = ss > 0.0 ? sqrt(ts.x * ts.x + ts.y * ts.y) / sqrt(tt * ss) : 1.0;
  if (cosang < stab) om = (stab / cosang) * om;
  sc[r].omega = D2(om);
}

void launch_bicg_omega(const void* tt, const void* s, int t, size_t n, size_t rs, int nrhs, double2* part,
                       BicgScal* sc, double stab, hipStream_t st) {
  const void* a[3] = {tt, tt, s};
  const void* b[3] = {s, tt, s};
  launch_dots_partial(3, a, b, t, n, rs, nrhs, part, st, &sc->active, sizeof(BicgScal) / sizeof(int));
  k_bicg_omega_fin<<<nrhs, 64, 0, st>>>(part, reduce_nwg(n), sc, stab);
}

// x += alpha p + omega s;  r = s - omega t;  partial <rt, r>, <r, r>
template <class T, class R>
__global__ __launch_bounds__(RED_THREADS) void k_bicg_xr(T* x, T* r, const T* p, const T* s, const T* t,
                                                         const T* rt, size_t n, size_t rs, const BicgScal* sc,
                                                         double2* part) {
  const int rr = blockIdx.y;
  const bool act = sc[rr].active;
  const size_t off = rr * rs;
  cplx<R> al = {(R)sc[rr].alpha.x, (R)sc[rr].alpha.y}, om = {(R)sc[rr].omega.x, (R)sc[rr].omega.y};
  double v[3] = {0, 0, 0};
  if (act) {
    for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * RED_THREADS) {
      cplx<R> ss = ld<R>(s + off, i);
      if (x) st(x + off, i, ld<R>(x + off, i) + al * ld<R>(p + off, i) + om * ss);
      cplx<R> rn = ss - om * ld<R>(t + off, i);
      st(r + off, i, rn);
      cplx<double> rd = ld<double>(r + off, i);  // stored value
      cplx<double> q = ld<double>(rt + off, i);
      v[0] += q.x * rd.x + q.y * rd.y;
      v[1] += q.x * rd.y - q.y * rd.x;
      v[2] += rd.x * rd.x + rd.y * rd.y;
    }
  }
  block_sum<3>(v);
  if (threadIdx.x == 0) {
    part[((size_t)rr * gridDim.x + blockIdx.x) * 2 + 0] = make_double2(v[0], v[1]);
    part[((size_t)rr * gridDim.x + blockIdx.x) * 2 + 1] = make_double2(v[2], 0.0);
  }
}

__global__ void k_bicg_rho_fin(const double2* part, int nwg, BicgScal* sc) {
  int r = blockIdx.x;
  if (threadIdx.x != 0 || !sc[r].active) return;
  BicgScal s = sc[r];
  cplx<double> rho = sum_parts(part, nwg, 2, r, 0);
  double r2 = sum_parts(part, nwg, 2, r, 1).x;
  s.rho_old = s.rho;
  s.rho = D2(rho);
  s.rnorm2 = r2;
  s.iters += 1;
  if (s.final_step || r2 <= s.tol2 * s.bnorm2 || (rho.x == 0.0 && rho.y == 0.0) ||
      (s.omega.x == 0.0 && s.omega.y == 0.0)) {
    s.active = 0;
  } else {
    s.beta = D2(cdiv(rho, C(s.rho_old)) * cdiv(C(s.alpha), C(s.omega)));
  }
  sc[r] = s;
}

void launch_bicg_xr(void* x, void* r, const void* p, const void* s, const void* tt, const void* rt, int t, size_t n,
                    size_t rs, int nrhs, double2* part, BicgScal* sc, hipStream_t st) {
  dim3 grid(reduce_nwg(n), nrhs);
  if (t == C128)
    k_bicg_xr<double2, double><<<grid, RED_THREADS, 0, st>>>((double2*)x, (double2*)r, (const double2*)p,
                                                             (const double2*)s, (const double2*)tt,
                                                             (const double2*)rt, n, rs, sc, part);
  else
    k_bicg_xr<float2, float><<<grid, RED_THREADS, 0, st>>>((float2*)x, (float2*)r, (const float2*)p,
                                                           (const float2*)s, (const float2*)tt, (const float2*)rt, n,
                                                           rs, sc, part);
  k_bicg_rho_fin<<<nrhs, 64, 0, st>>>(part, reduce_nwg(n), sc);
}

// x += alpha M p + omega M s (the flexible BiCGStab's update of the iterate:
// the preconditioned vectors, FP32 or FP64, into the FP64 iterate)
template <class TZ>
__global__ __launch_bounds__(256) void k_fbicg_x(double2* x, const TZ* mp, const TZ* ms, size_t n, size_t rs,
                                                 const BicgScal* sc) {
  const int rr = blockIdx.y;
  if (!sc[rr].active) return;
  const size_t off = rr * rs;
  const cplx<double> al = {sc[rr].alpha.x, sc[rr].alpha.y}, om = {sc[rr].omega.x, sc[rr].omega.y};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    st(x + off, i, ld<double>(x + off, i) + al * ld<double>(mp + off, i) + om * ld<double>(ms + off, i));
}

void launch_fbicg_x(double2* x, const void* mp, const void* ms, int zt, size_t n, size_t rs, int nrhs,
                    const BicgScal* sc, hipStream_t st) {
  if (zt == C128)
    k_fbicg_x<double2><<<ew_grid(n, nrhs), 256, 0, st>>>(x, (const double2*)mp, (const double2*)ms, n, rs, sc);
  else if (zt == C64)
    k_fbicg_x<float2><<<ew_grid(n, nrhs), 256, 0, st>>>(x, (const float2*)mp, (const float2*)ms, n, rs, sc);
  else
    throw std::runtime_error("launch_fbicg_x: preconditioned vectors must be FP64 or FP32");
}

// ---------------------------------------------------------------- FGMRES (FP64 basis)
// One Gram-Schmidt sweep over a chunk of NQ basis vectors Q_k (compile-time
// count, so that all loads of an element are issued before the first use),
// the new Arnoldi vector w and, in the two-vector modes, the pending vector p.
// Each thread owns one complex number of one right-hand side per step of the
// grid-stride loop; the partial sums of a workgroup go to part[r][block][NOUT].
// Streaming accesses: every element of the sweeps is touched once per launch.
__device__ __forceinline__ cplx<double> ld_nt(const double2* p) {
  return {__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}
__device__ __forceinline__ void st_nt(double2* p, cplx<double> v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

template <int NQ, int MODE>
__global__ __launch_bounds__(RED_THREADS) void k_gs(GsArgs a) {
  constexpr bool TWO = MODE == GS_DOT2 || MODE == GS_COMB2;
  constexpr bool AXPY = MODE == GS_AXPY_DOT || MODE == GS_AXPY_NORM || MODE == GS_COMB2;
  constexpr int NOUT = MODE == GS_DOT || MODE == GS_AXPY_DOT ? NQ : MODE == GS_DOT2 ? 2 * NQ + 3 : 1;
  constexpr int NO = NOUT > 0 ? NOUT : 1;
  constexpr int NC = NQ + (TWO ? 1 : 0);  // coefficients per right-hand side
  const int r = blockIdx.y;
  const size_t off = r * a.rs;
  // negated update coefficients of w (-c for the AXPY modes, -c2 for COMB2)
  // and the coefficients of the new p (COMB2)
  cplx<double> cw[NC > 0 ? NC : 1], cp[NC > 0 ? NC : 1];
  if constexpr (AXPY) {
    const double2* src = MODE == GS_COMB2 ? a.c2 : a.c1;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      double2 v = src[(size_t)k * a.nrhs + r];
      cw[k] = {-v.x, -v.y};
    }
  }
  if constexpr (MODE == GS_COMB2) {
#pragma unroll
    for (int k = 0; k < NC; ++k) cp[k] = C(a.c1[(size_t)k * a.nrhs + r]);
  }
  double acc[2 * NO];
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) acc[k] = 0;
  auto cjacc = [&](int k, cplx<double> u, cplx<double> v) {  // acc_k += conj(u) v
    acc[2 * k] = fma(u.x, v.x, fma(u.y, v.y, acc[2 * k]));
    acc[2 * k + 1] = fma(u.x, v.y, fma(-u.y, v.x, acc[2 * k + 1]));
  };
  const double2* Q = a.Q + off;
  double2* P = a.p + off;
  double2* W = a.w + off;
  // COMB2: the new w, times vscale, also as the FP32 input of the next V-cycle
  float2* VI = a.vin ? a.vin + off : nullptr;
  const double vsc = a.vin ? a.vscale[r] : 0.0;
  for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < a.n; i += (size_t)gridDim.x * RED_THREADS) {
    cplx<double> q[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[k] = ld_nt(Q + (size_t)k * a.vs + i);
    cplx<double> pv = {0, 0};
    if constexpr (TWO) pv = ld_nt(P + i);
    cplx<double> wv = ld_nt(W + i);
    if constexpr (MODE == GS_DOT) {
#pragma unroll
      for (int k = 0; k < NQ; ++k) cjacc(k, q[k], wv);
    } else if constexpr (MODE == GS_DOT2) {
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        cjacc(k, q[k], wv);
        cjacc(NQ + k, q[k], pv);
      }
      cjacc(2 * NQ, pv, wv);
      cjacc(2 * NQ + 1, pv, pv);
      acc[2 * (2 * NQ + 2)] = fma(wv.x, wv.x, fma(wv.y, wv.y, acc[2 * (2 * NQ + 2)]));
    } else {
      if constexpr (MODE == GS_COMB2) {
        cplx<double> pn = cp[NQ] * pv;
        cmac(wv, cw[NQ], pv);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          cmac(pn, cp[k], q[k]);
          cmac(wv, cw[k], q[k]);
        }
        if (a.write_p) st_nt(P + i, pn);
      } else {
#pragma unroll
        for (int k = 0; k < NQ; ++k) cmac(wv, cw[k], q[k]);
      }
      st_nt(W + i, wv);
      if constexpr (MODE == GS_COMB2) {
        if (VI) st(VI, i, vsc * wv);
      }
      if constexpr (MODE == GS_AXPY_DOT) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) cjacc(k, q[k], wv);
      } else {
        acc[0] = fma(wv.x, wv.x, fma(wv.y, wv.y, acc[0]));
      }
    }
  }
  block_sum<2 * NO>(acc);
  if (threadIdx.x == 0) {
    double2* out = a.part + ((size_t)r * gridDim.x + blockIdx.x) * NOUT;
#pragma unroll
    for (int k = 0; k < NOUT; ++k) out[k] = make_double2(acc[2 * k], acc[2 * k + 1]);
  }
}

// Sum of the partial sums of k_gs in a fixed order: thread t adds output
// t % 64 over the workgroups t / 64, t / 64 + 4, ... and the four groups are
// added in order; one workgroup per right-hand side.
__global__ __launch_bounds__(256) void k_gs_fin(GsArgs a, int mode, int nwg, int nout) {
  __shared__ double2 red[4][64];
  const int r = blockIdx.x, k = threadIdx.x & 63, g = threadIdx.x >> 6;
  double2 s = make_double2(0.0, 0.0);
  if (k < nout)
    for (int w = g; w < nwg; w += 4) {
      double2 v = a.part[((size_t)r * nwg + w) * nout + k];
      s.x += v.x;
      s.y += v.y;
    }
  red[g][k] = s;
  __syncthreads();
  if (g != 0 || k >= nout) return;
  for (int q = 1; q < 4; ++q) {
    s.x += red[q][k].x;
    s.y += red[q][k].y;
  }
  const size_t nr = a.nrhs;
  if (mode == GS_AXPY_NORM || mode == GS_COMB2) {
    if (a.norm2) a.norm2[r] = s.x;
  } else if (k < a.nq) {
    a.h1[k * nr + r] = s;
  } else if (k < 2 * a.nq) {
    a.h2[(k - a.nq) * nr + r] = s;
  } else if (k == 2 * a.nq) {
    a.h1p[r] = s;
  } else if (k == 2 * a.nq + 1) {
    a.h2p[r] = s;
  } else if (a.ww) {
    a.ww[r] = s.x;
  }
}

template <int MODE, int... K>
static void gs_launch(std::integer_sequence<int, K...>, const GsArgs& a, dim3 grid, hipStream_t st) {
  using F = void (*)(GsArgs);
  static const F tab[] = {&k_gs<K, MODE>...};
  hipLaunchKernelGGL(tab[a.nq], grid, dim3(RED_THREADS), 0, st, a);
}

void launch_gs(int mode, const GsArgs& a, hipStream_t st) {
  const bool two = mode == GS_DOT2 || mode == GS_COMB2;
  if (a.nq < (two ? 0 : 1) || a.nq > GS_CHUNK) throw std::runtime_error("launch_gs: basis chunk out of range");
  if (!a.part) throw std::runtime_error("launch_gs: no partial-sum buffer");
  // 256 workgroups per right-hand side: measured the fastest for these
  // read-write streams (512 and more cost 3-7%)
  const int nwg = std::min(reduce_nwg(a.n), 256);
  const dim3 grid(nwg, a.nrhs);
  auto seq = std::make_integer_sequence<int, GS_CHUNK + 1>{};
  switch (mode) {
    case GS_DOT: gs_launch<GS_DOT>(seq, a, grid, st); break;
    case GS_AXPY_DOT: gs_launch<GS_AXPY_DOT>(seq, a, grid, st); break;
    case GS_AXPY_NORM: gs_launch<GS_AXPY_NORM>(seq, a, grid, st); break;
    case GS_DOT2: gs_launch<GS_DOT2>(seq, a, grid, st); break;
    case GS_COMB2: gs_launch<GS_COMB2>(seq, a, grid, st); break;
    default: throw std::runtime_error("launch_gs: unknown mode");
  }
  const int nout = mode == GS_DOT || mode == GS_AXPY_DOT ? a.nq : mode == GS_DOT2 ? 2 * a.nq + 3 : 1;
  if ((mode == GS_AXPY_NORM || mode == GS_COMB2) && !a.norm2) return;
  k_gs_fin<<<a.nrhs, 256, 0, st>>>(a, mode, nwg, nout);
}

__global__ __launch_bounds__(256) void k_scale(const double2* w, const double* scale, double2* out, float2* out32,
                                               size_t n, size_t rs) {
  const int r = blockIdx.y;
  const size_t off = r * rs;
  double sc = scale[r];
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    double2 a = w[off + i];
    double2 b = make_double2(a.x * sc, a.y * sc);
    if (out) out[off + i] = b;
    if (out32) out32[off + i] = make_float2((float)b.x, (float)b.y);
  }
}

void launch_scale(const double2* w, const double* scale, double2* out, float2* out32, size_t n, size_t rs, int nrhs,
                  hipStream_t st) {
  k_scale<<<ew_grid(n, nrhs), 256, 0, st>>>(w, scale, out, out32, n, rs);
}

template <class TZ>
__global__ __launch_bounds__(256) void k_update_x(double2* x, const TZ* Z, size_t zs, int nk, const double2* y,
                                                  size_t n, size_t rs, int nrhs) {
  const int r = blockIdx.y;
  const size_t off = r * rs;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    cplx<double> acc = ld<double>(x + off, i);
    for (int k = 0; k < nk; ++k) cmac(acc, C(y[(size_t)k * nrhs + r]), ld<double>(Z + (size_t)k * zs + off, i));
    st(x + off, i, acc);
  }
}

void launch_update_x(double2* x, const void* Z, int z_t, size_t zs, int nk, const double2* y, size_t n, size_t rs,
                     int nrhs, hipStream_t st) {
  if (z_t == C128)
    k_update_x<double2><<<ew_grid(n, nrhs), 256, 0, st>>>(x, (const double2*)Z, zs, nk, y, n, rs, nrhs);
  else
    k_update_x<float2><<<ew_grid(n, nrhs), 256, 0, st>>>(x, (const float2*)Z, zs, nk, y, n, rs, nrhs);
}

// ---------------------------------------------------------------- MR smoother (coarse levels)
// alpha[r] = <p, r> / <p, p> (0 when p = 0), from partials of (<p,r>, <p,p>)
__global__ void k_mr_fin(const double2* part, int nwg, double2* alpha) {
  int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  cplx<double> pr = sum_parts(part, nwg, 2, r, 0);
  double pp = sum_parts(part, nwg, 2, r, 1).x;
  alpha[r] = pp > 0 ? make_double2(pr.x / pp, pr.y / pp) : make_double2(0.0, 0.0);
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_mr_update(T* x, T* r, const T* p, const double2* alpha, size_t n,
                                                   size_t rs) {
  const int rr = blockIdx.y;
  const size_t off = rr * rs;
  cplx<R> al = {(R)alpha[rr].x, (R)alpha[rr].y};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    cplx<R> ri = ld<R>(r + off, i);
    st(x + off, i, ld<R>(x + off, i) + al * ri);
    st(r + off, i, ri - al * ld<R>(p + off, i));
  }
}

void launch_mr_alpha(const void* p, const void* r, int t, size_t n, size_t rs, int nrhs, double2* part,
                     double2* alpha, hipStream_t st) {
  const void* a[2] = {p, p};
  const void* b[2] = {r, p};
  launch_dots_partial(2, a, b, t, n, rs, nrhs, part, st);
  k_mr_fin<<<nrhs, 64, 0, st>>>(part, reduce_nwg(n), alpha);
}

void launch_mr_update(void* x, void* r, const void* p, const double2* alpha, int t, size_t n, size_t rs, int nrhs,
                      hipStream_t st) {
  if (t == C128)
    k_mr_update<double2, double><<<ew_grid(n, nrhs), 256, 0, st>>>((double2*)x, (double2*)r, (const double2*)p,
                                                                   alpha, n, rs);
  else
    k_mr_update<float2, float><<<ew_grid(n, nrhs), 256, 0, st>>>((float2*)x, (float2*)r, (const float2*)p, alpha,
                                                                 n, rs);
}

// ---------------------------------------------------------------- seeded Gaussian vectors
// Counter-based: element i of stream `seed` takes two 64-bit words from the
// SplitMix64 finaliser (Steele, Lea, Flood 2014) of seed*2^32 + 2i and + 2i+1,
// maps them to uniforms in (0, 1] and applies the Box-Muller transform.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

template <class T>
__global__ __launch_bounds__(256) void k_gauss(T* out, size_t n, unsigned long long seed) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    unsigned long long base = (seed << 32) + 2 * (unsigned long long)i;
    double u1 = ((splitmix64(base) >> 11) + 1) * (1.0 / 9007199254740992.0);
    double u2 = (splitmix64(base + 1) >> 11) * (1.0 / 9007199254740992.0);
    double rad = sqrt(-2.0 * log(u1));
    double ph = 6.283185307179586 * u2;
    st(out, i, cplx<double>{rad * cos(ph), rad * sin(ph)});
  }
}

void launch_gauss(void* out, int t, size_t n, unsigned long long seed, hipStream_t st) {
  unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  if (t == C128)
    k_gauss<double2><<<nb, 256, 0, st>>>((double2*)out, n, seed);
  else
    k_gauss<float2><<<nb, 256, 0, st>>>((float2*)out, n, seed);
}

}  // namespace wc
