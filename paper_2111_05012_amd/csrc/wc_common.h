// Internal definitions shared by the HIP kernels of libwcamg (complex
// arithmetic, storage types, lattice geometry of the blocked site order).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace wc {

// ---------------------------------------------------------------------------
// Complex numbers in registers; storage types in memory
// ---------------------------------------------------------------------------
template <class R>
struct cplx {
  R x, y;
};

template <class R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__host__ __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return {s * a.x, s * a.y}; }
template <class R>
__host__ __device__ __forceinline__ cplx<R> cj(cplx<R> a) { return {a.x, -a.y}; }
// a += b * c
template <class R>
__host__ __device__ __forceinline__ void cmac(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(-b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(b.y, c.x, a.y);
}
// a += conj(b) * c
template <class R>
__host__ __device__ __forceinline__ void cjmac(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(-b.y, c.x, a.y);
}
// Multiplication by a unit u in {1, i, -1, -i} (code 0..3), folded at compile time.
template <int U, class R>
__host__ __device__ __forceinline__ cplx<R> unit(cplx<R> a) {
  if constexpr (U == 0) return a;
  else if constexpr (U == 1) return {-a.y, a.x};
  else if constexpr (U == 2) return {-a.x, -a.y};
  else return {a.y, -a.x};
}

struct alignas(4) half2_t {
  _Float16 x, y;
};

// load one complex number from storage, converted to the register precision R
template <class R>
__device__ __forceinline__ cplx<R> ld(const double2* p, size_t i) {
  double2 v = p[i];
  return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cplx<R> ld(const float2* p, size_t i) {
  float2 v = p[i];
  return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cplx<R> ld(const half2_t* p, size_t i) {
  half2_t v = p[i];
  return {(R)(float)v.x, (R)(float)v.y};
}
template <class R>
__device__ __forceinline__ void st(double2* p, size_t i, cplx<R> v) { p[i] = make_double2((double)v.x, (double)v.y); }
template <class R>
__device__ __forceinline__ void st(float2* p, size_t i, cplx<R> v) { p[i] = make_float2((float)v.x, (float)v.y); }
template <class R>
__device__ __forceinline__ void st(half2_t* p, size_t i, cplx<R> v) {
  half2_t h;
  h.x = (_Float16)v.x;  // round to nearest even, directly from R
  h.y = (_Float16)v.y;
  p[i] = h;
}

// ---------------------------------------------------------------------------
// Blocked site order.  A lattice of extents L[mu] (mu = x,y,z,t) is cut into
// blocks of extents B[mu] (the SAP domains and multigrid aggregates).  The
// internal site index is s = blk * Vb + loc with blk and loc both
// lexicographic (x fastest) over the block grid NB and inside the block.
// ---------------------------------------------------------------------------
struct Geo {
  int L[4], B[4], NB[4];
  int sB[4];  // strides of loc
  int sN[4];  // strides of blk
  int V, Vb, nblk;
  int bc[4];
};

inline Geo make_geo(const int* L, const int* B, const int* bc) {
  Geo g;
  for (int m = 0; m < 4; ++m) {
    g.L[m] = L[m];
    g.B[m] = B[m];
    g.NB[m] = L[m] / B[m];
    g.bc[m] = bc[m];
  }
  g.sB[0] = 1;
  g.sN[0] = 1;
  for (int m = 1; m < 4; ++m) {
    g.sB[m] = g.sB[m - 1] * B[m - 1];
    g.sN[m] = g.sN[m - 1] * g.NB[m - 1];
  }
  g.Vb = B[0] * B[1] * B[2] * B[3];
  g.nblk = g.NB[0] * g.NB[1] * g.NB[2] * g.NB[3];
  g.V = g.Vb * g.nblk;
  return g;
}

struct SiteCoord {
  int blk, loc;
  int lc[4];  // coordinate inside the block
  int bk[4];  // block coordinate
};

__host__ __device__ __forceinline__ SiteCoord decompose(const Geo& g, int s) {
  SiteCoord c;
  c.blk = s / g.Vb;
  c.loc = s - c.blk * g.Vb;
  int l = c.loc, b = c.blk;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    int q = l / g.B[m];
    c.lc[m] = l - q * g.B[m];
    l = q;
    int p = b / g.NB[m];
    c.bk[m] = b - p * g.NB[m];
    b = p;
  }
  c.lc[3] = l;
  c.bk[3] = b;
  return c;
}

// Field storage.  A site field of K planes (K = 12 spin-colour components
// for spinors and test vectors, 36 for the links [mu][row][col] and for the
// packed clover) is stored block-major, [blk][K][Vb]: the K planes of one
// block are contiguous.  Everything a block (an SAP domain, a multigrid
// aggregate) touches is then one contiguous range, and the planes of a site
// are Vb elements apart instead of V (at lattice volumes that are large powers
// of two, planes V apart all fall into the same cache set).  Plane q of site s
// = blk * Vb + loc lies at fbase(g, K, s) + q * Vb.
__host__ __device__ __forceinline__ size_t fbase_b(const Geo& g, int K, int s, int blk) {
  return (size_t)s + (size_t)blk * (K - 1) * g.Vb;
}
__host__ __device__ __forceinline__ size_t fbase(const Geo& g, int K, int s) {
  return fbase_b(g, K, s, s / g.Vb);
}

// Neighbour of site s (coordinates c) in direction +mu (FWD) or -mu.  Sets
// sign to bc[mu] when the hop crosses the lattice boundary, inblk to whether
// the neighbour lies in the same block and nblk to the neighbour's block.
template <bool FWD>
__host__ __device__ __forceinline__ int neighbour(const Geo& g, int s, const SiteCoord& c, int mu, int& sign,
                                                  bool& inblk, int& nblk_out) {
  sign = 1;
  nblk_out = c.blk;
  if (FWD) {
    if (c.lc[mu] < g.B[mu] - 1) {
      inblk = true;
      return s + g.sB[mu];
    }
    int nloc = c.loc - (g.B[mu] - 1) * g.sB[mu];
    int nblk;
    if (c.bk[mu] < g.NB[mu] - 1) {
      nblk = c.blk + g.sN[mu];
    } else {
      nblk = c.blk - (g.NB[mu] - 1) * g.sN[mu];
      sign = g.bc[mu];
    }
    inblk = (nblk == c.blk);
    nblk_out = nblk;
    return nblk * g.Vb + nloc;
  } else {
    if (c.lc[mu] > 0) {
      inblk = true;
      return s - g.sB[mu];
    }
    int nloc = c.loc + (g.B[mu] - 1) * g.sB[mu];
    int nblk;
    if (c.bk[mu] > 0) {
      nblk = c.blk - g.sN[mu];
    } else {
      nblk = c.blk + (g.NB[mu] - 1) * g.sN[mu];
      sign = g.bc[mu];
    }
    inblk = (nblk == c.blk);
    nblk_out = nblk;
    return nblk * g.Vb + nloc;
  }
}
template <bool FWD>
__host__ __device__ __forceinline__ int neighbour(const Geo& g, int s, const SiteCoord& c, int mu, int& sign,
                                                  bool& inblk) {
  int nblk;
  return neighbour<FWD>(g, s, c, mu, sign, inblk, nblk);
}

// Map a launch's workgroup index so that consecutive logical tiles land on
// the same XCD (workgroups are dispatched round-robin over the 8 XCDs, each
// with its own L2): logical = (id % 8) * ceil(n / 8) + id / 8.  The launch
// must have 8 * ceil(n / 8) workgroups (a bijection onto [0, 8 ceil(n/8)));
// the kernel skips logical indices >= n.
__device__ __forceinline__ int xcd_remap(int id, int n) {
  int per = (n + 7) >> 3;
  return (id & 7) * per + (id >> 3);
}

}  // namespace wc
