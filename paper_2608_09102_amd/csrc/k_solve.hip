// k_solve.hip -- solve-phase kernels: V-cycle level operations (damped block
// Jacobi, residual, restriction, prolongation), the FP64 outer block SpMV,
// the Gram-Schmidt passes of the Arnoldi step, the small FGMRES scalar work
// and the projection.  All of them are bound by HBM bandwidth: one thread per
// block row, one wavefront per 64-row slice, coalesced slot-major loads, and
// reductions in a fixed tree so results are bitwise reproducible.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "llg_internal.h"

namespace llg {

namespace {

constexpr int TPB = 256;
constexpr int MAXV_S = 32;  // largest FGMRES restart

// sliced-ELL kernels: 256-thread blocks for large levels, one slice per block
// for small ones so that the blocks spread over all CUs
inline int tpb_rows(int64_t n) { return n >= 65536 ? 256 : 64; }

inline unsigned nblk(int64_t n, int t = TPB) { return (unsigned)ceil_div(n > 0 ? n : 1, t); }


template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
__device__ inline V3<T> ld3(const T* p, int64_t i) {
  return V3<T>{p[3 * i], p[3 * i + 1], p[3 * i + 2]};
}
template <typename T>
__device__ inline void st3(T* p, int64_t i, V3<T> v) {
  p[3 * i] = v.x;
  p[3 * i + 1] = v.y;
  p[3 * i + 2] = v.z;
}

// x value of node j under the level's x mode
template <typename T, int XMODE>
__device__ inline V3<T> xval(const T* x, const T* b, T omega, int64_t j) {
  if (XMODE == 0) return ld3(x, j);
  if (XMODE == 1) {
    V3<T> v = ld3(b, j);
    return V3<T>{omega * v.x, omega * v.y, omega * v.z};
  }
  return V3<T>{T(0), T(0), T(0)};
}

// acc += blk * v for a 3x3 block stored slot-major
template <typename T, typename TV, typename TA>
__device__ inline void blk_mv(const T* __restrict__ val, int64_t vb, V3<TV> v, TA& a0, TA& a1, TA& a2) {
  const TA x = (TA)v.x, y = (TA)v.y, z = (TA)v.z;
  a0 += (TA)val[vb + 0 * SL] * x + (TA)val[vb + 1 * SL] * y + (TA)val[vb + 2 * SL] * z;
  a1 += (TA)val[vb + 3 * SL] * x + (TA)val[vb + 4 * SL] * y + (TA)val[vb + 5 * SL] * z;
  a2 += (TA)val[vb + 6 * SL] * x + (TA)val[vb + 7 * SL] * y + (TA)val[vb + 8 * SL] * z;
}

// Nine zero entries per lane at the slot stride: the block that padding slots
// of the lane-group row product read instead of their own (never stored)
// values.
__device__ double g_zero_block[9 * SL];

// Row i of a sliced-ELL matrix times x: the slot loop is unrolled by four so
// that the column indices of four slots are loaded together; a slot's values
// and x entries are loaded only for a stored block (padding slots cost no
// memory traffic, which matters on the large levels where rows run about
// 1.4 times shorter than their slice).  FP32 values: the four slots' loads
// are all issued before any product; FP64 values: slot by slot, which
// measured faster for FP64 (the four-slot form needs about twice the
// registers).
template <typename T, typename TA, typename XF>
__device__ inline void sell_row_mv(const int32_t* __restrict__ col, const T* __restrict__ val, int64_t cb,
                                   int w, int l, XF xf, TA& a0, TA& a1, TA& a2) {
  for (int t = 0; t < w; t += 4) {
    int32_t c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = (t + q < w) ? col[cb + (int64_t)(t + q) * SL + l] : -1;
    if constexpr (sizeof(T) == 8) {  // FP64 values: one slot's loads at a time (fewer registers)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (c[q] >= 0) blk_mv(val, cb * 9 + (int64_t)(t + q) * 9 * SL + l, xf(c[q]), a0, a1, a2);
      continue;
    }
    using XV = decltype(xf(0));
    T v[4][9];
    XV xq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (c[q] >= 0) {
        const int64_t vb = cb * 9 + (int64_t)(t + q) * 9 * SL + l;
#pragma unroll
        for (int e = 0; e < 9; ++e) v[q][e] = val[vb + e * SL];
        xq[q] = xf(c[q]);
      } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) v[q][e] = T(0);
        xq[q] = XV{0, 0, 0};
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const TA x = (TA)xq[q].x, y = (TA)xq[q].y, z = (TA)xq[q].z;
      a0 += (TA)v[q][0] * x + (TA)v[q][1] * y + (TA)v[q][2] * z;
      a1 += (TA)v[q][3] * x + (TA)v[q][4] * y + (TA)v[q][5] * z;
      a2 += (TA)v[q][6] * x + (TA)v[q][7] * y + (TA)v[q][8] * z;
    }
  }
}

template <typename T>
__device__ inline V3<T> dmv(const T* __restrict__ d, int64_t db, V3<T> v) {
  return V3<T>{d[db + 0 * SL] * v.x + d[db + 1 * SL] * v.y + d[db + 2 * SL] * v.z,
               d[db + 3 * SL] * v.x + d[db + 4 * SL] * v.y + d[db + 5 * SL] * v.z,
               d[db + 6 * SL] * v.x + d[db + 7 * SL] * v.y + d[db + 8 * SL] * v.z};
}

// Row handled by this thread (XCD-aware block order).  With G > 1, G
// consecutive lanes share one row (small levels: their rows are latency
// bound, so the row's slots are spread over the lanes); sub is the lane's
// index within its group.
struct RowPos {
  int64_t i, s;
  int l, sub;
};
template <int G>
__device__ inline RowPos row_pos() {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t t = (int64_t)blk * blockDim.x + threadIdx.x;
  RowPos p;
  p.i = t / G;
  p.sub = (int)(t - p.i * G);
  p.s = p.i / SL;
  p.l = (int)(p.i - p.s * SL);
  return p;
}

// Row product with the slots of the row split over the G lanes of a group,
// then a butterfly sum inside the group (every lane ends with the total).
// These levels are latency bound, so two slots per lane are loaded with no
// branch between them: a padding slot reads the zero block and x of node 0.
template <int G, typename T, typename TA, typename XF>
__device__ inline void sell_row_mv_g(const int32_t* __restrict__ col, const T* __restrict__ val, int64_t cb,
                                     int w, int l, int sub, XF xf, TA& a0, TA& a1, TA& a2) {
  if (G == 1) {
    sell_row_mv(col, val, cb, w, l, xf, a0, a1, a2);
    return;
  }
  const T* zero = (const T*)g_zero_block + l;
  for (int t = sub; t < w; t += 2 * G) {
    const int32_t c0 = col[cb + (int64_t)t * SL + l];
    const int32_t c1 = t + G < w ? col[cb + (int64_t)(t + G) * SL + l] : -1;
    const bool ok0 = c0 >= 0, ok1 = c1 >= 0;
    const T* v0 = ok0 ? val + cb * 9 + (int64_t)t * 9 * SL + l : zero;
    const T* v1 = ok1 ? val + cb * 9 + (int64_t)(t + G) * 9 * SL + l : zero;
    blk_mv(v0, 0, xf(ok0 ? c0 : 0), a0, a1, a2);
    blk_mv(v1, 0, xf(ok1 ? c1 : 0), a0, a1, a2);
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, G);
    a1 += __shfl_xor(a1, off, G);
    a2 += __shfl_xor(a2, off, G);
  }
}

// ------------------------------------------------------------- level kernels
// x = omega D^{-1} b (first pre-smoothing sweep from x = 0)
template <typename T>
__global__ void k_smooth_first(int64_t n, const T* __restrict__ dinv, T omega, const T* __restrict__ b,
                               T* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = i / SL;
  const int l = (int)(i - s * SL);
  V3<T> d = dmv(dinv, s * 9 * SL + l, ld3(b, i));
  st3(x, i, V3<T>{omega * d.x, omega * d.y, omega * d.z});
}

// r = b - A x
template <typename T, int XMODE, int G>
__global__ void k_residual(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                           const T* __restrict__ val, T omega, const T* __restrict__ b,
                           const T* __restrict__ x, T* __restrict__ r) {
  const RowPos p = row_pos<G>();
  if (p.i >= n) return;
  const int64_t cb = sl[p.s];
  const int w = (int)((sl[p.s + 1] - cb) / SL);
  T a0 = 0, a1 = 0, a2 = 0;
  sell_row_mv_g<G>(col, val, cb, w, p.l, p.sub, [&](int32_t c) { return xval<T, XMODE>(x, b, omega, c); }, a0,
                   a1, a2);
  if (p.sub != 0) return;
  const V3<T> bi = ld3(b, p.i);
  st3(r, p.i, V3<T>{bi.x - a0, bi.y - a1, bi.z - a2});
}

// Restriction bc_I = sum of r_i over the members of aggregate I, ascending,
// fused with the first pre-smoothing sweep of the coarse level,
// xc_I = omega Dc_I^{-1} bc_I (when xc != NULL).
template <typename T>
__global__ void k_restrict(int64_t nc, const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                           const T* __restrict__ r, T* __restrict__ bc, const T* __restrict__ cdinv, T omega,
                           T* __restrict__ xc) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  T a0 = 0, a1 = 0, a2 = 0;
  for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
    const V3<T> v = ld3(r, (int64_t)mem[q]);
    a0 += v.x;
    a1 += v.y;
    a2 += v.z;
  }
  st3(bc, I, V3<T>{a0, a1, a2});
  if (xc) {
    const int64_t cs = I / SL;
    const V3<T> d = dmv(cdinv, cs * 9 * SL + (I - cs * SL), V3<T>{a0, a1, a2});
    st3(xc, I, V3<T>{omega * d.x, omega * d.y, omega * d.z});
  }
}

// out_i = x'_i + omega D_i^{-1} (b_i - sum_j A_ij x'_j), x'_j = xbase_j + ec[agg_j]
template <typename T, int XMODE, bool UNIT, int G>
__global__ void k_post_smooth(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                              const T* __restrict__ val, const T* __restrict__ dinv, T omega,
                              const T* __restrict__ b, const T* __restrict__ x,
                              const int32_t* __restrict__ agg, const T* __restrict__ ec,
                              T* __restrict__ out) {
  const RowPos p = row_pos<G>();
  if (p.i >= n) return;
  const int64_t cb = sl[p.s];
  const int w = (int)((sl[p.s + 1] - cb) / SL);
  auto xp = [&](int64_t c) {
    V3<T> xj = xval<T, XMODE>(x, b, omega, c);
    if (ec) {
      const V3<T> e = ld3(ec, (int64_t)agg[c]);
      xj.x += e.x;
      xj.y += e.y;
      xj.z += e.z;
    }
    return xj;
  };
  T a0 = 0, a1 = 0, a2 = 0;
  sell_row_mv_g<G>(col, val, cb, w, p.l, p.sub, [&](int32_t c) { return xp(c); }, a0, a1, a2);
  if (p.sub != 0) return;
  const V3<T> xi = xp(p.i);
  const V3<T> bi = ld3(b, p.i);
  V3<T> res{bi.x - a0, bi.y - a1, bi.z - a2};
  if (!UNIT) res = dmv(dinv, p.s * 9 * SL + p.l, res);
  st3(out, p.i, V3<T>{xi.x + omega * res.x, xi.y + omega * res.y, xi.z + omega * res.z});
}

// ------------------------------------------------ CSR-ordered large levels
// A coarse level that feeds a Galerkin product also keeps its blocks in CSR
// order (nine contiguous values per block, a row's blocks contiguous in
// ascending column order).  The row products of the large coarse levels read
// that copy: their rows vary in length, so their slices hold about 1.4 times
// the stored blocks, and a slot line is fetched whole as soon as one row of
// the slice reaches it.  G lanes share a row: lane sub takes the blocks
// rp[i] + sub, + G, ..., U = 2 per pass (the column indices, then the
// values, then the x gathers of the U blocks, each group of loads in flight
// together), and the group's partial sums are added by a butterfly (every
// lane ends with the total).
template <int G, typename T, typename XF>
__device__ inline void csr_row_mv_g(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    const T* __restrict__ vt, int64_t i, int sub, XF xf, T& a0, T& a1, T& a2) {
  constexpr int U = 2;  // blocks per lane and pass
  const int32_t k1 = rp[i + 1];
  for (int32_t k = rp[i] + sub; k < k1; k += U * G) {
    int32_t kk[U], cc[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = k + u * G < k1;
      kk[u] = ok[u] ? k + u * G : k;  // a missing block re-reads the first
      cc[u] = ci[kk[u]];
    }
    T p[U][9];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 9; ++e) p[u][e] = vt[(int64_t)kk[u] * 9 + e];
    V3<T> xx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xx[u] = xf(cc[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      a0 += p[u][0] * xx[u].x + p[u][1] * xx[u].y + p[u][2] * xx[u].z;
      a1 += p[u][3] * xx[u].x + p[u][4] * xx[u].y + p[u][5] * xx[u].z;
      a2 += p[u][6] * xx[u].x + p[u][7] * xx[u].y + p[u][8] * xx[u].z;
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, G);
    a1 += __shfl_xor(a1, off, G);
    a2 += __shfl_xor(a2, off, G);
  }
}

// r = b - A x, A in CSR order
template <typename T, int XMODE, int G>
__global__ void k_residual_csr(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const T* __restrict__ vt, T omega, const T* __restrict__ b, const T* __restrict__ x,
                               T* __restrict__ r) {
  const RowPos p = row_pos<G>();
  if (p.i >= n) return;  // the G lanes of a row leave together
  T a0 = 0, a1 = 0, a2 = 0;
  csr_row_mv_g<G>(rp, ci, vt, p.i, p.sub, [&](int32_t c) { return xval<T, XMODE>(x, b, omega, c); }, a0, a1, a2);
  if (p.sub != 0) return;
  const V3<T> bi = ld3(b, p.i);
  st3(r, p.i, V3<T>{bi.x - a0, bi.y - a1, bi.z - a2});
}

// out_i = x_i + omega D_i^{-1} (b_i - sum_j A_ij x_j), A in CSR order (the
// coarse correction is prolonged into x beforehand, in its own pass)
template <typename T, int XMODE, int G>
__global__ void k_post_smooth_csr(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const T* __restrict__ vt, const T* __restrict__ dinv, T omega,
                                  const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ out) {
  const RowPos p = row_pos<G>();
  if (p.i >= n) return;
  T a0 = 0, a1 = 0, a2 = 0;
  csr_row_mv_g<G>(rp, ci, vt, p.i, p.sub, [&](int32_t c) { return xval<T, XMODE>(x, b, omega, c); }, a0, a1, a2);
  if (p.sub != 0) return;
  const V3<T> xi = xval<T, XMODE>(x, b, omega, p.i);
  const V3<T> bi = ld3(b, p.i);
  const V3<T> res = dmv(dinv, p.s * 9 * SL + p.l, V3<T>{bi.x - a0, bi.y - a1, bi.z - a2});
  st3(out, p.i, V3<T>{xi.x + omega * res.x, xi.y + omega * res.y, xi.z + omega * res.z});
}

// One block Gauss-Seidel sweep over a colour class, in place.  The rows of a
// class are not coupled to each other, so every row reads only rows of other
// classes (settled by earlier launches) and its own entry.  FIRST: x = 0
// everywhere before the sweep, so x_i = D_i^{-1} b_i without reading A.
template <typename T, bool UNIT, bool FIRST, int G>
__global__ void k_gs_sweep(int64_t n, const int32_t* __restrict__ rows, const int32_t* __restrict__ sl,
                           const int32_t* __restrict__ col, const T* __restrict__ val, const T* __restrict__ dinv,
                           const T* __restrict__ b, T* x) {
  const RowPos p = row_pos<G>();
  if (p.i >= n) return;
  const int64_t i = rows[p.i];
  T a0 = 0, a1 = 0, a2 = 0;
  if (!FIRST) {
    const int64_t cb = sl[p.s];
    const int w = (int)((sl[p.s + 1] - cb) / SL);
    sell_row_mv_g<G>(col, val, cb, w, p.l, p.sub, [&](int32_t c) { return ld3((const T*)x, (int64_t)c); }, a0,
                     a1, a2);
  }
  if (p.sub != 0) return;
  const V3<T> bi = ld3(b, i);
  V3<T> res{bi.x - a0, bi.y - a1, bi.z - a2};
  if (!UNIT) res = dmv(dinv, p.s * 9 * SL + p.l, res);
  if (FIRST) {
    st3(x, i, res);
  } else {
    const V3<T> xi = ld3((const T*)x, i);
    st3(x, i, V3<T>{xi.x + res.x, xi.y + res.y, xi.z + res.z});
  }
}

template <typename T>
__global__ void k_fill_zero(T* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

template <typename T, int XMODE>
__global__ void k_prolong(int64_t n, T omega, const T* __restrict__ b, const T* __restrict__ x,
                          const int32_t* __restrict__ agg, const T* __restrict__ ec, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V3<T> xi = xval<T, XMODE>(x, b, omega, i);
  const V3<T> e = ld3(ec, (int64_t)agg[i]);
  st3(out, i, V3<T>{xi.x + e.x, xi.y + e.y, xi.z + e.z});
}

template <typename T>
__global__ void k_scale_in(int64_t n, const double* __restrict__ dinv0, int left_scale,
                           const double* __restrict__ v, const double* __restrict__ vs, T* __restrict__ b0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V3<double> x = ld3(v, i);
  if (vs) {
    const double f = vs[0];
    x = V3<double>{x.x * f, x.y * f, x.z * f};
  }
  if (left_scale) {
    const int64_t s = i / SL;
    x = dmv(dinv0, s * 9 * SL + (i - s * SL), x);
  }
  st3(b0, i, V3<T>{(T)x.x, (T)x.y, (T)x.z});
}

// ------------------------------------------------------------- outer (FP64)
template <typename TZ>
__global__ void k_spmv_outer(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                             const double* __restrict__ val, const TZ* __restrict__ z,
                             double* __restrict__ w) {
  const RowPos p = row_pos<1>();
  if (p.i >= n) return;
  const int64_t cb = sl[p.s];
  const int wd = (int)((sl[p.s + 1] - cb) / SL);
  double a0 = 0, a1 = 0, a2 = 0;
  sell_row_mv(col, val, cb, wd, p.l, [&](int32_t c) { return ld3(z, (int64_t)c); }, a0, a1, a2);
  st3(w, p.i, V3<double>{a0, a1, a2});
}

// Sum of NS per-thread values over the workgroup in a fixed tree (wave
// shuffles, then the waves in order); results land in out[0..NS) of thread 0.
template <int NS>
__device__ inline void block_sums(const double* v, double* sh, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double a = v[q];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0) sh[wv * NS + q] = a;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    double r = 0;
    for (int k = 0; k < nw; ++k) r += sh[k * NS + threadIdx.x];
    out[threadIdx.x] = r;
  }
  __syncthreads();
}

__global__ void k_resid_outer(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                              const double* __restrict__ val, const double* __restrict__ b,
                              const double* __restrict__ u, double* __restrict__ r,
                              double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  __shared__ double res[1];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double nrm = 0;
  if (i < n) {
    const int64_t s = i / SL;
    const int l = (int)(i - s * SL);
    const int64_t cb = sl[s];
    const int wd = (int)((sl[s + 1] - cb) / SL);
    double a0 = 0, a1 = 0, a2 = 0;
    sell_row_mv(col, val, cb, wd, l, [&](int32_t c) { return ld3(u, (int64_t)c); }, a0, a1, a2);
    const V3<double> bi = ld3(b, i);
    const V3<double> ri{bi.x - a0, bi.y - a1, bi.z - a2};
    st3(r, i, ri);
    nrm = (ri.x * ri.x + ri.y * ri.y) + ri.z * ri.z;
  }
  block_sums<1>(&nrm, sh, res);
  if (threadIdx.x == 0) part[blockIdx.x] = res[0];
}

// ------------------------------------------------------- factored fine level
// On the grid level every off-diagonal block of row p is one 3x3 block:
// A_pq = Mh_p = (dt/h^2) M_p for each in-grid neighbour q, A_pp = I + s_pp M_p
// with s_pp = -deg_p dt/h^2 = -deg_p (dt/h^2); the left-scaled operator has
// Atilde_pq = K_p = D_p^{-1} Mh_p and Atilde_pp = I.  One block per node in
// the [slice][9][64] layout, neighbours from the grid:
//   (A z)_p = z_p + Mh_p (sum_q z_q - deg_p z_p),   (Atilde x)_p = x_p + K_p sum_q x_q.
struct GridPos {
  int64_t p;
  bool ok;
};
// Node of this thread.  2D: XCD-aware block order over the node index.  3D:
// XCD x (= blockIdx mod 8, the dispatch order of the chip) takes the y rows
// [x ny/8, (x+1) ny/8) of every plane and walks them plane by plane.  The
// planes k-1, k, k+1 that a stencil row reads then stay in that XCD's L2: a
// contiguous z-slab per XCD keeps whole planes in flight, and at 256^3 their
// three-plane reuse window (4.7 MB of FP64 vector) overflows the L2, so each
// vector entry was fetched about three times.  Launched with grid_blocks().
template <int DIM>
__device__ inline GridPos grid_pos(const GridDims& gd) {
  GridPos g;
  if (DIM == 2) {
    g.p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    g.ok = g.p < (int64_t)gd.nx * gd.ny;
    return g;
  }
  const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
  const uint32_t nx = (uint32_t)gd.nx, ny = (uint32_t)gd.ny;
  const uint32_t j0 = (x * ny) >> 3, j1 = ((x + 1) * ny) >> 3;
  const uint32_t row = (j1 - j0) * nx;  // nodes of the band in one plane
  const uint32_t t = k * TPB + threadIdx.x;
  g.ok = t < row * (uint32_t)gd.nz;
  const uint32_t kz = g.ok ? t / row : 0, r = t - kz * row;
  const uint32_t jj = r / nx, i = r - jj * nx;
  g.p = ((int64_t)kz * ny + j0 + jj) * nx + i;
  return g;
}

// In-grid neighbours of p in ascending index order (k-1, j-1, i-1, i+1,
// j+1, k+1): h[t] tells whether neighbour t exists, q[t] is its index or p
// itself when it does not (so that every load can be issued without a branch).
template <int DIM>
struct Nbrs {
  bool h[6];
  int64_t q[6];
};
template <int DIM>
__device__ inline Nbrs<DIM> nbrs(int nx, int ny, int nz, int64_t p) {
  const uint32_t up = (uint32_t)p, unx = (uint32_t)nx, uny = (uint32_t)ny;
  uint32_t i, j, k = 0;
  if (DIM == 3) {
    const uint32_t nxy = unx * uny;
    k = up / nxy;
    const uint32_t rem = up - k * nxy;
    j = rem / unx;
    i = rem - j * unx;
  } else {
    j = up / unx;
    i = up - j * unx;
  }
  const int64_t sxy = (int64_t)nx * ny;
  Nbrs<DIM> n;
  n.h[0] = DIM == 3 && k > 0;
  n.h[1] = j > 0;
  n.h[2] = i > 0;
  n.h[3] = i + 1 < unx;
  n.h[4] = j + 1 < uny;
  n.h[5] = DIM == 3 && k + 1 < (uint32_t)nz;
  const int64_t off[6] = {-sxy, -(int64_t)nx, -1, 1, (int64_t)nx, sxy};
#pragma unroll
  for (int t = 0; t < 6; ++t) n.q[t] = n.h[t] ? p + off[t] : p;
  return n;
}
__device__ constexpr bool nbr_used(int dim, int t) { return dim == 3 || (t != 0 && t != 5); }

// Sum of f(q) over the in-grid neighbours (missing ones contribute zero);
// deg receives their number.
template <int DIM, typename T, typename XF>
__device__ inline V3<T> nbr_sum(int nx, int ny, int nz, int64_t p, XF f, int& deg) {
  const Nbrs<DIM> n = nbrs<DIM>(nx, ny, nz, p);
  V3<T> v[6];
#pragma unroll
  for (int t = 0; t < 6; ++t)
    if (nbr_used(DIM, t)) v[t] = f(n.q[t]);
  V3<T> a{T(0), T(0), T(0)};
  int d = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t)
    if (nbr_used(DIM, t)) {
      a.x += n.h[t] ? v[t].x : T(0);
      a.y += n.h[t] ? v[t].y : T(0);
      a.z += n.h[t] ? v[t].z : T(0);
      d += n.h[t] ? 1 : 0;
    }
  deg = d;
  return a;
}

// the nine entries of a per-node block ([slice][9][64] layout)
template <typename T>
struct B9 {
  T e[9];
};
template <typename T>
__device__ inline B9<T> ld9(const T* __restrict__ d, int64_t db) {
  B9<T> b;
#pragma unroll
  for (int q = 0; q < 9; ++q) b.e[q] = d[db + q * SL];
  return b;
}
template <typename T, typename TV>
__device__ inline V3<TV> mv9(const B9<T>& b, V3<TV> v) {
  return V3<TV>{(TV)b.e[0] * v.x + (TV)b.e[1] * v.y + (TV)b.e[2] * v.z,
                (TV)b.e[3] * v.x + (TV)b.e[4] * v.y + (TV)b.e[5] * v.z,
                (TV)b.e[6] * v.x + (TV)b.e[7] * v.y + (TV)b.e[8] * v.z};
}

// The blocks of node p recomputed from its frozen field (24 B instead of the
// 72 B of a stored block; the same values, see grid_blocks).
template <int DIM>
__device__ inline int nbr_count(const Nbrs<DIM>& n) {
  int d = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t)
    if (nbr_used(DIM, t)) d += n.h[t] ? 1 : 0;
  return d;
}
__device__ inline B9<double> node_Mh(const GridDims& gd, int64_t p, int deg) {
  double v[9];
  grid_blocks(gd.mt + 3 * p, gd.prm[0], gd.prm[1], gd.inv_h2, deg, v, nullptr, nullptr);
  B9<double> b;
#pragma unroll
  for (int e = 0; e < 9; ++e) b.e[e] = v[e];
  return b;
}
template <typename T>
__device__ inline B9<T> node_K(const GridDims& gd, const double* mt, int deg) {
  double v[9];
  grid_blocks(mt, gd.prm[0], gd.prm[1], gd.inv_h2, deg, nullptr, nullptr, v);
  B9<T> b;
#pragma unroll
  for (int e = 0; e < 9; ++e) b.e[e] = (T)v[e];
  return b;
}
// The FP32-AMG level-1 products: K from the frozen field rounded to FP32,
// evaluated in FP32 (the products are FP32; the FP64 evaluation of the same
// formula costs more than the product's memory traffic hides).  Same steps as
// grid_blocks: M, D = I + s_pp M, its adjugate inverse, K = D^{-1} (s M).
template <typename T>
__device__ inline B9<T> node_K(const GridDims& gd, const float* mt, int deg) {
  const float a = (float)gd.prm[0], s_off = (float)(gd.prm[1] * gd.inv_h2);
  const float s_diag = (float)(gd.prm[1] * (-(double)deg * gd.inv_h2));
  const float m1 = mt[0], m2 = mt[1], m3 = mt[2];
  float M[9];
  M[0] = -(a * (m2 * m2 + m3 * m3));
  M[1] = -m3 + a * (m1 * m2);
  M[2] = m2 + a * (m1 * m3);
  M[3] = m3 + a * (m1 * m2);
  M[4] = -(a * (m1 * m1 + m3 * m3));
  M[5] = -m1 + a * (m2 * m3);
  M[6] = -m2 + a * (m1 * m3);
  M[7] = m1 + a * (m2 * m3);
  M[8] = -(a * (m1 * m1 + m2 * m2));
  float D[9], B[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const float v = s_diag * M[e];
    D[e] = (e == 0 || e == 4 || e == 8) ? 1.0f + v : v;
    B[e] = s_off * M[e];
  }
  float adj[9];
  adj[0] = D[4] * D[8] - D[5] * D[7];
  adj[1] = D[2] * D[7] - D[1] * D[8];
  adj[2] = D[1] * D[5] - D[2] * D[4];
  adj[3] = D[5] * D[6] - D[3] * D[8];
  adj[4] = D[0] * D[8] - D[2] * D[6];
  adj[5] = D[2] * D[3] - D[0] * D[5];
  adj[6] = D[3] * D[7] - D[4] * D[6];
  adj[7] = D[1] * D[6] - D[0] * D[7];
  adj[8] = D[0] * D[4] - D[1] * D[3];
  const float rdet = 1.0f / ((D[0] * adj[0] + D[1] * adj[3]) + D[2] * adj[6]);
  B9<T> k;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      k.e[3 * r + q] = (T)(rdet * ((adj[3 * r] * B[q] + adj[3 * r + 1] * B[3 + q]) + adj[3 * r + 2] * B[6 + q]));
  return k;
}

// The same with D^{-1} recomputed from the frozen field (factored grid level)
template <int DIM, typename T>
__global__ void k_scale_in_grid(GridDims gd, const double* __restrict__ v, const double* __restrict__ vs,
                                T* __restrict__ b0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)gd.nx * gd.ny * gd.nz) return;
  V3<double> x = ld3(v, i);
  if (vs) {
    const double f = vs[0];
    x = V3<double>{x.x * f, x.y * f, x.z * f};
  }
  double di[9];
  grid_blocks(gd.mt + 3 * i, gd.prm[0], gd.prm[1], gd.inv_h2, nbr_count<DIM>(nbrs<DIM>(gd.nx, gd.ny, gd.nz, i)),
              nullptr, di, nullptr);
  const V3<double> y{(di[0] * x.x + di[1] * x.y) + di[2] * x.z, (di[3] * x.x + di[4] * x.y) + di[5] * x.z,
                     (di[6] * x.x + di[7] * x.y) + di[8] * x.z};
  st3(b0, i, V3<T>{(T)y.x, (T)y.y, (T)y.z});
}

template <int DIM, typename TZ>
__global__ void k_fact_outer(GridDims gd, const TZ* __restrict__ z, double* __restrict__ w) {
  const int nx = gd.nx, ny = gd.ny, nz = gd.nz;
  const GridPos g = grid_pos<DIM>(gd);
  if (!g.ok) return;
  const B9<double> m = node_Mh(gd, g.p, nbr_count<DIM>(nbrs<DIM>(nx, ny, nz, g.p)));
  auto zd = [&](int64_t q) {
    const V3<TZ> t = ld3(z, q);
    return V3<double>{(double)t.x, (double)t.y, (double)t.z};
  };
  int deg;
  const V3<double> sz = nbr_sum<DIM, double>(nx, ny, nz, g.p, zd, deg);
  const V3<double> zp = zd(g.p);
  const double dg = (double)deg;
  const V3<double> md = mv9(m, V3<double>{sz.x - dg * zp.x, sz.y - dg * zp.y, sz.z - dg * zp.z});
  st3(w, g.p, V3<double>{zp.x + md.x, zp.y + md.y, zp.z + md.z});
}

// r = b - A u with the partial sums of |r|^2 per workgroup
template <int DIM>
__global__ void k_fact_resid_outer(GridDims gd, const double* __restrict__ b, const double* __restrict__ u,
                                   double* __restrict__ r, double* __restrict__ part) {
  const int nx = gd.nx, ny = gd.ny, nz = gd.nz;
  __shared__ double sh[TPB / 64];
  __shared__ double res[1];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  double nrm = 0;
  if (p < N) {
    const B9<double> m = node_Mh(gd, p, nbr_count<DIM>(nbrs<DIM>(nx, ny, nz, p)));
    int deg;
    const V3<double> su = nbr_sum<DIM, double>(nx, ny, nz, p, [&](int64_t q) { return ld3(u, q); }, deg);
    const V3<double> up = ld3(u, p);
    const double dg = (double)deg;
    const V3<double> md = mv9(m, V3<double>{su.x - dg * up.x, su.y - dg * up.y, su.z - dg * up.z});
    const V3<double> bi = ld3(b, p);
    const V3<double> ri{bi.x - (up.x + md.x), bi.y - (up.y + md.y), bi.z - (up.z + md.z)};
    st3(r, p, ri);
    nrm = (ri.x * ri.x + ri.y * ri.y) + ri.z * ri.z;
  }
  block_sums<1>(&nrm, sh, res);
  if (threadIdx.x == 0) part[blockIdx.x] = res[0];
}

// r = b - Atilde x on the grid level
template <int DIM, typename T, int XMODE>
__global__ void k_fact_residual(GridDims gd, T omega, const T* __restrict__ b, const T* __restrict__ x,
                                T* __restrict__ r) {
  const int nx = gd.nx, ny = gd.ny, nz = gd.nz;
  const GridPos g = grid_pos<DIM>(gd);
  if (!g.ok) return;
  const B9<T> kb = node_K<T>(gd, gd.mt + 3 * g.p, nbr_count<DIM>(nbrs<DIM>(nx, ny, nz, g.p)));
  int deg;
  const V3<T> sx =
      nbr_sum<DIM, T>(nx, ny, nz, g.p, [&](int64_t q) { return xval<T, XMODE>(x, b, omega, q); }, deg);
  const V3<T> kx = mv9(kb, sx);
  const V3<T> xp = xval<T, XMODE>(x, b, omega, g.p);
  const V3<T> bi = ld3(b, g.p);
  st3(r, g.p, V3<T>{bi.x - (xp.x + kx.x), bi.y - (xp.y + kx.y), bi.z - (xp.z + kx.z)});
}

// out = x' + omega (b - Atilde x'), x'_q = xbase_q + ec[agg_q] (EC) or xbase_q.
// The aggregate numbers of the row's nodes are loaded first, then all the
// x and ec entries together.
template <int DIM, typename T, int XMODE, bool EC>
__global__ void k_fact_post_smooth(GridDims gd, T omega, const T* __restrict__ b, const T* __restrict__ x,
                                   const int32_t* __restrict__ agg, const T* __restrict__ ec, T* __restrict__ out) {
  const int nx = gd.nx, ny = gd.ny, nz = gd.nz;
  const GridPos g = grid_pos<DIM>(gd);
  if (!g.ok) return;
  const Nbrs<DIM> n = nbrs<DIM>(nx, ny, nz, g.p);
  const B9<T> kb = node_K<T>(gd, gd.mt + 3 * g.p, nbr_count<DIM>(n));
  int32_t a[7];
  if (EC) {
#pragma unroll
    for (int t = 0; t < 6; ++t)
      if (nbr_used(DIM, t)) a[t] = agg[n.q[t]];
    a[6] = agg[g.p];
  }
  V3<T> v[7];
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    if (t < 6 && !nbr_used(DIM, t)) continue;
    const int64_t q = t < 6 ? n.q[t] : g.p;
    v[t] = xval<T, XMODE>(x, b, omega, q);
    if (EC) {
      const V3<T> e = ld3(ec, (int64_t)a[t]);
      v[t].x += e.x;
      v[t].y += e.y;
      v[t].z += e.z;
    }
  }
  V3<T> sx{T(0), T(0), T(0)};
#pragma unroll
  for (int t = 0; t < 6; ++t)
    if (nbr_used(DIM, t)) {
      sx.x += n.h[t] ? v[t].x : T(0);
      sx.y += n.h[t] ? v[t].y : T(0);
      sx.z += n.h[t] ? v[t].z : T(0);
    }
  const V3<T> kx = mv9(kb, sx);
  const V3<T> xi = v[6];
  const V3<T> bi = ld3(b, g.p);
  const V3<T> res{bi.x - (xi.x + kx.x), bi.y - (xi.y + kx.y), bi.z - (xi.z + kx.z)};
  st3(out, g.p, V3<T>{xi.x + omega * res.x, xi.y + omega * res.y, xi.z + omega * res.z});
}

// partial sums of x.x over a fixed grid of RED_BLOCKS-bounded blocks
__global__ void k_norm_part(int64_t m, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  __shared__ double res[1];
  double a = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    a += x[k] * x[k];
  block_sums<1>(&a, sh, res);
  if (threadIdx.x == 0) part[blockIdx.x] = res[0];
}

// part[q][blk] = V_q . w (q < NV), part[NV][blk] = w . w; one sweep over w and V
template <int NV>
__global__ void __launch_bounds__(TPB) k_mdot(int64_t m, const double* __restrict__ V, int64_t ldv,
                                              const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[(TPB / 64) * (NV + 1)];
  __shared__ double res[NV + 1];
  const int G = gridDim.x;
  double acc[NV + 1];
#pragma unroll
  for (int q = 0; q <= NV; ++q) acc[q] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    const double wk = w[k];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] += V[q * ldv + k] * wk;
    acc[NV] += wk * wk;
  }
  block_sums<NV + 1>(acc, sh, res);
  if (threadIdx.x <= NV) part[(int64_t)threadIdx.x * G + blockIdx.x] = res[threadIdx.x];
}

// w -= sum_q h_q V_q; in the same sweep (V_q still in registers)
// part[q][blk] = V_q . w_new when want_dots, and part[NV][blk] = w_new . w_new.
// skip: when non-NULL and *skip == 0 the pass is not needed and returns.
template <int NV>
__global__ void __launch_bounds__(TPB) k_mupdate_dot(int64_t m, const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ h, double* __restrict__ w,
                                                     double* __restrict__ part, int want_dots,
                                                     const double* __restrict__ skip) {
  if (skip && skip[0] == 0.0) return;
  __shared__ double sh[(TPB / 64) * (NV + 1)];
  __shared__ double res[NV + 1];
  double hs[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) hs[q] = h[q];
  const int G = gridDim.x;
  double acc[NV + 1];
#pragma unroll
  for (int q = 0; q <= NV; ++q) acc[q] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    double v[NV];
    double wk = w[k];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      v[q] = V[q * ldv + k];
      wk -= hs[q] * v[q];
    }
    w[k] = wk;
    if (want_dots) {
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] += v[q] * wk;
    }
    acc[NV] += wk * wk;
  }
  block_sums<NV + 1>(acc, sh, res);
  if (threadIdx.x <= NV && (want_dots || threadIdx.x == NV))
    part[(int64_t)threadIdx.x * G + blockIdx.x] = res[threadIdx.x];
}

// Delayed reorthogonalization (classical Gram-Schmidt with the second pass of
// v_j lagged into the next iteration, after Swirydowicz, Langou, Ananthan,
// Yang and Thomas 2021).  Slot j of V holds u = h_j v~_j: the once
// orthogonalized vector times its norm h_j.  One sweep gives all the dots of
// the iteration, a second sweep finishes v_j and forms the next w'.
// part[q] = V_q . u and part[NV + q] = V_q . w (q < NV), part[2NV] = u.u,
// part[2NV + 1] = u.w, part[2NV + 2] = w.w, one column per workgroup.
template <int NV>
__global__ void __launch_bounds__(TPB) k_dcgs_dots(int64_t m, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ u, const double* __restrict__ w,
                                                   double* __restrict__ part) {
  constexpr int NS = 2 * NV + 3;
  __shared__ double sh[(TPB / 64) * NS];
  __shared__ double res[NS];
  const int G = gridDim.x;
  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    const double uk = u[k], wk = w[k];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double v = V[q * ldv + k];
      acc[q] += v * uk;
      acc[NV + q] += v * wk;
    }
    acc[2 * NV] += uk * uk;
    acc[2 * NV + 1] += uk * wk;
    acc[2 * NV + 2] += wk * wk;
  }
  block_sums<NS>(acc, sh, res);
  if (threadIdx.x < NS) part[(int64_t)threadIdx.x * G + blockIdx.x] = res[threadIdx.x];
}

// v_j = du u - sum_q d_q V_q (over u, in place) and w' = w - sum_q c_q V_q - cu u
// (into wo), with part[blk] = w'.w'.  coef = d_0..d_{NV-1}, c_0..c_{NV-1}, du, cu.
template <int NV>
__global__ void __launch_bounds__(TPB) k_dcgs_update(int64_t m, const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ coef, double* __restrict__ u,
                                                     const double* __restrict__ w, double* __restrict__ wo,
                                                     double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  __shared__ double res[1];
  double d[NV > 0 ? NV : 1], cc[NV > 0 ? NV : 1];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    d[q] = coef[q];
    cc[q] = coef[NV + q];
  }
  const double du = coef[2 * NV], cu = coef[2 * NV + 1];
  const int G = gridDim.x;
  double acc = 0.0;
  // The grid-stride passes run from the last to the first: the dots sweep
  // just before read the same vectors from the first pass to the last, so
  // its last passes are the ones still in the Infinity Cache (the basis
  // outgrows it); all lanes of a wavefront stay on one pass.
  const int64_t stride = (int64_t)G * blockDim.x;
  const int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = (m - 1) / stride; r >= 0; --r) {
    const int64_t k = r * stride + k0;
    if (k >= m) continue;
    const double uk = u[k], wk = w[k];
    double vj = du * uk, wp = wk - cu * uk;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double v = V[q * ldv + k];
      vj -= d[q] * v;
      wp -= cc[q] * v;
    }
    u[k] = vj;
    wo[k] = wp;
    acc += wp * wp;
  }
  block_sums<1>(&acc, sh, res);
  if (threadIdx.x == 0) part[blockIdx.x] = res[0];
}

template <typename TS, typename TD>
__global__ void k_cast(int64_t m, const TS* __restrict__ x, TD* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) y[k] = (TD)x[k];
}

__global__ void k_scale_vec(int64_t m, const double* __restrict__ x, const double* __restrict__ s,
                            double* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) y[k] = x[k] * s[0];
}

template <typename TZ>
__global__ void k_zy(int64_t m, int kk, const TZ* __restrict__ Z, int64_t ldz, const double* __restrict__ y,
                     double* __restrict__ u) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double a = u[k];
  for (int q = 0; q < kk; ++q) a += y[q] * (double)Z[q * ldz + k];
  u[k] = a;
}

__global__ void k_project(int64_t n, const double* __restrict__ u, double* __restrict__ out, int project,
                          int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const V3<double> v = ld3(u, i);
  if (!project) {
    st3(out, i, v);
    if (!isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z)) atomicOr(flag, 4);
    return;
  }
  const double nrm = sqrt((v.x * v.x + v.y * v.y) + v.z * v.z);
  if (!(nrm > 0.0) || !isfinite(nrm)) atomicOr(flag, 4);
  st3(out, i, V3<double>{v.x / nrm, v.y / nrm, v.z / nrm});
}

// ------------------------------------------------------------- K-cycle
// Coarse correction of a Krylov-accelerated level: two minimal-residual (GCR)
// steps on A_c e = r with directions v1 = B r and v2 = B rho.  The dot
// products are reduced in a fixed order; the coefficients stay on the device
// (kc[0] = a1, kc[1] = w1.w1, kc[4] = w1.rho, kc[2], kc[3] = final weights).

// w = A v (level operator); part[q][blk]: q = 0 w.w, q = 1 w.d1, q = 2 w.d2
template <typename T, int ND, int G>
__global__ void k_spmv_dots(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                            const T* __restrict__ val, const T* __restrict__ v, T* __restrict__ w,
                            const T* __restrict__ d1, const T* __restrict__ d2, double* __restrict__ part) {
  __shared__ double sh[(TPB / 64) * (ND + 1)];
  __shared__ double res[ND + 1];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / G;
  const int sub = (int)(t - i * G);
  double acc[ND + 1];
#pragma unroll
  for (int q = 0; q <= ND; ++q) acc[q] = 0.0;
  if (i < n) {
    const int64_t s = i / SL;
    const int l = (int)(i - s * SL);
    const int64_t cb = sl[s];
    const int wd = (int)((sl[s + 1] - cb) / SL);
    T a0 = 0, a1 = 0, a2 = 0;
    sell_row_mv_g<G>(col, val, cb, wd, l, sub, [&](int32_t c) { return ld3(v, (int64_t)c); }, a0, a1, a2);
    if (sub == 0) {
      st3(w, i, V3<T>{a0, a1, a2});
      const double x0 = a0, x1 = a1, x2 = a2;
      acc[0] = (x0 * x0 + x1 * x1) + x2 * x2;
      if (ND >= 1) {
        const V3<T> d = ld3(d1, i);
        acc[1 % (ND + 1)] = (x0 * (double)d.x + x1 * (double)d.y) + x2 * (double)d.z;
      }
      if (ND >= 2) {
        const V3<T> d = ld3(d2, i);
        acc[2 % (ND + 1)] = (x0 * (double)d.x + x1 * (double)d.y) + x2 * (double)d.z;
      }
    }
  }
  block_sums<ND + 1>(acc, sh, res);
  if (threadIdx.x <= ND) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = res[threadIdx.x];
}

// ------------------------------------------------ level 1 from the grid level
// Over a grid level stored per node (Atilde_ii = I, Atilde_ij = K_i for each
// grid neighbour j), the Galerkin block (I, J) of level 1 is
// [I = J] |I| I3 + sum over members i of I of n_iJ K_i, where n_iJ counts
// the grid neighbours of i in aggregate J.  So
//   (A1 x)_I = |I| x_I + sum_{i in I} K_i sum_{j ~ i} x_agg(j),
// which reads 72 B (FP64) per grid node instead of the stored level-1 blocks
// (about 150 B per grid node).  The stored blocks are still formed (for the
// next Galerkin product and the diagonal inverse D1); only the products use
// this form, so they differ from the stored-block products by rounding.
// mtq holds the frozen field in member order (mtq[q] = mt[mem[q]], rounded
// to T: in the FP32-AMG form the products are FP32 and their blocks come
// from the rounded field; the blocks K_i are recomputed from it) and nagg
// the level-1 aggregates of the
// members' grid neighbours ([slice][6][64] by member, -1 where the neighbour
// is missing), so that the lanes of a wavefront read consecutive entries and
// only the x gathers depend on loaded indices.
// MODE 0: r = b - A1 x.  MODE 1: out = x' + omega D1^{-1} (b - A1 x') with
// x'_J = x_J + ec[agg2_J] (ec may be NULL; XZ: x = 0).  MODE 2: w = A1 v with
// the K-cycle's partial sums (q = 0 w.w, 1 w.d1, 2 w.d2).  A workgroup
// takes L1_AGG consecutive aggregates and their members (an aggregate of two
// matching passes has at most four): L1_MPT members per thread for the
// products, their loads in flight together (the kernel waits on its
// gathers), then one thread per aggregate sums its members' products from
// LDS in the fixed order ((p0 + p2) + (p1 + p3)).
constexpr int L1_G = 4;                          // members of an aggregate, at most
constexpr int L1_MPT = 2;                        // members per thread
constexpr int L1_AGG = TPB * L1_MPT / L1_G;      // aggregates per workgroup
static_assert(TPB / L1_AGG == L1_LANES, "workgroups per aggregate count");
template <int DIM, typename T, int MODE, bool XZ, int ND>
__global__ void __launch_bounds__(TPB) k_l1(GridDims gd, int64_t n1, const int32_t* __restrict__ mptr,
                                            const int32_t* __restrict__ nagg, const T* __restrict__ mtq,
                                            const T* __restrict__ x, const T* __restrict__ b,
                                            const T* __restrict__ dinv1, const int32_t* __restrict__ agg2,
                                            const T* __restrict__ ec, T omega, T* __restrict__ out,
                                            const T* __restrict__ d1, const T* __restrict__ d2,
                                            double* __restrict__ part) {
  __shared__ T pm[3][TPB * L1_MPT];  // member products, by member slot in the workgroup
  __shared__ double sh[(TPB / 64) * (ND + 1)];
  __shared__ double res[ND + 1];
  // XCD-contiguous aggregate ranges: the neighbour aggregates a member
  // gathers (ids near its own, one grid row and one grid plane away) are then
  // read by the same XCD, from its L2
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t I0 = (int64_t)blk * L1_AGG;
  const int64_t I1 = min(I0 + (int64_t)L1_AGG, n1);
  const int32_t qa = mptr[I0], qb = mptr[I1];  // the workgroup's members
  const int tid = (int)threadIdx.x;
  auto xv = [&](int64_t J) {
    V3<T> v = XZ ? V3<T>{T(0), T(0), T(0)} : ld3(x, J);
    if (MODE == 1 && ec) {
      const V3<T> e = ld3(ec, (int64_t)agg2[J]);
      v.x += e.x;
      v.y += e.y;
      v.z += e.z;
    }
    return v;
  };
  // the aggregate's own operands (threads 0..L1_AGG-1), issued before the member work
  const int64_t I = I0 + tid;
  const bool own = tid < L1_AGG && I < I1;
  int32_t m0 = 0, m1 = 0;
  V3<T> xI{T(0), T(0), T(0)}, bI{T(0), T(0), T(0)}, dd1{T(0), T(0), T(0)}, dd2{T(0), T(0), T(0)};
  if (own) {
    m0 = mptr[I];
    m1 = mptr[I + 1];
    xI = xv(I);
    if (MODE != 2) bI = ld3(b, I);
    if (MODE == 2 && ND >= 1) dd1 = ld3(d1, I);
    if (MODE == 2 && ND >= 2) dd2 = ld3(d2, I);
  }
  // L1_MPT members per thread: K_i sum_{j~i} x'_agg(j)
  {
    int32_t a[L1_MPT][6];
    int deg[L1_MPT];
    bool hv[L1_MPT];
#pragma unroll
    for (int mm = 0; mm < L1_MPT; ++mm) {
      const int32_t q = qa + tid + mm * TPB;
      hv[mm] = q < qb;
      const int64_t sq = q / SL, lq = q - sq * SL;
      deg[mm] = 0;
#pragma unroll
      for (int u = 0; u < 2 * DIM; ++u) {
        a[mm][u] = hv[mm] ? nagg[sq * 6 * SL + u * SL + lq] : -1;
        deg[mm] += a[mm][u] >= 0 ? 1 : 0;
      }
    }
    V3<T> v[L1_MPT][6];
#pragma unroll
    for (int mm = 0; mm < L1_MPT; ++mm)
#pragma unroll
      for (int u = 0; u < 2 * DIM; ++u) v[mm][u] = xv((int64_t)(a[mm][u] >= 0 ? a[mm][u] : 0));
#pragma unroll
    for (int mm = 0; mm < L1_MPT; ++mm) {
      const int32_t q = qa + tid + mm * TPB;
      V3<T> kx{T(0), T(0), T(0)};
      if (hv[mm]) {
        const B9<T> kb = node_K<T>(gd, mtq + 3 * (int64_t)q, deg[mm]);  // field in member order
        V3<T> sx{T(0), T(0), T(0)};
#pragma unroll
        for (int u = 0; u < 2 * DIM; ++u) {
          sx.x += a[mm][u] >= 0 ? v[mm][u].x : T(0);
          sx.y += a[mm][u] >= 0 ? v[mm][u].y : T(0);
          sx.z += a[mm][u] >= 0 ? v[mm][u].z : T(0);
        }
        const V3<T> p = mv9(kb, sx);
        kx = V3<T>{T(0) + p.x, T(0) + p.y, T(0) + p.z};
      }
      pm[0][tid + mm * TPB] = kx.x;
      pm[1][tid + mm * TPB] = kx.y;
      pm[2][tid + mm * TPB] = kx.z;
    }
  }
  __syncthreads();
  double dots[ND + 1];
#pragma unroll
  for (int q = 0; q <= ND; ++q) dots[q] = 0.0;
  if (own) {
    // the member sums in the fixed order ((p0 + p2) + (p1 + p3)), absent members 0
    V3<T> p[L1_G];
#pragma unroll
    for (int k = 0; k < L1_G; ++k) {
      const bool h = m0 + k < m1;
      const int sl = h ? m0 + k - qa : 0;
      p[k] = h ? V3<T>{pm[0][sl], pm[1][sl], pm[2][sl]} : V3<T>{T(0), T(0), T(0)};
    }
    const V3<T> acc{(p[0].x + p[2].x) + (p[1].x + p[3].x), (p[0].y + p[2].y) + (p[1].y + p[3].y),
                    (p[0].z + p[2].z) + (p[1].z + p[3].z)};
    const T m = (T)(m1 - m0);
    const V3<T> ax{m * xI.x + acc.x, m * xI.y + acc.y, m * xI.z + acc.z};
    if (MODE == 0) {
      st3(out, I, V3<T>{bI.x - ax.x, bI.y - ax.y, bI.z - ax.z});
    } else if (MODE == 1) {
      const int64_t s1 = I / SL;
      const V3<T> d = dmv(dinv1, s1 * 9 * SL + (I - s1 * SL), V3<T>{bI.x - ax.x, bI.y - ax.y, bI.z - ax.z});
      st3(out, I, V3<T>{xI.x + omega * d.x, xI.y + omega * d.y, xI.z + omega * d.z});
    } else {
      st3(out, I, ax);
      const double w0 = ax.x, w1 = ax.y, w2 = ax.z;
      dots[0] = (w0 * w0 + w1 * w1) + w2 * w2;
      if (ND >= 1) dots[1 % (ND + 1)] = (w0 * (double)dd1.x + w1 * (double)dd1.y) + w2 * (double)dd1.z;
      if (ND >= 2) dots[2 % (ND + 1)] = (w0 * (double)dd2.x + w1 * (double)dd2.y) + w2 * (double)dd2.z;
    }
  }
  if (MODE == 2) {
    block_sums<ND + 1>(dots, sh, res);
    if (threadIdx.x <= ND) part[(int64_t)threadIdx.x * gridDim.x + blk] = res[threadIdx.x];
  }
}

// nagg[q][t] = agg(t-th grid neighbour of mem[q]) or -1 ([slice][6][64])
template <int DIM>
__global__ void k_member_nbr_aggs(int nx, int ny, int nz, const int32_t* __restrict__ mem,
                                  const int32_t* __restrict__ agg, int32_t* __restrict__ nagg) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (q >= N) return;
  const Nbrs<DIM> nb = nbrs<DIM>(nx, ny, nz, mem[q]);
  const int64_t sq = q / SL, lq = q - sq * SL;
  int u = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t)
    if (nbr_used(DIM, t)) nagg[sq * 6 * SL + (u++) * SL + lq] = nb.h[t] ? agg[nb.q[t]] : -1;
}

// mtq[q] = mt[mem[q]]: the frozen field in the member order of the aggregates
// (rounded to T: FP32 in the FP32-AMG form, where the level-1 products are FP32)
template <typename T>
__global__ void k_member_fields(int64_t n, const int32_t* __restrict__ mem, const double* __restrict__ mt,
                                T* __restrict__ mtq) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t i = mem[q];
#pragma unroll
  for (int c = 0; c < 3; ++c) mtq[3 * q + c] = (T)mt[3 * i + c];
}

// rho = r - a1 w1, x = omega D^{-1} rho (first sweep of the second inner
// cycle, when x != NULL); part[blk] = w1 . rho
template <typename T>
__global__ void k_kc_update(int64_t n, const T* __restrict__ r, const T* __restrict__ w1,
                            const double* __restrict__ kc, T* __restrict__ rho, const T* __restrict__ dinv,
                            T omega, T* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  __shared__ double res[1];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    const T a1 = (T)kc[0];
    const V3<T> ri = ld3(r, i), wi = ld3(w1, i);
    const V3<T> p{ri.x - a1 * wi.x, ri.y - a1 * wi.y, ri.z - a1 * wi.z};
    st3(rho, i, p);
    acc = ((double)wi.x * p.x + (double)wi.y * p.y) + (double)wi.z * p.z;
    if (x) {
      const int64_t s = i / SL;
      const V3<T> d = dmv(dinv, s * 9 * SL + (i - s * SL), p);
      st3(x, i, V3<T>{omega * d.x, omega * d.y, omega * d.z});
    }
  }
  block_sums<1>(&acc, sh, res);
  if (threadIdx.x == 0) part[blockIdx.x] = res[0];
}

template <typename T>
__global__ void k_kc_combine(int64_t n, const T* __restrict__ v1, const T* __restrict__ v2,
                             const double* __restrict__ kc, T* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  const T c1 = (T)kc[2], c2 = (T)kc[3];
  e[i] = c1 * v1[i] + c2 * v2[i];
}

// ------------------------------------------------------------- scalar work
// One wavefront sums nparts partials in a fixed order (lane-strided sums,
// four independent accumulators, then a shuffle tree); valid in lane 0.
// Sum of nparts partial sums by one wave.  Sixteen loads per lane are in
// flight at once (a vector reduction leaves 1024 partials: one round trip),
// added in a fixed tree, so the result is reproducible.
__device__ inline double wave_sum(const double* __restrict__ part, int64_t nparts) {
  const int lane = threadIdx.x & 63;
  double a[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) a[u] = 0.0;
  for (int64_t k0 = 0; k0 < nparts; k0 += 1024) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t k = k0 + 64 * u + lane;
      v[u] = k < nparts ? part[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] += v[u];
  }
#pragma unroll
  for (int w = 8; w > 0; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) a[u] += a[u + w];
  double r = a[0];
  for (int off = 32; off > 0; off >>= 1) r += __shfl_down(r, off, 64);
  return r;
}

// Sums of NQ columns of n partial sums each (column q at part + q ld) by the
// whole workgroup (TPB-multiple size): every thread loads its entries of all
// columns before the first add; lanes, then waves, are added in a fixed
// tree.  The totals land in tot[0..NQ) (shared), valid after the call.
template <int NQ>
__device__ inline void group_sums(const double* __restrict__ part, int64_t ld, int64_t n, double* tot) {
  __shared__ double ws[32][NQ];
  const int nt = (int)blockDim.x, nw = nt >> 6, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double a[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) a[q][u] = 0.0;
  for (int64_t k0 = 0; k0 < n; k0 += 4 * (int64_t)nt) {
    double v[NQ][4];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t k = k0 + (int64_t)u * nt + threadIdx.x;
        v[q][u] = k < n ? part[q * ld + k] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) a[q][u] += v[q][u];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double r = (a[q][0] + a[q][1]) + (a[q][2] + a[q][3]);
    for (int off = 32; off > 0; off >>= 1) r += __shfl_down(r, off, 64);
    if (lane == 0) ws[wv][q] = r;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += ws[w][threadIdx.x];
    tot[threadIdx.x] = r;
  }
  __syncthreads();
}

// K-cycle coefficients from the partial sums of one workgroup per block.
// Stage 1: a1 = (w1.r)/(w1.w1) from w1.w1 and w1.r.  Stage 3: the weights of
// e = a1 v1 + a2 (v2 - gamma v1), gamma = (w1.w2)/(w1.w1),
// a2 = (w2'.rho)/(w2'.w2') with w2' = w2 - gamma w1, from w2.w2, w2.w1,
// w2.rho (part, G per column) and w1.rho (part2, G2 partials that the update
// of rho wrote; summed here rather than in a launch of its own).
__global__ void k_kc_coef(const double* part, int64_t G, int stage, double* kc, const double* part2, int64_t G2) {
  __shared__ double s[3];
  __shared__ double s2[1];
  if (stage == 1) {
    group_sums<2>(part, G, G, s);
  } else {
    group_sums<3>(part, G, G, s);
    __syncthreads();
    group_sums<1>(part2, G2, G2, s2);
  }
  if (threadIdx.x != 0) return;
  if (stage == 1) {
    kc[1] = s[0];
    kc[0] = s[1] / s[0];
  } else {
    const double w1rho = s2[0];
    kc[4] = w1rho;
    const double w11 = kc[1], w22 = s[0], w12 = s[1], w2r = s[2];
    const double gamma = w12 / w11;
    const double num = w2r - gamma * w1rho;
    const double den = (w22 - 2.0 * gamma * w12) + gamma * gamma * w11;
    const double a2 = num / den;
    kc[2] = kc[0] - a2 * gamma;
    kc[3] = a2;
  }
}

__global__ void k_norm_finish(const double* part, int64_t nparts, int slot, double* sc, double* host) {
  const double s = wave_sum(part, nparts);
  if (threadIdx.x == 0) {
    const double v = sqrt(s);
    sc[slot] = v;
    sc[1] = 1.0 / v;
    if (host) host[slot] = v;
  }
}

// Pass-1 sums: hcol[q] = sum part[q] (q < nv), sc[5] = ||w||^2 (entry nv).
__global__ void k_dots_finish(const double* part, int64_t nparts, int nv, double* hcol, double* sc) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int q = wv; q <= nv; q += nw) {
    const double s = wave_sum(part + (int64_t)q * nparts, nparts);
    if ((threadIdx.x & 63) == 0) {
      if (q < nv)
        hcol[q] = s;
      else
        sc[5] = s;
    }
  }
}

// Pass-2 sums and the reorthogonalization test: the first classical
// Gram-Schmidt pass is kept when ||w'|| >= ||w|| / sqrt(2) (Kahan-Parlett
// "twice is enough"); otherwise the second-pass coefficients go to delta,
// are added to hcol, and sc[7] = 1 asks for the second update.
__global__ void k_reorth_finish(const double* part, int64_t nparts, int nv, double* hcol, double* delta,
                                double* sc) {
  __shared__ double s[MAXV_S + 1];
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int q = wv; q <= nv; q += nw) {
    const double v = wave_sum(part + (int64_t)q * nparts, nparts);
    if ((threadIdx.x & 63) == 0) s[q] = v;
  }
  __syncthreads();
  const bool again = !(s[nv] >= 0.5 * sc[5]);
  for (int q = threadIdx.x; q < nv; q += blockDim.x) {
    if (again) {
      delta[q] = s[q];
      hcol[q] += s[q];
    } else {
      delta[q] = 0.0;
    }
  }
  if (threadIdx.x == 0) sc[7] = again ? 1.0 : 0.0;
}

// New Hessenberg column, previous Givens rotations, the new rotation and the
// residual estimate.  The column and the rotations are staged in LDS so the
// serial part runs on one lane without global-memory round trips.
__global__ void k_arnoldi_finish(const double* part, int64_t nparts, int j, int R, KrylovScalars ks,
                                 double* host) {
  __shared__ double col[MAXV_S + 2], c_s[MAXV_S], s_s[MAXV_S];
  const double s = wave_sum(part + (int64_t)(j + 1) * nparts, nparts);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    col[i] = ks.hcol[i];
    if (i < j) {
      c_s[i] = ks.cs[i];
      s_s[i] = ks.sn[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(s);
    col[j + 1] = hn;
    const double wnorm0 = sqrt(ks.sc[5]);
    const int breakdown = hn <= 1e-14 * wnorm0 ? 1 : 0;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], c = col[i + 1];
      col[i] = c_s[i] * a + s_s[i] * c;
      col[i + 1] = -s_s[i] * a + c_s[i] * c;
    }
    const double a = col[j], c = col[j + 1];
    const double rho = hypot(a, c);
    const double cj = a / rho, sj = c / rho;
    ks.cs[j] = cj;
    ks.sn[j] = sj;
    col[j] = rho;
    col[j + 1] = 0.0;
    const double gj = ks.g[j];
    ks.g[j + 1] = -sj * gj;
    ks.g[j] = cj * gj;
    const double est = fabs(sj * gj);
    ks.sc[3] = est;
    ks.sc[4] = hn;
    ks.sc[1] = 1.0 / hn;
    host[3] = est;
    host[6] = (double)breakdown;
    host[7] += ks.sc[7];  // second Gram-Schmidt passes in this solve
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) ks.H[i * R + j] = col[i];
}

// Final column `col` (unrotated, rows 0..jj+1) of the Hessenberg matrix:
// the previous rotations, a new one, the rotated column into H and the
// right-hand side g updated.  Returns the residual estimate |g_{jj+1}|.
// One thread.
__device__ inline double givens_column(double* col, int jj, int R, KrylovScalars ks) {
  for (int i = 0; i < jj; ++i) {
    const double a = col[i], c = col[i + 1];
    col[i] = ks.cs[i] * a + ks.sn[i] * c;
    col[i + 1] = -ks.sn[i] * a + ks.cs[i] * c;
  }
  const double a = col[jj], c = col[jj + 1];
  const double rho = hypot(a, c);
  const double cj = a / rho, sj = c / rho;
  ks.cs[jj] = cj;
  ks.sn[jj] = sj;
  col[jj] = rho;
  col[jj + 1] = 0.0;
  const double gj = ks.g[jj];
  ks.g[jj + 1] = -sj * gj;
  ks.g[jj] = cj * gj;
  for (int i = 0; i <= jj + 1; ++i) ks.H[i * R + jj] = col[i];
  return fabs(sj * gj);
}

// After the dots sweep of iteration j: s = V^T v~_j, nu = |v~_j - V s| (by
// Pythagoras), the coefficients of w against the final v_0..v_j, the final
// column j-1 (its last entries change with v~_j = V s + nu v_j), and the
// coefficients of the update sweep.
__global__ void k_dcgs_finish1(const double* part, int64_t nparts, int j, int R, KrylovScalars ks, double* host) {
  __shared__ double a[MAXV_S + 1], b[MAXV_S + 1], e3[3], col[MAXV_S + 2];
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ns = 2 * j + 3;
  for (int q = wv; q < ns; q += nw) {
    const double v = wave_sum(part + (int64_t)q * nparts, nparts);
    if ((threadIdx.x & 63) == 0) {
      if (q < j)
        a[q] = v;
      else if (q < 2 * j)
        b[q - j] = v;
      else
        e3[q - 2 * j] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double h = ks.hs[j];
  double nu = 1.0, ss = 0.0;
  if (j > 0) {
    for (int q = 0; q < j; ++q) {
      a[q] /= h;  // s_q
      ss += a[q] * a[q];
    }
    const double nu2 = e3[0] / (h * h) - ss;
    nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
  }
  double st = 0.0;
  for (int q = 0; q < j; ++q) st += a[q] * b[q];
  const double hjj = nu > 0.0 ? (e3[1] / h - st) / nu : 0.0;
  if (j > 0) {  // column j-1 is final now
    for (int q = 0; q < j; ++q) col[q] = ks.hcol[q] + h * a[q];
    col[j] = h * nu;
    ks.sc[3] = givens_column(col, j - 1, R, ks);
    host[7] += 1.0;  // delayed second passes in this solve
  }
  for (int q = 0; q < j; ++q) ks.hcol[q] = b[q];
  ks.hcol[j] = hjj;
  // update sweep: v_j = u / (h nu) - V s / nu, w' = w - V (t - s hjj / nu) - u hjj / (h nu)
  const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
  for (int q = 0; q < j; ++q) {
    ks.coef[q] = a[q] * inv;
    ks.coef[j + q] = b[q] - a[q] * hjj * inv;
  }
  ks.coef[2 * j] = inv / h;
  ks.coef[2 * j + 1] = hjj * inv / h;
  ks.sc[5] = e3[2];  // ||w||^2
  ks.sc[8] = nu > 0.0 ? 0.0 : 1.0;
}

// After the update sweep: h_{j+1} = |w'|, the provisional column j (its
// first-pass entries) rotated by the final rotations for the residual
// estimate, and the breakdown test.
__global__ void k_dcgs_finish2(const double* part, int64_t nparts, int j, int R, KrylovScalars ks, double* host) {
  const double s = wave_sum(part, nparts);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(s);
  ks.hs[j + 1] = hn;
  ks.hinv[j + 1] = 1.0 / hn;  // slot j+1 times this is the next preconditioner input
  ks.sc[4] = hn;
  // rotation i changes entries i and i+1 of the column; only the running
  // entry (i+1, the next rotation's input) is needed, and entry j+1 = hn is
  // untouched by rotations 0..j-1
  double t = ks.hcol[0];
  for (int i = 0; i < j; ++i) t = -ks.sn[i] * t + ks.cs[i] * ks.hcol[i + 1];
  const double rho = hypot(t, hn);
  const double est = fabs(hn / rho * ks.g[j]);
  const int breakdown = (hn <= 1e-14 * sqrt(ks.sc[5]) || ks.sc[8] != 0.0) ? 1 : 0;
  ks.sc[9] = (double)breakdown;
  host[3] = est;
  host[6] = (double)breakdown;
}

// End of a cycle after k iterations: the last column (k-1) made final with
// the dots of slot k against v_0..v_{k-1} (part from k_dcgs_dots<k> with
// u = w = slot k); without correction after a breakdown.
__global__ void k_dcgs_last(const double* part, int64_t nparts, int k, int R, KrylovScalars ks, double* host) {
  __shared__ double a[MAXV_S + 1], uu[1], col[MAXV_S + 2];
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int q = wv; q <= k; q += nw) {
    const int idx = q < k ? q : 2 * k;
    const double v = wave_sum(part + (int64_t)idx * nparts, nparts);
    if ((threadIdx.x & 63) == 0) {
      if (q < k)
        a[q] = v;
      else
        uu[0] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double h = ks.hs[k];
  const int j = k - 1;
  if (ks.sc[9] != 0.0 || !(h > 0.0)) {
    for (int q = 0; q <= j; ++q) col[q] = ks.hcol[q];
    col[j + 1] = h;
  } else {
    double ss = 0.0;
    for (int q = 0; q < k; ++q) {
      a[q] /= h;
      ss += a[q] * a[q];
    }
    const double nu2 = uu[0] / (h * h) - ss;
    for (int q = 0; q <= j; ++q) col[q] = ks.hcol[q] + h * a[q];
    col[j + 1] = h * (nu2 > 0.0 ? sqrt(nu2) : 0.0);
    host[7] += 1.0;
  }
  ks.sc[3] = givens_column(col, j, R, ks);
  host[3] = ks.sc[3];
}

__global__ void k_cycle_start(int R, KrylovScalars ks) {
  for (int i = threadIdx.x; i <= R; i += blockDim.x) ks.g[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    ks.g[0] = ks.sc[0];
    ks.sc[1] = 1.0 / ks.sc[0];
    ks.hs[0] = 1.0;  // v_0 = r / beta is final
    ks.hinv[0] = 1.0;
    ks.sc[9] = 0.0;
  }
}

// y = H(0:k, 0:k)^{-1} g(0:k), upper triangular back substitution
__global__ void k_solve_y(int k, int R, KrylovScalars ks) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = ks.g[i];
    for (int q = i + 1; q < k; ++q) s -= ks.H[i * R + q] * ks.y[q];
    ks.y[i] = s / ks.H[i * R + i];
  }
}

// ------------------------------------------------------ fused coarse cycle
// The rows of one level of the fused cycle, G lanes per row as in the level
// kernels; f(i, s, l, a0, a1, a2) runs on the group's first lane with the row
// product sum_j A_ij x_j, x in LDS.
template <int G, typename T, typename F>
__device__ inline void tail_rows_g(const TailLevel<T>& L, const T* x, F f) {
  constexpr int R = TAIL_T / G;  // rows per pass
  const int sub = (int)(threadIdx.x % G);
  for (int i0 = 0; i0 < L.n; i0 += R) {
    const int i = i0 + (int)(threadIdx.x / G);
    if (i >= L.n) break;  // the lanes of a group share i
    const int s = i / SL, l = i - s * SL;
    const int64_t cb = L.sl[s];
    const int w = (int)((L.sl[s + 1] - cb) / SL);
    T a0 = 0, a1 = 0, a2 = 0;
    sell_row_mv_g<G>(L.col, L.val, cb, w, l, sub, [&](int32_t c) { return ld3(x, (int64_t)c); }, a0, a1, a2);
    if (sub == 0) f(i, s, l, a0, a1, a2);
  }
}
template <typename T, typename F>
__device__ inline void tail_rows(const TailLevel<T>& L, const T* x, F f) {
  if (L.G == 16)
    tail_rows_g<16>(L, x, f);
  else if (L.G == 8)
    tail_rows_g<8>(L, x, f);
  else
    tail_rows_g<1>(L, x, f);
}

// y = x + omega D^{-1} (b - A x), the damped block-Jacobi sweep
template <typename T>
__device__ inline void tail_sweep(const TailLevel<T>& L, const T* b, const T* x, T* y, T om) {
  tail_rows(L, x, [&](int i, int s, int l, T a0, T a1, T a2) {
    const V3<T> xi = ld3(x, (int64_t)i);
    const V3<T> bi = ld3(b, (int64_t)i);
    V3<T> res{bi.x - a0, bi.y - a1, bi.z - a2};
    res = dmv(L.dinv, (int64_t)s * 9 * SL + l, res);
    st3(y, (int64_t)i, V3<T>{xi.x + om * res.x, xi.y + om * res.y, xi.z + om * res.z});
  });
}

// bc_I = sum of r_i over the members of aggregate I, ascending
template <typename T>
__device__ inline V3<T> tail_restrict_row(const int32_t* mptr, const int32_t* mem, const T* r, int I) {
  T a0 = 0, a1 = 0, a2 = 0;
  for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
    const V3<T> v = ld3(r, (int64_t)mem[q]);
    a0 += v.x;
    a1 += v.y;
    a2 += v.z;
  }
  return V3<T>{a0, a1, a2};
}

// The V-cycle of levels s..L-1 (Sec. 3) in one workgroup: restriction of the
// residual of level s-1, then per level the first pre-smoothing sweep from
// x = 0, further pre-sweeps, residual and restriction; the exact solve on the
// coarsest level; per level upwards the prolongation of the correction and
// the post-smoothing sweeps.  Between the steps a workgroup barrier stands
// where the per-level path has a kernel boundary.
template <typename T>
__global__ void __launch_bounds__(TAIL_T) k_tail(const TailArgs<T> a, const T* __restrict__ rab,
                                                 const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                                                 T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  auto vec = [&](int32_t off) { return (T*)(tail_lds + off); };
  const int tid = (int)threadIdx.x;
  const T om = a.omega;
  const bool xz = a.nu_pre == 0;  // no pre-smoothing: x = 0
  // after nu_pre - 1 further pre-sweeps x sits in the level's ox (even count) or oy
  const bool xswap = a.nu_pre >= 2 && (a.nu_pre - 1) % 2 == 1;
  // restriction onto tail level kn, with that level's first pre-smoothing
  // sweep from x = 0, x = omega D^{-1} b, taken by the thread that formed b
  // (as the per-level restriction kernel does)
  auto restrict_to = [&](int kn, const int32_t* mp, const int32_t* me, const T* r) {
    const TailLevel<T>& N = a.lv[kn];
    T* Bn = vec(N.ob);
    T* Xn = vec(N.ox);
    for (int I = tid; I < N.n; I += TAIL_T) {
      const V3<T> b = tail_restrict_row(mp, me, r, I);
      st3(Bn, (int64_t)I, b);
      if (!xz) {
        const int s = I / SL, l = I - s * SL;
        const V3<T> d = dmv(N.dinv, (int64_t)s * 9 * SL + l, b);
        st3(Xn, (int64_t)I, V3<T>{om * d.x, om * d.y, om * d.z});
      }
    }
  };
  restrict_to(0, mptr, mem, rab);
  __syncthreads();
  for (int k = 0; k < a.nlev; ++k) {
    const TailLevel<T>& L = a.lv[k];
    const T* B = vec(L.ob);
    T* X = vec(L.ox);
    T* Y = vec(L.oy);
    for (int q = 1; q < a.nu_pre; ++q) {
      tail_sweep(L, B, X, Y, om);
      __syncthreads();
      T* t = X;
      X = Y;
      Y = t;
    }
    const T* rs = B;
    if (!xz) {
      tail_rows(L, X, [&](int i, int, int, T a0, T a1, T a2) {
        const V3<T> bi = ld3(B, (int64_t)i);
        st3(Y, (int64_t)i, V3<T>{bi.x - a0, bi.y - a1, bi.z - a2});
      });
      __syncthreads();
      rs = Y;
    }
    if (k + 1 < a.nlev) {
      restrict_to(k + 1, L.mptr, L.mem, rs);
    } else {
      double* bd = (double*)(tail_lds + a.obd);
      for (int I = tid; I < a.nc; I += TAIL_T) {
        const V3<T> v = tail_restrict_row(L.mptr, L.mem, rs, I);
        bd[3 * I] = (double)v.x;
        bd[3 * I + 1] = (double)v.y;
        bd[3 * I + 2] = (double)v.z;
      }
    }
    __syncthreads();
  }
  {
    // coarsest: e = A_c^{-1} b, one wave per row, unfused multiply-add as in
    // the standalone coarsest solve
#pragma clang fp contract(off)
    const double* bd = (const double*)(tail_lds + a.obd);
    T* E = vec(a.oe);
    const int nd = 3 * a.nc;
    const int lane = tid & 63, wv = tid >> 6;
    for (int row = wv; row < nd; row += TAIL_T / 64) {
      double s = 0.0;
      for (int c = lane; c < nd; c += 64) s += a.inv[(int64_t)row * nd + c] * bd[c];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if (lane == 0) E[row] = (T)s;
    }
  }
  __syncthreads();
  int32_t eo = a.oe;  // LDS offset of the correction of the level below
  for (int k = a.nlev - 1; k >= 0; --k) {
    const TailLevel<T>& L = a.lv[k];
    const T* B = vec(L.ob);
    T* X = vec(xswap ? L.oy : L.ox);
    T* Y = vec(xswap ? L.ox : L.oy);
    const T* ec = vec(eo);
    for (int i = tid; i < L.n; i += TAIL_T) {
      V3<T> xi = xz ? V3<T>{T(0), T(0), T(0)} : ld3((const T*)X, (int64_t)i);
      const V3<T> e = ld3(ec, (int64_t)L.agg[i]);
      xi.x += e.x;
      xi.y += e.y;
      xi.z += e.z;
      st3(X, (int64_t)i, xi);
    }
    __syncthreads();
    for (int q = 0; q < a.nu_post; ++q) {
      tail_sweep(L, B, X, Y, om);
      __syncthreads();
      T* t = X;
      X = Y;
      Y = t;
    }
    eo = (int32_t)((unsigned char*)X - tail_lds);
    if (k == 0)
      for (int i = tid; i < 3 * L.n; i += TAIL_T) out[i] = X[i];
  }
}

}  // namespace

// ------------------------------------------------------------- launchers
template <typename T>
void launch_smooth_first(hipStream_t st, Sell A, const T* dinv, double omega, const T* b, T* x) {
  if (A.n > 0) hipLaunchKernelGGL((k_smooth_first<T>), dim3(nblk(A.n)), dim3(TPB), 0, st, A.n, dinv, (T)omega, b, x);
}

template <typename T>
void launch_residual(hipStream_t st, Sell A, const T* val, int xmode, double omega, const T* b,
                     const T* x, T* r, int G) {
  if (A.n <= 0) return;
  const int64_t nt = A.n * G;
  const int tb = tpb_rows(A.n);
  const dim3 g(nblk(nt, tb)), t(tb);
  const T om = (T)omega;
#define LLG_RS(XM, GG) \
  hipLaunchKernelGGL((k_residual<T, XM, GG>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, om, b, x, r)
#define LLG_RSG(GG)                      \
  if (xmode == 0) LLG_RS(0, GG);         \
  else if (xmode == 1) LLG_RS(1, GG);    \
  else LLG_RS(2, GG);
  if (G == 16) {
    LLG_RSG(16)
  } else if (G == 8) {
    LLG_RSG(8)
  } else {
    LLG_RSG(1)
  }
#undef LLG_RSG
#undef LLG_RS
}

template <typename T>
void launch_restrict(hipStream_t st, int64_t nc, const int32_t* mptr, const int32_t* mem, const T* r, T* bc,
                     const T* cdinv, double omega, T* xc) {
  const int tb = tpb_rows(nc);
  if (nc > 0)
    hipLaunchKernelGGL((k_restrict<T>), dim3(nblk(nc, tb)), dim3(tb), 0, st, nc, mptr, mem, r, bc, cdinv,
                       (T)omega, xc);
}

template <typename T>
void launch_post_smooth(hipStream_t st, Sell A, const T* val, const T* dinv, int unit, int xmode,
                        double omega, const T* b, const T* x, const int32_t* agg, const T* ec, T* out, int G) {
  if (A.n <= 0) return;
  const int64_t nt = A.n * G;
  const int tb = tpb_rows(A.n);
  const dim3 g(nblk(nt, tb)), t(tb);
  const T om = (T)omega;
#define LLG_PS(XM, U, GG)                                                                                   \
  hipLaunchKernelGGL((k_post_smooth<T, XM, U, GG>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, dinv, om, b, x, \
                     agg, ec, out)
#define LLG_PSG(GG)                                \
  if (unit) {                                      \
    if (xmode == 0) LLG_PS(0, true, GG);           \
    else if (xmode == 1) LLG_PS(1, true, GG);      \
    else LLG_PS(2, true, GG);                      \
  } else {                                         \
    if (xmode == 0) LLG_PS(0, false, GG);          \
    else if (xmode == 1) LLG_PS(1, false, GG);     \
    else LLG_PS(2, false, GG);                     \
  }
  if (G == 16) {
    LLG_PSG(16)
  } else if (G == 8) {
    LLG_PSG(8)
  } else {
    LLG_PSG(1)
  }
#undef LLG_PSG
#undef LLG_PS
}

template <typename T>
void launch_prolong(hipStream_t st, int64_t n, int xmode, double omega, const T* b, const T* x,
                    const int32_t* agg, const T* ec, T* out) {
  if (n <= 0) return;
  const int tb = tpb_rows(n);
  const dim3 g(nblk(n, tb)), t(tb);
  if (xmode == 0)
    hipLaunchKernelGGL((k_prolong<T, 0>), g, t, 0, st, n, (T)omega, b, x, agg, ec, out);
  else if (xmode == 1)
    hipLaunchKernelGGL((k_prolong<T, 1>), g, t, 0, st, n, (T)omega, b, x, agg, ec, out);
  else
    hipLaunchKernelGGL((k_prolong<T, 2>), g, t, 0, st, n, (T)omega, b, x, agg, ec, out);
}

// the large-level products on the CSR-ordered copy: G = CSR_G lanes per row
template <typename T>
void launch_residual_csr(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const T* vt, int xmode,
                         double omega, const T* b, const T* x, T* r) {
  if (n <= 0) return;
  const int tb = tpb_rows(n);
  const dim3 g(nblk(n * CSR_G, tb)), t(tb);
  const T om = (T)omega;
  if (xmode == 0)
    hipLaunchKernelGGL((k_residual_csr<T, 0, CSR_G>), g, t, 0, st, n, rp, ci, vt, om, b, x, r);
  else if (xmode == 1)
    hipLaunchKernelGGL((k_residual_csr<T, 1, CSR_G>), g, t, 0, st, n, rp, ci, vt, om, b, x, r);
  else
    hipLaunchKernelGGL((k_residual_csr<T, 2, CSR_G>), g, t, 0, st, n, rp, ci, vt, om, b, x, r);
}

template <typename T>
void launch_post_smooth_csr(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const T* vt,
                            const T* dinv, int xmode, double omega, const T* b, const T* x, T* out) {
  if (n <= 0) return;
  const int tb = tpb_rows(n);
  const dim3 g(nblk(n * CSR_G, tb)), t(tb);
  const T om = (T)omega;
  if (xmode == 0)
    hipLaunchKernelGGL((k_post_smooth_csr<T, 0, CSR_G>), g, t, 0, st, n, rp, ci, vt, dinv, om, b, x, out);
  else if (xmode == 1)
    hipLaunchKernelGGL((k_post_smooth_csr<T, 1, CSR_G>), g, t, 0, st, n, rp, ci, vt, dinv, om, b, x, out);
  else
    hipLaunchKernelGGL((k_post_smooth_csr<T, 2, CSR_G>), g, t, 0, st, n, rp, ci, vt, dinv, om, b, x, out);
}

template <typename T>
void launch_tail(hipStream_t st, const TailArgs<T>& a, const T* rabove, const int32_t* mptr, const int32_t* mem,
                 T* out) {
  hipLaunchKernelGGL((k_tail<T>), dim3(1), dim3(TAIL_T), (size_t)a.lds, st, a, rabove, mptr, mem, out);
}
template void launch_tail<double>(hipStream_t, const TailArgs<double>&, const double*, const int32_t*,
                                  const int32_t*, double*);
template void launch_tail<float>(hipStream_t, const TailArgs<float>&, const float*, const int32_t*, const int32_t*,
                                 float*);

bool tail_prepare() {
  const bool ok = hipFuncSetAttribute((const void*)k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      TAIL_LDS) == hipSuccess &&
                  hipFuncSetAttribute((const void*)k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      TAIL_LDS) == hipSuccess;
  (void)hipGetLastError();
  return ok;
}

template <typename T>
void launch_gs_sweep(hipStream_t st, Sell C, const int32_t* rows, const T* cval, const T* cdinv, int unit,
                     int first, const T* b, T* x, int G) {
  if (C.n <= 0) return;
  if (first) G = 1;
  const int64_t nt = C.n * G;
  const int tb = tpb_rows(C.n);
  const dim3 g(nblk(nt, tb)), t(tb);
#define LLG_GS(U, F, GG) \
  hipLaunchKernelGGL((k_gs_sweep<T, U, F, GG>), g, t, 0, st, C.n, rows, C.sl_ptr, C.col, cval, cdinv, b, x)
#define LLG_GSG(GG)                 \
  if (unit) {                       \
    if (first) LLG_GS(true, true, GG); \
    else LLG_GS(true, false, GG);   \
  } else {                          \
    if (first) LLG_GS(false, true, GG); \
    else LLG_GS(false, false, GG);  \
  }
  if (G == 16) {
    LLG_GSG(16)
  } else if (G == 8) {
    LLG_GSG(8)
  } else {
    LLG_GSG(1)
  }
#undef LLG_GSG
#undef LLG_GS
}

template <typename T>
void launch_fill(hipStream_t st, T* p, int64_t n) {
  if (n > 0) hipLaunchKernelGGL((k_fill_zero<T>), dim3(nblk(n)), dim3(TPB), 0, st, p, n);
}

template <typename T>
void launch_scale_in(hipStream_t st, int64_t n, const double* dinv0, int left_scale, const double* v,
                     const double* vs, T* b0) {
  if (n > 0)
    hipLaunchKernelGGL((k_scale_in<T>), dim3(nblk(n)), dim3(TPB), 0, st, n, dinv0, left_scale, v, vs, b0);
}
template <typename T>
void launch_scale_in_grid(hipStream_t st, GridDims g, const double* v, const double* vs, T* b0) {
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  if (g.nz > 1)
    hipLaunchKernelGGL((k_scale_in_grid<3, T>), dim3(nblk(N)), dim3(TPB), 0, st, g, v, vs, b0);
  else
    hipLaunchKernelGGL((k_scale_in_grid<2, T>), dim3(nblk(N)), dim3(TPB), 0, st, g, v, vs, b0);
}
template void launch_scale_in_grid<double>(hipStream_t, GridDims, const double*, const double*, double*);
template void launch_scale_in_grid<float>(hipStream_t, GridDims, const double*, const double*, float*);

#define LLG_INST(T)                                                                                         \
  template void launch_smooth_first<T>(hipStream_t, Sell, const T*, double, const T*, T*);                  \
  template void launch_residual<T>(hipStream_t, Sell, const T*, int, double, const T*, const T*, T*, int); \
  template void launch_restrict<T>(hipStream_t, int64_t, const int32_t*, const int32_t*, const T*, T*,     \
                                   const T*, double, T*);                                                   \
  template void launch_post_smooth<T>(hipStream_t, Sell, const T*, const T*, int, int, double, const T*,   \
                                      const T*, const int32_t*, const T*, T*, int);                         \
  template void launch_prolong<T>(hipStream_t, int64_t, int, double, const T*, const T*, const int32_t*,   \
                                  const T*, T*);                                                            \
  template void launch_residual_csr<T>(hipStream_t, int64_t, const int32_t*, const int32_t*, const T*, int,  \
                                       double, const T*, const T*, T*);                                     \
  template void launch_post_smooth_csr<T>(hipStream_t, int64_t, const int32_t*, const int32_t*, const T*,   \
                                          const T*, int, double, const T*, const T*, T*);                   \
  template void launch_scale_in<T>(hipStream_t, int64_t, const double*, int, const double*, const double*, \
                                   T*);                                                                     \
  template void launch_gs_sweep<T>(hipStream_t, Sell, const int32_t*, const T*, const T*, int, int, const T*, \
                                   T*, int);                                                                \
  template void launch_fill<T>(hipStream_t, T*, int64_t);
LLG_INST(double)
LLG_INST(float)
#undef LLG_INST

template <typename TZ>
void launch_spmv_outer(hipStream_t st, Sell A, const double* val, const TZ* z, double* w, hipEvent_t e0,
                       hipEvent_t e1) {
  if (A.n <= 0) return;
  const int tb = tpb_rows(A.n);
  if (e0)
    hipExtLaunchKernelGGL((k_spmv_outer<TZ>), dim3(nblk(A.n, tb)), dim3(tb), 0, st, e0, e1, 0, A.n, A.sl_ptr, A.col,
                          val, z, w);
  else
    hipLaunchKernelGGL((k_spmv_outer<TZ>), dim3(nblk(A.n, tb)), dim3(tb), 0, st, A.n, A.sl_ptr, A.col, val, z, w);
}
template void launch_spmv_outer<double>(hipStream_t, Sell, const double*, const double*, double*, hipEvent_t,
                                        hipEvent_t);
template void launch_spmv_outer<float>(hipStream_t, Sell, const double*, const float*, double*, hipEvent_t,
                                       hipEvent_t);

void launch_resid_outer(hipStream_t st, Sell A, const double* val, const double* b, const double* u,
                        double* r, double* part) {
  hipLaunchKernelGGL(k_resid_outer, dim3(nblk(A.n)), dim3(TPB), 0, st, A.n, A.sl_ptr, A.col, val, b, u, r, part);
}

// workgroups of the grid-level stencil kernels (the node order of grid_pos)
inline unsigned grid_blocks(const GridDims& g) {
  if (g.nz <= 1) return nblk((int64_t)g.nx * g.ny);
  return 8u * nblk((int64_t)((g.ny + 7) / 8) * g.nx * g.nz);
}

template <typename TZ>
void launch_fact_outer(hipStream_t st, GridDims g, const TZ* z, double* w, hipEvent_t e0, hipEvent_t e1) {
  if (e0 && g.nz > 1)
    hipExtLaunchKernelGGL((k_fact_outer<3, TZ>), dim3(grid_blocks(g)), dim3(TPB), 0, st, e0, e1, 0, g, z, w);
  else if (e0)
    hipExtLaunchKernelGGL((k_fact_outer<2, TZ>), dim3(grid_blocks(g)), dim3(TPB), 0, st, e0, e1, 0, g, z, w);
  else if (g.nz > 1)
    hipLaunchKernelGGL((k_fact_outer<3, TZ>), dim3(grid_blocks(g)), dim3(TPB), 0, st, g, z, w);
  else
    hipLaunchKernelGGL((k_fact_outer<2, TZ>), dim3(grid_blocks(g)), dim3(TPB), 0, st, g, z, w);
}
template void launch_fact_outer<double>(hipStream_t, GridDims, const double*, double*, hipEvent_t, hipEvent_t);
template void launch_fact_outer<float>(hipStream_t, GridDims, const float*, double*, hipEvent_t, hipEvent_t);

void launch_fact_resid_outer(hipStream_t st, GridDims g, const double* b, const double* u, double* r, double* part) {
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  if (g.nz > 1)
    hipLaunchKernelGGL(k_fact_resid_outer<3>, dim3(nblk(N)), dim3(TPB), 0, st, g, b, u, r, part);
  else
    hipLaunchKernelGGL(k_fact_resid_outer<2>, dim3(nblk(N)), dim3(TPB), 0, st, g, b, u, r, part);
}

template <typename T>
void launch_fact_residual(hipStream_t st, GridDims g, int xmode, double omega, const T* b, const T* x, T* r) {
  const dim3 gr(grid_blocks(g)), t(TPB);
#define LLG_FR(D, XM) hipLaunchKernelGGL((k_fact_residual<D, T, XM>), gr, t, 0, st, g, (T)omega, b, x, r)
#define LLG_FRD(D)        \
  if (xmode == 0)         \
    LLG_FR(D, 0);         \
  else if (xmode == 1)    \
    LLG_FR(D, 1);         \
  else                    \
    LLG_FR(D, 2);
  if (g.nz > 1) {
    LLG_FRD(3)
  } else {
    LLG_FRD(2)
  }
#undef LLG_FRD
#undef LLG_FR
}

template <typename T>
void launch_fact_post_smooth(hipStream_t st, GridDims g, int xmode, double omega, const T* b, const T* x,
                             const int32_t* agg, const T* ec, T* out) {
  const dim3 gr(grid_blocks(g)), t(TPB);
#define LLG_FP(D, XM)                                                                                          \
  if (ec)                                                                                                        \
    hipLaunchKernelGGL((k_fact_post_smooth<D, T, XM, true>), gr, t, 0, st, g, (T)omega, b, x, agg, ec, out);    \
  else                                                                                                           \
    hipLaunchKernelGGL((k_fact_post_smooth<D, T, XM, false>), gr, t, 0, st, g, (T)omega, b, x, agg, ec, out)
#define LLG_FPD(D)        \
  if (xmode == 0)         \
    LLG_FP(D, 0);         \
  else if (xmode == 1)    \
    LLG_FP(D, 1);         \
  else                    \
    LLG_FP(D, 2);
  if (g.nz > 1) {
    LLG_FPD(3)
  } else {
    LLG_FPD(2)
  }
#undef LLG_FPD
#undef LLG_FP
}
template void launch_fact_residual<double>(hipStream_t, GridDims, int, double, const double*, const double*, double*);
template void launch_fact_residual<float>(hipStream_t, GridDims, int, double, const float*, const float*, float*);
template void launch_fact_post_smooth<double>(hipStream_t, GridDims, int, double, const double*, const double*,
                                              const int32_t*, const double*, double*);
template void launch_fact_post_smooth<float>(hipStream_t, GridDims, int, double, const float*, const float*,
                                             const int32_t*, const float*, float*);

int64_t red_blocks(int64_t m) { return std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, ceil_div(m, TPB * 4))); }

void launch_norm_part(hipStream_t st, int64_t m, const double* x, double* part) {
  hipLaunchKernelGGL(k_norm_part, dim3((unsigned)red_blocks(m)), dim3(TPB), 0, st, m, x, part);
}

#define LLG_NV_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

void launch_mdot(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* w,
                 double* part) {
  const dim3 g((unsigned)red_blocks(m)), t(TPB);
  switch (nv) {
#define X(K) \
  case K: hipLaunchKernelGGL((k_mdot<K>), g, t, 0, st, m, V, ldv, w, part); break;
    LLG_NV_CASES(X)
#undef X
    default: break;
  }
}

void launch_mupdate_dot(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* h,
                        double* w, double* part, int want_dots, const double* skip) {
  const dim3 g((unsigned)red_blocks(m)), t(TPB);
  switch (nv) {
#define X(K) \
  case K: hipLaunchKernelGGL((k_mupdate_dot<K>), g, t, 0, st, m, V, ldv, h, w, part, want_dots, skip); break;
    LLG_NV_CASES(X)
#undef X
    default: break;
  }
}

#define LLG_NV0_CASES(X) X(0) LLG_NV_CASES(X)

void launch_dcgs_dots(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* u,
                      const double* w, double* part) {
  const dim3 g((unsigned)red_blocks(m)), t(TPB);
  switch (nv) {
#define X(K) \
  case K: hipLaunchKernelGGL((k_dcgs_dots<K>), g, t, 0, st, m, V, ldv, u, w, part); break;
    LLG_NV0_CASES(X)
#undef X
    default: break;
  }
}

void launch_dcgs_update(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* coef,
                        double* u, const double* w, double* wo, double* part) {
  const dim3 g((unsigned)red_blocks(m)), t(TPB);
  switch (nv) {
#define X(K) \
  case K: hipLaunchKernelGGL((k_dcgs_update<K>), g, t, 0, st, m, V, ldv, coef, u, w, wo, part); break;
    LLG_NV0_CASES(X)
#undef X
    default: break;
  }
}

void launch_dcgs_finish1(hipStream_t st, const double* part, int64_t nparts, int j, int R, KrylovScalars ks,
                         double* host) {
  hipLaunchKernelGGL(k_dcgs_finish1, dim3(1), dim3(1024), 0, st, part, nparts, j, R, ks, host);
}
void launch_dcgs_finish2(hipStream_t st, const double* part, int64_t nparts, int j, int R, KrylovScalars ks,
                         double* host) {
  hipLaunchKernelGGL(k_dcgs_finish2, dim3(1), dim3(64), 0, st, part, nparts, j, R, ks, host);
}
void launch_dcgs_last(hipStream_t st, const double* part, int64_t nparts, int k, int R, KrylovScalars ks,
                      double* host) {
  hipLaunchKernelGGL(k_dcgs_last, dim3(1), dim3(1024), 0, st, part, nparts, k, R, ks, host);
}

void launch_scale_vec(hipStream_t st, int64_t m, const double* x, const double* s, double* y) {
  if (m > 0) hipLaunchKernelGGL(k_scale_vec, dim3(nblk(m)), dim3(TPB), 0, st, m, x, s, y);
}
template <typename TS, typename TD>
void launch_cast(hipStream_t st, int64_t m, const TS* x, TD* y) {
  if (m > 0) hipLaunchKernelGGL((k_cast<TS, TD>), dim3(nblk(m)), dim3(TPB), 0, st, m, x, y);
}
template void launch_cast<float, double>(hipStream_t, int64_t, const float*, double*);
template void launch_cast<double, double>(hipStream_t, int64_t, const double*, double*);

template <typename TZ>
void launch_zy(hipStream_t st, int64_t m, int k, const TZ* Z, int64_t ldz, const double* y, double* u) {
  if (m > 0 && k > 0) hipLaunchKernelGGL((k_zy<TZ>), dim3(nblk(m)), dim3(TPB), 0, st, m, k, Z, ldz, y, u);
}
template void launch_zy<double>(hipStream_t, int64_t, int, const double*, int64_t, const double*, double*);
template void launch_zy<float>(hipStream_t, int64_t, int, const float*, int64_t, const double*, double*);

void launch_project(hipStream_t st, int64_t n, const double* u, double* out, int project, int32_t* flag) {
  if (n > 0) hipLaunchKernelGGL(k_project, dim3(nblk(n)), dim3(TPB), 0, st, n, u, out, project, flag);
}

void launch_norm_finish_n(hipStream_t st, const double* part, int64_t nparts, int slot, double* sc,
                          double* host) {
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(64), 0, st, part, nparts, slot, sc, host);
}
void launch_dots_finish_n(hipStream_t st, const double* part, int64_t nparts, int nv, double* hcol, double* sc) {
  hipLaunchKernelGGL(k_dots_finish, dim3(1), dim3(1024), 0, st, part, nparts, nv, hcol, sc);
}
void launch_reorth_finish_n(hipStream_t st, const double* part, int64_t nparts, int nv, double* hcol,
                            double* delta, double* sc) {
  hipLaunchKernelGGL(k_reorth_finish, dim3(1), dim3(1024), 0, st, part, nparts, nv, hcol, delta, sc);
}
void launch_arnoldi_finish_n(hipStream_t st, const double* part, int64_t nparts, int j, int R,
                             KrylovScalars ks, double* host) {
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, st, part, nparts, j, R, ks, host);
}
void launch_cycle_start(hipStream_t st, int R, KrylovScalars ks) {
  hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(64), 0, st, R, ks);
}
void launch_solve_y(hipStream_t st, int k, int R, KrylovScalars ks) {
  hipLaunchKernelGGL(k_solve_y, dim3(1), dim3(64), 0, st, k, R, ks);
}

template <typename T>
void launch_spmv_dots(hipStream_t st, Sell A, const T* val, const T* v, T* w, const T* d1, const T* d2,
                      double* part, int G) {
  const dim3 g(nblk(A.n * G)), t(TPB);
#define LLG_SD(ND, GG) \
  hipLaunchKernelGGL((k_spmv_dots<T, ND, GG>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, v, w, d1, d2, part)
#define LLG_SDG(GG)     \
  if (d2) LLG_SD(2, GG); \
  else LLG_SD(1, GG);
  if (G == 16) {
    LLG_SDG(16)
  } else if (G == 8) {
    LLG_SDG(8)
  } else {
    LLG_SDG(1)
  }
#undef LLG_SDG
#undef LLG_SD
}
template <typename T>
void launch_kc_update(hipStream_t st, int64_t n, const T* r, const T* w1, const double* kc, T* rho,
                      const T* dinv, double omega, T* x, double* part) {
  hipLaunchKernelGGL((k_kc_update<T>), dim3(nblk(n)), dim3(TPB), 0, st, n, r, w1, kc, rho, dinv, (T)omega, x,
                     part);
}
template <typename T>
void launch_kc_combine(hipStream_t st, int64_t n, const T* v1, const T* v2, const double* kc, T* e) {
  hipLaunchKernelGGL((k_kc_combine<T>), dim3(nblk(3 * n)), dim3(TPB), 0, st, n, v1, v2, kc, e);
}
void launch_kc_coef(hipStream_t st, const double* part, int64_t G, int stage, double* kc, const double* part2,
                    int64_t G2) {
  hipLaunchKernelGGL(k_kc_coef, dim3(1), dim3(1024), 0, st, part, G, stage, kc, part2, G2);
}
int64_t rows_blocks(int64_t n, int G) { return ceil_div(n > 0 ? n * G : 1, TPB); }

void launch_member_nbr_aggs(hipStream_t st, GridDims g, const int32_t* mem, const int32_t* agg, int32_t* nagg) {
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  if (g.nz > 1)
    hipLaunchKernelGGL(k_member_nbr_aggs<3>, dim3(nblk(N)), dim3(TPB), 0, st, g.nx, g.ny, g.nz, mem, agg, nagg);
  else
    hipLaunchKernelGGL(k_member_nbr_aggs<2>, dim3(nblk(N)), dim3(TPB), 0, st, g.nx, g.ny, g.nz, mem, agg, nagg);
}

template <typename T>
void launch_member_fields(hipStream_t st, int64_t n, const int32_t* mem, const double* mt, T* mtq) {
  if (n > 0) hipLaunchKernelGGL((k_member_fields<T>), dim3(nblk(n)), dim3(TPB), 0, st, n, mem, mt, mtq);
}
template void launch_member_fields<double>(hipStream_t, int64_t, const int32_t*, const double*, double*);
template void launch_member_fields<float>(hipStream_t, int64_t, const int32_t*, const double*, float*);

template <typename T>
void launch_l1(hipStream_t st, GridDims g, int mode, int xzero, int64_t n1, const int32_t* mptr, const int32_t* nagg,
               const T* mtq, const T* x, const T* b, const T* dinv1, const int32_t* agg2, const T* ec,
               double omega, T* out, const T* d1, const T* d2, double* part, hipEvent_t e0, hipEvent_t e1) {
  if (n1 <= 0) return;
  const dim3 gr((unsigned)ceil_div(n1, L1_AGG)), t(TPB);
  const T om = (T)omega;
#define LLG_L1(D, M, XZ, ND)                                                                                      \
  hipExtLaunchKernelGGL((k_l1<D, T, M, XZ, ND>), gr, t, 0, st, e0, e1, 0, g, n1, mptr, nagg, mtq, x, b, dinv1, agg2, \
                        ec, om, out, d1, d2, part)
#define LLG_L1D(D)                                 \
  if (mode == 0) LLG_L1(D, 0, false, 0);           \
  else if (mode == 1 && xzero) LLG_L1(D, 1, true, 0); \
  else if (mode == 1) LLG_L1(D, 1, false, 0);      \
  else if (d2) LLG_L1(D, 2, false, 2);             \
  else LLG_L1(D, 2, false, 1);
  if (g.nz > 1) {
    LLG_L1D(3)
  } else {
    LLG_L1D(2)
  }
#undef LLG_L1D
#undef LLG_L1
}
template void launch_l1<double>(hipStream_t, GridDims, int, int, int64_t, const int32_t*, const int32_t*,
                                const double*, const double*, const double*, const double*, const int32_t*,
                                const double*, double, double*, const double*, const double*, double*, hipEvent_t,
                                hipEvent_t);
template void launch_l1<float>(hipStream_t, GridDims, int, int, int64_t, const int32_t*, const int32_t*,
                               const float*, const float*, const float*, const float*, const int32_t*, const float*,
                               double, float*, const float*, const float*, double*, hipEvent_t,
                               hipEvent_t);
#define LLG_INST_K(T)                                                                                    \
  template void launch_spmv_dots<T>(hipStream_t, Sell, const T*, const T*, T*, const T*, const T*, double*, int); \
  template void launch_kc_update<T>(hipStream_t, int64_t, const T*, const T*, const double*, T*, const T*, \
                                    double, T*, double*);                                                 \
  template void launch_kc_combine<T>(hipStream_t, int64_t, const T*, const T*, const double*, T*);
LLG_INST_K(double)
LLG_INST_K(float)
#undef LLG_INST_K

}  // namespace llg
