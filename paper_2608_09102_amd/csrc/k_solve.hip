// k_solve.hip -- solve-phase kernels: V-cycle level operations (damped block
// Jacobi, residual, restriction, prolongation), the FP64 outer block SpMV,
// the Gram-Schmidt passes of the Arnoldi step, the small FGMRES scalar work
// and the projection.  All of them are bound by HBM bandwidth: one thread per
// block row, one wavefront per 64-row slice, coalesced slot-major loads, and
// reductions in a fixed tree so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "llg_internal.h"

namespace llg {

namespace {

constexpr int TPB = 256;

inline unsigned nblk(int64_t n, int t = TPB) { return (unsigned)ceil_div(n > 0 ? n : 1, t); }

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; give each
// XCD a contiguous range of slices so that neighbouring rows (which share x
// entries) are served from the same L2.
__device__ inline unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned per = nb / 8, rem = nb % 8;
  const unsigned xcd = b % 8, k = b / 8;
  // blocks [0, 8*per) are spread evenly; the remainder keeps its index
  if (b < 8 * per) return xcd * per + k;
  (void)rem;
  return b;
}

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

template <typename T>
__device__ inline V3<T> dmv(const T* __restrict__ d, int64_t db, V3<T> v) {
  return V3<T>{d[db + 0 * SL] * v.x + d[db + 1 * SL] * v.y + d[db + 2 * SL] * v.z,
               d[db + 3 * SL] * v.x + d[db + 4 * SL] * v.y + d[db + 5 * SL] * v.z,
               d[db + 6 * SL] * v.x + d[db + 7 * SL] * v.y + d[db + 8 * SL] * v.z};
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
template <typename T, int XMODE>
__global__ void k_residual(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                           const T* __restrict__ val, T omega, const T* __restrict__ b,
                           const T* __restrict__ x, T* __restrict__ r) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = i / SL;
  const int l = (int)(i - s * SL);
  const int64_t cb = sl[s];
  const int w = (int)((sl[s + 1] - cb) / SL);
  T a0 = 0, a1 = 0, a2 = 0;
  for (int t = 0; t < w; ++t) {
    const int32_t c = col[cb + (int64_t)t * SL + l];
    if (c < 0) break;
    blk_mv(val, cb * 9 + (int64_t)t * 9 * SL + l, xval<T, XMODE>(x, b, omega, c), a0, a1, a2);
  }
  const V3<T> bi = ld3(b, i);
  st3(r, i, V3<T>{bi.x - a0, bi.y - a1, bi.z - a2});
}

// bc_I = sum of r_i over the members of aggregate I, ascending
template <typename T>
__global__ void k_restrict(int64_t nc, const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                           const T* __restrict__ r, T* __restrict__ bc) {
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
}

// out_i = x'_i + omega D_i^{-1} (b_i - sum_j A_ij x'_j), x'_j = xbase_j + ec[agg_j]
template <typename T, int XMODE, bool UNIT>
__global__ void k_post_smooth(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                              const T* __restrict__ val, const T* __restrict__ dinv, T omega,
                              const T* __restrict__ b, const T* __restrict__ x,
                              const int32_t* __restrict__ agg, const T* __restrict__ ec,
                              T* __restrict__ out) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = i / SL;
  const int l = (int)(i - s * SL);
  const int64_t cb = sl[s];
  const int w = (int)((sl[s + 1] - cb) / SL);
  T a0 = 0, a1 = 0, a2 = 0;
  for (int t = 0; t < w; ++t) {
    const int32_t c = col[cb + (int64_t)t * SL + l];
    if (c < 0) break;
    V3<T> xj = xval<T, XMODE>(x, b, omega, c);
    if (ec) {
      const V3<T> e = ld3(ec, (int64_t)agg[c]);
      xj.x += e.x;
      xj.y += e.y;
      xj.z += e.z;
    }
    blk_mv(val, cb * 9 + (int64_t)t * 9 * SL + l, xj, a0, a1, a2);
  }
  V3<T> xi = xval<T, XMODE>(x, b, omega, i);
  if (ec) {
    const V3<T> e = ld3(ec, (int64_t)agg[i]);
    xi.x += e.x;
    xi.y += e.y;
    xi.z += e.z;
  }
  const V3<T> bi = ld3(b, i);
  V3<T> res{bi.x - a0, bi.y - a1, bi.z - a2};
  if (!UNIT) res = dmv(dinv, s * 9 * SL + l, res);
  st3(out, i, V3<T>{xi.x + omega * res.x, xi.y + omega * res.y, xi.z + omega * res.z});
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
                           const double* __restrict__ v, T* __restrict__ b0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V3<double> x = ld3(v, i);
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
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = i / SL;
  const int l = (int)(i - s * SL);
  const int64_t cb = sl[s];
  const int wd = (int)((sl[s + 1] - cb) / SL);
  double a0 = 0, a1 = 0, a2 = 0;
  for (int t = 0; t < wd; ++t) {
    const int32_t c = col[cb + (int64_t)t * SL + l];
    if (c < 0) break;
    blk_mv(val, cb * 9 + (int64_t)t * 9 * SL + l, ld3(z, (int64_t)c), a0, a1, a2);
  }
  st3(w, i, V3<double>{a0, a1, a2});
}

// block sum of v over 256 threads, fixed tree; result valid in thread 0
__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
  }
  __syncthreads();
  return r;
}

__global__ void k_resid_outer(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                              const double* __restrict__ val, const double* __restrict__ b,
                              const double* __restrict__ u, double* __restrict__ r,
                              double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double nrm = 0;
  if (i < n) {
    const int64_t s = i / SL;
    const int l = (int)(i - s * SL);
    const int64_t cb = sl[s];
    const int wd = (int)((sl[s + 1] - cb) / SL);
    double a0 = 0, a1 = 0, a2 = 0;
    for (int t = 0; t < wd; ++t) {
      const int32_t c = col[cb + (int64_t)t * SL + l];
      if (c < 0) break;
      blk_mv(val, cb * 9 + (int64_t)t * 9 * SL + l, ld3(u, (int64_t)c), a0, a1, a2);
    }
    const V3<double> bi = ld3(b, i);
    const V3<double> ri{bi.x - a0, bi.y - a1, bi.z - a2};
    st3(r, i, ri);
    nrm = (ri.x * ri.x + ri.y * ri.y) + ri.z * ri.z;
  }
  const double t = block_sum(nrm, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// partial sums of x.x over a fixed grid of RED_BLOCKS-bounded blocks
__global__ void k_norm_part(int64_t m, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  double a = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    a += x[k] * x[k];
  const double t = block_sum(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

constexpr int MAXV = 33;  // restart <= 32, plus the squared norm

// part[i][blk] = V_i . w (i < nv), part[nv][blk] = w . w; one sweep over w and V
__global__ void __launch_bounds__(TPB) k_mdot(int64_t m, int nv, const double* __restrict__ V, int64_t ldv,
                                              const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  const int G = gridDim.x;
  double acc[MAXV];
#pragma unroll
  for (int q = 0; q < MAXV; ++q) acc[q] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    const double wk = w[k];
#pragma unroll
    for (int q = 0; q < MAXV; ++q) {
      if (q < nv) acc[q] += V[q * ldv + k] * wk;
    }
    acc[MAXV - 1] += wk * wk;
  }
  for (int q = 0; q < nv; ++q) {
    double t = 0;
#pragma unroll
    for (int r = 0; r < MAXV - 1; ++r)
      if (r == q) t = acc[r];
    t = block_sum(t, sh);
    if (threadIdx.x == 0) part[(int64_t)q * G + blockIdx.x] = t;
  }
  const double t = block_sum(acc[MAXV - 1], sh);
  if (threadIdx.x == 0) part[(int64_t)nv * G + blockIdx.x] = t;
}

// w -= sum_i h_i V_i, then (same sweep, V_i still in registers)
// part[i][blk] = V_i . w_new when want_dots, part[nv][blk] = w_new . w_new
__global__ void __launch_bounds__(TPB) k_mupdate_dot(int64_t m, int nv, const double* __restrict__ V,
                                                     int64_t ldv, const double* __restrict__ h,
                                                     double* __restrict__ w, double* __restrict__ part,
                                                     int want_dots) {
  __shared__ double sh[TPB / 64];
  __shared__ double hs[MAXV];
  if (threadIdx.x < MAXV) hs[threadIdx.x] = (int)threadIdx.x < nv ? h[threadIdx.x] : 0.0;
  __syncthreads();
  const int G = gridDim.x;
  double acc[MAXV];
#pragma unroll
  for (int q = 0; q < MAXV; ++q) acc[q] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    double v[MAXV - 1];
    double wk = w[k];
#pragma unroll
    for (int q = 0; q < MAXV - 1; ++q) {
      v[q] = q < nv ? V[q * ldv + k] : 0.0;
      wk -= hs[q] * v[q];
    }
    w[k] = wk;
    if (want_dots) {
#pragma unroll
      for (int q = 0; q < MAXV - 1; ++q) acc[q] += v[q] * wk;
    }
    acc[MAXV - 1] += wk * wk;
  }
  if (want_dots) {
    for (int q = 0; q < nv; ++q) {
      double t = 0;
#pragma unroll
      for (int r = 0; r < MAXV - 1; ++r)
        if (r == q) t = acc[r];
      t = block_sum(t, sh);
      if (threadIdx.x == 0) part[(int64_t)q * G + blockIdx.x] = t;
    }
  }
  const double t = block_sum(acc[MAXV - 1], sh);
  if (threadIdx.x == 0) part[(int64_t)nv * G + blockIdx.x] = t;
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

// ------------------------------------------------------------- scalar work
// Sum of nparts partials in a fixed order: strided per-thread sums, then a
// fixed tree over the workgroup.
__device__ inline double wg_sum(const double* part, int64_t nparts, double* sh) {
  double a = 0;
  for (int64_t k = threadIdx.x; k < nparts; k += blockDim.x) a += part[k];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void k_norm_finish(const double* part, int64_t nparts, int slot, double* sc, double* host) {
  __shared__ double sh[TPB];
  const double s = wg_sum(part, nparts, sh);
  if (threadIdx.x == 0) {
    const double v = sqrt(s);
    sc[slot] = v;
    sc[1] = 1.0 / v;
    if (host) host[slot] = v;
  }
}

__global__ void k_dots_finish(const double* part, int64_t nparts, int nv, double* hcol, double* delta,
                              int accumulate, double* normsq) {
  __shared__ double sh[TPB];
  for (int i = 0; i <= nv; ++i) {
    const double s = wg_sum(part + (int64_t)i * nparts, nparts, sh);
    if (threadIdx.x == 0) {
      if (i == nv) {
        if (normsq) *normsq = s;
      } else if (accumulate) {
        delta[i] = s;
        hcol[i] += s;
      } else {
        hcol[i] = s;
      }
    }
  }
}

__global__ void k_arnoldi_finish(const double* part, int64_t nparts, int j, int R, KrylovScalars ks,
                                 double* host) {
  __shared__ double sh[TPB];
  const double s = wg_sum(part + (int64_t)(j + 1) * nparts, nparts, sh);
  if (threadIdx.x != 0) return;
  double* H = ks.H;
  const double hn = sqrt(s);
  for (int i = 0; i <= j; ++i) H[i * R + j] = ks.hcol[i];
  H[(j + 1) * R + j] = hn;
  const double wnorm0 = sqrt(ks.sc[5]);
  const int breakdown = hn <= 1e-14 * wnorm0 ? 1 : 0;
  for (int i = 0; i < j; ++i) {
    const double a = H[i * R + j], c = H[(i + 1) * R + j];
    H[i * R + j] = ks.cs[i] * a + ks.sn[i] * c;
    H[(i + 1) * R + j] = -ks.sn[i] * a + ks.cs[i] * c;
  }
  const double a = H[j * R + j], c = H[(j + 1) * R + j];
  const double rho = hypot(a, c);
  ks.cs[j] = a / rho;
  ks.sn[j] = c / rho;
  H[j * R + j] = rho;
  H[(j + 1) * R + j] = 0.0;
  ks.g[j + 1] = -ks.sn[j] * ks.g[j];
  ks.g[j] = ks.cs[j] * ks.g[j];
  const double est = fabs(ks.g[j + 1]);
  ks.sc[3] = est;
  ks.sc[4] = hn;
  ks.sc[1] = 1.0 / hn;
  host[3] = est;
  host[6] = (double)breakdown;
}

__global__ void k_cycle_start(int R, KrylovScalars ks) {
  for (int i = threadIdx.x; i <= R; i += blockDim.x) ks.g[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    ks.g[0] = ks.sc[0];
    ks.sc[1] = 1.0 / ks.sc[0];
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

}  // namespace

// ------------------------------------------------------------- launchers
template <typename T>
void launch_smooth_first(hipStream_t st, Sell A, const T* dinv, double omega, const T* b, T* x) {
  if (A.n > 0) hipLaunchKernelGGL((k_smooth_first<T>), dim3(nblk(A.n)), dim3(TPB), 0, st, A.n, dinv, (T)omega, b, x);
}

template <typename T>
void launch_residual(hipStream_t st, Sell A, const T* val, int xmode, double omega, const T* b,
                     const T* x, T* r) {
  if (A.n <= 0) return;
  const dim3 g(nblk(A.n)), t(TPB);
  if (xmode == 0)
    hipLaunchKernelGGL((k_residual<T, 0>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, (T)omega, b, x, r);
  else if (xmode == 1)
    hipLaunchKernelGGL((k_residual<T, 1>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, (T)omega, b, x, r);
  else
    hipLaunchKernelGGL((k_residual<T, 2>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, (T)omega, b, x, r);
}

template <typename T>
void launch_restrict(hipStream_t st, int64_t nc, const int32_t* mptr, const int32_t* mem, const T* r, T* bc) {
  if (nc > 0) hipLaunchKernelGGL((k_restrict<T>), dim3(nblk(nc)), dim3(TPB), 0, st, nc, mptr, mem, r, bc);
}

template <typename T>
void launch_post_smooth(hipStream_t st, Sell A, const T* val, const T* dinv, int unit, int xmode,
                        double omega, const T* b, const T* x, const int32_t* agg, const T* ec, T* out) {
  if (A.n <= 0) return;
  const dim3 g(nblk(A.n)), t(TPB);
  const T om = (T)omega;
#define LLG_PS(XM, U)                                                                                  \
  hipLaunchKernelGGL((k_post_smooth<T, XM, U>), g, t, 0, st, A.n, A.sl_ptr, A.col, val, dinv, om, b, x, \
                     agg, ec, out)
  if (unit) {
    if (xmode == 0) LLG_PS(0, true);
    else if (xmode == 1) LLG_PS(1, true);
    else LLG_PS(2, true);
  } else {
    if (xmode == 0) LLG_PS(0, false);
    else if (xmode == 1) LLG_PS(1, false);
    else LLG_PS(2, false);
  }
#undef LLG_PS
}

template <typename T>
void launch_prolong(hipStream_t st, int64_t n, int xmode, double omega, const T* b, const T* x,
                    const int32_t* agg, const T* ec, T* out) {
  if (n <= 0) return;
  const dim3 g(nblk(n)), t(TPB);
  if (xmode == 0)
    hipLaunchKernelGGL((k_prolong<T, 0>), g, t, 0, st, n, (T)omega, b, x, agg, ec, out);
  else if (xmode == 1)
    hipLaunchKernelGGL((k_prolong<T, 1>), g, t, 0, st, n, (T)omega, b, x, agg, ec, out);
  else
    hipLaunchKernelGGL((k_prolong<T, 2>), g, t, 0, st, n, (T)omega, b, x, agg, ec, out);
}

template <typename T>
void launch_scale_in(hipStream_t st, int64_t n, const double* dinv0, int left_scale, const double* v, T* b0) {
  if (n > 0) hipLaunchKernelGGL((k_scale_in<T>), dim3(nblk(n)), dim3(TPB), 0, st, n, dinv0, left_scale, v, b0);
}

#define LLG_INST(T)                                                                                         \
  template void launch_smooth_first<T>(hipStream_t, Sell, const T*, double, const T*, T*);                  \
  template void launch_residual<T>(hipStream_t, Sell, const T*, int, double, const T*, const T*, T*);      \
  template void launch_restrict<T>(hipStream_t, int64_t, const int32_t*, const int32_t*, const T*, T*);    \
  template void launch_post_smooth<T>(hipStream_t, Sell, const T*, const T*, int, int, double, const T*,   \
                                      const T*, const int32_t*, const T*, T*);                              \
  template void launch_prolong<T>(hipStream_t, int64_t, int, double, const T*, const T*, const int32_t*,   \
                                  const T*, T*);                                                            \
  template void launch_scale_in<T>(hipStream_t, int64_t, const double*, int, const double*, T*);
LLG_INST(double)
LLG_INST(float)
#undef LLG_INST

template <typename TZ>
void launch_spmv_outer(hipStream_t st, Sell A, const double* val, const TZ* z, double* w) {
  if (A.n > 0)
    hipLaunchKernelGGL((k_spmv_outer<TZ>), dim3(nblk(A.n)), dim3(TPB), 0, st, A.n, A.sl_ptr, A.col, val, z, w);
}
template void launch_spmv_outer<double>(hipStream_t, Sell, const double*, const double*, double*);
template void launch_spmv_outer<float>(hipStream_t, Sell, const double*, const float*, double*);

void launch_resid_outer(hipStream_t st, Sell A, const double* val, const double* b, const double* u,
                        double* r, double* part) {
  hipLaunchKernelGGL(k_resid_outer, dim3(nblk(A.n)), dim3(TPB), 0, st, A.n, A.sl_ptr, A.col, val, b, u, r, part);
}

int64_t red_blocks(int64_t m) { return std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, ceil_div(m, TPB * 4))); }

void launch_norm_part(hipStream_t st, int64_t m, const double* x, double* part) {
  hipLaunchKernelGGL(k_norm_part, dim3((unsigned)red_blocks(m)), dim3(TPB), 0, st, m, x, part);
}
void launch_mdot(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* w,
                 double* part) {
  hipLaunchKernelGGL(k_mdot, dim3((unsigned)red_blocks(m)), dim3(TPB), 0, st, m, nv, V, ldv, w, part);
}
void launch_mupdate_dot(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv,
                        const double* h, double* w, double* part, int want_dots) {
  hipLaunchKernelGGL(k_mupdate_dot, dim3((unsigned)red_blocks(m)), dim3(TPB), 0, st, m, nv, V, ldv, h, w,
                     part, want_dots);
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
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(TPB), 0, st, part, nparts, slot, sc, host);
}
void launch_dots_finish_n(hipStream_t st, const double* part, int64_t nparts, int nv, double* hcol,
                          double* delta, int accumulate, double* normsq) {
  hipLaunchKernelGGL(k_dots_finish, dim3(1), dim3(TPB), 0, st, part, nparts, nv, hcol, delta, accumulate,
                     normsq);
}
void launch_arnoldi_finish_n(hipStream_t st, const double* part, int64_t nparts, int j, int R,
                             KrylovScalars ks, double* host) {
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(TPB), 0, st, part, nparts, j, R, ks, host);
}
void launch_cycle_start(hipStream_t st, int R, KrylovScalars ks) {
  hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(64), 0, st, R, ks);
}
void launch_solve_y(hipStream_t st, int k, int R, KrylovScalars ks) {
  hipLaunchKernelGGL(k_solve_y, dim3(1), dim3(64), 0, st, k, R, ks);
}

}  // namespace llg
