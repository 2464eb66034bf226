// k_krylov.hip -- vector and scalar kernels of the unpreconditioned Krylov
// baselines (BiCGstab, TFQMR) that the paper compares its multigrid solve
// against.  FP64 throughout; HBM-bound streaming kernels with partial sums in
// a fixed tree, and one-workgroup scalar steps that keep every coefficient on
// the device so an iteration replays as one graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "llg_internal.h"

namespace llg {

namespace {

constexpr int TPB = 256;

// Sum of NS per-thread values over the workgroup in a fixed order.
template <int NS>
__device__ inline void wg_sums(const double* v, double* sh, double* out) {
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

__device__ inline double coef(const KTerm& t) { return t.s * (t.c ? t.c[0] : 1.0); }

// y = sum of up to three terms s_i c_i x_i (y may be one of the x_i), with
// the partial sums of y.d0, y.d1 and y.y.
__global__ void __launch_bounds__(TPB) k_lin3(int64_t m, KTerm t0, KTerm t1, KTerm t2, double* y,
                                              const double* d0, const double* d1, double* part) {
  __shared__ double sh[(TPB / 64) * 3];
  __shared__ double res[3];
  const double a0 = coef(t0), a1 = t1.x ? coef(t1) : 0.0, a2 = t2.x ? coef(t2) : 0.0;
  double acc[3] = {0.0, 0.0, 0.0};
  const int G = gridDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    double v = a0 * t0.x[k];
    if (t1.x) v += a1 * t1.x[k];
    if (t2.x) v += a2 * t2.x[k];
    y[k] = v;
    if (d0) acc[0] += v * d0[k];
    if (d1) acc[1] += v * d1[k];
    acc[2] += v * v;
  }
  wg_sums<3>(acc, sh, res);
  if (threadIdx.x < 3) part[(int64_t)threadIdx.x * G + blockIdx.x] = res[threadIdx.x];
}

// partial sums of x0.y0 and x1.y1 (the second pair optional)
__global__ void __launch_bounds__(TPB) k_dot2(int64_t m, const double* x0, const double* y0, const double* x1,
                                              const double* y1, double* part) {
  __shared__ double sh[(TPB / 64) * 2];
  __shared__ double res[2];
  double acc[2] = {0.0, 0.0};
  const int G = gridDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)G * blockDim.x) {
    acc[0] += x0[k] * y0[k];
    if (x1) acc[1] += x1[k] * y1[k];
  }
  wg_sums<2>(acc, sh, res);
  if (threadIdx.x < 2) part[(int64_t)threadIdx.x * G + blockIdx.x] = res[threadIdx.x];
}

__global__ void k_copy(int64_t m, const double* x, double* y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) y[k] = x[k];
}

__global__ void k_scale_copy(int64_t m, const double* x, const double* s, double* y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) y[k] = s ? x[k] * s[0] : x[k];
}

__device__ inline double psum(const double* part, int64_t nparts, int q) {
  double a = 0.0;
  const int lane = threadIdx.x & 63;
  for (int64_t k = lane; k < nparts; k += 64) a += part[(int64_t)q * nparts + k];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  return a;
}

// One scalar step of a baseline on the state kb (see KB_* in the header).
// part holds the partial sums of the preceding vector kernel.
__global__ void k_kb_step(const double* part, int64_t nparts, int op, double* kb, double* host) {
  const double p0 = psum(part, nparts, 0);
  const double p1 = psum(part, nparts, 1);
  const double p2 = psum(part, nparts, 2);
  if (threadIdx.x != 0) return;
  auto bad = [&](double x) { return !(x == x) || isinf(x); };
  switch (op) {
    case KB_START:  // p0 = r.r^ (or r.rs), p1 = r.r: rho, tau and the flags
      kb[KB_RHO] = p0;
      kb[KB_TAU] = sqrt(p1);
      kb[KB_THETA] = 0.0;
      kb[KB_ETA] = 0.0;
      kb[KB_HALF] = 0.0;
      kb[KB_FLAG] = 0.0;
      kb[KB_MINB] = INFINITY;
      break;
    case KB_ALPHA: {  // p0 = v.r^
      const double a = kb[KB_RHO] / p0;
      if (p0 == 0.0 || bad(a)) kb[KB_FLAG] = 1.0;
      kb[KB_ALPHA] = kb[KB_FLAG] != 0.0 ? 0.0 : a;
      break;
    }
    case KB_OMEGA: {  // p0 = t.s, p1 = t.t
      const double w = p1 > 0.0 ? p0 / p1 : 0.0;
      if (bad(w) || w == 0.0) kb[KB_FLAG] = 1.0;
      kb[KB_OMEGA] = kb[KB_FLAG] != 0.0 ? 0.0 : w;
      break;
    }
    case KB_BICG_END: {  // after r = s - omega t: p0 = r.r^, p2 = r.r
      const double beta = (p0 / kb[KB_RHO]) * (kb[KB_ALPHA] / kb[KB_OMEGA]);
      if (p0 == 0.0 || bad(beta)) kb[KB_FLAG] = 1.0;
      kb[KB_BETA] = kb[KB_FLAG] != 0.0 ? 0.0 : beta;
      kb[KB_BW] = kb[KB_BETA] * kb[KB_OMEGA];
      kb[KB_RHO] = p0;
      host[3] = sqrt(p2);
      host[6] = kb[KB_FLAG];
      break;
    }
    case KB_TF_F:  // coefficient of d in d = u + (theta^2 / alpha) eta d
      kb[KB_F] = (kb[KB_THETA] * kb[KB_THETA] / kb[KB_ALPHA]) * kb[KB_ETA];
      break;
    case KB_TF_HALF: {  // after the w update: p2 = w.w
      const double theta = sqrt(p2) / kb[KB_TAU];
      const double c = 1.0 / sqrt(1.0 + theta * theta);
      kb[KB_THETA] = theta;
      kb[KB_TAU] = kb[KB_TAU] * theta * c;
      kb[KB_ETA] = c * c * kb[KB_ALPHA];
      kb[KB_HALF] += 1.0;
      // bound on the true residual after this half-step
      kb[KB_MINB] = fmin(kb[KB_MINB], kb[KB_TAU] * sqrt(kb[KB_HALF] + 1.0));
      break;
    }
    case KB_TF_END: {  // p0 = w.rs
      const double beta = p0 / kb[KB_RHO];
      if (bad(beta)) kb[KB_FLAG] = 1.0;
      kb[KB_BETA] = kb[KB_FLAG] != 0.0 ? 0.0 : beta;
      kb[KB_B2] = kb[KB_BETA] * kb[KB_BETA];
      kb[KB_RHO] = p0;
      host[3] = kb[KB_MINB];  // the smaller bound of the two half-steps
      host[6] = kb[KB_FLAG];
      kb[KB_MINB] = INFINITY;
      break;
    }
    default:
      break;
  }
}

}  // namespace

void launch_lin3(hipStream_t st, int64_t m, KTerm t0, KTerm t1, KTerm t2, double* y, const double* d0,
                 const double* d1, double* part) {
  hipLaunchKernelGGL(k_lin3, dim3((unsigned)red_blocks(m)), dim3(TPB), 0, st, m, t0, t1, t2, y, d0, d1, part);
}
void launch_dot2(hipStream_t st, int64_t m, const double* x0, const double* y0, const double* x1,
                 const double* y1, double* part) {
  hipLaunchKernelGGL(k_dot2, dim3((unsigned)red_blocks(m)), dim3(TPB), 0, st, m, x0, y0, x1, y1, part);
}
void launch_copy(hipStream_t st, int64_t m, const double* x, double* y) {
  if (m > 0) hipLaunchKernelGGL(k_copy, dim3((unsigned)ceil_div(m, TPB)), dim3(TPB), 0, st, m, x, y);
}
void launch_scale_copy(hipStream_t st, int64_t m, const double* x, const double* s, double* y) {
  if (m > 0) hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)ceil_div(m, TPB)), dim3(TPB), 0, st, m, x, s, y);
}
void launch_kb_step(hipStream_t st, const double* part, int64_t nparts, int op, double* kb, double* host) {
  hipLaunchKernelGGL(k_kb_step, dim3(1), dim3(64), 0, st, part, nparts, op, kb, host);
}

}  // namespace llg
