// k_field.hip -- the explicit field of the full model (Sec. 2): uniaxial
// anisotropy, a uniform external field and the stray field of the
// magnetization, entering the right-hand side of the scheme.
//
// The stray field is h = -N * m, the discrete convolution of m with the
// cell-averaged demagnetizing tensor of the grid's cubic cells (Newell,
// Williams and Dunlop 1993; the point-dipole tensor beyond 16 cells), taken as
// a cyclic convolution on the grid zero-padded to powers of two P >= 2n - 1
// per axis: forward FFTs of the three components, a pointwise product with
// the (real) transform of the tensor, inverse FFTs.  The FFTs are radix-2,
// one workgroup per line with the line in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "llg_internal.h"

namespace llg {

namespace {

constexpr int TPB = 256;
inline unsigned nblk(int64_t n, int t = TPB) { return (unsigned)ceil_div(n > 0 ? n : 1, t); }

// ------------------------------------------------------------ demag tensor
__device__ double newell_f(double x, double y, double z) {
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  if (R == 0.0) return 0.0;
  double r = 0.0;
  if (y > 0.0 && z2 != x2) r += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
  if (z > 0.0 && y2 != x2) r += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
  if (x > 0.0 && y > 0.0 && z > 0.0) r -= x * y * z * atan(y * z / (x * R));
  r += (2.0 * x2 - y2 - z2) * R / 6.0;
  return r;
}

__device__ double newell_g(double x, double y, double z) {
  const double sgn = (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) * (y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0));
  if (sgn == 0.0) return 0.0;
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double r = 0.0;
  if (z > 0.0) r += x * y * z * asinh(z / sqrt(x2 + y2));
  r += (y / 6.0) * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
  r += (x / 6.0) * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
  if (z > 0.0) {
    r -= (z2 * z / 6.0) * atan(x * y / (z * R));
    r -= (z * y2 / 2.0) * atan(x * z / (y * R));
    r -= (z * x2 / 2.0) * atan(y * z / (x * R));
  }
  r -= x * y * R / 3.0;
  return sgn * r;
}

// second difference over the 27 neighbouring corners, over 4 pi a b c
template <bool OFF>
__device__ double newell_sum(double X, double Y, double Z, double a, double b, double c) {
  const double w[3] = {-1.0, 2.0, -1.0};
  double acc = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        const double x = X + (i - 1) * a, y = Y + (j - 1) * b, z = Z + (k - 1) * c;
        acc += w[i] * w[j] * w[k] * (OFF ? newell_g(x, y, z) : newell_f(x, y, z));
      }
  return acc / (4.0 * M_PI * a * b * c);
}

// component comp (0..5: xx yy zz xy xz yz) between cells (X, Y, Z) apart
__device__ double demag(int comp, double X, double Y, double Z, double d) {
  const double far = fmax(fabs(X), fmax(fabs(Y), fabs(Z))) / d;
  if (far > 16.0) {
    const double r2 = X * X + Y * Y + Z * Z, r = sqrt(r2);
    const double k = -(d * d * d) / (4.0 * M_PI * r2 * r);
    switch (comp) {
      case 0: return k * (3.0 * X * X / r2 - 1.0);
      case 1: return k * (3.0 * Y * Y / r2 - 1.0);
      case 2: return k * (3.0 * Z * Z / r2 - 1.0);
      case 3: return k * 3.0 * X * Y / r2;
      case 4: return k * 3.0 * X * Z / r2;
      default: return k * 3.0 * Y * Z / r2;
    }
  }
  switch (comp) {
    case 0: return newell_sum<false>(X, Y, Z, d, d, d);
    case 1: return newell_sum<false>(Y, X, Z, d, d, d);
    case 2: return newell_sum<false>(Z, Y, X, d, d, d);
    case 3: return newell_sum<true>(X, Y, Z, d, d, d);
    case 4: return newell_sum<true>(X, Z, Y, d, d, d);
    default: return newell_sum<true>(Y, Z, X, d, d, d);
  }
}

// offset of padded index a along an axis of n cells padded to P (cyclic):
// a < n: +a; a > P - n: a - P; otherwise outside every cell pair (flag)
__device__ inline bool wrap(int64_t a, int64_t n, int64_t P, int64_t& off) {
  if (a < n) {
    off = a;
    return true;
  }
  if (a > P - n) {
    off = a - P;
    return true;
  }
  return false;
}

// components c0..c0+2 of the tensor on the padded grid, as complex values
__global__ void k_demag_grid(FieldDims f, int c0, double h, double2* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = f.px * f.py * f.pz;
  if (p >= P) return;
  const int64_t a = p % f.px, b = (p / f.px) % f.py, c = p / (f.px * f.py);
  int64_t X, Y, Z;
  const bool in = wrap(a, f.nx, f.px, X) && wrap(b, f.ny, f.py, Y) && wrap(c, f.nz, f.pz, Z);
  for (int k = 0; k < 3; ++k) {
    const double v = in ? demag(c0 + k, X * h, Y * h, Z * h, h) : 0.0;
    out[k * P + p] = make_double2(v, 0.0);
  }
}

// Nhat[c0 + k] = real part of the transformed component k
__global__ void k_take_real(int64_t P, int c0, const double2* in, double* nhat) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  for (int k = 0; k < 3; ++k) nhat[(c0 + k) * P + p] = in[k * P + p].x;
}

// ------------------------------------------------------------ FFT
__device__ inline unsigned bitrev(unsigned i, int bits) { return __brev(i) >> (32 - bits); }

// One radix-2 transform of length L = 2^bits per workgroup, of the line
// starting at base(line) with element stride s; dir = -1 forward, +1 inverse
// (then scaled by `scale`).  The line is held in LDS.
__global__ void k_fft_lines(double2* data, int bits, int64_t s, int64_t n_inner, int64_t inner_stride,
                            int64_t outer_stride, int dir, double scale) {
  extern __shared__ double2 sm[];
  const int64_t L = (int64_t)1 << bits;
  const int64_t line = blockIdx.x;
  const int64_t base = (line % n_inner) * inner_stride + (line / n_inner) * outer_stride;
  for (int64_t i = threadIdx.x; i < L; i += blockDim.x) sm[bitrev((unsigned)i, bits)] = data[base + i * s];
  __syncthreads();
  for (int64_t len = 2; len <= L; len <<= 1) {
    const int64_t half = len >> 1;
    for (int64_t q = threadIdx.x; q < L / 2; q += blockDim.x) {
      const int64_t g = q / half, k = q - g * half;
      const int64_t i = g * len + k, j = i + half;
      double sn, cs;
      sincospi((double)dir * 2.0 * (double)k / (double)len, &sn, &cs);
      const double2 v = sm[j], u = sm[i];
      const double2 t = make_double2(cs * v.x - sn * v.y, cs * v.y + sn * v.x);
      sm[i] = make_double2(u.x + t.x, u.y + t.y);
      sm[j] = make_double2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < L; i += blockDim.x) {
    const double2 v = sm[i];
    data[base + i * s] = make_double2(v.x * scale, v.y * scale);
  }
}

// ------------------------------------------------------------ field terms
// the three components of m~ (m^n, or 2 m^n - m^{n-1}) on the padded grid
__global__ void k_pad_field(FieldDims f, const double* m, const double* mprev, double2* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = f.px * f.py * f.pz;
  if (p >= P) return;
  const int64_t a = p % f.px, b = (p / f.px) % f.py, c = p / (f.px * f.py);
  const bool in = a < f.nx && b < f.ny && c < f.nz;
  const int64_t node = a + f.nx * (b + f.ny * c);
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    if (in) v = mprev ? 2.0 * m[3 * node + k] - mprev[3 * node + k] : m[3 * node + k];
    out[k * P + p] = make_double2(v, 0.0);
  }
}

// pointwise H = Nhat M (Nhat real, symmetric), in place
__global__ void k_demag_mul(int64_t P, const double* nhat, double2* w) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double xx = nhat[p], yy = nhat[P + p], zz = nhat[2 * P + p];
  const double xy = nhat[3 * P + p], xz = nhat[4 * P + p], yz = nhat[5 * P + p];
  const double2 a = w[p], b = w[P + p], c = w[2 * P + p];
  w[p] = make_double2(xx * a.x + xy * b.x + xz * c.x, xx * a.y + xy * b.y + xz * c.y);
  w[P + p] = make_double2(xy * a.x + yy * b.x + yz * c.x, xy * a.y + yy * b.y + yz * c.y);
  w[2 * P + p] = make_double2(xz * a.x + yz * b.x + zz * c.x, xz * a.y + yz * b.y + zz * c.y);
}

// h = -N * m: the physical part of the inverse transform, negated
__global__ void k_stray_out(FieldDims f, const double2* w, double* h) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = f.nx * f.ny * f.nz;
  if (node >= N) return;
  const int64_t P = f.px * f.py * f.pz;
  const int64_t a = node % f.nx, b = (node / f.nx) % f.ny, c = node / (f.nx * f.ny);
  const int64_t p = a + f.px * (b + f.py * c);
  for (int k = 0; k < 3; ++k) h[3 * node + k] = -w[k * P + p].x;
}

// b -= dt' (m~ x f + alpha m~ x (m~ x f)), f = (h_s + h_e) - q (0, m~2, m~3);
// prm: [0] alpha, [2] dt', [3] q, [4..6] h_e
__global__ void k_field_rhs(int64_t N, const double* prm, const double* m, const double* mprev, FieldDims f,
                            const double2* w, double* b) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const double alpha = prm[0], dtp = prm[2], q = prm[3];
  double x[3], hs[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3; ++k) x[k] = mprev ? 2.0 * m[3 * node + k] - mprev[3 * node + k] : m[3 * node + k];
  if (w) {
    const int64_t P = f.px * f.py * f.pz;
    const int64_t a = node % f.nx, bb = (node / f.nx) % f.ny, c = node / (f.nx * f.ny);
    const int64_t p = a + f.px * (bb + f.py * c);
    for (int k = 0; k < 3; ++k) hs[k] = -w[k * P + p].x;
  }
  const double fp[3] = {hs[0] + prm[4], (hs[1] + prm[5]) - q * x[1], (hs[2] + prm[6]) - q * x[2]};
  const double c1[3] = {x[1] * fp[2] - x[2] * fp[1], x[2] * fp[0] - x[0] * fp[2], x[0] * fp[1] - x[1] * fp[0]};
  const double c2[3] = {x[1] * c1[2] - x[2] * c1[1], x[2] * c1[0] - x[0] * c1[2], x[0] * c1[1] - x[1] * c1[0]};
  for (int k = 0; k < 3; ++k) b[3 * node + k] = b[3 * node + k] - dtp * (c1[k] + alpha * c2[k]);
}

int ilog2(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

// forward (dir -1) or inverse (+1, scaled by 1/P) transform of the three
// padded components, axis by axis
void fft3(hipStream_t st, FieldDims f, double2* w, int dir) {
  const int64_t P = f.px * f.py * f.pz;
  const double scale = dir > 0 ? 1.0 / (double)P : 1.0;
  for (int k = 0; k < 3; ++k) {
    double2* d = w + k * P;
    struct Axis {
      int64_t L, s, n_inner, inner_stride, outer_stride;
    } ax[3] = {{f.px, 1, f.py * f.pz, f.px, 0},      // lines along x: consecutive
               {f.py, f.px, f.px, 1, f.px * f.py},   // along y: start (x, z)
               {f.pz, f.px * f.py, f.px * f.py, 1, 0}};  // along z: start (x, y)
    int last = -1;  // the last transformed axis carries the inverse scaling
    for (int a = 0; a < 3; ++a)
      if (ax[a].L > 1) last = a;
    for (int a = 0; a < 3; ++a) {
      if (ax[a].L <= 1) continue;
      const int bits = ilog2(ax[a].L);
      const int64_t lines = P / ax[a].L;
      const int t = (int)std::min<int64_t>(256, std::max<int64_t>(64, ax[a].L / 2));
      hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)lines), dim3(t), ax[a].L * sizeof(double2), st, d, bits, ax[a].s,
                         ax[a].n_inner, ax[a].inner_stride, ax[a].outer_stride, dir, a == last ? scale : 1.0);
    }
  }
}

}  // namespace

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

FieldDims field_dims(int nx, int ny, int nz) {
  FieldDims f;
  f.nx = nx;
  f.ny = ny;
  f.nz = nz;
  f.px = next_pow2(2 * (int64_t)nx - 1);
  f.py = next_pow2(2 * (int64_t)ny - 1);
  f.pz = nz > 1 ? next_pow2(2 * (int64_t)nz - 1) : 1;
  return f;
}

void init_field_attributes() {
  (void)hipFuncSetAttribute((const void*)k_fft_lines, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(FFT_MAX_LEN * sizeof(double2)));
}

void launch_demag_setup(hipStream_t st, FieldDims f, double h, double2* work, double* nhat) {
  const int64_t P = f.px * f.py * f.pz;
  for (int c0 = 0; c0 < 6; c0 += 3) {
    hipLaunchKernelGGL(k_demag_grid, dim3(nblk(P)), dim3(TPB), 0, st, f, c0, h, work);
    fft3(st, f, work, -1);
    hipLaunchKernelGGL(k_take_real, dim3(nblk(P)), dim3(TPB), 0, st, P, c0, work, nhat);
  }
}

void launch_stray(hipStream_t st, FieldDims f, const double* m, const double* mprev, const double* nhat,
                  double2* work) {
  const int64_t P = f.px * f.py * f.pz;
  hipLaunchKernelGGL(k_pad_field, dim3(nblk(P)), dim3(TPB), 0, st, f, m, mprev, work);
  fft3(st, f, work, -1);
  hipLaunchKernelGGL(k_demag_mul, dim3(nblk(P)), dim3(TPB), 0, st, P, nhat, work);
  fft3(st, f, work, +1);
}

void launch_stray_out(hipStream_t st, FieldDims f, const double2* work, double* h) {
  const int64_t N = f.nx * f.ny * f.nz;
  hipLaunchKernelGGL(k_stray_out, dim3(nblk(N)), dim3(TPB), 0, st, f, work, h);
}

void launch_field_rhs(hipStream_t st, int64_t N, const double* prm, const double* m, const double* mprev,
                      FieldDims f, const double2* work, double* b) {
  hipLaunchKernelGGL(k_field_rhs, dim3(nblk(N)), dim3(TPB), 0, st, N, prm, m, mprev, f, work, b);
}

}  // namespace llg
