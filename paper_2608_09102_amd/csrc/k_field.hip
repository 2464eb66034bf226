// k_field.hip -- the explicit field of the full model (Sec. 2): uniaxial
// anisotropy, a uniform external field and the stray field of the
// magnetization, entering the right-hand side of the scheme.
//
// The stray field is h = -N * m, the discrete convolution of m with the
// cell-averaged demagnetizing tensor of the grid's cubic cells (Newell,
// Williams and Dunlop 1993; the point-dipole tensor beyond 16 cells), taken as
// a cyclic convolution on the grid zero-padded to powers of two P >= 2n - 1
// per axis.  The three real components travel as two complex planes
// (m1 + i m2, m3); the forward transform reads only the n-box and skips the
// lines that are zero, the product with the (real) transformed tensor
// separates the packed pair by conjugate symmetry, and the inverse transform
// writes only the n-box.  Line transforms are mixed-radix Stockham passes in
// registers and LDS, several lines per workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "llg.h"
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

// ------------------------------------------------------------ FFT
// Line transforms by a mixed-radix Stockham scheme: a line of L = 2^BITS
// complex values is held by T = L / 8 threads, eight values each.  The first
// pass (radix 2, 4 or 8, no twiddles) works on the values as loaded from HBM,
// the radix-8 passes after it exchange through LDS, and the last one stores
// straight to HBM in natural order.  C lines share a workgroup (512 threads);
// for strided lines the C lines are adjacent in memory and lanes run across
// them first, so that a row of C values is read together.
struct FftPass {
  int64_t n_inner, inner_stride, outer_stride, s, plane_stride;
  int n_load, n_store, dir;
  double scale;
};

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// times dir * i
__device__ inline double2 cmul_i(double2 a, double dir) { return make_double2(-dir * a.y, dir * a.x); }

// DFT of 2, 4 or 8 values with kernel exp(dir 2 pi i n k / R), in place
__device__ inline void dft4(double2& a0, double2& a1, double2& a2, double2& a3, double dir) {
  const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = cmul_i(csub(a1, a3), dir);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}
template <int R>
__device__ inline void dft(double2* v, double dir) {
  if constexpr (R == 2) {
    const double2 t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3], dir);
  } else {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3, dir);
    dft4(o0, o1, o2, o3, dir);
    const double r2 = 0.70710678118654752440;
    o1 = make_double2(r2 * (o1.x - dir * o1.y), r2 * (o1.y + dir * o1.x));     // (1 + dir i) / sqrt 2
    o2 = cmul_i(o2, dir);                                                       // dir i
    o3 = make_double2(r2 * (-o3.x - dir * o3.y), r2 * (-o3.y + dir * o3.x));   // (-1 + dir i) / sqrt 2
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  }
}

// v[r] *= w^r, w = exp(i pi th), for r = 1..7
__device__ inline void twiddle8(double2* v, double th) {
  double s1, c1, s2, c2, s4, c4;
  sincospi(th, &s1, &c1);
  sincospi(2.0 * th, &s2, &c2);
  sincospi(4.0 * th, &s4, &c4);
  const double2 w1 = make_double2(c1, s1), w2 = make_double2(c2, s2), w4 = make_double2(c4, s4);
  const double2 w3 = cmul(w1, w2);
  v[1] = cmul(v[1], w1);
  v[2] = cmul(v[2], w2);
  v[3] = cmul(v[3], w3);
  v[4] = cmul(v[4], w4);
  v[5] = cmul(v[5], cmul(w1, w4));
  v[6] = cmul(v[6], cmul(w2, w4));
  v[7] = cmul(v[7], cmul(w3, w4));
}

template <int BITS, bool CF>
__global__ __launch_bounds__(512) void k_fft(double2* __restrict__ data, FftPass p) {
  constexpr int L = 1 << BITS;
  constexpr int T = L >= 8 ? L / 8 : 1;  // threads per line
  constexpr int NR = L >= 8 ? 8 : L;     // values per thread
  constexpr int C = 512 / T;             // lines per workgroup
  constexpr int R0 = (BITS % 3 == 0) ? 8 : (1 << (BITS % 3));
  constexpr int NMID = BITS > 3 ? (BITS - (R0 == 8 ? 3 : BITS % 3)) / 3 - 1 : -1;  // radix-8 passes between
  constexpr int LP = L + (L >> 3);       // padded line in LDS
  __shared__ double2 sm[L >= 16 ? C * LP : 1];
  const int t = threadIdx.x;
  const int c = CF ? t % C : t / T;
  const int j = CF ? t / C : t % T;
  int64_t g = blockIdx.x;
  if (CF && (gridDim.x & 31) == 0) g = (g & ~(int64_t)31) | ((g & 7) << 2) | ((g >> 3) & 3);
  const int64_t gpo = (p.n_inner + C - 1) / C;
  const int64_t outer = g / gpo;
  const int64_t inner = (g - outer * gpo) * C + c;
  const bool live = inner < p.n_inner;
  double2* line = data + (int64_t)blockIdx.y * p.plane_stride + (live ? inner : 0) * p.inner_stride +
                  outer * p.outer_stride;
  const double dir = (double)p.dir;
  auto lds = [&](int i) -> double2& { return CF ? sm[(i + (i >> 3)) * C + c] : sm[c * LP + i + (i >> 3)]; };
  double2 v[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int i = j + q * T;
    v[q] = (live && i < p.n_load) ? line[(int64_t)i * p.s] : make_double2(0.0, 0.0);
  }
  if constexpr (L <= 8) {  // one pass
    dft<NR>(v, dir);
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (live && q < p.n_store) line[(int64_t)q * p.s] = make_double2(v[q].x * p.scale, v[q].y * p.scale);
    return;
  } else {
    // first pass: butterflies u of radix R0 on registers u + r (8 / R0)
    constexpr int U = 8 / R0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double2 w[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) w[r] = v[u + r * U];
      dft<R0>(w, dir);
      const int jj = j + u * T;
#pragma unroll
      for (int r = 0; r < R0; ++r) lds(jj * R0 + r) = w[r];
    }
    int ns = R0;
#pragma unroll
    for (int m = 0; m < NMID; ++m) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = lds(j + r * T);
      __syncthreads();
      const int k = j % ns;
      twiddle8(v, dir * 2.0 * (double)k / (double)(8 * ns));
      dft<8>(v, dir);
      const int d = (j / ns) * ns * 8 + k;
#pragma unroll
      for (int r = 0; r < 8; ++r) lds(d + r * ns) = v[r];
      ns *= 8;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = lds(j + r * T);
    twiddle8(v, dir * 2.0 * (double)j / (double)L);  // ns = L / 8 = T, so k = j
    dft<8>(v, dir);
    if (live) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = j + r * T;
        if (i < p.n_store) line[(int64_t)i * p.s] = make_double2(v[r].x * p.scale, v[r].y * p.scale);
      }
    }
  }
}

template <int BITS, bool CF>
void launch_fft_t(hipStream_t st, double2* data, const FftPass& p, int64_t n_outer, int planes) {
  constexpr int L = 1 << BITS;
  constexpr int T = L >= 8 ? L / 8 : 1;
  constexpr int C = 512 / T;
  const int64_t groups = ((p.n_inner + C - 1) / C) * n_outer;
  hipLaunchKernelGGL((k_fft<BITS, CF>), dim3((unsigned)groups, (unsigned)planes), dim3(512), 0, st, data, p);
}

template <bool CF>
void launch_fft_cf(hipStream_t st, int bits, double2* data, const FftPass& p, int64_t n_outer, int planes) {
  switch (bits) {
    case 1: return launch_fft_t<1, CF>(st, data, p, n_outer, planes);
    case 2: return launch_fft_t<2, CF>(st, data, p, n_outer, planes);
    case 3: return launch_fft_t<3, CF>(st, data, p, n_outer, planes);
    case 4: return launch_fft_t<4, CF>(st, data, p, n_outer, planes);
    case 5: return launch_fft_t<5, CF>(st, data, p, n_outer, planes);
    case 6: return launch_fft_t<6, CF>(st, data, p, n_outer, planes);
    case 7: return launch_fft_t<7, CF>(st, data, p, n_outer, planes);
    case 8: return launch_fft_t<8, CF>(st, data, p, n_outer, planes);
    case 9: return launch_fft_t<9, CF>(st, data, p, n_outer, planes);
    case 10: return launch_fft_t<10, CF>(st, data, p, n_outer, planes);
    case 11: return launch_fft_t<11, CF>(st, data, p, n_outer, planes);
    case 12: return launch_fft_t<12, CF>(st, data, p, n_outer, planes);
    default: throw LLG_ERR_UNSUPPORTED;  // lengths are checked when the context is created
  }
}

int ilog2(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

// One transform along one axis, lines (inner, outer) of `planes` planes of P
// values: elements i < n_load are read (the rest taken as zero), i < n_store
// written; the inverse pass that ends a transform is scaled by 1 / P.
void fft_axis(hipStream_t st, double2* data, int64_t P, int planes, int64_t L, int64_t s, int64_t n_inner,
              int64_t inner_stride, int64_t n_outer, int64_t outer_stride, int64_t n_load, int64_t n_store, int dir,
              double scale) {
  if (L <= 1) return;
  FftPass p;
  p.n_inner = n_inner;
  p.inner_stride = inner_stride;
  p.outer_stride = outer_stride;
  p.s = s;
  p.plane_stride = P;
  p.n_load = (int)n_load;
  p.n_store = (int)n_store;
  p.dir = dir;
  p.scale = scale;
  if (s == 1)
    launch_fft_cf<false>(st, ilog2(L), data, p, n_outer, planes);
  else
    launch_fft_cf<true>(st, ilog2(L), data, p, n_outer, planes);
}

// Forward transform of `planes` planes holding values on the n-box only (the
// rest of the padded grid is never read: zero by construction), every axis
// pruned to the lines that can hold nonzero values.
void fft_forward_box(hipStream_t st, FieldDims f, double2* w, int planes) {
  const int64_t P = f.px * f.py * f.pz, pxy = f.px * f.py;
  fft_axis(st, w, P, planes, f.px, 1, f.ny, f.px, f.nz, pxy, f.nx, f.px, -1, 1.0);
  fft_axis(st, w, P, planes, f.py, f.px, f.px, 1, f.nz, pxy, f.ny, f.py, -1, 1.0);
  fft_axis(st, w, P, planes, f.pz, pxy, pxy, 1, 1, 0, f.nz, f.pz, -1, 1.0);
}

// Inverse transform, scaled by 1 / P, of which only the n-box is written.
void fft_inverse_box(hipStream_t st, FieldDims f, double2* w, int planes) {
  const int64_t P = f.px * f.py * f.pz, pxy = f.px * f.py;
  const double sc = 1.0 / (double)P;
  const bool z = f.pz > 1;
  if (z) fft_axis(st, w, P, planes, f.pz, pxy, pxy, 1, 1, 0, f.pz, f.nz, +1, 1.0);
  fft_axis(st, w, P, planes, f.py, f.px, f.px, 1, f.nz, pxy, f.py, f.ny, +1, 1.0);
  fft_axis(st, w, P, planes, f.px, 1, f.ny, f.px, f.nz, pxy, f.px, f.nx, +1, sc);
}

// Forward transform of `planes` full padded planes.
void fft_forward_full(hipStream_t st, FieldDims f, double2* w, int planes) {
  const int64_t P = f.px * f.py * f.pz, pxy = f.px * f.py;
  fft_axis(st, w, P, planes, f.px, 1, f.py, f.px, f.pz, pxy, f.px, f.px, -1, 1.0);
  fft_axis(st, w, P, planes, f.py, f.px, f.px, 1, f.pz, pxy, f.py, f.py, -1, 1.0);
  fft_axis(st, w, P, planes, f.pz, pxy, pxy, 1, 1, 0, f.pz, f.pz, -1, 1.0);
}

// Two tensor components packed as one complex plane, a + i b: both are real
// and even up to rounding, so their transforms are real and the packed
// transform's real and imaginary parts are the two transforms.
__global__ void k_demag_grid2(FieldDims f, int c0, int c1, double h, double2* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = f.px * f.py * f.pz;
  if (p >= P) return;
  const int64_t a = p % f.px, b = (p / f.px) % f.py, c = p / (f.px * f.py);
  int64_t X, Y, Z;
  const bool in = wrap(a, f.nx, f.px, X) && wrap(b, f.ny, f.py, Y) && wrap(c, f.nz, f.pz, Z);
  double v0 = 0.0, v1 = 0.0;
  if (in) {
    v0 = demag(c0, X * h, Y * h, Z * h, h);
    v1 = demag(c1, X * h, Y * h, Z * h, h);
  }
  out[p] = make_double2(v0, v1);
}

__global__ void k_take_pair(int64_t P, int c0, int c1, const double2* in, double* nhat) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double2 v = in[p];
  nhat[c0 * P + p] = v.x;
  nhat[c1 * P + p] = v.y;
}

// ------------------------------------------------------------ field terms
// m~ (m^n, or 2 m^n - m^{n-1}) into two padded planes: m~1 + i m~2 and m~3,
// on the n-box only
__global__ void k_pad_field(FieldDims f, const double* m, const double* mprev, double2* out) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = f.nx * f.ny * f.nz;
  if (node >= N) return;
  const int64_t P = f.px * f.py * f.pz;
  const int64_t a = node % f.nx, b = (node / f.nx) % f.ny, c = node / (f.nx * f.ny);
  const int64_t p = a + f.px * (b + f.py * c);
  double x[3];
  for (int k = 0; k < 3; ++k) x[k] = mprev ? 2.0 * m[3 * node + k] - mprev[3 * node + k] : m[3 * node + k];
  out[p] = make_double2(x[0], x[1]);
  out[P + p] = make_double2(x[2], 0.0);
}

// The product H = Nhat M on the packed transforms.  Plane 0 holds
// Z = M1 + i M2, so M1(k) = (Z(k) + conj Z(-k)) / 2 and
// M2(k) = (Z(k) - conj Z(-k)) / 2i; plane 1 holds M3.  The result is packed
// the same way (H1 + i H2, H3); each thread does the pair k, -k.
__device__ inline void demag_apply(const double* nhat, int64_t P, int64_t p, double2 z, double2 zm, double2 m3,
                                   double2& o0, double2& o1) {
  const double2 m1 = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
  const double2 m2 = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
  const double xx = nhat[p], yy = nhat[P + p], zz = nhat[2 * P + p];
  const double xy = nhat[3 * P + p], xz = nhat[4 * P + p], yz = nhat[5 * P + p];
  const double2 h1 = make_double2(xx * m1.x + xy * m2.x + xz * m3.x, xx * m1.y + xy * m2.y + xz * m3.y);
  const double2 h2 = make_double2(xy * m1.x + yy * m2.x + yz * m3.x, xy * m1.y + yy * m2.y + yz * m3.y);
  o1 = make_double2(xz * m1.x + yz * m2.x + zz * m3.x, xz * m1.y + yz * m2.y + zz * m3.y);
  o0 = make_double2(h1.x - h2.y, h1.y + h2.x);
}

__global__ void k_demag_mul(FieldDims f, const double* nhat, double2* w) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = f.px * f.py * f.pz;
  if (p >= P) return;
  const int64_t a = p % f.px, b = (p / f.px) % f.py, c = p / (f.px * f.py);
  const int64_t q = ((f.px - a) & (f.px - 1)) + f.px * (((f.py - b) & (f.py - 1)) + f.py * ((f.pz - c) & (f.pz - 1)));
  if (q < p) return;  // done by the partner
  const double2 zp = w[p], zq = w[q], m3p = w[P + p], m3q = w[P + q];
  double2 o0, o1;
  demag_apply(nhat, P, p, zp, zq, m3p, o0, o1);
  if (q != p) {
    double2 r0, r1;
    demag_apply(nhat, P, q, zq, zp, m3q, r0, r1);
    w[q] = r0;
    w[P + q] = r1;
  }
  w[p] = o0;
  w[P + p] = o1;
}

// h = -N * m from the inverse transform: plane 0 = h1 + i h2, plane 1 = h3
__global__ void k_stray_out(FieldDims f, const double2* w, double* h) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = f.nx * f.ny * f.nz;
  if (node >= N) return;
  const int64_t P = f.px * f.py * f.pz;
  const int64_t a = node % f.nx, b = (node / f.nx) % f.ny, c = node / (f.nx * f.ny);
  const int64_t p = a + f.px * (b + f.py * c);
  const double2 v = w[p];
  h[3 * node] = -v.x;
  h[3 * node + 1] = -v.y;
  h[3 * node + 2] = -w[P + p].x;
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
    const double2 v = w[p];
    hs[0] = -v.x;
    hs[1] = -v.y;
    hs[2] = -w[P + p].x;
  }
  const double fp[3] = {hs[0] + prm[4], (hs[1] + prm[5]) - q * x[1], (hs[2] + prm[6]) - q * x[2]};
  const double c1[3] = {x[1] * fp[2] - x[2] * fp[1], x[2] * fp[0] - x[0] * fp[2], x[0] * fp[1] - x[1] * fp[0]};
  const double c2[3] = {x[1] * c1[2] - x[2] * c1[1], x[2] * c1[0] - x[0] * c1[2], x[0] * c1[1] - x[1] * c1[0]};
  for (int k = 0; k < 3; ++k) b[3 * node + k] = b[3 * node + k] - dtp * (c1[k] + alpha * c2[k]);
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

void init_field_attributes() {}

void launch_demag_setup(hipStream_t st, FieldDims f, double h, double2* work, double* nhat) {
  const int64_t P = f.px * f.py * f.pz;
  const int pairs[3][2] = {{0, 1}, {2, 3}, {4, 5}};
  for (int r = 0; r < 3; ++r) {
    hipLaunchKernelGGL(k_demag_grid2, dim3(nblk(P)), dim3(TPB), 0, st, f, pairs[r][0], pairs[r][1], h, work);
    fft_forward_full(st, f, work, 1);
    hipLaunchKernelGGL(k_take_pair, dim3(nblk(P)), dim3(TPB), 0, st, P, pairs[r][0], pairs[r][1], work, nhat);
  }
}

void launch_stray(hipStream_t st, FieldDims f, const double* m, const double* mprev, const double* nhat,
                  double2* work) {
  const int64_t P = f.px * f.py * f.pz, N = f.nx * f.ny * f.nz;
  hipLaunchKernelGGL(k_pad_field, dim3(nblk(N)), dim3(TPB), 0, st, f, m, mprev, work);
  fft_forward_box(st, f, work, 2);
  hipLaunchKernelGGL(k_demag_mul, dim3(nblk(P)), dim3(TPB), 0, st, f, nhat, work);
  fft_inverse_box(st, f, work, 2);
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
