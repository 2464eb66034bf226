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
#include <mutex>

#include "llg.h"
#include "llg_internal.h"

namespace llg {

namespace {

constexpr int TPB = 256;
inline unsigned nblk(int64_t n, int t = TPB) { return (unsigned)ceil_div(n > 0 ? n : 1, t); }

// ------------------------------------------------------------ demag tensor
// With m constant on the cubic cells of side h and the field averaged over
// each cell, the stray field of eq. stray_field is h_i = -sum_j N(k_i - k_j) m_j,
// where for the cell offset k (in cells, r = k h)
//   N_ab(k) = -(1/4pi) int_{[-1,1]^3} prod_d (1 - |s_d|) K_ab(k + s) ds,
//   K_ab(y) = d_a d_b (1/|y|) = (3 y_a y_b - delta_ab |y|^2) / |y|^5:
// averaging the field of one uniformly magnetized cube over another is the
// convolution of the point kernel with the autocorrelation of the cube, a tent
// of half-width one cell along each axis.  N does not depend on h.  The offset
// is handled by range (max norm of k):
//  - |k| <= 1, cells that touch or coincide (the integrand is singular):
//    closed form.  Along an axis where the kernel is differentiated twice the
//    tent average is the second difference of the kernel; along an axis where
//    it is not, the second difference of a second antiderivative.  So N is the
//    27-point second difference (weights 2 at 0, -1 at +-1 per axis), over
//    4 pi, of a generating function whose mixed derivatives give 1/|y| (Newell,
//    Williams and Dunlop 1993); the six generating functions are evaluated
//    together at each lattice point from the three logarithms and three
//    arctangents they share (gen6).
//  - 2 <= |k| <= 16: the integral above by Gauss-Legendre quadrature.  The
//    nearest point of the other cell is a cell away, so the integrand is
//    analytic on the domain; each axis is folded onto [0, 1], which leaves
//    the tent as the weight (1 - s).  Twelve nodes per folded axis reproduce
//    the closed form evaluated at 40 digits to about 1e-18 at |k| = 2, and
//    better beyond.
//  - |k| > 16: the point dipole -(1/4pi) K(k).
// Entries: 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz.  The diagonal entries are even
// in every coordinate of k; the xy entry is odd in k_x and k_y and even in
// k_z, and so on, so the positive octant determines the tensor.

constexpr int DEMAG_NEAR = 1, DEMAG_FAR = 16, GL_NODES = 12, GL_AXIS = 2 * GL_NODES;

// Nodes and weights of the folded rule on [0, 1] for the weight (1 - s).
struct GlRule {
  double t[GL_NODES], w[GL_NODES];
};

// The six generating values at a lattice point (coordinates taken by
// absolute value; the off-diagonal ones are odd in their first two
// arguments, applied by the caller).  With R = |y|, l_a = log((y_a + R) / rho_a)
// (rho_a the distance to the a axis; set to 0 where rho_a = 0, where each of
// its coefficients vanishes) and t_a = atan2(y_b y_c, y_a R):
//   F_aa = y_b (y_c^2 - y_a^2) l_b / 2 + y_c (y_b^2 - y_a^2) l_c / 2
//          - y_a y_b y_c t_a + (2 y_a^2 - y_b^2 - y_c^2) R / 6,
//   F_ab = y_a y_b y_c l_c + y_b (3 y_c^2 - y_b^2) l_a / 6 + y_a (3 y_c^2 - y_a^2) l_b / 6
//          - y_c^3 t_c / 6 - y_c y_b^2 t_b / 2 - y_c y_a^2 t_a / 2 - y_a y_b R / 3
// for (a, b, c) a cyclic or the matching order of (x, y, z).
__device__ void gen6(double x, double y, double z, double F[6]) {
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double xx = x * x, yy = y * y, zz = z * z;
  const double R = sqrt(xx + yy + zz);
  if (R == 0.0) {
    for (int c = 0; c < 6; ++c) F[c] = 0.0;
    return;
  }
  const double ryz = sqrt(yy + zz), rxz = sqrt(xx + zz), rxy = sqrt(xx + yy);
  const double lx = ryz > 0.0 ? log((x + R) / ryz) : 0.0;
  const double ly = rxz > 0.0 ? log((y + R) / rxz) : 0.0;
  const double lz = rxy > 0.0 ? log((z + R) / rxy) : 0.0;
  const double tx = atan2(y * z, x * R), ty = atan2(x * z, y * R), tz = atan2(x * y, z * R);
  const double xyz = x * y * z, R6 = R / 6.0;
  F[0] = 0.5 * y * (zz - xx) * ly + 0.5 * z * (yy - xx) * lz - xyz * tx + (2.0 * xx - yy - zz) * R6;
  F[1] = 0.5 * x * (zz - yy) * lx + 0.5 * z * (xx - yy) * lz - xyz * ty + (2.0 * yy - xx - zz) * R6;
  F[2] = 0.5 * y * (xx - zz) * ly + 0.5 * x * (yy - zz) * lx - xyz * tz + (2.0 * zz - xx - yy) * R6;
  F[3] = xyz * lz + y * (3.0 * zz - yy) * lx / 6.0 + x * (3.0 * zz - xx) * ly / 6.0 - z * zz * tz / 6.0 -
         0.5 * z * yy * ty - 0.5 * z * xx * tx - x * y * R / 3.0;
  F[4] = xyz * ly + z * (3.0 * yy - zz) * lx / 6.0 + x * (3.0 * yy - xx) * lz / 6.0 - y * yy * ty / 6.0 -
         0.5 * y * zz * tz - 0.5 * y * xx * tx - x * z * R / 3.0;
  F[5] = xyz * lx + z * (3.0 * xx - zz) * ly / 6.0 + y * (3.0 * xx - yy) * lz / 6.0 - x * xx * tx / 6.0 -
         0.5 * x * zz * tz - 0.5 * x * yy * ty - y * z * R / 3.0;
}

__device__ inline double sgn(int64_t v) { return v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0); }

// closed form for |k| <= 1
__device__ void demag_near(int64_t X, int64_t Y, int64_t Z, double t[6]) {
  for (int c = 0; c < 6; ++c) t[c] = 0.0;
  for (int k = -1; k <= 1; ++k)
    for (int j = -1; j <= 1; ++j)
      for (int i = -1; i <= 1; ++i) {
        const double W = (i ? -1.0 : 2.0) * (j ? -1.0 : 2.0) * (k ? -1.0 : 2.0);
        const int64_t a = X + i, b = Y + j, c = Z + k;
        double F[6];
        gen6((double)a, (double)b, (double)c, F);
        const double sab = sgn(a) * sgn(b), sac = sgn(a) * sgn(c), sbc = sgn(b) * sgn(c);
        t[0] += W * F[0];
        t[1] += W * F[1];
        t[2] += W * F[2];
        t[3] += W * sab * F[3];
        t[4] += W * sac * F[4];
        t[5] += W * sbc * F[5];
      }
  for (int c = 0; c < 6; ++c) t[c] = t[c] / (4.0 * M_PI);
}

// -(1/4pi) K(y) (the point dipole; also the quadrature's integrand)
__device__ inline void dipole(double x, double y, double z, double t[6]) {
  const double r2 = x * x + y * y + z * z;
  const double s = -1.0 / (4.0 * M_PI * r2 * r2 * sqrt(r2));
  t[0] = s * (3.0 * x * x - r2);
  t[1] = s * (3.0 * y * y - r2);
  t[2] = s * (3.0 * z * z - r2);
  t[3] = s * 3.0 * x * y;
  t[4] = s * 3.0 * x * z;
  t[5] = s * 3.0 * y * z;
}

// The positive octant of offsets, T[c][node] on the n-box: the near and far
// ranges, one thread per offset (the quadrature range is k_demag_mid's).
__global__ void k_demag_octant(FieldDims f, double* __restrict__ T) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = f.nx * f.ny * f.nz;
  if (node >= N) return;
  const int64_t X = node % f.nx, Y = (node / f.nx) % f.ny, Z = node / (f.nx * f.ny);
  const int64_t far = X > Y ? (X > Z ? X : Z) : (Y > Z ? Y : Z);
  double t[6];
  if (far <= DEMAG_NEAR)
    demag_near(X, Y, Z, t);
  else if (far > DEMAG_FAR)
    dipole((double)X, (double)Y, (double)Z, t);
  else
    return;
  for (int c = 0; c < 6; ++c) T[c * N + node] = t[c];
}

// The quadrature range, one workgroup per offset of the box
// [0, min(n, 17))^3; GL_AXIS^3 points (both halves of every folded axis).
constexpr int MID_TPB = 256;
__global__ __launch_bounds__(MID_TPB) void k_demag_mid(FieldDims f, GlRule q, double* __restrict__ T) {
  const int64_t mx = f.nx < DEMAG_FAR + 1 ? f.nx : DEMAG_FAR + 1;
  const int64_t my = f.ny < DEMAG_FAR + 1 ? f.ny : DEMAG_FAR + 1;
  const int64_t X = blockIdx.x % mx, Y = (blockIdx.x / mx) % my, Z = blockIdx.x / (mx * my);
  const int64_t far = X > Y ? (X > Z ? X : Z) : (Y > Z ? Y : Z);
  if (far <= DEMAG_NEAR) return;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < GL_AXIS * GL_AXIS * GL_AXIS; p += MID_TPB) {
    const int a = p % GL_AXIS, b = (p / GL_AXIS) % GL_AXIS, c = p / (GL_AXIS * GL_AXIS);
    const double sa = a < GL_NODES ? q.t[a] : -q.t[a - GL_NODES];
    const double sb = b < GL_NODES ? q.t[b] : -q.t[b - GL_NODES];
    const double sc = c < GL_NODES ? q.t[c] : -q.t[c - GL_NODES];
    const double W = q.w[a % GL_NODES] * q.w[b % GL_NODES] * q.w[c % GL_NODES];
    double t[6];
    dipole((double)X + sa, (double)Y + sb, (double)Z + sc, t);
    for (int k = 0; k < 6; ++k) acc[k] += W * t[k];
  }
  __shared__ double red[6][MID_TPB];
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = MID_TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t N = f.nx * f.ny * f.nz, node = X + f.nx * (Y + f.ny * Z);
    for (int k = 0; k < 6; ++k) T[k * N + node] = red[k][0];
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

// Two tensor components packed as one complex plane, a + i b, on the padded
// grid (cyclic offsets), from the octant table by the parities of the
// entries: both are real and even up to sign flips that the transform sees
// as real, so the packed transform's real and imaginary parts are the two
// transforms.
__global__ void k_demag_pair(FieldDims f, int c0, int c1, const double* __restrict__ T, double2* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = f.px * f.py * f.pz;
  if (p >= P) return;
  const int64_t a = p % f.px, b = (p / f.px) % f.py, c = p / (f.px * f.py);
  int64_t X, Y, Z;
  double v[2] = {0.0, 0.0};
  if (wrap(a, f.nx, f.px, X) && wrap(b, f.ny, f.py, Y) && wrap(c, f.nz, f.pz, Z)) {
    const int64_t N = f.nx * f.ny * f.nz;
    const int64_t node = (X < 0 ? -X : X) + f.nx * ((Y < 0 ? -Y : Y) + f.ny * (Z < 0 ? -Z : Z));
    const int cc[2] = {c0, c1};
    for (int r = 0; r < 2; ++r) {
      const int comp = cc[r];
      double s = 1.0;
      if (comp == 3) s = (X < 0 ? -1.0 : 1.0) * (Y < 0 ? -1.0 : 1.0);
      if (comp == 4) s = (X < 0 ? -1.0 : 1.0) * (Z < 0 ? -1.0 : 1.0);
      if (comp == 5) s = (Y < 0 ? -1.0 : 1.0) * (Z < 0 ? -1.0 : 1.0);
      v[r] = s * T[comp * N + node];
    }
  }
  out[p] = make_double2(v[0], v[1]);
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

// Gauss-Legendre nodes x_i and weights on [-1, 1] by Newton's method on the
// Legendre polynomial (three-term recurrence), mapped to [0, 1] with the
// weight (1 - s) folded into the weights.
GlRule folded_rule() {
  GlRule q;
  const int n = GL_NODES;
  for (int i = 0; i < n; ++i) {
    double x = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    const double w = 2.0 / ((1.0 - x * x) * dp * dp);
    const double t = 0.5 * (x + 1.0);
    q.t[i] = t;
    q.w[i] = 0.5 * w * (1.0 - t);
  }
  return q;
}

// The octant table T[6][N] (N = nx ny nz doubles each) of the tensor.
void launch_demag_table(hipStream_t st, FieldDims f, double* T) {
  const int64_t N = f.nx * f.ny * f.nz;
  hipLaunchKernelGGL(k_demag_octant, dim3(nblk(N)), dim3(TPB), 0, st, f, T);
  const int64_t mx = std::min<int64_t>(f.nx, DEMAG_FAR + 1), my = std::min<int64_t>(f.ny, DEMAG_FAR + 1),
                mz = std::min<int64_t>(f.nz, DEMAG_FAR + 1);
  hipLaunchKernelGGL(k_demag_mid, dim3((unsigned)(mx * my * mz)), dim3(MID_TPB), 0, st, f, folded_rule(), T);
}

// Components c0 (real part) and c1 (imaginary part) on the padded grid.
void launch_demag_pair(hipStream_t st, FieldDims f, int c0, int c1, const double* T, double2* out) {
  const int64_t P = f.px * f.py * f.pz;
  hipLaunchKernelGGL(k_demag_pair, dim3(nblk(P)), dim3(TPB), 0, st, f, c0, c1, T, out);
}

// The octant table goes to the second work plane (16 P bytes >= 48 N: every
// padded length is at least twice the grid's), the packed pairs to the first.
void launch_demag_setup(hipStream_t st, FieldDims f, double2* work, double* nhat) {
  const int64_t P = f.px * f.py * f.pz;
  double* T = (double*)(work + P);
  launch_demag_table(st, f, T);
  const int pairs[3][2] = {{0, 1}, {2, 3}, {4, 5}};
  for (int r = 0; r < 3; ++r) {
    launch_demag_pair(st, f, pairs[r][0], pairs[r][1], T, work);
    fft_forward_full(st, f, work, 1);
    hipLaunchKernelGGL(k_take_pair, dim3(nblk(P)), dim3(TPB), 0, st, P, pairs[r][0], pairs[r][1], work, nhat);
  }
}

// ------------------------------------------------------------ no-allocation stray field
// The stray field of a device field without a context: the transformed tensor
// (6 P doubles) and the two work planes (4 P doubles) live in one static
// device array, so the call allocates nothing.  Each device holds its own
// copy of the array; its address is looked up once per device.  The array
// keeps the last call's contents: the transformed tensor is reused when the
// grid dimensions repeat.  Calls that overlap on one device race.
constexpr size_t NOALLOC_BYTES = LLG_STRAY_NOALLOC_MAX_BYTES;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEV] = {};
int64_t g_noalloc_dims[NOALLOC_MAX_DEV][3] = {};
}  // namespace

size_t stray_noalloc_bytes(FieldDims f) { return (size_t)(f.px * f.py * f.pz) * 10 * sizeof(double); }

hipError_t stray_noalloc(FieldDims f, const double* m, double* h, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[dev] = p;
  }
  const int64_t P = f.px * f.py * f.pz;
  double* nhat = (double*)g_noalloc_ptr[dev];
  double2* work = (double2*)(nhat + 6 * P);
  const bool same = g_noalloc_dims[dev][0] == f.nx && g_noalloc_dims[dev][1] == f.ny && g_noalloc_dims[dev][2] == f.nz;
  if (!same) {
    g_noalloc_dims[dev][0] = 0;  // invalid until the new tensor is in place
    launch_demag_setup(st, f, work, nhat);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  launch_stray(st, f, m, nullptr, nhat, work);
  launch_stray_out(st, f, work, h);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  g_noalloc_dims[dev][0] = f.nx;
  g_noalloc_dims[dev][1] = f.ny;
  g_noalloc_dims[dev][2] = f.nz;
  return hipSuccess;
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
