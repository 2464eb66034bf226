// llg_internal.h -- internal declarations shared by the HIP translation units
// of the library (device helpers, matrix views, kernel launchers).
//
// Matrix storage (every AMG level and the outer operator): 3x3-block sliced
// ELL with 64-row slices, one wavefront per slice.  Slice s covers rows
// 64s .. 64s+63 and has width W_s = max row length in the slice; its block
// slots occupy sl_ptr[s] .. sl_ptr[s+1] = sl_ptr[s] + 64 W_s.  Slot t of row
// 64s+l is at index sl_ptr[s] + 64 t + l in col[] (column or -1 after the
// row's last block) and its nine values at 9 sl_ptr[s] + 64 (9 t + e) + l in
// val[], so that the 64 lanes of a wavefront read 64 consecutive words for
// every (slot, entry).  Columns of a row are ascending; the diagonal block is
// always present.  Per-node 3x3 blocks (inverse diagonals) use the layout
// [slice][9][64].  Vectors are [N][3], node-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace llg {

constexpr int SL = 64;          // rows per slice (wavefront size)
constexpr int MAX_PASS = 3;     // pairwise matching passes per level
constexpr int PRM_WORDS = 12;   // the step's parameter block (8 values, 3 input addresses, 1 spare)
constexpr int RED_BLOCKS = 1024;  // fixed partial-sum count of grid reductions

struct Sell {
  int64_t n = 0;        // rows
  int64_t nslices = 0;  // ceil(n / 64)
  int64_t nslots = 0;   // sl_ptr[nslices]
  int32_t* sl_ptr = nullptr;
  int32_t* col = nullptr;
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; give each
// XCD a contiguous range of blocks so that neighbouring rows (which share
// vector entries) are served from the same L2.  A bijection of [0, nb).
__device__ inline unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned per = nb / 8;
  const unsigned xcd = b % 8, k = b / 8;
  // blocks [0, 8*per) are spread evenly; the remainder keeps its index
  if (b < 8 * per) return xcd * per + k;
  return b;
}

// Grid sizes, and the source of the grid level's blocks for the solve
// kernels: the frozen field mt (N x 3), prm[0] = alpha, prm[1] = dt' eps, and
// 1/h^2 (the blocks are recomputed per node with grid_blocks).
struct GridDims {
  int nx, ny, nz;
  const double* mt = nullptr;
  const double* prm = nullptr;
  double inv_h2 = 0.0;
};

// ---------------------------------------------------------- grid-level blocks
// Row r of M collects the coefficients of (Lap u1, Lap u2, Lap u3) in
// equation r of the damped component-wise system (Sec. 2.1):
//   M = [ -a(m2^2+m3^2)     -m3 + a m1 m2     m2 + a m1 m3 ]
//       [  m3 + a m1 m2    -a(m1^2+m3^2)     -m1 + a m2 m3 ]
//       [ -m2 + a m1 m3     m1 + a m2 m3    -a(m1^2+m2^2)  ]
// These functions are evaluated without contraction in every file, so that
// the solve kernels recompute bit for bit the blocks the assembly stores.
__device__ inline void block_M(double m1, double m2, double m3, double a, double* M) {
#pragma clang fp contract(off)
  M[0] = -(a * (m2 * m2 + m3 * m3));
  M[1] = -m3 + a * (m1 * m2);
  M[2] = m2 + a * (m1 * m3);
  M[3] = m3 + a * (m1 * m2);
  M[4] = -(a * (m1 * m1 + m3 * m3));
  M[5] = -m1 + a * (m2 * m3);
  M[6] = -m2 + a * (m1 * m3);
  M[7] = m1 + a * (m2 * m3);
  M[8] = -(a * (m1 * m1 + m2 * m2));
}

// 3x3 inverse: adjugate times the reciprocal of the determinant (cofactor
// expansion along the first row).
__device__ inline void inv3(const double* D, double* R) {
#pragma clang fp contract(off)
  const double a = D[0], b = D[1], c = D[2], d = D[3], e = D[4], f = D[5], g = D[6], h = D[7],
               i = D[8];
  double adj[9];
  adj[0] = e * i - f * h;
  adj[1] = c * h - b * i;
  adj[2] = b * f - c * e;
  adj[3] = f * g - d * i;
  adj[4] = a * i - c * g;
  adj[5] = c * d - a * f;
  adj[6] = d * h - e * g;
  adj[7] = b * g - a * h;
  adj[8] = a * e - b * d;
  const double det = (a * adj[0] + b * adj[3]) + c * adj[6];
  const double rdet = 1.0 / det;
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = adj[k] * rdet;
}

// The grid level's blocks of a node with frozen field mt and deg in-grid
// neighbours: Mh = s M (s = dt'/h^2, the off-diagonal block of A),
// D = I + s_pp M (s_pp = -deg s, the diagonal block), Di = D^{-1} and
// K = Di Mh (entry (r, q) summed over k = 0, 1, 2 in order; the off-diagonal
// block of D^{-1} A).  Mh, Di or K may be NULL when not needed.
__device__ inline void grid_blocks(const double* mt, double alpha, double dt, double inv_h2, int deg, double* Mh,
                                   double* Di, double* K) {
#pragma clang fp contract(off)
  double M[9];
  block_M(mt[0], mt[1], mt[2], alpha, M);
  const double s_off = dt * inv_h2;
  const double s_diag = dt * (-(double)deg * inv_h2);
  double D[9], R[9], B[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double v = s_diag * M[e];
    if (e == 0 || e == 4 || e == 8) v = 1.0 + v;
    D[e] = v;
    B[e] = s_off * M[e];
  }
  inv3(D, R);
  if (Mh) {
#pragma unroll
    for (int e = 0; e < 9; ++e) Mh[e] = B[e];
  }
  if (Di) {
#pragma unroll
    for (int e = 0; e < 9; ++e) Di[e] = R[e];
  }
  if (K) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) K[3 * r + q] = (R[3 * r] * B[q] + R[3 * r + 1] * B[3 + q]) + R[3 * r + 2] * B[6 + q];
  }
}

// ----------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns nothing; launch errors are
// collected by the caller with hipGetLastError().

// integer utilities
void launch_fill_i32(hipStream_t st, int32_t* p, int64_t n, int32_t v);
void launch_fill_f64(hipStream_t st, double* p, int64_t n, double v);
// exclusive scan of n int32 values (in may equal out); out[n] is NOT written,
// the total goes to *total.  tmp needs scan_tmp_ints(n) ints.
int64_t scan_tmp_ints(int64_t n);
void launch_scan_excl(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                      int32_t* tmp);
// device flag |= (a[0] != expect)
void launch_check_eq(hipStream_t st, const int32_t* a, int32_t expect, int32_t* flag, int32_t bit);
// *p[k] == v[k] for k < n (n <= CHECK_BATCH), in one launch; else flag |= bit
constexpr int CHECK_BATCH = 64;
void launch_check_many(hipStream_t st, const int32_t* const* p, const int32_t* v, int n, int32_t* flag, int32_t bit);

// grid graph and patterns
void launch_grid_degree(hipStream_t st, int nx, int ny, int nz, int32_t* deg);
void launch_grid_graph(hipStream_t st, int nx, int ny, int nz, const int32_t* grp, int32_t* gci,
                       int32_t* gw);
void launch_pattern_rp(hipStream_t st, int64_t n, const int32_t* grp, int32_t* brp);
void launch_pattern_cols(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci,
                         const int32_t* brp, int32_t* bci);
// sliced-ELL structure of rows[0..n) of a CSR pattern (rows == NULL: rows 0..n)
void launch_slice_width(hipStream_t st, int64_t n, const int32_t* rows, const int32_t* brp, int32_t* wslots);
void launch_sell_cols(hipStream_t st, int64_t n, const int32_t* rows, const int32_t* brp, const int32_t* bci,
                      const int32_t* sl_ptr, int32_t* col);

// colour classes of the multicolour Gauss-Seidel smoother
constexpr int MAX_COLOURS = 128;
void launch_parity_colour(hipStream_t st, int nx, int ny, int nz, int32_t* col);
// one Jones-Plassmann round; *pending is set non-zero when a node stays uncoloured
void launch_jp_round(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci, const uint64_t* rank,
                     int32_t r, int32_t* cround, int32_t* col, int32_t* pending);
void launch_colour_max(hipStream_t st, int64_t n, const int32_t* col, int32_t* ncol);
// counting sort by colour: hist has ncol * colour_blocks(n) entries (+1 for the total)
int64_t colour_blocks(int64_t n);
void launch_colour_hist(hipStream_t st, int64_t n, const int32_t* col, int32_t ncol, int32_t* hist);
void launch_colour_place(hipStream_t st, int64_t n, const int32_t* col, int32_t ncol, const int32_t* hist,
                         int32_t* perm);
// values (and inverse diagonal blocks when dinv != NULL) of the class rows[0..n)
// (fk != NULL: the level is the factored grid level, as in launch_galerkin)
template <typename T>
void launch_cls_gather(hipStream_t st, int64_t n, const int32_t* rows, Sell A, const T* val, const T* dinv,
                       Sell C, T* cval, T* cdinv, const T* fk);

// pairwise matching (one pass)
void launch_node_rank(hipStream_t st, int64_t n, uint64_t salt, uint64_t* rank);
// prop[i] = proposed partner or -1; *any is set non-zero when some node proposes
// Matching state of a node, one 8-byte record so that a candidate costs one
// load: its largest edge weight and its mate (-1 while unmatched; the
// proposal rounds mark a free node without candidates -2 in the mate array
// only, which the record does not need to know).  The visiting rank is a
// hash of the node's index, computed where it is compared (cheaper than the
// 16-byte record that held it: 256^3 proposal rounds 13.3 -> 12.8 ms).
struct alignas(8) NodeSt {
  int32_t mx;
  int32_t mate;
};
// ns[i] = {max_k w_ik, -1}; mate[i] = -1; prop[i] = -1 (no proposal yet)
void launch_match_init(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gw, uint64_t salt,
                       NodeSt* ns, int32_t* mate, int32_t* prop);
void launch_propose(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci, const int32_t* gw,
                    int32_t* mate, const NodeSt* ns, uint64_t salt, int32_t bnum, int32_t bden, int32_t* prop,
                    int32_t* any, int lanes);
// The same round on the grid graph of an nx x ny x nz grid (weights 1): the
// neighbours are computed, the visiting ranks read from rank (node_rank of
// every node under salt), no records are read.  The first round (first)
// also sets mate of every node; prop and mate need no initialisation.
void launch_propose_grid(hipStream_t st, int nx, int ny, int nz, int32_t* mate, const uint64_t* rank,
                         uint64_t salt, int32_t bnum, int32_t bden, int32_t* prop, int32_t* any, bool first);
// Every round of the matching of a small level (n <= MATCH_SMALL) in one
// workgroup, with 2 lanes per node (G >= 2) or 1; raises flag bit if it did
// not end within n rounds.
constexpr int64_t MATCH_SMALL = 512;
void launch_match_small(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci, const int32_t* gw,
                        int32_t* mate, NodeSt* ns, uint64_t salt, int32_t bnum, int32_t bden, int32_t* prop,
                        int32_t* flag, int32_t bit, int G);
// mutual proposals are matched (mate and ns[].mate); propose marks a free
// node without candidates dead (mate -2, unmatched for every reader)
void launch_accept(hipStream_t st, int64_t n, const int32_t* prop, int32_t* mate, NodeSt* ns);
void launch_leader_flag(hipStream_t st, int64_t n, const int32_t* mate, int32_t* flag);
void launch_assign(hipStream_t st, int64_t n, const int32_t* mate, const int32_t* id, int32_t* agg,
                   int32_t* lead);
void launch_cg_count(hipStream_t st, int64_t nc, const int32_t* lead, const int32_t* mate,
                     const int32_t* grp, int32_t* cnt);
// Coarse graph rows, written tile by tile (cg_tile_rows(shape) rows per
// tile) from the tile's candidate offset cptr[first row]: nrp[I] = row I's
// offset in its tile, ttot[tile] = the tile's length.  wide: the coarse
// levels of a 3D grid (rows of up to about 50 candidates); grid: {nx, ny,
// nz} when the graph is the grid graph itself (the grid level's first pass;
// its rows are then computed, at most twelve candidates), else null.  shape:
// 1 wide, 2 grid, 0 the others.  nsn, maten, propn (or null): the next
// matching pass's state of the coarse nodes, set as launch_match_init would
// set it on the new graph.
int cg_tile_rows(int shape);
void launch_cg_fill(hipStream_t st, int64_t nc, const int32_t* lead, const int32_t* mate,
                    const int32_t* grp, const int32_t* gci, const int32_t* gw, const int32_t* agg,
                    const int32_t* cptr, int32_t* cj, int32_t* cw, int32_t* nrp, int32_t* ttot, bool wide,
                    const int* grid, NodeSt* nsn, int32_t* maten, int32_t* propn);
// After an exclusive scan of ttot into tbase (total at tbase[tiles]): the
// tiles moved to nci/nw end to end, nrp made the row pointers (nrp[nc] the
// edge count).
void launch_cg_copy(hipStream_t st, int64_t nc, int shape, const int32_t* cptr, const int32_t* cj,
                    const int32_t* cw, const int32_t* tbase, int32_t* nrp, int32_t* nci, int32_t* nw);
// Members of the composite aggregates of a level after np passes, from each
// pass's leaders (lead[q][a]: the leader of aggregate a of pass q, a node of
// pass q's graph) and mates: cnt[I] = the number of fine nodes of aggregate
// I; then, with mptr the exclusive scan of cnt, mem[mptr[I]..] = its fine
// nodes ascending and acc[i] = the aggregate of fine node i.
void launch_member_count(hipStream_t st, int64_t nc, int np, const int32_t* const* lead,
                         const int32_t* const* mate, int32_t* cnt);
void launch_member_fill(hipStream_t st, int64_t nc, int np, const int32_t* const* lead,
                        const int32_t* const* mate, const int32_t* mptr, int32_t* mem, int32_t* acc);

// assembly of the fine operator (FP64 A) and the scaled level-0 operator,
// the right-hand side b and the initial guess u; the frozen field is m
// (mprev == NULL) or 2 m - mprev (BDF2, b = (4 m - mprev) / 3 + dt F).
// prm[0] = alpha, prm[1] = the time-step factor of the operator, prm[2] = the
// factor of the forcing and of the explicit field terms (device memory, so
// captured graphs stay valid)
// Factored form (fact): the per-node blocks are written instead of the
// sliced-ELL values Aval and Lval, each where its pointer is not null: Mh
// (FP64) and K (in T) sliced, Knm node-major (nine contiguous values per
// node).  dinv0 may be null (nothing reads it when the preconditioner's
// input scaling recomputes D^{-1} from the frozen field).
// The inputs m^n, m^{n-1} (or null) and F (or null) are read at the device
// addresses held, as bit patterns, in prm[8], prm[9] and prm[10], so that a
// captured setup serves every step's buffers.
template <typename T>
void launch_assemble(hipStream_t st, int nx, int ny, int nz, double inv_h2, const double* prm,
                     int left_scale, int x0_is_mn, Sell A, double* Aval, T* Lval, double* dinv0, T* ldinv,
                     double* b, double* u, int32_t* flag, bool fact, double* Mh, T* K, T* Knm, double* mt_out);
// The factored grid level's sliced blocks Mh (FP64) and K (in T) from the
// frozen field mt the assembly wrote, with the parameters in prm (the values
// the assembly computes; for callers that read the blocks back).
template <typename T>
void launch_fact_blocks(hipStream_t st, int nx, int ny, int nz, double inv_h2, const double* prm, const double* mt,
                        double* Mh, T* K);

// Where a Galerkin product reads the fine blocks, and where it leaves a copy
// of the coarse ones.  fk != NULL: the fine level is the factored grid level,
// whose block (i, j) is the identity when j == i and K_i otherwise; K_i is
// read from knm (node-major, nine contiguous values) when it is not NULL,
// else from fk.  Otherwise the blocks are read from fvt (the level's blocks
// in slot order, nine contiguous values per slot) when it is not NULL, else
// from the sliced-ELL values fval.  cvt != NULL receives the coarse blocks
// in slot order.
template <typename T>
struct GalSrc {
  const T* fval = nullptr;     // fine blocks, sliced ELL (the grid level stored as BSR)
  const T* fvt = nullptr;      // fine blocks in the fine level's CSR order (coarse levels)
  const T* fk = nullptr;
  const T* knm = nullptr;
  const int32_t* frp = nullptr;  // fine CSR pattern: row pointers and ascending columns
  const int32_t* fci = nullptr;
  T* cvt = nullptr;            // coarse blocks in the coarse level's CSR order (for the next product)
  const int32_t* crp = nullptr;  // coarse CSR row pointers (positions of cvt)
  const int32_t* cci = nullptr;  // coarse CSR columns (ascending; the sliced-ELL slot order)
};
// Galerkin block sums P^T A P and the inverse diagonal blocks of the result
template <typename T>
void launch_galerkin(hipStream_t st, Sell C, T* cval, T* cdinv, const int32_t* mptr, const int32_t* mem, Sell F,
                     const int32_t* agg, const GalSrc<T>& g);

// one-time kernel attribute setup (large dynamic LDS for the coarsest inverse)
void init_kernel_attributes();

// coarsest level: dense copy and in-place Gauss-Jordan inverse
template <typename T>
void launch_dense_scatter(hipStream_t st, Sell C, const T* cval, double* dense);
void launch_gauss_jordan(hipStream_t st, int64_t nd, double* dense, int32_t* piv, int32_t* flag);
template <typename T>
void launch_dense_apply(hipStream_t st, int64_t nd, const double* inv, const T* b, T* x);
// restriction of r onto the coarsest level (nc nodes) and x = A_c^{-1} P^T r
template <typename T>
void launch_restrict_dense(hipStream_t st, int64_t nc, const int32_t* mptr, const int32_t* mem, const T* r,
                           const double* inv, T* x);

// V-cycle level kernels.  xmode: 0 = x stored, 1 = x = omega b (unit
// diagonal, first sweep from zero), 2 = x = 0.
template <typename T>
void launch_smooth_first(hipStream_t st, Sell A, const T* dinv, double omega, const T* b, T* x);
// G = lanes per row (1, 8 or 16; more lanes for small, latency-bound levels)
template <typename T>
void launch_residual(hipStream_t st, Sell A, const T* val, int xmode, double omega, const T* b,
                     const T* x, T* r, int G);
// bc = P^T r (members ascending); xc = omega Dc^{-1} bc when xc != NULL (the
// first pre-smoothing sweep of the coarse level)
template <typename T>
void launch_restrict(hipStream_t st, int64_t nc, const int32_t* mptr, const int32_t* mem, const T* r, T* bc,
                     const T* cdinv, double omega, T* xc);
// out = x' + omega D^{-1} (b - A x') with x' = xbase + P ec (ec may be NULL)
template <typename T>
void launch_post_smooth(hipStream_t st, Sell A, const T* val, const T* dinv, int unit, int xmode,
                        double omega, const T* b, const T* x, const int32_t* agg, const T* ec,
                        T* out, int G);
// The same two products on a level's CSR-ordered blocks (rp, ci: the level's
// block pattern; vt: nine contiguous values per block, in pattern order),
// CSR_G lanes per row; the post-smoothing sweep takes no coarse correction
// (prolong it into x first).  CSR_G: lanes per row (the large coarse levels
// hold about 15 blocks per row in 3D; eight lanes measured faster than two or four).
constexpr int CSR_G = 8;
template <typename T>
void launch_residual_csr(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const T* vt, int xmode,
                         double omega, const T* b, const T* x, T* r);
template <typename T>
void launch_post_smooth_csr(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const T* vt,
                            const T* dinv, int xmode, double omega, const T* b, const T* x, T* out);
// One block Gauss-Seidel sweep over a colour class (C: the class as a
// sliced-ELL matrix, rows: its level rows): x_i += D_i^{-1} (b_i - sum_j A_ij x_j),
// in place.  first: x is zero everywhere, so x_i = D_i^{-1} b_i.
template <typename T>
void launch_gs_sweep(hipStream_t st, Sell C, const int32_t* rows, const T* cval, const T* cdinv, int unit,
                     int first, const T* b, T* x, int G);
template <typename T>
void launch_fill(hipStream_t st, T* p, int64_t n);
// out = xbase + P ec
template <typename T>
void launch_prolong(hipStream_t st, int64_t n, int xmode, double omega, const T* b, const T* x,
                    const int32_t* agg, const T* ec, T* out);
// The V-cycle of the small coarse levels s..L-1 in one workgroup (block
// Jacobi smoothing): the level vectors live in LDS, the matrices are read
// from global memory.  The launch takes the residual of level s-1 and the
// aggregates of level s-1, and writes the coarse correction e_s; the
// arithmetic of every step is that of the per-level kernels (same row
// products, lane groups, summation orders), so the result is the same.
constexpr int TAIL_T = 1024;    // threads of the workgroup
constexpr int TAIL_MAX = 16;    // levels
constexpr int TAIL_LDS = 152 * 1024;  // LDS budget (bytes)
template <typename T>
struct TailLevel {
  const int32_t* sl;
  const int32_t* col;
  const T* val;
  const T* dinv;
  const int32_t* mptr;  // aggregates of this level (the next level's rows), members ascending
  const int32_t* mem;
  const int32_t* agg;   // node -> aggregate
  int32_t n, G;         // rows; lanes per row (1, 8 or 16)
  int32_t ob, ox, oy;   // LDS byte offsets of b, x and the third work vector (3 n each)
};
template <typename T>
struct TailArgs {
  TailLevel<T> lv[TAIL_MAX];  // smoothed levels s..L-2
  const double* inv;          // coarsest level: dense inverse (nd x nd, nd = 3 nc)
  int32_t nlev, nc;
  int32_t obd, oe;            // LDS byte offsets: coarsest b (FP64) and its solution (T)
  int32_t nu_pre, nu_post;
  int32_t lds;                // LDS bytes
  T omega;
};
// rabove: residual of level s-1; mptr/mem: its aggregates (the rows of level s)
template <typename T>
void launch_tail(hipStream_t st, const TailArgs<T>& a, const T* rabove, const int32_t* mptr, const int32_t* mem,
                 T* out);
// the tail kernel's LDS limit; false when the device refuses it
bool tail_prepare();

// b0 = D0^{-1} (v vs[0]) (or v vs[0]; vs NULL: 1), cast to T
template <typename T>
void launch_scale_in(hipStream_t st, int64_t n, const double* dinv0, int left_scale, const double* v,
                     const double* vs, T* b0);
// the same with D^{-1} recomputed from the frozen field g.mt (factored grid level)
template <typename T>
void launch_scale_in_grid(hipStream_t st, GridDims g, const double* v, const double* vs, T* b0);

// K-cycle coarse correction (two minimal-residual steps); partial sums over
// rows_blocks(n) blocks, coefficients in kc (see k_solve.hip)
int64_t rows_blocks(int64_t n, int G);
template <typename T>
void launch_spmv_dots(hipStream_t st, Sell A, const T* val, const T* v, T* w, const T* d1, const T* d2,
                      double* part, int G);
template <typename T>
void launch_kc_update(hipStream_t st, int64_t n, const T* r, const T* w1, const double* kc, T* rho,
                      const T* dinv, double omega, T* x, double* part);
template <typename T>
void launch_kc_combine(hipStream_t st, int64_t n, const T* v1, const T* v2, const double* kc, T* e);
void launch_kc_coef(hipStream_t st, const double* part, int64_t G, int stage, double* kc,
                    const double* part2 = nullptr, int64_t G2 = 0);

// Factored grid level (one 3x3 block per node, [slice][9][64]): Mh_p is
// every off-diagonal block of row p of A (A_pp = I - deg_p Mh_p), K_p every
// off-diagonal block of the left-scaled operator (unit diagonal).
// Level-1 products from the grid level's per-node blocks K (see k_solve.hip):
// mode 0 r = b - A1 x; mode 1 post-smoothing sweep (xzero: x = 0; ec, agg2
// the coarse correction or NULL); mode 2 w = A1 x with the K-cycle partial
// sums (d1, optional d2) over rows_blocks(n1, L1_LANES) workgroups of 256
constexpr int L1_LANES = 2;
// mtq[q] = mt[mem[q]] for the n grid nodes (the field in the level-1 member order)
template <typename T>
void launch_member_fields(hipStream_t st, int64_t n, const int32_t* mem, const double* mt, T* mtq);
template <typename T>
void launch_l1(hipStream_t st, GridDims g, int mode, int xzero, int64_t n1, const int32_t* mptr, const int32_t* nagg,
               const T* mtq, const T* x, const T* b, const T* dinv1, const int32_t* agg2, const T* ec,
               double omega, T* out, const T* d1, const T* d2, double* part, hipEvent_t e0 = nullptr,
               hipEvent_t e1 = nullptr);
// nagg[q][t]: level-1 aggregate of the t-th grid neighbour of member q ([slice][6][64], -1 if missing)
void launch_member_nbr_aggs(hipStream_t st, GridDims g, const int32_t* mem, const int32_t* agg, int32_t* nagg);
template <typename TZ>
void launch_fact_outer(hipStream_t st, GridDims g, const TZ* z, double* w, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
void launch_fact_resid_outer(hipStream_t st, GridDims g, const double* b, const double* u, double* r, double* part);
template <typename T>
void launch_fact_residual(hipStream_t st, GridDims g, int xmode, double omega, const T* b, const T* x, T* r);
template <typename T>
void launch_fact_post_smooth(hipStream_t st, GridDims g, int xmode, double omega, const T* b, const T* x,
                             const int32_t* agg, const T* ec, T* out);

// Krylov baselines (BiCGstab, TFQMR): a term s c x of a linear combination
// (c: device scalar or NULL for 1), the combination with its dots, plain
// copies, and the scalar steps on the state kb.
struct KTerm {
  const double* x;
  const double* c;
  double s;
};
enum {
  KB_RHO = 0, KB_ALPHA, KB_OMEGA, KB_BETA, KB_BW, KB_TAU, KB_THETA, KB_ETA, KB_F, KB_HALF, KB_FLAG, KB_B2,
  KB_MINB, KB_SIZE = 16
};
enum { KB_START = 0, KB_BICG_END = 3, KB_TF_F = 4, KB_TF_HALF = 5, KB_TF_END = 6 };
// (op codes KB_ALPHA and KB_OMEGA reuse the state indices of their results)
void launch_lin3(hipStream_t st, int64_t m, KTerm t0, KTerm t1, KTerm t2, double* y, const double* d0,
                 const double* d1, double* part);
void launch_dot2(hipStream_t st, int64_t m, const double* x0, const double* y0, const double* x1,
                 const double* y1, double* part);
void launch_copy(hipStream_t st, int64_t m, const double* x, double* y);
void launch_scale_copy(hipStream_t st, int64_t m, const double* x, const double* s, double* y);
void launch_kb_step(hipStream_t st, const double* part, int64_t nparts, int op, double* kb, double* host);

// Full field (anisotropy, external and stray field).  The stray field is a
// cyclic convolution on the grid zero-padded to P = pow2 >= 2n - 1 per axis
// (P = 1 along z for a 2D grid); work holds three complex P-arrays, nhat the
// six real transformed tensor components.
constexpr int64_t FFT_MAX_LEN = 4096;
struct FieldDims {
  int64_t nx = 0, ny = 0, nz = 0, px = 0, py = 0, pz = 0;
};
int64_t next_pow2(int64_t v);
FieldDims field_dims(int nx, int ny, int nz);
void init_field_attributes();
// the transformed demagnetizing tensor (six real planes of P values) into
// nhat, using both work planes
void launch_demag_setup(hipStream_t st, FieldDims f, double2* work, double* nhat);
// the tensor on the positive octant of offsets, T[6][nx ny nz]; components
// c0 + i c1 on the padded grid (cyclic offsets) from it
void launch_demag_table(hipStream_t st, FieldDims f, double* T);
void launch_demag_pair(hipStream_t st, FieldDims f, int c0, int c1, const double* T, double2* out);
// work = the transformed-back product N^ M^ of m~ (m, or 2 m - mprev)
void launch_stray(hipStream_t st, FieldDims f, const double* m, const double* mprev, const double* nhat,
                  double2* work);
void launch_stray_out(hipStream_t st, FieldDims f, const double2* work, double* h);
// the stray field of a device field in the static device array (see
// llg_stray_field_noalloc); bytes it needs for a padded grid
size_t stray_noalloc_bytes(FieldDims f);
hipError_t stray_noalloc(FieldDims f, const double* m, double* h, hipStream_t st);
// b -= dt' (m~ x f + alpha m~ x (m~ x f)); work NULL: no stray field
void launch_field_rhs(hipStream_t st, int64_t N, const double* prm, const double* m, const double* mprev,
                      FieldDims f, const double2* work, double* b);

// outer Krylov kernels (FP64)
template <typename TZ>
void launch_spmv_outer(hipStream_t st, Sell A, const double* val, const TZ* z, double* w,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_resid_outer(hipStream_t st, Sell A, const double* val, const double* b, const double* u,
                        double* r, double* part);
void launch_norm_part(hipStream_t st, int64_t m, const double* x, double* part);
void launch_mdot(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* w,
                 double* part);
// w -= sum_q h_q V_q and, in the same sweep, the dots of the new w (when
// want_dots) and its squared norm; skipped when skip != NULL and *skip == 0
void launch_mupdate_dot(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv,
                        const double* h, double* w, double* part, int want_dots, const double* skip);
void launch_scale_vec(hipStream_t st, int64_t m, const double* x, const double* s, double* y);
template <typename TS, typename TD>
void launch_cast(hipStream_t st, int64_t m, const TS* x, TD* y);
template <typename TZ>
void launch_zy(hipStream_t st, int64_t m, int k, const TZ* Z, int64_t ldz, const double* y, double* u);
void launch_project(hipStream_t st, int64_t n, const double* u, double* out, int project,
                    int32_t* flag);

// FGMRES scalar work, one workgroup
struct KrylovScalars {
  double* H;      // (R+1) x R, row-major
  double* cs;     // R
  double* sn;     // R
  double* g;      // R+1
  double* hcol;   // R+1 (dots of the current pass)
  double* y;      // R
  double* sc;     // scalars: [0] beta, [1] 1/beta or 1/h, [2] bnorm, [3] est, [4] hn, [5] wnorm0,
                  // [7] second pass asked (two-pass form), [8] [9] breakdown flags (delayed form)
  double* hs;     // R+2: delayed form, slot j of V holds hs[j] times the once-orthogonalized v~_j
  double* hinv;   // R+2: the scale of slot j for the preconditioner input
  double* coef;   // 2R+4: coefficients of the update sweep
};
int64_t red_blocks(int64_t m);  // partial-sum count of the grid reductions over m doubles
void launch_norm_finish_n(hipStream_t st, const double* part, int64_t nparts, int slot, double* sc,
                          double* host);
// pass-1 sums: hcol[q] (q < nv) and sc[5] = ||w||^2
void launch_dots_finish_n(hipStream_t st, const double* part, int64_t nparts, int nv, double* hcol, double* sc);
// pass-2 sums and the reorthogonalization decision (sc[7]), delta = second coefficients
void launch_reorth_finish_n(hipStream_t st, const double* part, int64_t nparts, int nv, double* hcol,
                            double* delta, double* sc);
void launch_arnoldi_finish_n(hipStream_t st, const double* part, int64_t nparts, int j, int R,
                             KrylovScalars ks, double* host);
void launch_cycle_start(hipStream_t st, int R, KrylovScalars ks);
// Delayed reorthogonalization: the dots sweep (u = slot j, w = A z_j, nv = j),
// its scalar step, the update sweep (v_j over u, w' into wo = slot j+1), its
// scalar step; and at the end of a cycle of k iterations the dots of slot k
// (u = w = slot k, nv = k) and the final last column.
void launch_dcgs_dots(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* u,
                      const double* w, double* part);
void launch_dcgs_finish1(hipStream_t st, const double* part, int64_t nparts, int j, int R, KrylovScalars ks,
                         double* host);
void launch_dcgs_update(hipStream_t st, int64_t m, int nv, const double* V, int64_t ldv, const double* coef,
                        double* u, const double* w, double* wo, double* part);
void launch_dcgs_finish2(hipStream_t st, const double* part, int64_t nparts, int j, int R, KrylovScalars ks,
                         double* host);
void launch_dcgs_last(hipStream_t st, const double* part, int64_t nparts, int k, int R, KrylovScalars ks,
                      double* host);
void launch_solve_y(hipStream_t st, int k, int R, KrylovScalars ks);

}  // namespace llg
