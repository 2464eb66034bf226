/*
 * llgo.h -- FP64 CPU oracle for one semi-implicit BDF1 Landau-Lifshitz step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker that the HIP path is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the HIP library: everything here is written out
 * plainly, single threaded, in double precision, built with -ffp-contract=off.
 *
 * What it computes (paper references are to sections, equations, tables):
 *   - the damped semi-implicit BDF1 scheme of Sec. 2.1 (the component-wise
 *     form of the damped linear system) on a cell-centred finite-difference
 *     grid with homogeneous Neumann boundaries (Sec. 2.2 leaves the spatial
 *     discretization open; mirrored ghosts are the reading taken here);
 *   - the 3x3-block sparse operator A = I + dt * M_i * (L (x) I3);
 *   - an aggregation AMG hierarchy (Sec. 3.1, Sec. 3.1.1): two passes of
 *     pairwise matching per level, Boolean prolongation (eq. Pagg), Galerkin
 *     coarse operators computed by block sums (eq. galerkin, eq. Ac_direct);
 *   - one V-cycle (damped block Jacobi smoothing, or multicolour block
 *     Gauss-Seidel in the spirit of the Gauss-Seidel smoother of Sec. 3; exact
 *     dense LU at the coarsest level) as preconditioner of a restarted flexible GMRES,
 *     or of the preconditioned GCR of Algorithm 1 (Sec. 3.1.2);
 *   - the projection m <- m/|m| (Sec. 4.3).
 *
 * Layout: a field on the grid is double[N][3], node-major, node index
 * p = i + nx*(j + ny*k).  BSR matrices: int64 row_ptr[n+1], int32 col[nnzb]
 * (ascending within a row, diagonal always present), double val[nnzb][3][3]
 * row-major inside each block.  All pointers are host pointers owned by the
 * caller.  Functions return 0 on success and a negative code on failure.
 */
#ifndef LLGO_H
#define LLGO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  LLGO_OK = 0,
  LLGO_ERR_ARG = -1,          /* bad argument */
  LLGO_ERR_UNSUPPORTED = -2,  /* coarsest level too large for the dense solve */
  LLGO_ERR_NOT_CONVERGED = -5,
  LLGO_ERR_NONFINITE = -6
};

typedef struct {
  int32_t dim;   /* 2 or 3 */
  int32_t n[3];  /* points per axis; n[2] == 1 when dim == 2 */
  double h;      /* isotropic spacing */
} llgo_grid;

typedef struct {
  double rtol;          /* stop when ||b - A u|| <= rtol ||b|| */
  int32_t restart;      /* Krylov basis size per cycle */
  int32_t max_iters;    /* total iterations */
  int32_t nu_pre, nu_post;
  double omega;         /* Jacobi damping; <= 0 selects 4/5 (2D) or 6/7 (3D) */
  int32_t npass;        /* pairwise matching passes per level */
  int32_t beta_num, beta_den;  /* strength threshold beta = num/den */
  int32_t max_coarse;   /* stop coarsening at <= this many nodes */
  double stagnation;    /* stop if N_{l+1} > stagnation * N_l */
  int32_t max_levels;
  int32_t max_dense;    /* largest coarsest level (nodes) for the dense LU */
  int32_t left_scale;   /* build the hierarchy on D^{-1} A */
  int32_t project;      /* normalize the solution node by node */
  int32_t x0_is_mn;     /* initial guess m^n (else zero) */
  uint64_t agg_salt;
  int32_t krylov;       /* 0 = FGMRES + AMG, 1 = GCR + AMG (Algorithm 1); baselines without
                           preconditioner: 2 = GMRES(restart), 3 = BiCGstab, 4 = TFQMR */
  int32_t kcycle_depth; /* coarse corrections of levels 1..depth by the K-cycle (0: V-cycle) */
  int32_t smoother;     /* 0: damped block Jacobi; 1: multicolour block Gauss-Seidel */
} llgo_opts;

typedef struct {
  int32_t iters, restarts, levels, converged;
  double relres_est, relres_true;
} llgo_stats;

void llgo_default_opts(llgo_opts* o);

/* SplitMix64 finalizer applied to x + golden gamma (Steele, Lea, Flood 2014). */
uint64_t llgo_splitmix64(uint64_t x);

/* One pass of pairwise matching on an integer-weighted graph (CSR, no self
 * loops, symmetric).  agg[n] receives aggregate ids, mate[n] the partner or -1,
 * *nc the number of aggregates. */
int llgo_match_pass(int64_t n, const int64_t* rp, const int32_t* ci, const int64_t* w,
                    uint64_t salt, int32_t beta_num, int32_t beta_den,
                    int32_t* agg, int32_t* mate, int64_t* nc);

/* Galerkin product P^T A P of a 3x3 BSR matrix for Boolean P given by agg.
 * Call with out arrays NULL to get *nnzb_c; then call again with storage. */
/* The field-independent aggregation hierarchy of the grid graph alone (the
 * matching passes, coarse graphs and stopping rules of llgo_setup, without
 * any matrix values): *levels levels, level_nodes[0..levels-1] (at least
 * max_levels entries), and the aggregate maps of levels 0..levels-2
 * concatenated in agg (node -> aggregate on the next level; cap entries;
 * LLGO_ERR_ARG when it is too small). */
int llgo_aggregate_levels(const llgo_grid* g, const llgo_opts* o, int32_t* levels, int64_t* level_nodes,
                          int32_t* agg, int64_t cap);

int llgo_galerkin(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                  const int32_t* agg, int64_t nc,
                  int64_t* nnzb_c, int64_t* rp_c, int32_t* ci_c, double* val_c);

/* Assemble the unscaled operator A for the frozen field m_tilde. */
int llgo_assemble_nnzb(const llgo_grid* g, int64_t* nnzb);
int llgo_assemble(const llgo_grid* g, const double* m_tilde, double alpha, double dt,
                  int64_t* rp, int32_t* ci, double* val);

/* Hierarchy handle: assembly, scaling, aggregation and Galerkin levels. */
void* llgo_setup(const llgo_grid* g, const llgo_opts* o, const double* m_tilde,
                 double alpha, double dt, int* status);
void llgo_free(void* h);
int llgo_num_levels(void* h);
/* level -1 is the unscaled fine operator A; level 0.. are the hierarchy. */
int llgo_level_info(void* h, int level, int64_t* n, int64_t* nnzb);
int llgo_level_matrix(void* h, int level, int64_t* rp, int32_t* ci, double* val);
int llgo_level_dinv(void* h, int level, double* dinv);
int llgo_level_agg(void* h, int level, int32_t* agg);  /* map level -> level+1 */
/* Colour of every node of a smoothed level (multicolour Gauss-Seidel only);
 * *ncol receives the number of colours. */
int llgo_level_colour(void* h, int level, int32_t* colour, int32_t* ncol);
int llgo_apply_A(void* h, const double* x, double* y);
int llgo_precond(void* h, const double* v, double* z);
int llgo_solve(void* h, const double* b, const double* u0, double* u, llgo_stats* st);

/* One full step: m_np1 = P(A^{-1} (m_n + dt F)), F may be NULL. */
int llgo_step(const llgo_grid* g, const llgo_opts* o, const double* m_n, double alpha,
              double dt, const double* F, double* m_np1, llgo_stats* st);

/* One BDF2 step with m~ = 2 m^n - m^{n-1}: the system of llgo_step frozen at
 * m~ with dt' = 2 dt / 3 and right-hand side (4 m^n - m^{n-1}) / 3 + dt' F. */
int llgo_step2(const llgo_grid* g, const llgo_opts* o, const double* m_n, const double* m_nm1,
               double alpha, double dt, const double* F, double* m_np1, llgo_stats* st);

/* Full field of the nondimensional model (Sec. 2): exchange coefficient eps,
 * uniaxial anisotropy q along e1, uniform external field h_ext, and the stray
 * field of the magnetization (stray != 0). */
typedef struct {
  double eps;
  double q;
  double h_ext[3];
  int32_t stray;
} llgo_field;

/* Cell-averaged demagnetizing tensor between two cuboid cells dx x dy x dz
 * whose centres differ by (X, Y, Z): N[0..5] = xx, yy, zz, xy, xz, yz.  Newell,
 * Williams and Dunlop (1993) when max(|X|/dx, |Y|/dy, |Z|/dz) <= 16, the
 * point-dipole tensor -(V / 4 pi)(3 r r^T / r^2 - I) / r^3 beyond. */
void llgo_demag_tensor(double X, double Y, double Z, double dx, double dy, double dz, double* N);

/* Stray field h = -sum_j N(x_i - x_j) m_j of a field on the grid (cubic cells
 * of side h; a 2D grid is one layer of cells). */
int llgo_stray_field(const llgo_grid* g, const double* m, double* h);

/* The same sum at `count` cells only (h[count][3]): each cell's field summed
 * directly over every cell of the grid, for grids too large for the full
 * O(N^2) form. */
int llgo_stray_field_at(const llgo_grid* g, const double* m, const int64_t* cells, int64_t count, double* h);

/* One step of the full model: u + dt' eps (m~ x Lap u + alpha m~ x (m~ x Lap u))
 * = b0 - dt' (m~ x f + alpha m~ x (m~ x f)), f = -q (0, m~2, m~3) + h_ext + h_s(m~),
 * with BDF1 (m_nm1 NULL: m~ = m^n, b0 = m^n, dt' = dt) or BDF2 (m~ = 2 m^n - m^{n-1},
 * b0 = (4 m^n - m^{n-1}) / 3, dt' = 2 dt / 3); F adds dt' F to b0. */
int llgo_step_field(const llgo_grid* g, const llgo_opts* o, const double* m_n, const double* m_nm1, double alpha,
                    double dt, const llgo_field* fld, const double* F, double* m_np1, llgo_stats* st);

#ifdef __cplusplus
}
#endif
#endif
