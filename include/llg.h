/*
 * llg.h -- C ABI of the MI355X library for one semi-implicit BDF1 step of the
 * damped Landau-Lifshitz equation, solved by aggregation-AMG-preconditioned
 * flexible GMRES on the GPU.
 *
 * The operation (paper, Sec. 2.1 and Sec. 2.2): given the magnetization m^n on
 * a uniform finite-difference grid with homogeneous Neumann boundaries, the
 * damping alpha and the time step dt, compute m^{n+1} from
 *
 *     (I + dt m^n x Delta_h + alpha dt m^n x (m^n x Delta_h)) u = m^n + dt F,
 *     m^{n+1} = u / |u|            (node by node; the projection of Sec. 4.3)
 *
 * where m^n is frozen in the operator (the semi-implicit linearization of
 * eq. BDF1_linearized, extended to the damped scheme).  The linear system
 * (eq. linear_system) is assembled as a 3x3-block sparse matrix and solved by
 * FGMRES preconditioned with one V-cycle of aggregation AMG (Sec. 3, Sec. 3.1:
 * two passes of pairwise matching per level, Boolean prolongation P of
 * eq. Pagg, Galerkin coarse matrices P^T A P of eq. galerkin computed by the
 * block sums of eq. Ac_direct).  All of it runs in HIP kernels on the GPU.
 *
 * Conventions for every entry point:
 *   - Fields are double[N][3], node-major, contiguous, node p = i + nx*(j + ny*k)
 *     (x fastest), N = nx*ny*nz; node p is the cell centre ((i+1/2)h, (j+1/2)h,
 *     (k+1/2)h).  Pointers named d_* are DEVICE pointers on the context's
 *     device; pointers named h_* are HOST pointers.  The caller owns every
 *     buffer it passes; the library never frees or retains them past the call.
 *   - Every call returns llg_status.  LLG_ERR_DEVICE carries a message that
 *     llg_last_error() returns (thread-local).  Arguments are validated before
 *     any device work; on an argument error nothing is launched.
 *   - All device work of a context runs on the HIP stream given to
 *     llg_create() (and, with opts.overlap_rebuild, on a second stream of
 *     the context for the next step's structure rebuild).  llg_step() returns
 *     after the step's work is complete.  One
 *     context must not be used from two threads at once; distinct contexts are
 *     independent and may run concurrently on distinct streams.
 *   - Device memory: llg_create() and llg_step() allocate no device memory;
 *     the caller lends one workspace of llg_workspace_bytes() bytes for the
 *     context's lifetime.  llg_workspace_bytes() itself runs the (field
 *     independent) aggregation once on the current device, using temporary
 *     device memory that it frees before returning, and caches the result per
 *     grid and options.
 */
#ifndef LLG_H
#define LLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LLG_MAX_LEVELS 40

typedef enum {
  LLG_OK = 0,
  LLG_ERR_INVALID_ARG = 1,   /* null/misaligned pointer, bad size or option, aliasing */
  LLG_ERR_UNSUPPORTED = 2,   /* boundary condition, or coarsest level above max_dense */
  LLG_ERR_WORKSPACE = 3,     /* workspace smaller than llg_workspace_bytes() */
  LLG_ERR_DEVICE = 4,        /* HIP runtime error or failed device-side consistency check */
  LLG_ERR_NOT_CONVERGED = 5, /* max_iters reached; the output is still written */
  LLG_ERR_NONFINITE = 6      /* non-finite m^n, or |u_i| = 0 / non-finite at projection */
} llg_status;

typedef enum { LLG_BC_NEUMANN = 0 } llg_bc;

typedef enum {
  LLG_PREC_FP64 = 0,     /* whole solve in FP64 */
  LLG_PREC_FP32_AMG = 1  /* AMG hierarchy and V-cycle in FP32 inside FP64 FGMRES */
} llg_precision;

/* Smoother of every level but the coarsest.
 * JACOBI: x += omega D^{-1} (b - A x), all rows at once.
 * MCGS: block Gauss-Seidel, x_i += D_i^{-1} (b_i - sum_j A_ij x_j) with the
 * current x, taken colour class by colour class (ascending before the coarse
 * correction, descending after it).  The classes are independent sets of the
 * level's graph: on level 0 the parity of i + j + k; on coarse levels the
 * greedy colouring in the order of ascending (SplitMix64((v << 32 | v) ^ salt), v),
 * salt = agg_salt ^ (level << 8 | 0x80), each node taking the smallest colour
 * none of its earlier neighbours has.  At most 128 colours per level. */
typedef enum { LLG_SMOOTHER_JACOBI = 0, LLG_SMOOTHER_MCGS = 1 } llg_smoother;

/* Time discretization: first-order backward differentiation with the field
 * frozen at m^n (Sec. 2.1), or second order with m~ = 2 m^n - m^{n-1}. */
typedef enum { LLG_SCHEME_BDF1 = 0, LLG_SCHEME_BDF2 = 1 } llg_scheme;

/* Storage of the grid-level operators A and D^{-1} A.
 * BSR: 3x3-block sliced ELL, one block per stored (row, column) (default).
 * FACTORED: on the grid every off-diagonal block of row p is the same block,
 * Mh_p = (dt/h^2) M_p in A and K_p = D_p^{-1} Mh_p in D^{-1} A (whose diagonal
 * blocks are the identity), so one block per node is stored and the
 * neighbours come from the grid: (A z)_p = z_p + Mh_p (sum_q z_q - deg_p z_p),
 * (D^{-1} A x)_p = x_p + K_p sum_q x_q.  The coarse levels are identical in
 * both forms; the grid-level products differ by rounding.  Requires
 * left_scale (else UNSUPPORTED); a grid whose first level is already the
 * coarsest is stored as BSR. */
typedef enum { LLG_FINE_BSR = 0, LLG_FINE_FACTORED = 1 } llg_fine_operator;

/* Orthogonalization of the FGMRES basis (all FP64).
 * CGS2: classical Gram-Schmidt, a second pass when the first removes more
 * than half of |w|^2 (three sweeps over the basis per iteration).
 * DCGS2 (default): classical Gram-Schmidt with the second pass of each basis
 * vector delayed to the next iteration (Swirydowicz, Langou, Ananthan, Yang,
 * Thomas 2021): two sweeps per iteration; the Hessenberg column of an
 * iteration is made final one iteration later, the residual estimate of the
 * newest column uses its first-pass entries, and the last column of a cycle
 * is made final before the least-squares solve. */
typedef enum { LLG_ARNOLDI_CGS2 = 0, LLG_ARNOLDI_DCGS2 = 1 } llg_arnoldi;

/* The solver of the linear system.  FGMRES_AMG is the method (FGMRES(restart)
 * preconditioned by the AMG cycle).  The others are the unpreconditioned
 * Krylov solvers the paper compares against (Sec. 4): GMRES(restart), BiCGstab
 * (van der Vorst 1992) and TFQMR (Freund 1993) on A itself, FP64 only (else
 * UNSUPPORTED); no AMG hierarchy is built for them.  BiCGstab and TFQMR count
 * an iteration per two products with A and restart from the current iterate
 * after a breakdown or when their recurrence meets rtol and the true
 * residual does not. */
typedef enum {
  LLG_KRYLOV_FGMRES_AMG = 0,
  LLG_KRYLOV_GMRES = 2,
  LLG_KRYLOV_BICGSTAB = 3,
  LLG_KRYLOV_TFQMR = 4
} llg_krylov;

typedef struct {
  int32_t dim;   /* 2 or 3 */
  int32_t n[3];  /* points per axis, each >= 2; n[2] == 1 when dim == 2 */
  double h;      /* isotropic grid spacing, > 0 (the unit square/cube: h = 1/n) */
  int32_t bc;    /* llg_bc; only homogeneous Neumann */
} llg_grid;

typedef struct {
  double rtol;          /* converged when ||b - A u||_2 <= rtol ||b||_2 (true residual) */
  int32_t restart;      /* FGMRES basis size per cycle, 1..32 */
  int32_t max_iters;    /* total FGMRES iterations */
  int32_t precision;    /* llg_precision */
  int32_t nu_pre, nu_post;  /* smoothing sweeps before / after the coarse correction, each 0..4 */
  double omega;         /* Jacobi damping; <= 0 selects 4/5 (2D) or 6/7 (3D) */
  int32_t npass;        /* pairwise matching passes per level, 1..3 */
  int32_t beta_num, beta_den;  /* strong coupling: den * w >= num * max_w */
  int32_t max_coarse;   /* stop coarsening at <= this many nodes */
  double stagnation;    /* stop if N_{l+1} > stagnation * N_l */
  int32_t max_levels;   /* <= LLG_MAX_LEVELS */
  int32_t max_dense;    /* largest coarsest level (nodes) for the dense solve */
  int32_t left_scale;   /* build the hierarchy on D^{-1} A (block-diagonal scaling) */
  int32_t project;      /* normalize u node by node */
  int32_t x0_is_mn;     /* initial guess m~ (m^n for BDF1; else 0) */
  uint64_t agg_salt;    /* salt of the hashed matching order */
  int32_t rebuild_aggregates; /* 1: recompute the matching every step (default) */
  int32_t kcycle_depth; /* coarse corrections of levels 1..depth by the K-cycle (two
                           minimal-residual steps, Sec. 3.1); 0 = V-cycle; 0..8 */
  int32_t graphs;       /* 1: replay the step's setup and each FGMRES iteration as HIP
                           graphs captured once per context; 0: eager launches (default:
                           measured faster, the device stays ahead of the host either way) */
  int32_t smoother;     /* llg_smoother: damped block Jacobi (default) or multicolour
                           block Gauss-Seidel (Sec. 3 smooths by Gauss-Seidel) */
  int32_t scheme;       /* llg_scheme: BDF1 (default) or BDF2, see llg_step */
  int32_t fine_operator; /* llg_fine_operator: storage of the grid level, see below */
  int32_t arnoldi;      /* llg_arnoldi: orthogonalization of the FGMRES basis, see below */
  int32_t krylov;       /* llg_krylov: the solver; the default is FGMRES with the AMG cycle */
  int32_t stray_field;  /* 1: reserve the stray-field workspace (zero-padded FFT grids and the
                           transformed demagnetizing tensor) for llg_step_field; 2*n-1 padded to a
                           power of two must stay <= 4096 per axis (else UNSUPPORTED) */
  int32_t tail_nodes;   /* block-Jacobi cycles: the coarse levels below the K-cycle levels (and
                           below level 1 when it is applied through the grid level), each of at
                           most this many nodes, run their whole V-cycle in one workgroup with
                           the level vectors on chip (same arithmetic, one launch instead of
                           three per level); 0 switches it off */
  int32_t pipeline;     /* 1: FGMRES enqueues the preconditioner and product of the next
                           iteration before the host tests the current one's residual
                           estimate (skipped where convergence is predicted); 0: off */
  int32_t overlap_rebuild; /* 1 (with rebuild_aggregates, the AMG solver and graphs off): the
                           field-independent hierarchy structure (matching, coarse graphs,
                           patterns) is kept in two copies, and the copy the next step uses is
                           rebuilt on a second HIP stream while the current step assembles
                           and solves; the workspace holds the structure twice.  llg_step
                           still returns when its own step is complete; the rebuild may still
                           run then, and llg_destroy waits for it.  0: each step rebuilds
                           the structure before its assembly, on the context's stream */
  int32_t csr_levels;   /* 1: the row products of the large coarse levels (at least 32768 nodes,
                           block-Jacobi cycles, below the K-cycle levels, not the coarsest) read
                           the blocks in CSR order, the copy the next Galerkin product reads,
                           and no sliced-ELL values are kept for them; 0: sliced-ELL values */
} llg_opts;

typedef struct {
  int32_t iters, restarts, levels, converged;
  double relres_est, relres_true;
  int64_t level_nodes[LLG_MAX_LEVELS];
  int64_t level_nnzb[LLG_MAX_LEVELS];
  double ms_setup;   /* assembly + hierarchy + coarsest factorization */
  double ms_solve;   /* FGMRES */
  double ms_total;
  /* timing of one kernel class selected by llg_set_kernel_timing() */
  double kernel_ms;
  int64_t kernel_launches;
  int32_t reorth_passes;  /* Arnoldi steps that needed a second Gram-Schmidt pass */
  int32_t tail_level;     /* first level of the one-workgroup coarse cycle (opts.tail_nodes); 0 = none */
  double kernel_bytes;    /* algorithmic bytes of the timed launches (LLG_KT_LEVEL1: every launch's
                             operands read once and results written once), 0 for the other classes */
} llg_stats;

typedef struct llg_ctx llg_ctx;

/* Kernel classes that llg_set_kernel_timing() can time with HIP events. */
typedef enum {
  LLG_KT_NONE = 0,
  LLG_KT_OUTER_SPMV = 1,   /* w = A z, FP64 fine operator */
  LLG_KT_SMOOTH = 2,       /* damped block-Jacobi sweeps, all levels */
  LLG_KT_RESIDUAL = 3,     /* r = b - A x with restriction, all levels */
  LLG_KT_ARNOLDI = 4,      /* multi-dot and update passes of the Gram-Schmidt step */
  LLG_KT_GALERKIN = 5,     /* P^T A P values */
  LLG_KT_ASSEMBLE = 6,     /* fine operator assembly */
  LLG_KT_LEVEL1 = 7        /* level-1 products applied through the grid level's blocks (every mode) */
} llg_kernel_class;

/* Defaults: rtol 1e-10, restart 30, max_iters 1000, FP64, nu 1/1, omega by
 * dimension, npass 2, beta 1/4, max_coarse 40, stagnation 0.8, max_levels 40,
 * max_dense 512, left_scale 1, project 1, x0_is_mn 1, salt 0, rebuild 1,
 * K-cycle depth 0, graphs 0, Jacobi, BDF1, BSR grid level, DCGS2, FGMRES with
 * the AMG cycle, no stray-field workspace, tail_nodes 128, pipeline 1,
 * overlap_rebuild 1, csr_levels 1. */
void llg_default_opts(llg_opts* opts);

/* Exact device bytes a context for (grid, opts) needs.  Runs the aggregation
 * of the grid graph on the current device (field independent).  Errors:
 * INVALID_ARG, UNSUPPORTED, DEVICE. */
llg_status llg_workspace_bytes(const llg_grid* grid, const llg_opts* opts, size_t* bytes);

/* Create a context on the current device.  d_workspace: device memory of at
 * least llg_workspace_bytes() bytes, 256-byte aligned, lent until
 * llg_destroy().  hip_stream: a hipStream_t (NULL = default stream).
 * Builds the grid pattern and the aggregation hierarchy structure. */
llg_status llg_create(const llg_grid* grid, const llg_opts* opts, void* d_workspace,
                      size_t bytes, void* hip_stream, llg_ctx** out);

/* One time step.  d_m_n: m^n (N x 3); alpha >= 0 and dt > 0 finite;
 * d_forcing: F (N x 3) or NULL; d_m_np1: output m^{n+1}, must not overlap
 * d_m_n or d_m_nm1.  stats may be NULL.  NOT_CONVERGED still writes d_m_np1
 * (the projected last iterate) and stats.
 * BDF1 (Sec. 2.1): the system frozen at m~ = m^n, b = m^n + dt F; d_m_nm1 is
 * not read (may be NULL).
 * BDF2 (opts.scheme): (3 u - 4 m^n + m^{n-1}) / (2 dt) = -m~ x Lap u
 * - alpha m~ x (m~ x Lap u) + F with m~ = 2 m^n - m^{n-1}, i.e. the BDF1
 * operator frozen at m~ with dt' = 2 dt / 3 and b = (4 m^n - m^{n-1}) / 3
 * + dt' F.  d_m_nm1 = m^{n-1} (N x 3); when it is NULL the step is a BDF1
 * step (the usual start of a BDF2 run).  The initial guess is m~. */
llg_status llg_step(llg_ctx* ctx, const double* d_m_n, const double* d_m_nm1, double alpha,
                    double dt, const double* d_forcing, double* d_m_np1, llg_stats* stats);

/* The field of the full model (Sec. 2): m_t = -m x (eps Lap m + f) - alpha m x (m x (eps Lap m + f)),
 * f = -q (m2 e2 + m3 e3) + h_s + h_ext.  eps > 0 scales the Laplacian; q is the
 * uniaxial anisotropy along e1; h_ext a uniform external field; stray = 1 adds
 * the stray field h_s = -N * m of the magnetization, the convolution with the
 * cell-averaged demagnetizing tensor of the grid's cubic cells of side h
 * (Newell, Williams and Dunlop 1993; beyond 16 cells the point-dipole tensor;
 * a 2D grid is one layer of cells).  f is explicit, taken at m~. */
typedef struct {
  double eps;
  double q;
  double h_ext[3];
  int32_t stray;
} llg_field;

/* One step of the full model: the operator of llg_step with dt' eps in place
 * of dt' (dt' = dt for BDF1, 2 dt / 3 for BDF2) and the right-hand side
 * b - dt' (m~ x f + alpha m~ x (m~ x f)).  field NULL: llg_step.  stray = 1
 * needs a context created with opts.stray_field (else INVALID_ARG); the
 * tensor is transformed on the first such call.  Other arguments and errors
 * as llg_step. */
llg_status llg_step_field(llg_ctx* ctx, const double* d_m_n, const double* d_m_nm1, double alpha, double dt,
                          const llg_field* field, const double* d_forcing, double* d_m_np1, llg_stats* stats);

/* d_h = h_s(d_m), the stray field of a device field (N x 3 each), for a
 * context created with opts.stray_field (else INVALID_ARG).  Synchronizes the
 * stream. */
llg_status llg_stray_field(llg_ctx* ctx, const double* d_m, double* d_h);

/* The stray field without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid allocation):
 * d_h = h_s(d_m) on `grid` as llg_stray_field computes it, with the transformed
 * tensor and the FFT work planes in a static device array of
 * LLG_STRAY_NOALLOC_MAX_BYTES bytes that every device the library runs on
 * holds until the process ends.  The call allocates nothing.  It needs
 * 80 P bytes, P = the padded cell count (each axis of n > 1 cells padded to
 * the power of two >= 2 n - 1): 2D grids up to 512 x 512 and 3D grids up to
 * 64^3 fit; larger grids return UNSUPPORTED.  The array keeps the last call's
 * contents (the tensor is recomputed only when the grid's dimensions change);
 * calls that overlap on one device race.  All work runs on hip_stream (NULL =
 * the default stream), which is synchronized before returning.  d_m and d_h:
 * N x 3 doubles each.  Errors: INVALID_ARG, UNSUPPORTED, DEVICE. */
#define LLG_STRAY_NOALLOC_MAX_BYTES ((size_t)176160768) /* 168 MiB */
llg_status llg_stray_field_noalloc(const llg_grid* grid, const double* d_m, double* d_h, void* hip_stream);

/* Host copy of the cell-averaged demagnetizing tensor the stray field uses
 * (eq. stray_field with m constant on the cubic cells of side h; Newell,
 * Williams and Dunlop 1993 for cells within one cell of each other, the
 * cell average of the point-dipole kernel by quadrature up to 16 cells, the
 * point dipole beyond), as the device computes it, for every cell offset
 * k in [-(n_d - 1), n_d - 1] per axis: h_out[c][kz][ky][kx] with index
 * kx + (n_x - 1) fastest, c = 0..5 for xx, yy, zz, xy, xz, yz;
 * cap >= 6 (2 n_x - 1)(2 n_y - 1)(2 n_z - 1) doubles.  The entries do not
 * depend on h.  Needs a context created with opts.stray_field (else
 * INVALID_ARG).  Overwrites the stray-field work area (not the transformed
 * tensor).  Synchronizes the stream.  For parity tests. */
llg_status llg_get_demag_tensor(llg_ctx* ctx, double* h_out, int64_t cap);

/* Assemble the operator for the frozen field d_m_tilde and build the AMG
 * hierarchy values (what llg_step does before the Krylov solve).  Used with
 * the inspection calls below. */
llg_status llg_setup(llg_ctx* ctx, const double* d_m_tilde, double alpha, double dt);

/* Number of levels of the hierarchy, and the size of one level.  level -1 is
 * the unscaled fine operator A; levels 0.. are the hierarchy (level 0 is
 * D^{-1} A when left_scale is on). */
llg_status llg_num_levels(llg_ctx* ctx, int32_t* levels);
llg_status llg_level_info(llg_ctx* ctx, int32_t level, int64_t* n, int64_t* nnzb);

/* Host copy of a level in BSR form: h_row_ptr[n+1], h_col[nnzb] ascending per
 * row, h_vals[nnzb][3][3] row-major (FP32 levels are widened to double).  A
 * factored grid level is expanded to the blocks its products apply (the
 * diagonal block of level -1 is then I - deg_p Mh_p).
 * cap_nnzb is the capacity of h_col (blocks).  Synchronizes the stream. */
llg_status llg_get_level(llg_ctx* ctx, int32_t level, int32_t* h_row_ptr, int32_t* h_col,
                         double* h_vals, int64_t cap_nnzb);

/* Host copy of the aggregate map of `level` (node -> aggregate on level+1),
 * n entries.  Synchronizes the stream. */
llg_status llg_get_aggregates(llg_ctx* ctx, int32_t level, int32_t* h_out, int64_t n);

/* Host copy of the colour class of every node of `level` (multicolour
 * Gauss-Seidel smoother only; not the coarsest level), n entries, and the
 * number of classes in *h_ncol.  INVALID_ARG when the context smooths by
 * Jacobi.  Synchronizes the stream. */
llg_status llg_get_colours(llg_ctx* ctx, int32_t level, int32_t* h_out, int64_t n, int32_t* h_ncol);

/* z = B v: one V-cycle applied to D^{-1} v (the FGMRES preconditioner), both
 * FP64 device vectors of 3N entries.  Requires a prior llg_setup/llg_step. */
llg_status llg_apply_precond(llg_ctx* ctx, const double* d_v, double* d_z);

/* y = A x with the unscaled FP64 fine operator.  Requires a prior setup. */
llg_status llg_apply_A(llg_ctx* ctx, const double* d_x, double* d_y);

/* Time every launch of one kernel class with HIP events on the context's
 * stream; the totals are reported in llg_stats.kernel_ms/kernel_launches of
 * each subsequent llg_step.  LLG_KT_NONE switches timing off. */
llg_status llg_set_kernel_timing(llg_ctx* ctx, int32_t kernel_class);

/* Bytes the context uses inside its workspace. */
llg_status llg_ctx_bytes(llg_ctx* ctx, size_t* bytes);

llg_status llg_destroy(llg_ctx* ctx);

const char* llg_status_str(llg_status status);
const char* llg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LLG_H */
