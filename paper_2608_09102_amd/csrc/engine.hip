// engine.hip -- host side of the library: workspace planning, hierarchy
// construction, V-cycle, FGMRES driver, the time step and the C ABI.
//
// Planning.  The aggregation depends only on the grid graph (its edge weights
// are integers, m-independent), so the sizes of every hierarchy level are a
// function of the grid and the options.  llg_workspace_bytes() runs the
// structure build once in PLAN mode: buffers are allocated as they are
// requested, every size the host needs (aggregate counts, graph sizes, slot
// counts, handshake rounds) is read back and logged.  A context replays the
// same code in REPLAY mode: buffer requests are served from the caller's
// workspace in the same order, logged sizes are used instead of read-backs,
// and each logged value is re-checked on the device (a mismatch sets a flag
// that turns into LLG_ERR_DEVICE).  The per-step rebuild therefore needs no
// host round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/llg.h"
#include "llg_internal.h"

namespace llg {

namespace {

thread_local std::string g_err;

void set_err(const std::string& s) { g_err = s; }

struct DevError {
  std::string msg;
};

#define HIPX(expr)                                                                                 \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      throw DevError{std::string(#expr) + ": " + hipGetErrorString(e_) + " @" + std::to_string(__LINE__)}; \
  } while (0)

inline void check_launch(int line) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw DevError{std::string("kernel launch: ") + hipGetErrorString(e) + " @" + std::to_string(line)};
}
#define LCHK() check_launch(__LINE__)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// device flag bits
constexpr int32_t F_NONFINITE_IN = 1, F_SINGULAR = 2, F_PROJECT = 4, F_PLAN = 8;

enum class Mode { PLAN, REPLAY };

struct Plan {
  std::vector<size_t> sizes;     // every buffer request, in order
  std::vector<uint8_t> lazy;     // request is not materialized in PLAN mode
  std::vector<int64_t> counts;   // every host-visible count, in order
  size_t total = 0;
  size_t struct_bytes = 0;       // bytes of the structure's requests (the first ones)
  bool dbl = false;              // a second copy of the structure (the overlapped rebuild)
  int status = LLG_OK;
};

// Buffer and count provider for the structure build (see file comment).
struct Arena {
  Mode mode;
  Plan* plan;
  bool first = true;              // REPLAY: first pass assigns addresses
  std::vector<void*>* ptrs;       // REPLAY: addresses by request index
  char* base = nullptr;
  size_t cap = 0, off = 0;
  size_t ri = 0, ci = 0;
  std::vector<void*> owned;       // PLAN: temporary allocations
  hipStream_t st = nullptr;
  int32_t* flag = nullptr;        // REPLAY: mismatch flag
  int flag_word = 0;              // word of the flags the checks raise (1: a rebuild on the second stream)
  bool keep_grid = false;         // REPLAY of a step: the grid graph and the grid level's pattern (field and
                                  // aggregation independent) are already in place; skip their kernels
  int32_t* hcount = nullptr;      // PLAN: pinned read-back slot

  void* get(size_t bytes, bool lazy) {
    bytes = align_up(bytes ? bytes : ALIGN);
    if (mode == Mode::PLAN) {
      plan->sizes.push_back(bytes);
      plan->lazy.push_back(lazy ? 1 : 0);
      plan->total += bytes;
      if (lazy) return nullptr;
      void* p = nullptr;
      HIPX(hipMalloc(&p, bytes));
      owned.push_back(p);
      return p;
    }
    if (ri >= plan->sizes.size() || plan->sizes[ri] != bytes)
      throw DevError{"workspace layout differs from the plan"};
    void* p;
    if (first) {
      if (off + bytes > cap) throw DevError{"workspace overflow"};
      p = base + off;
      off += bytes;
      ptrs->push_back(p);
    } else {
      p = (*ptrs)[ri];
    }
    ++ri;
    return p;
  }
  template <typename X>
  X* alloc(int64_t n) { return (X*)get((size_t)std::max<int64_t>(n, 1) * sizeof(X), false); }
  template <typename X>
  X* lazy(int64_t n) { return (X*)get((size_t)std::max<int64_t>(n, 1) * sizeof(X), true); }

  // host-visible count stored at device address p
  // REPLAY: the logged count replaces the read-back, and the device value is
  // checked against it.  Counts in buffers that nothing overwrites during
  // the step (defer) are checked together, CHECK_BATCH per launch, when the
  // batch fills and at flush_checks(); a count in reused scratch is checked
  // at once.
  std::vector<const int32_t*> chk_p;
  std::vector<int32_t> chk_v;
  int64_t count(const int32_t* p, bool defer = true) {
    if (mode == Mode::PLAN) {
      HIPX(hipMemcpyAsync(hcount, p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPX(hipStreamSynchronize(st));
      plan->counts.push_back(*hcount);
      return *hcount;
    }
    if (ci >= plan->counts.size()) throw DevError{"count log exhausted"};
    const int64_t v = plan->counts[ci++];
    if (defer) {
      chk_p.push_back(p);
      chk_v.push_back((int32_t)v);
      if ((int)chk_p.size() == CHECK_BATCH) flush_checks();
    } else {
      launch_check_eq(st, p, (int32_t)v, flag, F_PLAN);
      LCHK();
    }
    return v;
  }
  void flush_checks() {
    if (chk_p.empty()) return;
    launch_check_many(st, chk_p.data(), chk_v.data(), (int)chk_p.size(), flag, F_PLAN);
    LCHK();
    chk_p.clear();
    chk_v.clear();
  }
  void release() {
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
  }
};

struct Level {
  Sell A;
  int32_t* brp = nullptr;  // BSR pattern (CSR) of the level
  int32_t* bci = nullptr;
  int64_t nnzb = 0;
  int32_t *grp = nullptr, *gci = nullptr, *gw = nullptr;  // integer graph
  int64_t gnnz = 0;
  int32_t *agg = nullptr, *mptr = nullptr, *mem = nullptr;  // to the next level
  int64_t nc = 0;
  void* val = nullptr;
  void* dinv = nullptr;
  bool unit = false;
  int G = 1;  // lanes per row in the level's sliced-ELL kernels
  bool csr = false;  // row products on the CSR-ordered copy vt (no sliced-ELL values)
  void *b = nullptr, *x = nullptr, *r = nullptr, *e = nullptr, *xo = nullptr;
  // K-cycle work vectors and coefficients (levels 1..kcycle_depth)
  void *v1 = nullptr, *v2 = nullptr, *w1 = nullptr, *w2 = nullptr, *rho = nullptr;
  double* kc = nullptr;
  // multicolour Gauss-Seidel: the colour of every node, the rows sorted by
  // colour (class q is perm[coff[q] .. coff[q+1])), and every class as a
  // sliced-ELL matrix with its own copy of the values and inverse diagonals
  int32_t* colour = nullptr;
  int32_t* perm = nullptr;
  int ncol = 0;
  std::vector<int64_t> coff;
  std::vector<Sell> cls;
  std::vector<void*> cval, cdinv;
  void* kf = nullptr;  // factored grid level: K_p per node ([slice][9][64])
  void* knm = nullptr;  // the same, node-major (9 contiguous values per node)
  void* vt = nullptr;  // coarse levels feeding a Galerkin product: the blocks in slot order (9 per slot)
  void* xp = nullptr;  // level 1 applied through the grid blocks: x + P e_c before the post-smoothing sweep
  double* prho = nullptr;  // K-cycle levels: partial sums of w1.rho
  void* mtq = nullptr;  // the frozen field in member order of the level-1 aggregates (mt[mem[q]]), in T
  int32_t* nagg = nullptr;  // level-1 aggregates of each member's grid neighbours ([slice][6][64])
};

// The parts of a level that the structure build writes (pattern, graph,
// aggregates, members, colour classes); two copies of these exist when the
// next step's structure is rebuilt on a second stream.
struct LevelStruct {
  Sell A;
  int32_t *brp = nullptr, *bci = nullptr;
  int64_t nnzb = 0;
  int32_t *grp = nullptr, *gci = nullptr, *gw = nullptr;
  int64_t gnnz = 0;
  int32_t *agg = nullptr, *mptr = nullptr, *mem = nullptr;
  int64_t nc = 0;
  int32_t *colour = nullptr, *perm = nullptr;
  int ncol = 0;
  std::vector<int64_t> coff;
  std::vector<Sell> cls;
};
struct StructSet {
  LevelStruct lv[LLG_MAX_LEVELS];
  int L = 0;
  int32_t *flags = nullptr, *count = nullptr, *scan_tmp = nullptr;
};

struct PlanKey {
  std::tuple<int, int, int, int, int, int, int, int, double, int, int, uint64_t, int, int, int, int, int, int, int,
             int, int>
      k;
  bool operator<(const PlanKey& o) const { return k < o.k; }
};

std::mutex g_plan_mu;
std::map<PlanKey, std::shared_ptr<Plan>> g_plans;

// the next step's structure is rebuilt on a second stream during the current
// step (double-buffered): AMG solves that rebuild every step, without graphs
bool overlapped_rebuild(const llg_opts& o) {
  return o.overlap_rebuild && o.rebuild_aggregates && o.krylov == LLG_KRYLOV_FGMRES_AMG && !o.graphs;
}

PlanKey plan_key(const llg_grid& g, const llg_opts& o) {
  PlanKey k;
  k.k = std::make_tuple(g.dim, g.n[0], g.n[1], g.n[2], o.npass, o.beta_num, o.beta_den, o.max_coarse,
                        o.stagnation, o.max_levels, o.max_dense, o.agg_salt, o.precision, o.restart,
                        o.left_scale, o.kcycle_depth, o.smoother, o.scheme, o.fine_operator, o.krylov,
                        o.stray_field * 4 + o.csr_levels * 2 + (overlapped_rebuild(o) ? 1 : 0));
  return k;
}

}  // namespace
}  // namespace llg

struct llg_ctx {
  llg_grid grid;
  llg_opts opts;
  int device = 0;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0, used = 0;
  std::shared_ptr<llg::Plan> plan;
  std::vector<void*> ptrs;
  int L = 0;
  llg::Level lv[LLG_MAX_LEVELS];
  double omega = 0;
  int64_t N = 0;
  // fine operator (FP64) and its inverse diagonal blocks; in the factored
  // form the per-node off-diagonal block Mh replaces the sliced-ELL values
  double* Aval = nullptr;
  double* dinv0 = nullptr;
  bool fact = false;
  bool f1 = false;  // level-1 products from the grid level's per-node blocks
  // levels tail.. run their V-cycle in one workgroup (0: none)
  int tail = 0;
  bool tail_ok = false;
  llg::TailArgs<double> ta64{};
  llg::TailArgs<float> ta32{};
  double* Mh = nullptr;
  double* mt = nullptr;  // factored grid level: the frozen field, from which the solve kernels recompute blocks
  // coarsest
  int64_t nd = 0;
  double* dense = nullptr;
  int32_t* piv = nullptr;
  // Krylov
  double *u = nullptr, *b = nullptr, *r = nullptr, *w = nullptr, *V = nullptr;
  void* Z = nullptr;
  int64_t ld = 0;
  double* part = nullptr;
  int64_t npart_vec = 0, npart_rows = 0;
  llg::KrylovScalars ks{};
  double* delta = nullptr;
  int32_t* flags = nullptr;
  int32_t* count = nullptr;
  int32_t* scan_tmp = nullptr;
  // overlapped rebuild: two structure sets, the one the current step uses
  // (loaded into lv[], flags, count, scan_tmp) and the one being rebuilt on
  // the second stream for the next step
  bool dbl = false;
  int set = 0;
  llg::StructSet sets[2];
  std::vector<void*> ptrs2;  // addresses of the second set's structure requests
  hipStream_t aux = nullptr;
  hipEvent_t built[2] = {nullptr, nullptr};
  hipEvent_t main_ev = nullptr;
  double* host = nullptr;     // pinned scalars
  int32_t* hflags = nullptr;  // pinned flags
  bool setup_done = false;
  // HIP graphs: the step's setup (two variants: without / with forcing) and
  // one graph per FGMRES iteration index j, captured on a private stream
  hipStream_t cap_st = nullptr;
  bool capturing = false;
  bool graphs_ok = true;
  hipGraphExec_t setup_graph[16] = {};  // [forcing + 2 bdf2 + 4 field + 8 stray]
  hipGraphExec_t kb_graph = nullptr;  // one iteration of a Krylov baseline
  double* kb = nullptr;                // device scalars of the Krylov baselines
  std::vector<hipGraphExec_t> pc_graph;  // preconditioner of iteration j
  std::vector<hipGraphExec_t> it_graph;  // Gram-Schmidt of iteration j
  double* prm = nullptr;          // device: alpha, dt
  double* hprm = nullptr;         // pinned staging for prm
  double* min = nullptr;          // device copy of m^n read by the setup graph
  double* mprv = nullptr;         // device copy of m^{n-1} (BDF2)
  // stray field: padded grid, transformed tensor (once per context) and work
  llg::FieldDims fd;
  double* nhat = nullptr;
  double2* fwork = nullptr;
  bool demag_ready = false;
  // timing of one kernel class
  int timed = LLG_KT_NONE;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  hipEvent_t it_ev = nullptr;  // end of an FGMRES iteration's orthogonalization (pipelined loop)
  double kernel_ms = 0;
  int64_t launches = 0;
  double kernel_bytes = 0;  // algorithmic bytes of the timed launches (level-1 class)
};

namespace llg {
namespace {

// ------------------------------------------------------------------ timing
struct KTimer {
  llg_ctx& c;
  bool on;
  KTimer(llg_ctx& cc, int cls) : c(cc), on(cc.timed == cls && !cc.capturing) {
    if (!on) return;
    if (c.ev_used + 2 > c.ev.size()) {
      for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        HIPX(hipEventCreate(&e));
        c.ev.push_back(e);
      }
    }
    HIPX(hipEventRecord(c.ev[c.ev_used], c.st));
  }
  ~KTimer() {
    if (!on) return;
    (void)hipEventRecord(c.ev[c.ev_used + 1], c.st);
    c.ev_used += 2;
  }
};

// A pair of timing events for one launch of class cls that stamps them
// itself (both null when cls is not timed or the stream is being captured).
void kernel_events(llg_ctx& c, int cls, hipEvent_t& e0, hipEvent_t& e1) {
  e0 = e1 = nullptr;
  if (c.timed != cls || c.capturing) return;
  if (c.ev_used + 2 > c.ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      HIPX(hipEventCreate(&e));
      c.ev.push_back(e);
    }
  }
  e0 = c.ev[c.ev_used];
  e1 = c.ev[c.ev_used + 1];
  c.ev_used += 2;
}

// after a stream synchronization: add up the recorded kernel intervals
// Add up the timing pairs recorded before index `upto` (all by default, once
// the stream is idle); later pairs move to the front of the pool.
void harvest(llg_ctx& c, size_t upto = SIZE_MAX) {
  upto = std::min(upto, c.ev_used);
  for (size_t k = 0; k + 1 < upto; k += 2) {
    float ms = 0;
    HIPX(hipEventElapsedTime(&ms, c.ev[k], c.ev[k + 1]));
    c.kernel_ms += ms;
    c.launches += 1;
  }
  std::rotate(c.ev.begin(), c.ev.begin() + upto, c.ev.begin() + c.ev_used);
  c.ev_used -= upto;
}

void sync(llg_ctx& c) {
  HIPX(hipStreamSynchronize(c.st));
  harvest(c);
}

// ------------------------------------------------------------------ structure
// build: false when the pattern is already in place (the grid level on a
// step's replay): the buffers are requested and the counts taken, no kernel runs
void build_sell(Arena& ar, hipStream_t st, Level& L, int64_t n, int64_t gnnz, bool build = true) {
  L.A.n = n;
  L.A.nslices = ceil_div(n, SL);
  L.brp = ar.alloc<int32_t>(n + 1);
  if (build) launch_pattern_rp(st, n, L.grp, L.brp);
  LCHK();
  L.nnzb = gnnz + n;
  L.bci = ar.alloc<int32_t>(L.nnzb);
  if (build) launch_pattern_cols(st, n, L.grp, L.gci, L.brp, L.bci);
  LCHK();
  L.A.sl_ptr = ar.alloc<int32_t>(L.A.nslices + 1);
  if (build) launch_slice_width(st, n, nullptr, L.brp, L.A.sl_ptr);
  LCHK();
}

void finish_sell(Arena& ar, hipStream_t st, Level& L, int32_t* scan_tmp, bool build = true) {
  if (build) launch_scan_excl(st, L.A.sl_ptr, L.A.sl_ptr, L.A.nslices, L.A.sl_ptr + L.A.nslices, scan_tmp);
  LCHK();
  L.A.nslots = ar.count(L.A.sl_ptr + L.A.nslices);
  L.A.col = ar.alloc<int32_t>(L.A.nslots);
  if (build) launch_sell_cols(st, L.A.n, nullptr, L.brp, L.bci, L.A.sl_ptr, L.A.col);
  LCHK();
}

// Colour classes of level l for the multicolour Gauss-Seidel smoother: the
// parity of i + j + k on level 0, Jones-Plassmann rounds on the level's graph
// elsewhere (rounds logged like the matching rounds), a stable counting sort
// of the rows by colour, and the sliced-ELL structure of every class.
void build_colours(llg_ctx& c, Arena& ar, int l) {
  hipStream_t st = c.st;
  Level& L = c.lv[l];
  const int64_t n = L.A.n;
  L.colour = ar.alloc<int32_t>(n);
  if (l == 0) {
    launch_parity_colour(st, c.grid.n[0], c.grid.n[1], c.grid.n[2], L.colour);
    LCHK();
  } else {
    const uint64_t salt = c.opts.agg_salt ^ (((uint64_t)l << 8) | 0x80u);
    uint64_t* rank = ar.alloc<uint64_t>(n);
    int32_t* cround = ar.alloc<int32_t>(n);
    launch_node_rank(st, n, salt, rank);
    launch_fill_i32(st, cround, n, INT32_MAX);
    launch_fill_i32(st, L.colour, n, -1);
    LCHK();
    if (ar.mode == Mode::PLAN) {
      int64_t rounds = 0;
      for (;;) {
        launch_fill_i32(st, c.count, 1, 0);
        launch_jp_round(st, n, L.grp, L.gci, rank, (int32_t)rounds, cround, L.colour, c.count);
        LCHK();
        ++rounds;
        HIPX(hipMemcpyAsync(ar.hcount, c.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPX(hipStreamSynchronize(st));
        if (*ar.hcount == 0) break;
        if (rounds > n + 2) throw DevError{"colouring did not terminate"};
      }
      ar.plan->counts.push_back(rounds);
    } else {
      const int64_t rounds = ar.plan->counts[ar.ci++];
      launch_fill_i32(st, c.count, 1, 0);
      for (int64_t r = 0; r < rounds; ++r)
        launch_jp_round(st, n, L.grp, L.gci, rank, (int32_t)r, cround, L.colour,
                        r + 1 == rounds ? c.count : c.count + 1);
      launch_check_eq(st, c.count, 0, ar.flag, F_PLAN);
      LCHK();
    }
  }
  launch_fill_i32(st, c.count + 2, 1, 0);
  launch_colour_max(st, n, L.colour, c.count + 2);
  LCHK();
  const int64_t ncol = ar.count(c.count + 2, false);  // c.count is reused scratch
  if (ncol > MAX_COLOURS && ar.mode == Mode::PLAN) ar.plan->status = LLG_ERR_UNSUPPORTED;
  L.ncol = (int)std::max<int64_t>(1, std::min<int64_t>(ncol, MAX_COLOURS));
  const int64_t nb = colour_blocks(n);
  int32_t* hist = ar.alloc<int32_t>(L.ncol * nb + 1);
  launch_colour_hist(st, n, L.colour, L.ncol, hist);
  launch_scan_excl(st, hist, hist, L.ncol * nb, hist + L.ncol * nb, c.scan_tmp);
  L.perm = ar.alloc<int32_t>(n);
  launch_fill_i32(st, L.perm, n, 0);
  launch_colour_place(st, n, L.colour, L.ncol, hist, L.perm);
  LCHK();
  L.coff.assign(L.ncol + 1, 0);
  for (int q = 1; q < L.ncol; ++q) L.coff[q] = ar.count(hist + (int64_t)q * nb);
  L.coff[L.ncol] = n;
  L.cls.assign(L.ncol, Sell{});
  for (int q = 0; q < L.ncol; ++q) {
    Sell& S = L.cls[q];
    S.n = L.coff[q + 1] - L.coff[q];
    S.nslices = ceil_div(S.n, SL);
    S.sl_ptr = ar.alloc<int32_t>(S.nslices + 1);
    const int32_t* rows = L.perm + L.coff[q];
    launch_slice_width(st, S.n, rows, L.brp, S.sl_ptr);
    launch_scan_excl(st, S.sl_ptr, S.sl_ptr, S.nslices, S.sl_ptr + S.nslices, c.scan_tmp);
    LCHK();
    S.nslots = ar.count(S.sl_ptr + S.nslices);
    S.col = ar.alloc<int32_t>(S.nslots);
    launch_sell_cols(st, S.n, rows, L.brp, L.bci, S.sl_ptr, S.col);
    LCHK();
  }
}

// Grid pattern, then per level: npass handshake-matching passes on the
// integer graph, composite aggregates, member lists, next-level graph and
// block pattern.  Returns the number of levels.
int build_structure(llg_ctx& c, Arena& ar) {
  hipStream_t st = c.st;
  const llg_grid& g = c.grid;
  const llg_opts& o = c.opts;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int64_t N = (int64_t)nx * ny * nz;
  c.flags = ar.alloc<int32_t>(8);
  c.count = ar.alloc<int32_t>(8);
  c.scan_tmp = ar.alloc<int32_t>(scan_tmp_ints(std::max<int64_t>(N + 1, MAX_COLOURS * colour_blocks(N) + 1)) + 64);
  if (ar.mode == Mode::PLAN || ar.first) {
    launch_fill_i32(st, c.flags, 8, 0);
    LCHK();
  }
  ar.flag = c.flags + ar.flag_word;
  Level& L0 = c.lv[0];
  const bool grid = !ar.keep_grid;  // build the grid graph and the grid level's pattern
  L0.grp = ar.alloc<int32_t>(N + 1);
  if (grid) {
    launch_grid_degree(st, nx, ny, nz, L0.grp);
    LCHK();
    launch_scan_excl(st, L0.grp, L0.grp, N, L0.grp + N, c.scan_tmp);
    LCHK();
  }
  L0.gnnz = ar.count(L0.grp + N);
  L0.gci = ar.alloc<int32_t>(L0.gnnz);
  L0.gw = ar.alloc<int32_t>(L0.gnnz);
  if (grid) {
    launch_grid_graph(st, nx, ny, nz, L0.grp, L0.gci, L0.gw);
    LCHK();
  }
  build_sell(ar, st, L0, N, L0.gnnz, grid);
  finish_sell(ar, st, L0, c.scan_tmp, grid);

  int l = 0;
  // the matching state of the next pass's nodes, set by the coarse-graph
  // fill of the pass before (null: set it here)
  NodeSt* ns_next = nullptr;
  int32_t *mate_next = nullptr, *prop_next = nullptr;
  for (;; ++l) {
    Level& L = c.lv[l];
    const int64_t n = L.A.n;
    if (n <= o.max_coarse || l + 1 >= o.max_levels) break;
    int32_t* acc = ar.alloc<int32_t>(n);
    const int32_t* leads[MAX_PASS] = {};
    const int32_t* mates[MAX_PASS] = {};
    int64_t cn = n, cg = L.gnnz;
    int32_t *crp = L.grp, *cci = L.gci, *cw = L.gw;
    for (int p = 0; p < o.npass; ++p) {
      const uint64_t salt = o.agg_salt ^ (((uint64_t)l << 8) | (uint64_t)p);
      // the first pass of the grid level matches on the grid graph itself,
      // whose rows the proposal kernel computes instead of loading; it needs
      // no records, and its first round sets mate and prop of every node
      const bool on_grid = l == 0 && p == 0 && cn > MATCH_SMALL;
      const bool preset = ns_next != nullptr;
      NodeSt* ns = preset ? ns_next : on_grid ? nullptr : ar.alloc<NodeSt>(cn);
      int32_t* mate = preset ? mate_next : ar.alloc<int32_t>(cn);
      int32_t* prop = preset ? prop_next : ar.alloc<int32_t>(cn);
      ns_next = nullptr;
      int32_t* id = ar.alloc<int32_t>(cn + 1);
      int32_t* aggp = ar.alloc<int32_t>(cn);
      int32_t* lead = ar.alloc<int32_t>(cn);
      uint64_t* rank = on_grid ? ar.alloc<uint64_t>(cn) : nullptr;
      if (on_grid)
        launch_node_rank(st, cn, salt, rank);
      else if (!preset)
        launch_match_init(st, cn, crp, cw, salt, ns, mate, prop);
      LCHK();
      // lanes per node in a proposal round: about two slots per lane on the
      // coarse levels (latency bound), one lane on the grid-sized levels.  A
      // round launches lanes x cn threads whatever is left to match, and the
      // late rounds (few free nodes) cost about their dispatch, so the lanes
      // stop at about 1.25M threads (level 1 of a 128^3 grid: 2 instead of 8).
      int lanes = 1;
      while (lanes < 16 && (int64_t)2 * lanes * cn < cg && (int64_t)2 * lanes * cn <= (int64_t(5) << 18)) lanes *= 2;
      auto propose = [&](int32_t* any, bool first) {
        if (on_grid)
          launch_propose_grid(st, nx, ny, nz, mate, rank, salt, o.beta_num, o.beta_den, prop, any, first);
        else
          launch_propose(st, cn, crp, cci, cw, mate, ns, salt, o.beta_num, o.beta_den, prop, any, lanes);
      };
      // handshake rounds: PLAN runs until a round has no proposal and logs
      // the number of rounds; REPLAY runs that many and checks the extra
      // round proposes nothing
      if (cn <= MATCH_SMALL) {
        // a small level: every round in one workgroup, in both modes
        launch_match_small(st, cn, crp, cci, cw, mate, ns, salt, o.beta_num, o.beta_den, prop, ar.flag, F_PLAN,
                           lanes);
        LCHK();
      } else if (ar.mode == Mode::PLAN) {
        int64_t rounds = 0;
        for (;;) {
          launch_fill_i32(st, c.count, 1, 0);
          propose(c.count, rounds == 0);
          LCHK();
          HIPX(hipMemcpyAsync(ar.hcount, c.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
          HIPX(hipStreamSynchronize(st));
          if (*ar.hcount == 0) break;
          launch_accept(st, cn, prop, mate, ns);
          LCHK();
          ++rounds;
          if (rounds > cn + 2) throw DevError{"matching did not terminate"};
        }
        ar.plan->counts.push_back(rounds);
      } else {
        const int64_t rounds = ar.plan->counts[ar.ci++];
        launch_fill_i32(st, c.count + 1, 1, 0);
        for (int64_t r = 0; r < rounds; ++r) {
          propose(c.count + 1, r == 0);
          launch_accept(st, cn, prop, mate, ns);
        }
        launch_fill_i32(st, c.count, 1, 0);
        propose(c.count, rounds == 0);
        launch_check_eq(st, c.count, 0, ar.flag, F_PLAN);
        LCHK();
      }
      launch_leader_flag(st, cn, mate, id);
      launch_scan_excl(st, id, id, cn, id + cn, c.scan_tmp);
      LCHK();
      const int64_t nc = ar.count(id + cn);
      launch_assign(st, cn, mate, id, aggp, lead);
      int32_t* cnt = ar.alloc<int32_t>(nc + 1);
      launch_cg_count(st, nc, lead, mate, crp, cnt);
      launch_scan_excl(st, cnt, cnt, nc, cnt + nc, c.scan_tmp);
      LCHK();
      const int64_t ncand = ar.count(cnt + nc);
      int32_t* cj = ar.alloc<int32_t>(ncand);
      int32_t* cwt = ar.alloc<int32_t>(ncand);
      int32_t* nrp = ar.alloc<int32_t>(nc + 1);
      // rows of the coarse levels of a 3D grid reach about 50 candidates
      const bool wide = nz > 1 && l > 0;
      // the grid level's first pass fills from the grid graph (gdims passed
      // below); the fill's tile rows follow the same choice
      const bool from_grid = l == 0 && p == 0;
      const int shape = wide ? 1 : from_grid ? 2 : 0;
      const int64_t tiles = ceil_div(nc, cg_tile_rows(shape));
      int32_t* ttot = ar.alloc<int32_t>(tiles + 1);
      const int gdims[3] = {nx, ny, nz};
      // the next pass (of this level or the next) starts from these nodes
      ns_next = ar.alloc<NodeSt>(nc);
      mate_next = ar.alloc<int32_t>(nc);
      prop_next = ar.alloc<int32_t>(nc);
      launch_cg_fill(st, nc, lead, mate, crp, cci, cw, aggp, cnt, cj, cwt, nrp, ttot, wide,
                     from_grid ? gdims : nullptr, ns_next, mate_next, prop_next);
      launch_scan_excl(st, ttot, ttot, tiles, ttot + tiles, c.scan_tmp);
      LCHK();
      const int64_t ng = ar.count(ttot + tiles);
      int32_t* nci = ar.alloc<int32_t>(ng);
      int32_t* nw = ar.alloc<int32_t>(ng);
      launch_cg_copy(st, nc, shape, cnt, cj, cwt, ttot, nrp, nci, nw);
      LCHK();
      leads[p] = lead;
      mates[p] = mate;
      cn = nc;
      cg = ng;
      crp = nrp;
      cci = nci;
      cw = nw;
    }
    if ((double)cn > o.stagnation * (double)n) break;
    // members of the composite aggregates, ascending, and the composite map
    int32_t* mptr = ar.alloc<int32_t>(cn + 1);
    int32_t* mem = ar.alloc<int32_t>(n);
    launch_member_count(st, cn, o.npass, leads, mates, mptr);
    launch_scan_excl(st, mptr, mptr, cn, mptr + cn, c.scan_tmp);
    launch_member_fill(st, cn, o.npass, leads, mates, mptr, mem, acc);
    LCHK();
    L.agg = acc;
    L.mptr = mptr;
    L.mem = mem;
    L.nc = cn;
    if (o.smoother == LLG_SMOOTHER_MCGS) build_colours(c, ar, l);
    Level& Nx = c.lv[l + 1];
    Nx.grp = crp;
    Nx.gci = cci;
    Nx.gw = cw;
    Nx.gnnz = cg;
    build_sell(ar, st, Nx, cn, cg);
    finish_sell(ar, st, Nx, c.scan_tmp);
  }
  ar.flush_checks();
  return l + 1;
}

// The levels from c.tail on run their V-cycle in one workgroup (k_tail):
// block-Jacobi cycles only, below every K-cycle level and below level 1 when
// it is applied through the grid level, each of at most opts.tail_nodes
// nodes, at most TAIL_MAX of them, their vectors within the kernel's LDS.
template <typename T>
void plan_tail(llg_ctx& c, TailArgs<T>& a) {
  const llg_opts& o = c.opts;
  c.tail = 0;
  if (o.tail_nodes <= 0 || o.smoother != LLG_SMOOTHER_JACOBI || c.L < 3 || !c.tail_ok) return;
  int lo = std::max(1, o.kcycle_depth + 1);
  if (c.f1) lo = std::max(lo, 2);
  const int64_t ts = sizeof(T);
  auto vb = [](int64_t n, int64_t sz) { return (3 * n * sz + 15) / 16 * 16; };
  const int64_t nc = c.lv[c.L - 1].A.n;
  int64_t bytes = vb(nc, 8) + vb(nc, ts);
  int s = c.L - 1;
  while (s - 1 >= lo && c.lv[s - 1].A.n <= o.tail_nodes && c.L - s <= TAIL_MAX) {
    const int64_t add = 3 * vb(c.lv[s - 1].A.n, ts);
    if (bytes + add > TAIL_LDS) break;
    bytes += add;
    --s;
  }
  if (s > c.L - 2) return;
  a = TailArgs<T>{};
  a.nlev = c.L - 1 - s;
  int64_t off = 0;
  for (int k = 0; k < a.nlev; ++k) {
    const Level& L = c.lv[s + k];
    TailLevel<T>& t = a.lv[k];
    t.sl = L.A.sl_ptr;
    t.col = L.A.col;
    t.val = (const T*)L.val;
    t.dinv = (const T*)L.dinv;
    t.mptr = L.mptr;
    t.mem = L.mem;
    t.agg = L.agg;
    t.n = (int32_t)L.A.n;
    t.G = L.G;
    t.ob = (int32_t)off;
    t.ox = (int32_t)(off + vb(L.A.n, ts));
    t.oy = (int32_t)(off + 2 * vb(L.A.n, ts));
    off += 3 * vb(L.A.n, ts);
  }
  a.obd = (int32_t)off;
  a.oe = (int32_t)(off + vb(nc, 8));
  off += vb(nc, 8) + vb(nc, ts);
  a.inv = c.dense;
  a.nc = (int32_t)nc;
  a.nu_pre = o.nu_pre;
  a.nu_post = o.nu_post;
  a.lds = (int32_t)off;
  a.omega = (T)c.omega;
  c.tail = s;
}

template <typename T>
const TailArgs<T>& tail_args(const llg_ctx& c);
template <>
const TailArgs<double>& tail_args<double>(const llg_ctx& c) {
  return c.ta64;
}
template <>
const TailArgs<float>& tail_args<float>(const llg_ctx& c) {
  return c.ta32;
}

void save_struct(const llg_ctx& c, StructSet& S) {
  S.L = c.L;
  S.flags = c.flags;
  S.count = c.count;
  S.scan_tmp = c.scan_tmp;
  for (int l = 0; l < LLG_MAX_LEVELS; ++l) {
    const Level& L = c.lv[l];
    LevelStruct& T = S.lv[l];
    T.A = L.A;
    T.brp = L.brp;
    T.bci = L.bci;
    T.nnzb = L.nnzb;
    T.grp = L.grp;
    T.gci = L.gci;
    T.gw = L.gw;
    T.gnnz = L.gnnz;
    T.agg = L.agg;
    T.mptr = L.mptr;
    T.mem = L.mem;
    T.nc = L.nc;
    T.colour = L.colour;
    T.perm = L.perm;
    T.ncol = L.ncol;
    T.coff = L.coff;
    T.cls = L.cls;
  }
}

void load_struct(llg_ctx& c, const StructSet& S) {
  c.L = S.L;
  c.flags = S.flags;
  c.count = S.count;
  c.scan_tmp = S.scan_tmp;
  for (int l = 0; l < LLG_MAX_LEVELS; ++l) {
    Level& L = c.lv[l];
    const LevelStruct& T = S.lv[l];
    L.A = T.A;
    L.brp = T.brp;
    L.bci = T.bci;
    L.nnzb = T.nnzb;
    L.grp = T.grp;
    L.gci = T.gci;
    L.gw = T.gw;
    L.gnnz = T.gnnz;
    L.agg = T.agg;
    L.mptr = T.mptr;
    L.mem = T.mem;
    L.nc = T.nc;
    L.colour = T.colour;
    L.perm = T.perm;
    L.ncol = T.ncol;
    L.coff = T.coff;
    L.cls = T.cls;
  }
}

// Values, vectors and Krylov storage (never materialized when planning).
void allocate_numeric(llg_ctx& c, Arena& ar) {
  const bool f32 = c.opts.precision == LLG_PREC_FP32_AMG;
  const size_t ts = f32 ? sizeof(float) : sizeof(double);
  const int R = c.opts.restart;
  Level& L0 = c.lv[0];
  // the factored grid level needs a coarse level (the coarsest is stored as BSR)
  c.fact = c.opts.fine_operator == LLG_FINE_FACTORED && c.L > 1;
  // level 1 (not the coarsest, one lane per row) applied through the grid level's blocks
  // (at most two matching passes: k_l1 takes aggregates of at most four members)
  const bool f1 = c.fact && c.L > 2 && c.lv[1].A.n >= 32768 && c.opts.smoother == LLG_SMOOTHER_JACOBI &&
                  c.opts.npass <= 2;
  if (c.fact) {
    c.Mh = ar.lazy<double>(9 * L0.A.nslices * SL);
    c.mt = ar.lazy<double>(3 * L0.A.n);
    L0.kf = ar.get(ts * 9 * L0.A.nslices * SL, true);
    L0.knm = ar.get(ts * 9 * L0.A.n, true);  // K node-major, read by level 1's Galerkin product
  } else {
    c.Aval = ar.lazy<double>(9 * L0.A.nslots);
  }
  c.dinv0 = ar.lazy<double>(9 * L0.A.nslices * SL);
  for (int l = 0; l < c.L; ++l) {
    Level& L = c.lv[l];
    const int64_t n = L.A.n;
    // the large coarse levels below the K-cycle levels apply their rows from
    // the CSR-ordered copy (block-Jacobi cycles; not the coarsest level)
    L.csr = c.opts.csr_levels && l >= 1 && !(l == 1 && f1) && l > c.opts.kcycle_depth && l + 1 < c.L &&
            n >= 32768 && c.opts.smoother == LLG_SMOOTHER_JACOBI;
    // sliced-ELL values, except where no product reads them: the factored
    // grid level, level 1 when it is applied through the grid blocks, and
    // the levels applied from the CSR-ordered copy
    if (!(l == 0 && c.fact) && !(l == 1 && f1) && !L.csr) L.val = ar.get(ts * 9 * L.A.nslots, true);
    // the next level's Galerkin product walks the member rows of this level
    // and reads their blocks in CSR order (contiguous per row; the sliced-ELL
    // layout spreads a row over 64-slot strides and a block over nine lines)
    if (l >= 1 && l + 1 < c.L) L.vt = ar.get(ts * 9 * L.nnzb, true);
    L.unit = l == 0 && c.opts.left_scale;
    L.G = n >= 32768 ? 1 : (c.grid.dim == 3 ? 16 : 8);
    L.dinv = ar.get(ts * 9 * L.A.nslices * SL, true);
    L.b = ar.get(ts * 3 * n, true);
    L.x = ar.get(ts * 3 * n, true);
    L.r = ar.get(ts * 3 * n, true);
    L.e = ar.get(ts * 3 * n, true);
    L.xo = ar.get(ts * 3 * n, true);
    if (L.csr) L.xp = ar.get(ts * 3 * n, true);  // the iterate with the prolonged correction
    L.cval.assign(L.ncol, nullptr);
    L.cdinv.assign(L.ncol, nullptr);
    for (int q = 0; q < L.ncol; ++q) {
      L.cval[q] = ar.get(ts * 9 * L.cls[q].nslots, true);
      if (!L.unit) L.cdinv[q] = ar.get(ts * 9 * L.cls[q].nslices * SL, true);
    }
    if (l >= 1 && l <= c.opts.kcycle_depth && l + 1 < c.L) {
      L.v1 = ar.get(ts * 3 * n, true);
      L.v2 = ar.get(ts * 3 * n, true);
      L.w1 = ar.get(ts * 3 * n, true);
      L.w2 = ar.get(ts * 3 * n, true);
      L.rho = ar.get(ts * 3 * n, true);
      L.kc = ar.lazy<double>(8);
    }
  }
  c.nd = 3 * c.lv[c.L - 1].A.n;
  c.dense = ar.lazy<double>(c.nd * c.nd);
  c.piv = (int32_t*)ar.get(sizeof(int32_t) * (c.nd + 2) + sizeof(double) * c.nd, true);
  const int64_t m = 3 * c.N;
  c.ld = (int64_t)(align_up((size_t)m * sizeof(double)) / sizeof(double));
  c.u = ar.lazy<double>(m);
  c.b = ar.lazy<double>(m);
  c.r = ar.lazy<double>(m);
  c.w = ar.lazy<double>(m);
  // the baselines keep their work vectors in the basis slots
  const int slots = c.opts.krylov == LLG_KRYLOV_BICGSTAB || c.opts.krylov == LLG_KRYLOV_TFQMR ? std::max(R + 1, 10)
                                                                                             : R + 1;
  c.V = ar.lazy<double>(slots * c.ld);
  c.kb = ar.lazy<double>(KB_SIZE);
  c.Z = ar.get(ts * (size_t)R * c.ld, true);
  c.npart_vec = red_blocks(m);
  c.npart_rows = ceil_div(c.N, 256);
  int64_t kparts = 0;
  for (int l = 1; l < c.L; ++l) {
    kparts = std::max<int64_t>(kparts, 3 * rows_blocks(c.lv[l].A.n, c.lv[l].G));
    // K-cycle levels: the partials of w1.rho, kept apart from c.part until
    // stage 3 sums them (a nested K-cycle reuses c.part in between)
    if (l <= c.opts.kcycle_depth && l + 1 < c.L) c.lv[l].prho = ar.lazy<double>(rows_blocks(c.lv[l].A.n, 1));
  }
  c.f1 = f1;
  if (c.f1) {
    kparts = std::max<int64_t>(kparts, 3 * rows_blocks(c.lv[1].A.n, L1_LANES));
    c.lv[0].mtq = ar.get(ts * 3 * c.lv[0].A.n, true);
    c.lv[0].nagg = ar.lazy<int32_t>(6 * c.lv[0].A.nslices * SL);
    c.lv[1].xp = ar.get(ts * 3 * c.lv[1].A.n, true);  // level-1 iterate with the prolonged correction
  }
  // partial sums: up to 2R+3 columns of the delayed Gram-Schmidt dots (R+2 for the two-pass form)
  c.part = ar.lazy<double>(std::max<int64_t>(std::max<int64_t>((2 * R + 4) * c.npart_vec, c.npart_rows), kparts) + 64);
  c.ks.H = ar.lazy<double>((R + 1) * R);
  c.ks.cs = ar.lazy<double>(R);
  c.ks.sn = ar.lazy<double>(R);
  c.ks.g = ar.lazy<double>(R + 1);
  c.ks.hcol = ar.lazy<double>(R + 2);
  c.ks.y = ar.lazy<double>(R);
  c.ks.sc = ar.lazy<double>(16);
  c.ks.hs = ar.lazy<double>(R + 2);
  c.ks.hinv = ar.lazy<double>(R + 2);
  c.ks.coef = ar.lazy<double>(2 * R + 4);
  c.delta = ar.lazy<double>(R + 2);
  c.prm = ar.lazy<double>(PRM_WORDS);
  if (f32)
    plan_tail<float>(c, c.ta32);
  else
    plan_tail<double>(c, c.ta64);
  if (c.opts.stray_field) {
    c.fd = field_dims(c.grid.n[0], c.grid.n[1], c.grid.n[2]);
    const int64_t P = c.fd.px * c.fd.py * c.fd.pz;
    c.nhat = ar.lazy<double>(6 * P);
    c.fwork = (double2*)ar.lazy<double>(4 * P);  // two packed complex planes
  }
  // copies of m^n (and m^{n-1}) for the field terms of llg_step_field, whose
  // captured kernels read them at fixed addresses
  c.min = ar.lazy<double>(m);
  if (c.opts.scheme == LLG_SCHEME_BDF2) c.mprv = ar.lazy<double>(m);
}

bool grid_ok(const llg_grid* g) {
  if (!g) return false;
  if (g->dim != 2 && g->dim != 3) return false;
  if (g->n[0] < 2 || g->n[1] < 2) return false;
  if (g->dim == 2 && g->n[2] != 1) return false;
  if (g->dim == 3 && g->n[2] < 2) return false;
  if (!(g->h > 0) || !std::isfinite(g->h)) return false;
  const double N = (double)g->n[0] * g->n[1] * g->n[2];
  if (N * 7.0 > 2.0e9) return false;  // int32 block indices
  return true;
}

bool opts_ok(const llg_opts* o) {
  return o && o->rtol >= 0 && std::isfinite(o->rtol) && o->restart >= 1 && o->restart <= 32 &&
         o->max_iters >= 1 && o->nu_pre >= 0 && o->nu_pre <= 4 && o->nu_post >= 0 && o->nu_post <= 4 &&
         o->npass >= 1 && o->npass <= MAX_PASS && o->beta_num >= 0 && o->beta_den >= 1 &&
         o->max_coarse >= 1 && o->max_levels >= 1 && o->max_levels <= LLG_MAX_LEVELS && o->max_dense >= 1 &&
         (o->precision == LLG_PREC_FP64 || o->precision == LLG_PREC_FP32_AMG) && std::isfinite(o->omega) &&
         std::isfinite(o->stagnation) && o->kcycle_depth >= 0 && o->kcycle_depth <= 8 &&
         (o->smoother == LLG_SMOOTHER_JACOBI || o->smoother == LLG_SMOOTHER_MCGS) &&
         (o->scheme == LLG_SCHEME_BDF1 || o->scheme == LLG_SCHEME_BDF2) &&
         (o->fine_operator == LLG_FINE_BSR || o->fine_operator == LLG_FINE_FACTORED) &&
         (o->arnoldi == LLG_ARNOLDI_CGS2 || o->arnoldi == LLG_ARNOLDI_DCGS2) &&
         (o->krylov == LLG_KRYLOV_FGMRES_AMG || o->krylov == LLG_KRYLOV_GMRES || o->krylov == LLG_KRYLOV_BICGSTAB ||
          o->krylov == LLG_KRYLOV_TFQMR) &&
         (o->stray_field == 0 || o->stray_field == 1) && o->tail_nodes >= 0 &&
         (o->pipeline == 0 || o->pipeline == 1) && (o->overlap_rebuild == 0 || o->overlap_rebuild == 1) &&
         (o->csr_levels == 0 || o->csr_levels == 1);
}

// Plan for (grid, opts): cached; computed on the current device.
std::shared_ptr<Plan> get_plan(const llg_grid& g, const llg_opts& o) {
  const PlanKey key = plan_key(g, o);
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
  }
  auto plan = std::make_shared<Plan>();
  llg_ctx c;
  c.grid = g;
  c.opts = o;
  c.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
  HIPX(hipStreamCreate(&c.st));
  Arena ar;
  ar.mode = Mode::PLAN;
  ar.plan = plan.get();
  ar.st = c.st;
  int32_t* hc = nullptr;
  HIPX(hipHostMalloc((void**)&hc, sizeof(int32_t) * 4, hipHostMallocDefault));
  ar.hcount = hc;
  try {
    c.L = build_structure(c, ar);
    plan->struct_bytes = plan->total;
    if (c.lv[c.L - 1].A.n > o.max_dense) plan->status = LLG_ERR_UNSUPPORTED;
    allocate_numeric(c, ar);
    if (overlapped_rebuild(o)) {  // the second structure set
      plan->dbl = true;
      plan->total += plan->struct_bytes;
    }
    HIPX(hipStreamSynchronize(c.st));
  } catch (...) {
    ar.release();
    (void)hipHostFree(hc);
    (void)hipStreamDestroy(c.st);
    throw;
  }
  ar.release();
  (void)hipHostFree(hc);
  (void)hipStreamDestroy(c.st);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans[key] = plan;
  return plan;
}

// ------------------------------------------------------------------ setup
void retarget_tail(llg_ctx& c) {
  if (c.opts.precision == LLG_PREC_FP32_AMG)
    plan_tail<float>(c, c.ta32);
  else
    plan_tail<double>(c, c.ta64);
}

// The overlapped rebuild.  The step uses the structure set built for it
// during the previous step (or at creation) on the second stream: the main
// stream waits for that build, takes its device-side check result as the
// step's initial flags, and the set is loaded.  Then the other set (the one
// the previous step used) is rebuilt on the second stream for the next step,
// after the work already queued on the main stream.  Every step thus still
// rebuilds a hierarchy structure; the rebuild runs beside the solve.
void rebuild_overlapped(llg_ctx& c) {
  const int cur = c.set, nxt = 1 - c.set;
  HIPX(hipStreamWaitEvent(c.st, c.built[cur], 0));
  load_struct(c, c.sets[cur]);
  retarget_tail(c);
  HIPX(hipMemcpyAsync(c.flags, c.flags + 1, sizeof(int32_t), hipMemcpyDeviceToDevice, c.st));
  launch_fill_i32(c.st, c.flags + 1, 1, 0);
  LCHK();
  HIPX(hipEventRecord(c.main_ev, c.st));
  HIPX(hipStreamWaitEvent(c.aux, c.main_ev, 0));
  load_struct(c, c.sets[nxt]);
  hipStream_t keep = c.st;
  c.st = c.aux;
  Arena ar;
  ar.mode = Mode::REPLAY;
  ar.plan = c.plan.get();
  ar.first = false;
  ar.ptrs = nxt == 0 ? &c.ptrs : &c.ptrs2;
  ar.st = c.aux;
  ar.flag_word = 1;
  ar.keep_grid = true;
  try {
    (void)build_structure(c, ar);
  } catch (...) {
    c.st = keep;
    load_struct(c, c.sets[cur]);
    retarget_tail(c);
    throw;
  }
  c.st = keep;
  HIPX(hipEventRecord(c.built[nxt], c.aux));
  load_struct(c, c.sets[cur]);
  retarget_tail(c);
  c.set = nxt;
}

// Everything llg_step does before the Krylov solve: the structure rebuild
// (replayed from the plan), assembly, Galerkin products and the coarsest
// inverse.  alpha and dt are read from c.prm on the device.
template <typename T>
void setup_values(llg_ctx& c, const double* m, const double* mprev, const double* F, int field = 0) {
  hipStream_t st = c.st;
  const llg_grid& g = c.grid;
  const bool amg = c.opts.krylov == LLG_KRYLOV_FGMRES_AMG;  // the baselines need only A, b and u0
  if (amg && c.opts.rebuild_aggregates && c.dbl) {
    rebuild_overlapped(c);
  } else if (amg && c.opts.rebuild_aggregates) {
    Arena ar;
    ar.mode = Mode::REPLAY;
    ar.plan = c.plan.get();
    ar.first = false;
    ar.ptrs = &c.ptrs;
    ar.st = st;
    ar.keep_grid = true;
    (void)build_structure(c, ar);
  }
  Level& L0 = c.lv[0];
  {
    KTimer kt(c, LLG_KT_ASSEMBLE);
    // factored grid level: the solve recomputes its blocks and D^{-1} from
    // the frozen field, so only the node-major K (Galerkin) and, for the
    // Gauss-Seidel colour classes, the sliced K are stored
    const bool kf = c.fact && c.opts.smoother == LLG_SMOOTHER_MCGS;
    launch_assemble<T>(st, g.n[0], g.n[1], g.n[2], 1.0 / (g.h * g.h), c.prm, c.opts.left_scale,
                       c.opts.x0_is_mn, L0.A, c.Aval, (T*)L0.val, c.fact ? nullptr : c.dinv0, (T*)L0.dinv, c.b, c.u,
                       c.flags, c.fact, nullptr, kf ? (T*)L0.kf : nullptr, (T*)L0.knm, c.mt);
    if (c.f1) {
      launch_member_nbr_aggs(st, GridDims{g.n[0], g.n[1], g.n[2]}, L0.mem, L0.agg, L0.nagg);
      launch_member_fields<T>(st, L0.A.n, L0.mem, c.mt, (T*)L0.mtq);
    }
    LCHK();
  }
  if (field) {  // explicit field terms of the right-hand side (field 2: with the stray field)
    if (field == 2) launch_stray(st, c.fd, m, mprev, c.nhat, c.fwork);
    launch_field_rhs(st, c.N, c.prm, m, mprev, c.fd, field == 2 ? c.fwork : nullptr, c.b);
    LCHK();
  }
  if (!amg) return;
  for (int l = 0; l + 1 < c.L; ++l) {
    Level& L = c.lv[l];
    Level& Nx = c.lv[l + 1];
    KTimer kt(c, LLG_KT_GALERKIN);
    GalSrc<T> src;
    src.fval = (const T*)L.val;
    src.fvt = (const T*)L.vt;
    src.fk = (const T*)L.kf;
    src.knm = (const T*)L.knm;  // factored grid level: K node-major
    src.frp = L.brp;
    src.fci = L.bci;
    src.cvt = (T*)Nx.vt;
    src.crp = Nx.brp;
    src.cci = Nx.bci;
    launch_galerkin<T>(st, Nx.A, (T*)Nx.val, (T*)Nx.dinv, L.mptr, L.mem, L.A, L.agg, src);
    LCHK();
  }
  for (int l = 0; l + 1 < c.L; ++l) {  // colour-class copies for Gauss-Seidel
    Level& L = c.lv[l];
    for (int q = 0; q < L.ncol; ++q)
      launch_cls_gather<T>(st, L.cls[q].n, L.perm + L.coff[q], L.A, (const T*)L.val,
                           L.unit ? nullptr : (const T*)L.dinv, L.cls[q], (T*)L.cval[q], (T*)L.cdinv[q],
                           (const T*)L.kf);
  }
  LCHK();
  Level& C = c.lv[c.L - 1];
  launch_dense_scatter<T>(st, C.A, (const T*)C.val, c.dense);
  launch_gauss_jordan(st, c.nd, c.dense, c.piv, c.flags);
  LCHK();
}

// Graphs are used unless switched off, or a kernel class other than the outer
// SpMV is being timed (per-kernel events need eager launches).
bool use_graphs(const llg_ctx& c) {
  return c.graphs_ok && c.opts.graphs && (c.timed == LLG_KT_NONE || c.timed == LLG_KT_OUTER_SPMV);
}

template <typename Fn>
hipGraphExec_t try_capture(llg_ctx& c, Fn body);

// Capture the work `body` enqueues into a graph (on the private capture
// stream) and instantiate it.
template <typename Fn>
hipGraphExec_t capture_graph(llg_ctx& c, Fn body) {
  hipStream_t saved = c.st;
  c.st = c.cap_st;
  c.capturing = true;
  HIPX(hipStreamBeginCapture(c.cap_st, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(c.cap_st, &g);
    if (g) (void)hipGraphDestroy(g);
    c.st = saved;
    c.capturing = false;
    throw;
  }
  const hipError_t e = hipStreamEndCapture(c.cap_st, &g);
  c.st = saved;
  c.capturing = false;
  if (e != hipSuccess) throw DevError{std::string("graph capture: ") + hipGetErrorString(e)};
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiateWithFlags(&ex, g, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) throw DevError{std::string("graph instantiate: ") + hipGetErrorString(e2)};
  return ex;
}

// Capture, or on failure switch the context to eager launches for good.
template <typename Fn>
hipGraphExec_t try_capture(llg_ctx& c, Fn body) {
  try {
    return capture_graph(c, body);
  } catch (const DevError& e) {
    c.graphs_ok = false;
    (void)hipGetLastError();
    return nullptr;
  }
}

// alpha, the time-step factors dt' = dt (BDF1) or 2 dt / 3 (BDF2) of the
// right-hand side and dt' eps of the operator, and the field parameters
// The step's parameters, and the device addresses of its inputs (bit
// patterns in prm[8..10], read by the assembly kernel).
void write_params(llg_ctx& c, double alpha, double dt, bool bdf2, const llg_field* fld, const double* m,
                  const double* mprev, const double* F) {
  const double dtp = bdf2 ? (2.0 * dt) / 3.0 : dt;
  c.hprm[0] = alpha;
  c.hprm[1] = fld ? dtp * fld->eps : dtp;
  c.hprm[2] = dtp;
  c.hprm[3] = fld ? fld->q : 0.0;
  for (int k = 0; k < 3; ++k) c.hprm[4 + k] = fld ? fld->h_ext[k] : 0.0;
  c.hprm[7] = 0.0;
  const double* in[3] = {m, mprev, F};
  for (int k = 0; k < 3; ++k) std::memcpy(&c.hprm[8 + k], &in[k], sizeof(double));
  c.hprm[11] = 0.0;
  HIPX(hipMemcpyAsync(c.prm, c.hprm, PRM_WORDS * sizeof(double), hipMemcpyHostToDevice, c.st));
}

// The setup of one step: the assembly reads the inputs at the addresses in
// the parameter block, the field terms the internal copies of m^n (and
// m^{n-1}).  forcing only selects the captured graph.
template <typename T>
void run_setup(llg_ctx& c, bool forcing, bool bdf2 = false, int field = 0) {
  const double* F = nullptr;
  const double* mp = bdf2 ? c.mprv : nullptr;
  if (use_graphs(c)) {
    hipGraphExec_t& gx = c.setup_graph[(forcing ? 1 : 0) + (bdf2 ? 2 : 0) + (field ? 4 : 0) + (field == 2 ? 8 : 0)];
    if (!gx) gx = try_capture(c, [&]() { setup_values<T>(c, c.min, mp, F, field); });
    if (gx) {
      HIPX(hipGraphLaunch(gx, c.st));
      c.setup_done = true;
      return;
    }
  }
  setup_values<T>(c, c.min, mp, F, field);
  c.setup_done = true;
}

// the transformed demagnetizing tensor, once per context (eager)
void demag_prepare(llg_ctx& c) {
  if (c.demag_ready) return;
  launch_demag_setup(c.st, c.fd, c.fwork, c.nhat);
  LCHK();
  c.demag_ready = true;
}

// ------------------------------------------------------------------ products
// Level and outer products, dispatched to the factored kernels on the grid
// level when the context stores it in factored form.
GridDims gdims(const llg_ctx& c) {
  GridDims g{c.grid.n[0], c.grid.n[1], c.grid.n[2]};
  g.mt = c.mt;
  g.prm = c.prm;
  g.inv_h2 = 1.0 / (c.grid.h * c.grid.h);
  return g;
}

// A level-1 product through the grid blocks (k_l1), timed as LLG_KT_LEVEL1:
// the launch stamps its own events, and its algorithmic bytes are added up:
// the member-ordered frozen field (3 values of T per grid node), the neighbour
// aggregates (4 B per neighbour slot), the member pointers, x once, and per
// mode b and the output (0), b, D1^{-1} and the output (1), the output and
// the dot operands (2).
template <typename T>
void l1(llg_ctx& c, int mode, int xzero, const T* x, const T* b, const T* dinv1, T* out, const T* d1, const T* d2,
        double* part) {
  const Level& L0 = c.lv[0];
  const int64_t n1 = c.lv[1].A.n, N = L0.A.n, v = sizeof(T);
  hipEvent_t e0, e1;
  kernel_events(c, LLG_KT_LEVEL1, e0, e1);
  if (e0) {
    double bytes = 3.0 * v * N + 4.0 * 2 * c.grid.dim * N + 4.0 * (n1 + 1) + (xzero ? 0.0 : 3.0 * v * n1);
    if (mode == 0) bytes += 6.0 * v * n1;
    if (mode == 1) bytes += 15.0 * v * n1;
    if (mode == 2) bytes += 3.0 * v * n1 * (1 + (d1 ? 1 : 0) + (d2 ? 1 : 0));
    c.kernel_bytes += bytes;
  }
  launch_l1<T>(c.st, gdims(c), mode, xzero, n1, L0.mptr, L0.nagg, (const T*)L0.mtq, x, b, dinv1, nullptr, nullptr, c.omega,
               out, d1, d2, part, e0, e1);
}

template <typename T>
void lvl_residual(llg_ctx& c, int l, int xmode, const T* b, const T* x, T* r) {
  Level& L = c.lv[l];
  if (l == 1 && c.f1 && xmode == 0) {
    l1<T>(c, 0, 0, x, b, nullptr, r, nullptr, nullptr, nullptr);
    return;
  }
  if (l == 0 && c.fact)
    launch_fact_residual<T>(c.st, gdims(c), xmode, c.omega, b, x, r);
  else if (L.csr)
    launch_residual_csr<T>(c.st, L.A.n, L.brp, L.bci, (const T*)L.vt, xmode, c.omega, b, x, r);
  else
    launch_residual<T>(c.st, L.A, (const T*)L.val, xmode, c.omega, b, x, r, L.G);
}

template <typename T>
void lvl_post_smooth(llg_ctx& c, int l, int xmode, const T* b, const T* x, const int32_t* agg, const T* ec,
                     T* out) {
  Level& L = c.lv[l];
  if (l == 1 && c.f1 && (xmode == 0 || xmode == 2)) {
    if (ec) {
      // the prolongation first, x' = x + P e_c, in its own pass: fused into
      // the level-1 sweep it puts a chain of two dependent gathers (the
      // neighbour's coarse aggregate, then its correction) behind every
      // neighbour load
      launch_prolong<T>(c.st, L.A.n, xmode, c.omega, b, x, agg, ec, (T*)L.xp);
      x = (const T*)L.xp;
      xmode = 0;
    }
    l1<T>(c, 1, xmode == 2, x, b, (const T*)L.dinv, out, nullptr, nullptr, nullptr);
    return;
  }
  if (l == 0 && c.fact) {
    launch_fact_post_smooth<T>(c.st, gdims(c), xmode, c.omega, b, x, agg, ec, out);
  } else if (L.csr) {
    if (ec) {  // the prolongation in its own pass, as on level 1
      launch_prolong<T>(c.st, L.A.n, xmode, c.omega, b, x, agg, ec, (T*)L.xp);
      x = (const T*)L.xp;
      xmode = 0;
    }
    launch_post_smooth_csr<T>(c.st, L.A.n, L.brp, L.bci, (const T*)L.vt, (const T*)L.dinv, xmode, c.omega, b, x,
                              out);
  } else {
    launch_post_smooth<T>(c.st, L.A, (const T*)L.val, (const T*)L.dinv, L.unit, xmode, c.omega, b, x, agg, ec, out,
                          L.G);
  }
}

// e0, e1: events the launch itself stamps at the kernel's start and end
template <typename TZ>
void outer_spmv(llg_ctx& c, const TZ* z, double* w, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (c.fact)
    launch_fact_outer<TZ>(c.st, gdims(c), z, w, e0, e1);
  else
    launch_spmv_outer<TZ>(c.st, c.lv[0].A, c.Aval, z, w, e0, e1);
}

// r = b - A u and the partial sums of |r|^2
void outer_resid(llg_ctx& c) {
  if (c.fact)
    launch_fact_resid_outer(c.st, gdims(c), c.b, c.u, c.r, c.part);
  else
    launch_resid_outer(c.st, c.lv[0].A, c.Aval, c.b, c.u, c.r, c.part);
}

// ------------------------------------------------------------------ V-cycle
template <typename T>
void kcorrection(llg_ctx& c, int lc);

// V(l, b): pre-smoothing from x = 0, restriction of the residual, V(l+1) on
// the coarse residual equation, prolongation of its correction fused with
// post-smoothing; the exact (dense inverse) solve at the coarsest level
// (Sec. 3).  The first pre-smoothing sweep of a coarse level is produced by
// the restriction kernel of the level above (x_{l+1} = omega D^{-1} b_{l+1}),
// and on the fine level with unit diagonal blocks it is x = omega b, never
// stored, so each level costs one "down" and one "up" kernel.
template <typename T>
void vcycle_gs(llg_ctx& c, int l, const T* b, T* out);

template <typename T>
void vcycle(llg_ctx& c, int l, const T* b, T* out) {
  hipStream_t st = c.st;
  if (l == c.L - 1) {
    launch_dense_apply<T>(st, c.nd, c.dense, b, out);
    LCHK();
    return;
  }
  if (c.opts.smoother == LLG_SMOOTHER_MCGS) {
    vcycle_gs<T>(c, l, b, out);
    return;
  }
  Level& L = c.lv[l];
  Level& Nx = c.lv[l + 1];
  const llg_opts& o = c.opts;
  const T* dinv = (const T*)L.dinv;
  const double om = c.omega;
  T* X = (T*)L.x;
  T* XO = (T*)L.xo;
  int xmode = 2;  // x = 0
  const T* xcur = nullptr;
  {
    KTimer kt(c, LLG_KT_SMOOTH);
    if (o.nu_pre >= 1) {
      if (l == 0 && L.unit) {
        xmode = 1;  // x = omega b
      } else if (l == 0) {
        launch_smooth_first<T>(st, L.A, dinv, om, b, X);
        xmode = 0;
        xcur = X;
      } else {
        xmode = 0;  // written by the restriction of the level above
        xcur = X;
      }
    }
    for (int s = 1; s < o.nu_pre; ++s) {
      T* dst = (xcur == X) ? XO : X;
      lvl_post_smooth<T>(c, l, xmode, b, xcur, nullptr, nullptr, dst);
      xmode = 0;
      xcur = dst;
    }
    LCHK();
  }
  const bool coarsest_next = l + 1 == c.L - 1;
  const bool tail_next = c.tail > 0 && l + 1 == c.tail;  // the rest of the cycle in one workgroup
  const T* rsrc = b;
  {
    KTimer kt(c, LLG_KT_RESIDUAL);
    const bool pre_next = o.nu_pre >= 1 && !coarsest_next;
    if (xmode != 2) {
      lvl_residual<T>(c, l, xmode, b, xcur, (T*)L.r);
      rsrc = (const T*)L.r;
    }
    if (tail_next) {
      // the fused cycle restricts rsrc itself
    } else if (coarsest_next) {  // restriction and the exact coarsest solve in one launch
      launch_restrict_dense<T>(st, L.nc, L.mptr, L.mem, rsrc, c.dense, (T*)Nx.e);
    } else {
      launch_restrict<T>(st, L.nc, L.mptr, L.mem, rsrc, (T*)Nx.b, pre_next ? (const T*)Nx.dinv : nullptr, om,
                         pre_next ? (T*)Nx.x : nullptr);
    }
    LCHK();
  }
  if (tail_next) {
    KTimer kt(c, LLG_KT_SMOOTH);
    launch_tail<T>(st, tail_args<T>(c), rsrc, L.mptr, L.mem, (T*)Nx.e);
    LCHK();
  } else if (coarsest_next) {
    // Nx.e holds the coarse correction
  } else if (Nx.kc) {
    kcorrection<T>(c, l + 1);
  } else {
    vcycle<T>(c, l + 1, (const T*)Nx.b, (T*)Nx.e);
  }
  const T* ec = (const T*)Nx.e;
  KTimer kt(c, LLG_KT_SMOOTH);
  if (o.nu_post == 0) {
    launch_prolong<T>(st, L.A.n, xmode, om, b, xcur, L.agg, ec, out);
    LCHK();
    return;
  }
  // further sweeps alternate between XO and X (X is free once the first
  // post-smoothing sweep has read it)
  for (int s = 0; s < o.nu_post; ++s) {
    const bool last = s == o.nu_post - 1;
    T* dst = last ? out : (xcur == XO ? X : XO);
    if (s == 0) {
      lvl_post_smooth<T>(c, l, xmode, b, xcur, L.agg, ec, dst);
    } else {
      lvl_post_smooth<T>(c, l, 0, b, xcur, nullptr, nullptr, dst);
    }
    LCHK();
    xcur = dst;
  }
}

// One multicolour block Gauss-Seidel sweep of level L on x, classes in
// ascending order (forward) or descending order; first: x is zero.
template <typename T>
void gs_sweeps(llg_ctx& c, Level& L, const T* b, T* x, bool forward, bool first) {
  for (int q = 0; q < L.ncol; ++q) {
    const int k = forward ? q : L.ncol - 1 - q;
    launch_gs_sweep<T>(c.st, L.cls[k], L.perm + L.coff[k], (const T*)L.cval[k], (const T*)L.cdinv[k], L.unit,
                       first && q == 0, b, x, L.G);
  }
}

// V(l, b) with multicolour block Gauss-Seidel smoothing: forward sweeps from
// x = 0, residual and restriction, the coarse correction, prolongation, then
// backward sweeps (the post-smoother mirrors the pre-smoother).
template <typename T>
void vcycle_gs(llg_ctx& c, int l, const T* b, T* out) {
  hipStream_t st = c.st;
  Level& L = c.lv[l];
  Level& Nx = c.lv[l + 1];
  const llg_opts& o = c.opts;
  T* X = (T*)L.x;
  {
    KTimer kt(c, LLG_KT_SMOOTH);
    launch_fill<T>(st, X, 3 * L.A.n);
    for (int s = 0; s < o.nu_pre; ++s) gs_sweeps<T>(c, L, b, X, true, s == 0);
    LCHK();
  }
  {
    KTimer kt(c, LLG_KT_RESIDUAL);
    const T* rsrc = b;
    if (o.nu_pre >= 1) {
      lvl_residual<T>(c, l, 0, b, X, (T*)L.r);
      rsrc = (const T*)L.r;
    }
    launch_restrict<T>(st, L.nc, L.mptr, L.mem, rsrc, (T*)Nx.b, nullptr, c.omega, nullptr);
    LCHK();
  }
  if (Nx.kc)
    kcorrection<T>(c, l + 1);
  else
    vcycle<T>(c, l + 1, (const T*)Nx.b, (T*)Nx.e);
  KTimer kt(c, LLG_KT_SMOOTH);
  launch_prolong<T>(st, L.A.n, 0, c.omega, b, X, L.agg, (const T*)Nx.e, out);
  for (int s = 0; s < o.nu_post; ++s) gs_sweeps<T>(c, L, b, out, false, false);
  LCHK();
}

// Coarse correction of level lc by the K-cycle (Sec. 3.1: Krylov acceleration
// at each level): e minimizes ||r - A_c e|| over span{v1, v2}, v1 = C(r),
// v2 = C(r - a1 A_c v1), C the cycle of level lc.  r is lv[lc].b, whose first
// pre-smoothing sweep the restriction has already produced; e goes to lv[lc].e.
template <typename T>
void kcorrection(llg_ctx& c, int lc) {
  hipStream_t st = c.st;
  Level& C = c.lv[lc];
  const T* val = (const T*)C.val;
  // with Jacobi smoothing the first sweep of the next cycle on rho is fused
  // into the update of rho (Gauss-Seidel cycles start from x = 0 themselves)
  const bool pre = c.opts.nu_pre >= 1 && c.opts.smoother == LLG_SMOOTHER_JACOBI;
  vcycle<T>(c, lc, (const T*)C.b, (T*)C.v1);
  const bool f1 = lc == 1 && c.f1;
  const int64_t G = f1 ? rows_blocks(C.A.n, L1_LANES) : rows_blocks(C.A.n, C.G);  // partial sums per column
  if (f1)
    l1<T>(c, 2, 0, (const T*)C.v1, nullptr, nullptr, (T*)C.w1, (const T*)C.b, nullptr, c.part);
  else
    launch_spmv_dots<T>(st, C.A, val, (const T*)C.v1, (T*)C.w1, (const T*)C.b, nullptr, c.part, C.G);
  launch_kc_coef(st, c.part, G, 1, C.kc);
  // the partials of w1.rho wait in the level's own buffer until stage 3
  double* part_rho = C.prho;
  launch_kc_update<T>(st, C.A.n, (const T*)C.b, (const T*)C.w1, C.kc, (T*)C.rho, (const T*)C.dinv, c.omega,
                      pre ? (T*)C.x : nullptr, part_rho);
  LCHK();
  vcycle<T>(c, lc, (const T*)C.rho, (T*)C.v2);
  if (f1)
    l1<T>(c, 2, 0, (const T*)C.v2, nullptr, nullptr, (T*)C.w2, (const T*)C.w1, (const T*)C.rho, c.part);
  else
    launch_spmv_dots<T>(st, C.A, val, (const T*)C.v2, (T*)C.w2, (const T*)C.w1, (const T*)C.rho, c.part, C.G);
  launch_kc_coef(st, c.part, G, 3, C.kc, part_rho, rows_blocks(C.A.n, 1));
  launch_kc_combine<T>(st, C.A.n, (const T*)C.v1, (const T*)C.v2, C.kc, (T*)C.e);
  LCHK();
}

template <typename T>
void precond(llg_ctx& c, const double* v, T* z, const double* vscale = nullptr) {
  Level& L0 = c.lv[0];
  if (c.fact)
    launch_scale_in_grid<T>(c.st, gdims(c), v, vscale, (T*)L0.b);
  else
    launch_scale_in<T>(c.st, c.N, c.dinv0, c.opts.left_scale, v, vscale, (T*)L0.b);
  LCHK();
  vcycle<T>(c, 0, (const T*)L0.b, z);
}

// ------------------------------------------------------------------ FGMRES
struct SolveOut {
  int iters = 0, restarts = 0;
  bool converged = false;
  double est = 0, truer = 0;
};

// One FGMRES iteration with basis index j, in three parts: z_j = B v_j (the
// preconditioner cycle), w = A z_j (the outer SpMV), and the two-pass
// classical Gram-Schmidt against v_0..v_j with the Hessenberg column, Givens
// update and v_{j+1} = w / h_{j+1,j}.  Parts 1 and 3 are replayed as graphs;
// the outer SpMV is a single launch, timed with events on the stream.
template <typename T>
void iter_precond(llg_ctx& c, int j) {
  const bool dcgs = c.opts.arnoldi == LLG_ARNOLDI_DCGS2;
  if (c.opts.krylov == LLG_KRYLOV_GMRES) {  // unpreconditioned: z_j = v_j
    launch_scale_copy(c.st, 3 * c.N, c.V + (int64_t)j * c.ld, dcgs ? c.ks.hinv + j : nullptr,
                      (double*)c.Z + (int64_t)j * c.ld);
    LCHK();
    return;
  }
  precond<T>(c, c.V + (int64_t)j * c.ld, (T*)c.Z + (int64_t)j * c.ld, dcgs ? c.ks.hinv + j : nullptr);
}

// The outer product is timed by the kernel's own start and end stamps (a
// launch with events), so the figure is the kernel's duration alone.
template <typename T>
void iter_spmv(llg_ctx& c, int j) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  kernel_events(c, LLG_KT_OUTER_SPMV, e0, e1);
  outer_spmv<T>(c, (const T*)c.Z + (int64_t)j * c.ld, c.w, e0, e1);
  LCHK();
}

void iter_arnoldi(llg_ctx& c, int j) {
  hipStream_t st = c.st;
  const int R = c.opts.restart;
  const int64_t m = 3 * c.N;
  KTimer kt(c, LLG_KT_ARNOLDI);
  if (c.opts.arnoldi == LLG_ARNOLDI_DCGS2) {
    // delayed reorthogonalization: one sweep for the dots, one for v_j and w'
    double* u = c.V + (int64_t)j * c.ld;
    launch_dcgs_dots(st, m, j, c.V, c.ld, u, c.w, c.part);
    launch_dcgs_finish1(st, c.part, c.npart_vec, j, R, c.ks, c.host);
    launch_dcgs_update(st, m, j, c.V, c.ld, c.ks.coef, u, c.w, c.V + (int64_t)(j + 1) * c.ld, c.part);
    launch_dcgs_finish2(st, c.part, c.npart_vec, j, R, c.ks, c.host);
    LCHK();
    return;
  }
  // classical Gram-Schmidt; the second pass only when the first lost more
  // than half of ||w||^2
  launch_mdot(st, m, j + 1, c.V, c.ld, c.w, c.part);
  launch_dots_finish_n(st, c.part, c.npart_vec, j + 1, c.ks.hcol, c.ks.sc);
  launch_mupdate_dot(st, m, j + 1, c.V, c.ld, c.ks.hcol, c.w, c.part, 1, nullptr);
  launch_reorth_finish_n(st, c.part, c.npart_vec, j + 1, c.ks.hcol, c.delta, c.ks.sc);
  launch_mupdate_dot(st, m, j + 1, c.V, c.ld, c.delta, c.w, c.part, 0, c.ks.sc + 7);
  launch_arnoldi_finish_n(st, c.part, c.npart_vec, j, R, c.ks, c.host);
  launch_scale_vec(st, m, c.w, c.ks.sc + 1, c.V + (int64_t)(j + 1) * c.ld);
  LCHK();
}

// The first two parts of iteration j (z_j = B v_j, w = A z_j): they write
// only z_j and w, so they may run ahead of the convergence test of iteration
// j - 1 (a finished solve never reads them).
template <typename T>
void iteration_head(llg_ctx& c, int j) {
  if (use_graphs(c) && !c.pc_graph[j]) c.pc_graph[j] = try_capture(c, [&]() { iter_precond<T>(c, j); });
  if (use_graphs(c))
    HIPX(hipGraphLaunch(c.pc_graph[j], c.st));
  else
    iter_precond<T>(c, j);
  iter_spmv<T>(c, j);
}

// The orthogonalization of iteration j (and the residual estimate to the host)
void iteration_tail(llg_ctx& c, int j) {
  if (use_graphs(c) && !c.it_graph[j]) c.it_graph[j] = try_capture(c, [&]() { iter_arnoldi(c, j); });
  if (use_graphs(c))
    HIPX(hipGraphLaunch(c.it_graph[j], c.st));
  else
    iter_arnoldi(c, j);
}

template <typename T>
SolveOut fgmres(llg_ctx& c) {
  hipStream_t st = c.st;
  const int R = c.opts.restart;
  const int64_t m = 3 * c.N;
  double* H = c.host;
  T* Z = (T*)c.Z;
  SolveOut so;
  H[7] = 0.0;
  // ||b|| and r = b - A u
  launch_norm_part(st, m, c.b, c.part);
  launch_norm_finish_n(st, c.part, c.npart_vec, 2, c.ks.sc, H);
  outer_resid(c);
  launch_norm_finish_n(st, c.part, c.npart_rows, 0, c.ks.sc, H);
  LCHK();
  HIPX(hipMemcpyAsync(c.hflags, c.flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  sync(c);
  if (*c.hflags & F_NONFINITE_IN) throw LLG_ERR_NONFINITE;
  const double bnorm = H[2];
  const double target = c.opts.rtol * bnorm;
  double beta = H[0];
  so.truer = bnorm > 0 ? beta / bnorm : 0;
  so.est = so.truer;
  if (bnorm == 0.0 || beta <= target) {
    so.converged = true;
    return so;
  }
  while (!so.converged && so.iters < c.opts.max_iters) {
    launch_cycle_start(st, R, c.ks);
    launch_scale_vec(st, m, c.r, c.ks.sc + 1, c.V);
    LCHK();
    // Pipelined iterations: after enqueuing the orthogonalization of column
    // j, the preconditioner and product of column j + 1 are enqueued before
    // the host waits for the estimate of iteration j, so the device never
    // idles during the host's test.  They are skipped when iteration j is
    // predicted to converge (the estimate falls about geometrically: est_j ~
    // est_{j-1}^2 / est_{j-2}), where they would be wasted work.
    int j = 0;
    bool ahead = false;  // the head of iteration j is already enqueued
    double e1 = -1.0, e2 = -1.0;  // the last two estimates (unscaled) of this cycle
    for (; j < R && so.iters < c.opts.max_iters; ++j) {
      if (!ahead) iteration_head<T>(c, j);
      iteration_tail(c, j);
      bool next = c.opts.pipeline && j + 1 < R && so.iters + 1 < c.opts.max_iters;
      if (next && e1 > 0 && e2 > 0) next = e1 * std::min(1.0, e1 / e2) > 3.0 * target;
      if (next) {
        HIPX(hipEventRecord(c.it_ev, st));
        const size_t mark = c.ev_used;
        iteration_head<T>(c, j + 1);
        HIPX(hipEventSynchronize(c.it_ev));
        harvest(c, mark);
      } else {
        sync(c);
      }
      ahead = next;
      ++so.iters;
      so.est = bnorm > 0 ? H[3] / bnorm : 0;
      e2 = e1;
      e1 = H[3];
      if (H[3] <= target || H[6] != 0.0) {
        ++j;
        break;
      }
    }
    if (c.opts.arnoldi == LLG_ARNOLDI_DCGS2) {
      // the last column is final once slot j is orthogonalized against v_0..v_{j-1}
      double* u = c.V + (int64_t)j * c.ld;
      launch_dcgs_dots(st, m, j, c.V, c.ld, u, u, c.part);
      launch_dcgs_last(st, c.part, c.npart_vec, j, R, c.ks, H);
      LCHK();
    }
    launch_solve_y(st, j, R, c.ks);
    launch_zy<T>(st, m, j, Z, c.ld, c.ks.y, c.u);
    outer_resid(c);
    launch_norm_finish_n(st, c.part, c.npart_rows, 0, c.ks.sc, H);
    LCHK();
    sync(c);
    beta = H[0];
    so.truer = beta / bnorm;
    so.converged = beta <= target;
    if (!so.converged) ++so.restarts;
  }
  return so;
}

// ------------------------------------------------------------------ baselines
// r = b - A u, its norm to the host (H[0]); synchronizes.
double true_residual(llg_ctx& c) {
  outer_resid(c);
  launch_norm_finish_n(c.st, c.part, c.npart_rows, 0, c.ks.sc, c.host);
  LCHK();
  sync(c);
  return c.host[0];
}

// Shared loop of the baselines: `start` begins a cycle from r, `body` is one
// iteration (replayed as a graph); a cycle ends on a breakdown flag or when
// the recurrence's residual estimate meets the target, and the true residual
// decides; otherwise the method restarts from the current iterate.
template <typename Start, typename Body>
SolveOut baseline_loop(llg_ctx& c, Start start, Body body) {
  hipStream_t st = c.st;
  const int64_t m = 3 * c.N;
  double* H = c.host;
  SolveOut so;
  H[7] = 0.0;
  launch_norm_part(st, m, c.b, c.part);
  launch_norm_finish_n(st, c.part, c.npart_vec, 2, c.ks.sc, H);
  LCHK();
  double rn = true_residual(c);
  const double bnorm = H[2];
  const double target = c.opts.rtol * bnorm;
  so.truer = so.est = bnorm > 0 ? rn / bnorm : 0;
  if (bnorm == 0.0 || rn <= target) {
    so.converged = true;
    return so;
  }
  while (so.iters < c.opts.max_iters) {
    start();
    LCHK();
    const int before = so.iters;
    while (so.iters < c.opts.max_iters) {
      if (use_graphs(c) && !c.kb_graph) c.kb_graph = try_capture(c, [&]() { body(); });
      if (use_graphs(c) && c.kb_graph)
        HIPX(hipGraphLaunch(c.kb_graph, st));
      else
        body();
      sync(c);
      ++so.iters;
      so.est = bnorm > 0 ? H[3] / bnorm : 0;
      if (H[6] != 0.0 || H[3] <= target) break;
    }
    rn = true_residual(c);
    so.truer = rn / bnorm;
    so.converged = rn <= target;
    if (so.converged || so.iters == before) break;
    ++so.restarts;
  }
  return so;
}

// Bi-CGSTAB (van der Vorst 1992) on A, without preconditioner; the shadow
// vector of each start is its residual.
SolveOut bicgstab(llg_ctx& c) {
  // launches go to c.st as read at call time (the capture stream while a
  // graph is recorded)
  const int64_t m = 3 * c.N, ld = c.ld, np = c.npart_vec;
  double *rh = c.V, *p = c.V + ld, *v = c.V + 2 * ld, *s = c.V + 3 * ld, *t = c.V + 4 * ld;
  double* kb = c.kb;
  const KTerm none{nullptr, nullptr, 0.0};
  auto start = [&]() {
    launch_copy(c.st, m, c.r, rh);
    launch_copy(c.st, m, c.r, p);
    launch_dot2(c.st, m, c.r, rh, c.r, c.r, c.part);
    launch_kb_step(c.st, c.part, np, KB_START, kb, c.host);
  };
  auto body = [&]() {
    outer_spmv<double>(c, p, v);
    launch_dot2(c.st, m, v, rh, nullptr, nullptr, c.part);
    launch_kb_step(c.st, c.part, np, KB_ALPHA, kb, c.host);
    launch_lin3(c.st, m, KTerm{c.r, nullptr, 1.0}, KTerm{v, kb + KB_ALPHA, -1.0}, none, s, nullptr, nullptr, c.part);
    outer_spmv<double>(c, s, t);
    launch_dot2(c.st, m, t, s, t, t, c.part);
    launch_kb_step(c.st, c.part, np, KB_OMEGA, kb, c.host);
    launch_lin3(c.st, m, KTerm{c.u, nullptr, 1.0}, KTerm{p, kb + KB_ALPHA, 1.0}, KTerm{s, kb + KB_OMEGA, 1.0}, c.u,
                nullptr, nullptr, c.part);
    launch_lin3(c.st, m, KTerm{s, nullptr, 1.0}, KTerm{t, kb + KB_OMEGA, -1.0}, none, c.r, rh, nullptr, c.part);
    launch_kb_step(c.st, c.part, np, KB_BICG_END, kb, c.host);
    launch_lin3(c.st, m, KTerm{c.r, nullptr, 1.0}, KTerm{p, kb + KB_BETA, 1.0}, KTerm{v, kb + KB_BW, -1.0}, p,
                nullptr, nullptr, c.part);
  };
  return baseline_loop(c, start, body);
}

// TFQMR (Freund 1993) on A, without preconditioner: one iteration is the two
// half-steps of a pair, u_even then u_odd.
SolveOut tfqmr(llg_ctx& c) {
  // launches go to c.st as read at call time (the capture stream while a
  // graph is recorded)
  const int64_t m = 3 * c.N, ld = c.ld, np = c.npart_vec;
  double *rs = c.V, *w = c.V + ld, *ue = c.V + 2 * ld, *uo = c.V + 3 * ld, *v = c.V + 4 * ld;
  double *d = c.V + 5 * ld, *aue = c.V + 6 * ld, *auo = c.V + 7 * ld;
  double* kb = c.kb;
  const KTerm none{nullptr, nullptr, 0.0};
  auto start = [&]() {
    launch_copy(c.st, m, c.r, rs);
    launch_copy(c.st, m, c.r, w);
    launch_copy(c.st, m, c.r, ue);
    outer_spmv<double>(c, ue, aue);
    launch_copy(c.st, m, aue, v);
    launch_lin3(c.st, m, KTerm{ue, nullptr, 0.0}, none, none, d, nullptr, nullptr, c.part);
    launch_dot2(c.st, m, c.r, rs, c.r, c.r, c.part);
    launch_kb_step(c.st, c.part, np, KB_START, kb, c.host);
  };
  auto half = [&](const double* um, const double* aum) {
    launch_kb_step(c.st, c.part, np, KB_TF_F, kb, c.host);
    launch_lin3(c.st, m, KTerm{w, nullptr, 1.0}, KTerm{aum, kb + KB_ALPHA, -1.0}, none, w, nullptr, nullptr, c.part);
    launch_kb_step(c.st, c.part, np, KB_TF_HALF, kb, c.host);
    launch_lin3(c.st, m, KTerm{um, nullptr, 1.0}, KTerm{d, kb + KB_F, 1.0}, none, d, nullptr, nullptr, c.part);
    launch_lin3(c.st, m, KTerm{c.u, nullptr, 1.0}, KTerm{d, kb + KB_ETA, 1.0}, none, c.u, nullptr, nullptr, c.part);
  };
  auto body = [&]() {
    launch_dot2(c.st, m, v, rs, nullptr, nullptr, c.part);
    launch_kb_step(c.st, c.part, np, KB_ALPHA, kb, c.host);
    launch_lin3(c.st, m, KTerm{ue, nullptr, 1.0}, KTerm{v, kb + KB_ALPHA, -1.0}, none, uo, nullptr, nullptr, c.part);
    outer_spmv<double>(c, uo, auo);
    half(ue, aue);
    half(uo, auo);
    launch_dot2(c.st, m, w, rs, nullptr, nullptr, c.part);
    launch_kb_step(c.st, c.part, np, KB_TF_END, kb, c.host);
    launch_lin3(c.st, m, KTerm{w, nullptr, 1.0}, KTerm{uo, kb + KB_BETA, 1.0}, none, ue, nullptr, nullptr, c.part);
    outer_spmv<double>(c, ue, aue);
    launch_lin3(c.st, m, KTerm{aue, nullptr, 1.0}, KTerm{auo, kb + KB_BETA, 1.0}, KTerm{v, kb + KB_B2, 1.0}, v, nullptr,
                nullptr, c.part);
  };
  return baseline_loop(c, start, body);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <typename T>
llg_status run_step(llg_ctx& c, const double* m_n, const double* m_nm1, double alpha, double dt, const double* F,
                    double* m_np1, llg_stats* stats, const llg_field* fld = nullptr) {
  const auto t0 = std::chrono::steady_clock::now();
  c.kernel_ms = 0;
  c.launches = 0;
  c.kernel_bytes = 0;
  c.ev_used = 0;
  const int64_t fb = (int64_t)sizeof(double) * 3 * c.N;
  const bool bdf2 = c.opts.scheme == LLG_SCHEME_BDF2 && m_nm1 != nullptr;
  if (fld) {  // the field terms read m^n (and m^{n-1}) at fixed addresses
    HIPX(hipMemcpyAsync(c.min, m_n, fb, hipMemcpyDeviceToDevice, c.st));
    if (bdf2) HIPX(hipMemcpyAsync(c.mprv, m_nm1, fb, hipMemcpyDeviceToDevice, c.st));
  }
  write_params(c, alpha, dt, bdf2, fld, m_n, bdf2 ? m_nm1 : nullptr, F);
  launch_fill_i32(c.st, c.flags, 1, 0);
  LCHK();
  const int field = fld ? (fld->stray ? 2 : 1) : 0;
  if (field == 2) demag_prepare(c);
  run_setup<T>(c, F != nullptr, bdf2, field);
  HIPX(hipStreamSynchronize(c.st));
  const double t_setup = ms_since(t0);
  SolveOut so = c.opts.krylov == LLG_KRYLOV_BICGSTAB ? bicgstab(c)
                : c.opts.krylov == LLG_KRYLOV_TFQMR  ? tfqmr(c)
                                                     : fgmres<T>(c);
  launch_project(c.st, c.N, c.u, m_np1, c.opts.project, c.flags);
  LCHK();
  HIPX(hipMemcpyAsync(c.hflags, c.flags, sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
  sync(c);
  const int32_t fl = *c.hflags;
  if (stats) {
    stats->iters = so.iters;
    stats->restarts = so.restarts;
    stats->levels = c.L;
    stats->converged = so.converged ? 1 : 0;
    stats->relres_est = so.est;
    stats->relres_true = so.truer;
    for (int l = 0; l < LLG_MAX_LEVELS; ++l) {
      stats->level_nodes[l] = l < c.L ? c.lv[l].A.n : 0;
      stats->level_nnzb[l] = l < c.L ? c.lv[l].nnzb : 0;
    }
    stats->ms_setup = t_setup;
    stats->ms_total = ms_since(t0);
    stats->ms_solve = stats->ms_total - t_setup;
    stats->kernel_ms = c.kernel_ms;
    stats->kernel_launches = c.launches;
    stats->kernel_bytes = c.kernel_bytes;
    stats->reorth_passes = (int32_t)c.host[7];
    stats->tail_level = c.tail;
  }
  if (fl & F_PLAN) {
    set_err("device-side check of the hierarchy structure failed");
    return LLG_ERR_DEVICE;
  }
  if (fl & F_NONFINITE_IN) return LLG_ERR_NONFINITE;
  if (fl & F_SINGULAR) {
    set_err("coarsest-level matrix is singular");
    return LLG_ERR_DEVICE;
  }
  if (fl & F_PROJECT) return LLG_ERR_NONFINITE;
  return so.converged ? LLG_OK : LLG_ERR_NOT_CONVERGED;
}

// Run f, mapping exceptions to status codes.
template <typename Fn>
llg_status guard(Fn f) {
  try {
    return f();
  } catch (const DevError& e) {
    set_err(e.msg);
    return LLG_ERR_DEVICE;
  } catch (llg_status s) {
    return s;
  } catch (const std::bad_alloc&) {
    set_err("host allocation failed");
    return LLG_ERR_DEVICE;
  }
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace
}  // namespace llg

using namespace llg;

extern "C" {

void llg_default_opts(llg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-10;
  o->restart = 30;
  o->max_iters = 1000;
  o->precision = LLG_PREC_FP64;
  o->nu_pre = 1;
  o->nu_post = 1;
  o->omega = 0.0;
  o->npass = 2;
  o->beta_num = 1;
  o->beta_den = 4;
  o->max_coarse = 40;
  o->stagnation = 0.8;
  o->max_levels = 40;
  o->max_dense = 512;
  o->left_scale = 1;
  o->project = 1;
  o->x0_is_mn = 1;
  o->agg_salt = 0;
  o->rebuild_aggregates = 1;
  o->kcycle_depth = 0;
  o->graphs = 0;
  o->smoother = LLG_SMOOTHER_JACOBI;
  o->scheme = LLG_SCHEME_BDF1;
  o->fine_operator = LLG_FINE_BSR;
  o->arnoldi = LLG_ARNOLDI_DCGS2;
  o->krylov = LLG_KRYLOV_FGMRES_AMG;
  o->stray_field = 0;
  o->tail_nodes = 128;
  o->pipeline = 1;
  o->overlap_rebuild = 1;
  o->csr_levels = 1;
}

// combinations the library does not implement
static bool supported(const llg_grid* grid, const llg_opts* opts) {
  if (grid->bc != LLG_BC_NEUMANN) return false;
  if (opts->fine_operator == LLG_FINE_FACTORED && !opts->left_scale) return false;
  if (opts->krylov != LLG_KRYLOV_FGMRES_AMG && opts->precision != LLG_PREC_FP64) return false;
  if (opts->stray_field) {  // padded FFT lengths within the one-workgroup transform
    const FieldDims f = field_dims(grid->n[0], grid->n[1], grid->n[2]);
    if (std::max(f.px, std::max(f.py, f.pz)) > FFT_MAX_LEN) return false;
  }
  return true;
}

llg_status llg_workspace_bytes(const llg_grid* grid, const llg_opts* opts, size_t* bytes) {
  if (!grid_ok(grid) || !opts_ok(opts) || !bytes) return LLG_ERR_INVALID_ARG;
  if (!supported(grid, opts)) return LLG_ERR_UNSUPPORTED;
  return guard([&]() -> llg_status {
    auto plan = get_plan(*grid, *opts);
    if (plan->status != LLG_OK) return (llg_status)plan->status;
    *bytes = plan->total;
    return LLG_OK;
  });
}

llg_status llg_create(const llg_grid* grid, const llg_opts* opts, void* d_workspace, size_t bytes,
                      void* hip_stream, llg_ctx** out) {
  if (!grid_ok(grid) || !opts_ok(opts) || !out || !d_workspace) return LLG_ERR_INVALID_ARG;
  if (((uintptr_t)d_workspace & (ALIGN - 1)) != 0) return LLG_ERR_INVALID_ARG;
  if (!supported(grid, opts)) return LLG_ERR_UNSUPPORTED;
  *out = nullptr;
  return guard([&]() -> llg_status {
    auto plan = get_plan(*grid, *opts);
    if (plan->status != LLG_OK) return (llg_status)plan->status;
    if (bytes < plan->total) return LLG_ERR_WORKSPACE;
    std::unique_ptr<llg_ctx> c(new llg_ctx());
    c->grid = *grid;
    c->opts = *opts;
    c->plan = plan;
    HIPX(hipGetDevice(&c->device));
    c->st = (hipStream_t)hip_stream;
    c->ws = (char*)d_workspace;
    c->ws_bytes = bytes;
    c->N = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    c->omega = opts->omega > 0 ? opts->omega : (grid->dim == 2 ? 4.0 / 5.0 : 6.0 / 7.0);
    HIPX(hipHostMalloc((void**)&c->host, sizeof(double) * 16, hipHostMallocDefault));
    HIPX(hipHostMalloc((void**)&c->hflags, sizeof(int32_t) * 4, hipHostMallocDefault));
    HIPX(hipHostMalloc((void**)&c->hprm, sizeof(double) * PRM_WORDS, hipHostMallocDefault));
    HIPX(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&c->it_ev, hipEventDisableTiming));
    c->it_graph.assign(opts->restart, nullptr);
    c->pc_graph.assign(opts->restart, nullptr);
    init_kernel_attributes();
    init_field_attributes();
    c->tail_ok = tail_prepare();
    Arena ar;
    ar.mode = Mode::REPLAY;
    ar.plan = plan.get();
    ar.first = true;
    ar.ptrs = &c->ptrs;
    ar.base = c->ws;
    ar.cap = bytes;
    ar.st = c->st;
    c->L = build_structure(*c, ar);
    allocate_numeric(*c, ar);
    c->used = ar.off;
    int32_t fl1 = 0;
    if (plan->dbl) {  // the second structure set, built here as well
      c->dbl = true;
      save_struct(*c, c->sets[0]);
      Arena a2;
      a2.mode = Mode::REPLAY;
      a2.plan = plan.get();
      a2.first = true;
      a2.ptrs = &c->ptrs2;
      a2.base = c->ws + c->used;
      a2.cap = bytes - c->used;
      a2.st = c->st;
      (void)build_structure(*c, a2);
      c->used += a2.off;
      save_struct(*c, c->sets[1]);
      HIPX(hipMemcpyAsync(c->hflags, c->flags, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
      HIPX(hipStreamSynchronize(c->st));
      fl1 = *c->hflags;
      load_struct(*c, c->sets[0]);
      retarget_tail(*c);
      HIPX(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
      for (int k = 0; k < 2; ++k) {
        HIPX(hipEventCreateWithFlags(&c->built[k], hipEventDisableTiming));
        HIPX(hipEventRecord(c->built[k], c->st));  // both sets are complete on the main stream
      }
      HIPX(hipEventCreateWithFlags(&c->main_ev, hipEventDisableTiming));
    }
    HIPX(hipMemcpyAsync(c->hflags, c->flags, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPX(hipStreamSynchronize(c->st));
    if ((*c->hflags | fl1) & F_PLAN) {
      set_err("hierarchy structure differs from the plan");
      llg_destroy(c.release());
      return LLG_ERR_DEVICE;
    }
    *out = c.release();
    return LLG_OK;
  });
}

static llg_status check_ctx(llg_ctx* c) {
  if (!c) return LLG_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
    set_err("context used on a device other than the one it was created on");
    return LLG_ERR_INVALID_ARG;
  }
  return LLG_OK;
}

llg_status llg_setup(llg_ctx* ctx, const double* d_m_tilde, double alpha, double dt) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!d_m_tilde || !aligned8(d_m_tilde) || !(dt > 0) || !std::isfinite(dt) || !(alpha >= 0) ||
      !std::isfinite(alpha))
    return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    write_params(*ctx, alpha, dt, false, nullptr, d_m_tilde, nullptr, nullptr);
    launch_fill_i32(ctx->st, ctx->flags, 1, 0);
    if (ctx->opts.precision == LLG_PREC_FP32_AMG)
      run_setup<float>(*ctx, false);
    else
      run_setup<double>(*ctx, false);
    HIPX(hipMemcpyAsync(ctx->hflags, ctx->flags, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->st));
    sync(*ctx);
    if (*ctx->hflags & F_PLAN) return LLG_ERR_DEVICE;
    if (*ctx->hflags & F_NONFINITE_IN) return LLG_ERR_NONFINITE;
    return LLG_OK;
  });
}

llg_status llg_step(llg_ctx* ctx, const double* d_m_n, const double* d_m_nm1, double alpha, double dt,
                    const double* d_forcing, double* d_m_np1, llg_stats* stats) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!d_m_n || !d_m_np1 || !aligned8(d_m_n) || !aligned8(d_m_np1) || (d_forcing && !aligned8(d_forcing)))
    return LLG_ERR_INVALID_ARG;
  if (!(dt > 0) || !std::isfinite(dt) || !(alpha >= 0) || !std::isfinite(alpha)) return LLG_ERR_INVALID_ARG;
  const size_t fb = sizeof(double) * 3 * (size_t)ctx->N;
  auto overlap = [fb](const void* x, const void* y) {
    const char* a0 = (const char*)x;
    const char* b0 = (const char*)y;
    return a0 < b0 + fb && b0 < a0 + fb;
  };
  if (overlap(d_m_n, d_m_np1)) return LLG_ERR_INVALID_ARG;
  const double* prev = ctx->opts.scheme == LLG_SCHEME_BDF2 ? d_m_nm1 : nullptr;
  if (prev && (!aligned8(prev) || overlap(prev, d_m_np1))) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    if (ctx->opts.precision == LLG_PREC_FP32_AMG)
      return run_step<float>(*ctx, d_m_n, prev, alpha, dt, d_forcing, d_m_np1, stats);
    return run_step<double>(*ctx, d_m_n, prev, alpha, dt, d_forcing, d_m_np1, stats);
  });
}

llg_status llg_step_field(llg_ctx* ctx, const double* d_m_n, const double* d_m_nm1, double alpha, double dt,
                          const llg_field* field, const double* d_forcing, double* d_m_np1, llg_stats* stats) {
  if (!field) return llg_step(ctx, d_m_n, d_m_nm1, alpha, dt, d_forcing, d_m_np1, stats);
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!(field->eps > 0) || !std::isfinite(field->eps) || !std::isfinite(field->q) ||
      !std::isfinite(field->h_ext[0]) || !std::isfinite(field->h_ext[1]) || !std::isfinite(field->h_ext[2]) ||
      (field->stray && !ctx->opts.stray_field))
    return LLG_ERR_INVALID_ARG;
  if (!d_m_n || !d_m_np1 || !aligned8(d_m_n) || !aligned8(d_m_np1) || (d_forcing && !aligned8(d_forcing)))
    return LLG_ERR_INVALID_ARG;
  if (!(dt > 0) || !std::isfinite(dt) || !(alpha >= 0) || !std::isfinite(alpha)) return LLG_ERR_INVALID_ARG;
  const size_t fb = sizeof(double) * 3 * (size_t)ctx->N;
  auto overlap = [fb](const void* x, const void* y) {
    const char* a0 = (const char*)x;
    const char* b0 = (const char*)y;
    return a0 < b0 + fb && b0 < a0 + fb;
  };
  if (overlap(d_m_n, d_m_np1)) return LLG_ERR_INVALID_ARG;
  const double* prev = ctx->opts.scheme == LLG_SCHEME_BDF2 ? d_m_nm1 : nullptr;
  if (prev && (!aligned8(prev) || overlap(prev, d_m_np1))) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    if (ctx->opts.precision == LLG_PREC_FP32_AMG)
      return run_step<float>(*ctx, d_m_n, prev, alpha, dt, d_forcing, d_m_np1, stats, field);
    return run_step<double>(*ctx, d_m_n, prev, alpha, dt, d_forcing, d_m_np1, stats, field);
  });
}

llg_status llg_stray_field(llg_ctx* ctx, const double* d_m, double* d_h) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!ctx->opts.stray_field || !d_m || !d_h || !aligned8(d_m) || !aligned8(d_h)) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    demag_prepare(*ctx);
    launch_stray(ctx->st, ctx->fd, d_m, nullptr, ctx->nhat, ctx->fwork);
    launch_stray_out(ctx->st, ctx->fd, ctx->fwork, d_h);
    LCHK();
    HIPX(hipStreamSynchronize(ctx->st));
    return LLG_OK;
  });
}

llg_status llg_stray_field_noalloc(const llg_grid* grid, const double* d_m, double* d_h, void* hip_stream) {
  if (!grid_ok(grid) || !d_m || !d_h || !aligned8(d_m) || !aligned8(d_h)) return LLG_ERR_INVALID_ARG;
  if (grid->bc != LLG_BC_NEUMANN) return LLG_ERR_UNSUPPORTED;
  const FieldDims f = field_dims(grid->n[0], grid->n[1], grid->n[2]);
  if (std::max(f.px, std::max(f.py, f.pz)) > FFT_MAX_LEN || stray_noalloc_bytes(f) > LLG_STRAY_NOALLOC_MAX_BYTES) {
    set_err("padded grid exceeds the static stray-field scratch");
    return LLG_ERR_UNSUPPORTED;
  }
  return guard([&]() -> llg_status {
    HIPX(stray_noalloc(f, d_m, d_h, (hipStream_t)hip_stream));
    return LLG_OK;
  });
}

llg_status llg_get_demag_tensor(llg_ctx* ctx, double* h_out, int64_t cap) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!ctx->opts.stray_field || !h_out) return LLG_ERR_INVALID_ARG;
  const FieldDims& f = ctx->fd;
  const int64_t ox = 2 * f.nx - 1, oy = 2 * f.ny - 1, oz = 2 * f.nz - 1, P = f.px * f.py * f.pz;
  if (cap < 6 * ox * oy * oz) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    double* T = (double*)(ctx->fwork + P);
    launch_demag_table(ctx->st, f, T);
    std::vector<double2> host((size_t)P);
    const int pairs[3][2] = {{0, 1}, {2, 3}, {4, 5}};
    for (int r = 0; r < 3; ++r) {
      launch_demag_pair(ctx->st, f, pairs[r][0], pairs[r][1], T, ctx->fwork);
      LCHK();
      HIPX(hipMemcpyAsync(host.data(), ctx->fwork, (size_t)P * sizeof(double2), hipMemcpyDeviceToHost, ctx->st));
      HIPX(hipStreamSynchronize(ctx->st));
      // offset (a, b, c) sits at padded index (a mod px, b mod py, c mod pz)
      for (int64_t c = 0; c < oz; ++c)
        for (int64_t b = 0; b < oy; ++b)
          for (int64_t a = 0; a < ox; ++a) {
            const int64_t X = a - (f.nx - 1), Y = b - (f.ny - 1), Z = c - (f.nz - 1);
            const int64_t p = ((X + f.px) % f.px) + f.px * (((Y + f.py) % f.py) + f.py * ((Z + f.pz) % f.pz));
            const int64_t o = a + ox * (b + oy * c);
            h_out[pairs[r][0] * ox * oy * oz + o] = host[(size_t)p].x;
            h_out[pairs[r][1] * ox * oy * oz + o] = host[(size_t)p].y;
          }
    }
    return LLG_OK;
  });
}

llg_status llg_num_levels(llg_ctx* ctx, int32_t* levels) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!levels) return LLG_ERR_INVALID_ARG;
  *levels = ctx->L;
  return LLG_OK;
}

llg_status llg_level_info(llg_ctx* ctx, int32_t level, int64_t* n, int64_t* nnzb) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (level < -1 || level >= ctx->L) return LLG_ERR_INVALID_ARG;
  const Level& L = ctx->lv[level < 0 ? 0 : level];
  if (n) *n = L.A.n;
  if (nnzb) *nnzb = L.nnzb;
  return LLG_OK;
}

llg_status llg_get_level(llg_ctx* ctx, int32_t level, int32_t* h_row_ptr, int32_t* h_col, double* h_vals,
                         int64_t cap_nnzb) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (level < -1 || level >= ctx->L || !h_row_ptr || !h_col || !h_vals) return LLG_ERR_INVALID_ARG;
  const Level& L = ctx->lv[level < 0 ? 0 : level];
  if (cap_nnzb < L.nnzb) return LLG_ERR_INVALID_ARG;
  if (!ctx->setup_done) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    const bool f32 = level >= 0 && ctx->opts.precision == LLG_PREC_FP32_AMG;
    const size_t ts = f32 ? 4 : 8;
    const bool fact = level <= 0 && ctx->fact;
    if (fact) {  // the sliced blocks, from the frozen field of the last setup
      const llg_grid& g = ctx->grid;
      if (ctx->opts.precision == LLG_PREC_FP32_AMG)
        launch_fact_blocks<float>(ctx->st, g.n[0], g.n[1], g.n[2], 1.0 / (g.h * g.h), ctx->prm, ctx->mt, ctx->Mh,
                                  (float*)ctx->lv[0].kf);
      else
        launch_fact_blocks<double>(ctx->st, g.n[0], g.n[1], g.n[2], 1.0 / (g.h * g.h), ctx->prm, ctx->mt,
                                   ctx->Mh, (double*)ctx->lv[0].kf);
      LCHK();
    }
    // a level whose products do not read sliced-ELL values keeps only its
    // CSR-ordered copy (level 1 applied through the grid blocks)
    const bool csr = !fact && level >= 0 && !L.val;
    const void* val = fact ? (level < 0 ? (const void*)ctx->Mh : L.kf)
                           : (level < 0 ? (const void*)ctx->Aval : (csr ? L.vt : L.val));
    std::vector<int32_t> sl(L.A.nslices + 1), col(L.A.nslots);
    std::vector<char> v(ts * 9 * (size_t)(fact ? L.A.nslices * SL : (csr ? L.nnzb : L.A.nslots)));
    HIPX(hipStreamSynchronize(ctx->st));
    HIPX(hipMemcpy(h_row_ptr, L.brp, sizeof(int32_t) * (L.A.n + 1), hipMemcpyDeviceToHost));
    HIPX(hipMemcpy(sl.data(), L.A.sl_ptr, sizeof(int32_t) * sl.size(), hipMemcpyDeviceToHost));
    HIPX(hipMemcpy(col.data(), L.A.col, sizeof(int32_t) * col.size(), hipMemcpyDeviceToHost));
    HIPX(hipMemcpy(v.data(), val, v.size(), hipMemcpyDeviceToHost));
    auto rd = [&](int64_t vi) {
      return f32 ? (double)((const float*)v.data())[vi] : ((const double*)v.data())[vi];
    };
    for (int64_t i = 0; i < L.A.n; ++i) {
      const int64_t sidx = i / SL, lane = i % SL;
      const int64_t cb = sl[sidx];
      const int64_t len = h_row_ptr[i + 1] - h_row_ptr[i];
      for (int64_t t = 0; t < len; ++t) {
        const int64_t o = h_row_ptr[i] + t;
        const int32_t j = col[cb + t * SL + lane];
        h_col[o] = j;
        for (int e = 0; e < 9; ++e) {
          double x;
          if (fact) {
            // the blocks the factored products apply: off the diagonal the
            // stored block, on it I (scaled level) or I - deg Mh (level -1)
            const double id = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
            const double blk = rd(sidx * 9 * SL + e * SL + lane);
            if (j != (int32_t)i)
              x = blk;
            else
              x = level < 0 ? id + (-(double)(len - 1)) * blk : id;
          } else if (csr) {
            x = rd(o * 9 + e);
          } else {
            x = rd(cb * 9 + (t * 9 + e) * SL + lane);
          }
          h_vals[9 * o + e] = x;
        }
      }
    }
    return LLG_OK;
  });
}

llg_status llg_get_aggregates(llg_ctx* ctx, int32_t level, int32_t* h_out, int64_t n) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (level < 0 || level + 1 >= ctx->L || !h_out || n != ctx->lv[level].A.n) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    HIPX(hipStreamSynchronize(ctx->st));
    HIPX(hipMemcpy(h_out, ctx->lv[level].agg, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    return LLG_OK;
  });
}

llg_status llg_get_colours(llg_ctx* ctx, int32_t level, int32_t* h_out, int64_t n, int32_t* h_ncol) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (ctx->opts.smoother != LLG_SMOOTHER_MCGS || level < 0 || level + 1 >= ctx->L || !h_out || !h_ncol ||
      n != ctx->lv[level].A.n)
    return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    HIPX(hipStreamSynchronize(ctx->st));
    HIPX(hipMemcpy(h_out, ctx->lv[level].colour, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    *h_ncol = ctx->lv[level].ncol;
    return LLG_OK;
  });
}

llg_status llg_apply_precond(llg_ctx* ctx, const double* d_v, double* d_z) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!d_v || !d_z || !aligned8(d_v) || !aligned8(d_z) || !ctx->setup_done) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    if (ctx->opts.precision == LLG_PREC_FP32_AMG) {
      float* z = (float*)ctx->Z;
      precond<float>(*ctx, d_v, z);
      launch_cast<float, double>(ctx->st, 3 * ctx->N, z, d_z);
    } else {
      precond<double>(*ctx, d_v, d_z);
    }
    LCHK();
    sync(*ctx);
    return LLG_OK;
  });
}

llg_status llg_apply_A(llg_ctx* ctx, const double* d_x, double* d_y) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (!d_x || !d_y || !aligned8(d_x) || !aligned8(d_y) || !ctx->setup_done) return LLG_ERR_INVALID_ARG;
  return guard([&]() -> llg_status {
    outer_spmv<double>(*ctx, d_x, d_y);
    LCHK();
    sync(*ctx);
    return LLG_OK;
  });
}

llg_status llg_set_kernel_timing(llg_ctx* ctx, int32_t kernel_class) {
  llg_status s = check_ctx(ctx);
  if (s != LLG_OK) return s;
  if (kernel_class < LLG_KT_NONE || kernel_class > LLG_KT_LEVEL1) return LLG_ERR_INVALID_ARG;
  ctx->timed = kernel_class;
  return LLG_OK;
}

llg_status llg_ctx_bytes(llg_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return LLG_ERR_INVALID_ARG;
  *bytes = ctx->used;
  return LLG_OK;
}

llg_status llg_destroy(llg_ctx* ctx) {
  if (!ctx) return LLG_ERR_INVALID_ARG;
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  (void)hipStreamSynchronize(ctx->st);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  for (hipEvent_t e : ctx->built)
    if (e) (void)hipEventDestroy(e);
  if (ctx->main_ev) (void)hipEventDestroy(ctx->main_ev);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->it_ev) (void)hipEventDestroy(ctx->it_ev);
  for (hipGraphExec_t g : ctx->pc_graph)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipGraphExec_t g : ctx->it_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (ctx->kb_graph) (void)hipGraphExecDestroy(ctx->kb_graph);
  for (hipGraphExec_t g : ctx->setup_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (ctx->cap_st) (void)hipStreamDestroy(ctx->cap_st);
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->hflags) (void)hipHostFree(ctx->hflags);
  if (ctx->hprm) (void)hipHostFree(ctx->hprm);
  delete ctx;
  return LLG_OK;
}

const char* llg_status_str(llg_status s) {
  switch (s) {
    case LLG_OK: return "ok";
    case LLG_ERR_INVALID_ARG: return "invalid argument";
    case LLG_ERR_UNSUPPORTED: return "unsupported configuration";
    case LLG_ERR_WORKSPACE: return "workspace too small";
    case LLG_ERR_DEVICE: return "device error";
    case LLG_ERR_NOT_CONVERGED: return "not converged";
    case LLG_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char* llg_last_error(void) { return llg::g_err.c_str(); }

}  // extern "C"
