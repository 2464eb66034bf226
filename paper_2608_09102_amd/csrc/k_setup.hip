// k_setup.hip -- setup kernels: grid pattern, fine-operator assembly,
// pairwise-matching aggregation, Galerkin coarse operators, dense coarsest
// inverse.  Built with -ffp-contract=off: the assembly and Galerkin sums are
// evaluated in the exact operation order stated in their comments.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "llg_internal.h"

namespace llg {

namespace {

constexpr int TPB = 256;

inline unsigned nblk(int64_t n, int t = TPB) { return (unsigned)ceil_div(n > 0 ? n : 1, t); }

// ---------------------------------------------------------------- utilities
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Exclusive scan, three phases: per-block sums of 1024 items, a single-block
// scan of the block sums, then per-block scans with the block offset added.
constexpr int SCAN_T = 256, SCAN_ITEMS = 4, SCAN_CHUNK = SCAN_T * SCAN_ITEMS;

__device__ inline int32_t block_excl_scan(int32_t v, int32_t* sh, int32_t* total) {
  // inclusive Hillis-Steele scan over 256 threads in LDS
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int32_t a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int32_t incl = sh[t];
  *total = sh[SCAN_T - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_reduce(const int32_t* in, int64_t n, int32_t* bsum) {
  __shared__ int32_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
  int32_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
    if (i < n) s += in[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = SCAN_T / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

__global__ void k_scan_top(int32_t* bsum, int64_t nb, int32_t* total) {
  __shared__ int32_t sh[SCAN_T];
  __shared__ int32_t tot;
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_T) {
    int64_t i = base + threadIdx.x;
    int32_t v = i < nb ? bsum[i] : 0;
    int32_t t;
    int32_t ex = block_excl_scan(v, sh, &t);
    if (threadIdx.x == 0) tot = t;
    __syncthreads();
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// Whole scan in one workgroup of 1024 threads for short arrays (n <= 16384):
// each thread sums its run of up to 16 items, the runs are scanned by wave
// shuffles and the 16 wave totals in LDS, then each thread writes its run.
// In place is fine: every thread reads its items before any are written.
constexpr int SCAN1_T = 1024, SCAN1_ITEMS = 16;
__global__ void __launch_bounds__(SCAN1_T) k_scan_single(const int32_t* in, int32_t* out, int64_t n,
                                                          int32_t* total) {
  __shared__ int32_t wsum[SCAN1_T / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t per = (n + SCAN1_T - 1) / SCAN1_T;
  const int64_t base = (int64_t)t * per;
  int32_t v[SCAN1_ITEMS];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN1_ITEMS; ++k) {
    v[k] = (k < per && base + k < n) ? in[base + k] : 0;
    sum += v[k];
  }
  int32_t incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (wv == 0) {
    int32_t x = lane < SCAN1_T / 64 ? wsum[lane] : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane < SCAN1_T / 64) wsum[lane] = x;  // inclusive over waves
  }
  __syncthreads();
  int32_t ex = incl - sum + (wv > 0 ? wsum[wv - 1] : 0);
#pragma unroll
  for (int k = 0; k < SCAN1_ITEMS; ++k) {
    if (k < per && base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (t == SCAN1_T - 1) *total = ex;
}

__global__ void k_scan_down(const int32_t* in, int32_t* out, int64_t n, const int32_t* bsum) {
  __shared__ int32_t sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int32_t tot;
  int32_t ex = block_excl_scan(s, sh, &tot) + bsum[blockIdx.x];
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
}

__global__ void k_check_eq(const int32_t* a, int32_t expect, int32_t* flag, int32_t bit) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && a[0] != expect) atomicOr(flag, bit);
}

struct CountChecks {
  const int32_t* p[CHECK_BATCH];
  int32_t v[CHECK_BATCH];
  int32_t n;
};
__global__ void k_check_many(const CountChecks c, int32_t* flag, int32_t bit) {
  const int k = (int)threadIdx.x;
  if (k < c.n && *c.p[k] != c.v[k]) atomicOr(flag, bit);
}

// ---------------------------------------------------------------- grid graph
// Neighbours of node p in ascending index order: k-1, j-1, i-1, i+1, j+1, k+1
// (homogeneous Neumann: missing neighbours are simply absent).
__device__ inline int grid_nbrs(int nx, int ny, int nz, int64_t p, int64_t* nb) {
  const int64_t nxy = (int64_t)nx * ny;
  const int64_t k = p / nxy, r = p - k * nxy;
  const int64_t j = r / nx, i = r - j * nx;
  int c = 0;
  if (k > 0) nb[c++] = p - nxy;
  if (j > 0) nb[c++] = p - nx;
  if (i > 0) nb[c++] = p - 1;
  if (i < nx - 1) nb[c++] = p + 1;
  if (j < ny - 1) nb[c++] = p + nx;
  if (k < nz - 1) nb[c++] = p + nxy;
  return c;
}

__global__ void k_grid_degree(int nx, int ny, int nz, int32_t* deg) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (p >= N) return;
  int64_t nb[6];
  deg[p] = grid_nbrs(nx, ny, nz, p, nb);
}

__global__ void k_grid_graph(int nx, int ny, int nz, const int32_t* grp, int32_t* gci, int32_t* gw) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (p >= N) return;
  int64_t nb[6];
  int c = grid_nbrs(nx, ny, nz, p, nb);
  int32_t o = grp[p];
  for (int t = 0; t < c; ++t) {
    gci[o + t] = (int32_t)nb[t];
    gw[o + t] = 1;
  }
}

// Block pattern of a level: the graph (no self loops) plus the diagonal.
__global__ void k_pattern_rp(int64_t n, const int32_t* grp, int32_t* brp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) brp[i] = grp[i] + (int32_t)i;
}

// Row i of the block pattern: the graph row (ascending, no self loop) with the
// diagonal inserted in column order.  PC_L lanes share a row: lane sub takes
// the entries sub, sub + PC_L, ...; an entry past the diagonal moves one slot
// right, and the lane holding the first such entry writes the diagonal in
// front of it (lane 0 writes it last when every entry precedes it).  The
// stores of a row's lanes are contiguous; one thread per row walked its row
// with a load and a store per step.
constexpr int PC_L = 8;
__global__ void k_pattern_cols(int64_t n, const int32_t* grp, const int32_t* gci, const int32_t* brp,
                               int32_t* bci) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / PC_L;
  const int sub = (int)(t - i * PC_L);
  if (i >= n) return;
  const int32_t k0 = grp[i], k1 = grp[i + 1], o = brp[i];
  for (int32_t k = k0 + sub; k < k1; k += PC_L) {
    const int32_t c = gci[k];
    const bool after = c > (int32_t)i;
    bci[o + (k - k0) + (after ? 1 : 0)] = c;
    if (after && (k == k0 || gci[k - 1] < (int32_t)i)) bci[o + (k - k0)] = (int32_t)i;
  }
  if (sub == 0 && (k1 == k0 || gci[k1 - 1] < (int32_t)i)) bci[o + (k1 - k0)] = (int32_t)i;
}

// Sliced-ELL structure of the rows rows[0..n) of a CSR pattern (rows == NULL:
// rows 0..n).  Slice widths first, then the column slots.
__global__ void k_slice_width(int64_t n, const int32_t* rows, const int32_t* brp, int32_t* wslots) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ns = ceil_div(n, SL);
  if (s >= ns) return;
  int32_t w = 0;
  for (int64_t k = s * SL; k < (s + 1) * SL && k < n; ++k) {
    const int64_t i = rows ? rows[k] : k;
    w = max(w, brp[i + 1] - brp[i]);
  }
  wslots[s] = w * SL;
}

__global__ void k_sell_cols(int64_t n, const int32_t* rows, const int32_t* brp, const int32_t* bci,
                            const int32_t* sl_ptr, int32_t* col) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ns = ceil_div(n, SL);
  if (k >= ns * SL) return;
  const int64_t s = k / SL;
  const int l = (int)(k - s * SL);
  const int32_t base = sl_ptr[s];
  const int w = (sl_ptr[s + 1] - base) / SL;
  const int64_t i = k < n ? (rows ? rows[k] : k) : -1;
  const int len = i >= 0 ? brp[i + 1] - brp[i] : 0;
  const int32_t r0 = i >= 0 ? brp[i] : 0;
  // eight slots at a time, their loads in flight together
  for (int t = 0; t < w; t += 8) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = t + u < len ? bci[r0 + t + u] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (t + u < w) col[base + (t + u) * SL + l] = v[u];
  }
}

// ---------------------------------------------------------------- matching
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): mix of x + golden gamma.
__device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ inline uint64_t node_rank(int64_t v, uint64_t salt) {
  return splitmix64((((uint64_t)v) << 32 | (uint64_t)v) ^ salt);
}

__global__ void k_node_rank(int64_t n, uint64_t salt, uint64_t* rank) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rank[i] = node_rank(i, salt);
}

struct EdgeKey {
  uint64_t rank;  // visiting rank of the first-visited endpoint
  int32_t first;
  int32_t w;
  int32_t lo, hi;
};

__device__ inline uint64_t edge_hash(int32_t lo, int32_t hi, uint64_t salt) {
  return splitmix64(((((uint64_t)lo) << 32) | (uint64_t)hi) ^ salt);
}

// true when a precedes b in the matching order: earlier first-visited
// endpoint, then larger weight, then larger edge hash, then smaller (lo, hi);
// the hashes are only evaluated when everything before them ties
__device__ inline bool key_before(const EdgeKey& a, const EdgeKey& b, uint64_t salt) {
  if (a.rank != b.rank) return a.rank < b.rank;
  if (a.first != b.first) return a.first < b.first;
  if (a.w != b.w) return a.w > b.w;
  const uint64_t ha = edge_hash(a.lo, a.hi, salt), hb = edge_hash(b.lo, b.hi, salt);
  if (ha != hb) return ha > hb;
  if (a.lo != b.lo) return a.lo < b.lo;
  return a.hi < b.hi;
}

// key_before with each key's edge hash evaluated at most once (ha, hb: the
// hashes once hav, hbv are set).  The grid pass uses it: its weights are all
// equal, so most comparisons of a walker's edges reach the hashes.
__device__ inline bool key_before_h(const EdgeKey& a, uint64_t& ha, bool& hav, const EdgeKey& b, uint64_t& hb,
                                    bool& hbv, uint64_t salt) {
  if (a.rank != b.rank) return a.rank < b.rank;
  if (a.first != b.first) return a.first < b.first;
  if (a.w != b.w) return a.w > b.w;
  if (!hav) {
    ha = edge_hash(a.lo, a.hi, salt);
    hav = true;
  }
  if (!hbv) {
    hb = edge_hash(b.lo, b.hi, salt);
    hbv = true;
  }
  if (ha != hb) return ha > hb;
  if (a.lo != b.lo) return a.lo < b.lo;
  return a.hi < b.hi;
}

// The earliest candidate edge of node i (largest weight mxi) over the row
// slots [kb, k1) that lane sub of its G lanes visits (every G-th slot); best
// and bk are updated in place.  Neighbours are examined U at a time so
// that their loads are in flight together.
template <int G, int U = 4>
__device__ inline void row_best(int64_t i, int sub, int32_t mxi, int32_t kb, int32_t k1,
                                const int32_t* __restrict__ gci, const int32_t* __restrict__ gw,
                                const NodeSt* __restrict__ ns, uint64_t salt, int32_t bnum, int32_t bden,
                                int32_t& best, EdgeKey& bk) {
  const uint64_t ri = node_rank(i, salt);
  for (int32_t k0 = kb + sub; k0 < k1; k0 += U * G) {
    int32_t jj[U], ww[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = k0 + u * G < k1;
      jj[u] = ok ? gci[k0 + u * G] : -1;
      ww[u] = ok ? gw[k0 + u * G] : 0;
    }
    // the candidates' records, all U loads issued together (a padding
    // slot reads node i's own record and is masked)
    NodeSt sj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) sj[u] = ns[jj[u] >= 0 ? jj[u] : i];
    bool fr[U];
    uint64_t rr[U];
    int32_t mj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      fr[u] = jj[u] >= 0 && sj[u].mate < 0;
      rr[u] = node_rank(jj[u] >= 0 ? jj[u] : i, salt);
      mj[u] = sj[u].mx;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!fr[u]) continue;
      const int32_t j = jj[u], w = ww[u];
      const uint64_t rj = rr[u];
      const bool ifirst = ri != rj ? ri < rj : i < j;
      const int32_t mf = ifirst ? mxi : mj[u];
      if ((int64_t)bden * w < (int64_t)bnum * mf) continue;
      EdgeKey e;
      e.rank = ifirst ? ri : rj;
      e.first = ifirst ? (int32_t)i : j;
      e.w = w;
      e.lo = (int32_t)min((int64_t)j, i);
      e.hi = (int32_t)max((int64_t)j, i);
      if (best < 0 || key_before(e, bk, salt)) {
        bk = e;
        best = j;
      }
    }
  }
}

// One handshake round: every free node proposes its earliest candidate edge
// (strong for its first-visited endpoint, other end free).  G lanes share a
// node (coarse levels: their rows are long and the dependent loads of a row
// walk are the round's latency); each lane walks every G-th slot, then a
// butterfly keeps the earliest key.  The order is strict, so the result does
// not depend on G.
// The proposal of node i (lanes sub = 0..G-1 of its group; i >= n: none) in
// one handshake round; returns whether it proposed (on lane 0).
template <int G>
__device__ inline bool propose_node(int64_t i, int sub, int64_t n, const int32_t* __restrict__ grp,
                                    const int32_t* __restrict__ gci, const int32_t* __restrict__ gw,
                                    int32_t* __restrict__ mate, const NodeSt* __restrict__ ns, uint64_t salt,
                                    int32_t bnum, int32_t bden, int32_t* __restrict__ prop) {
  int32_t best = -1;
  EdgeKey bk{};
  // matched nodes (most of them after the first rounds) read only their mate
  // and proposal; a free node then reads its record.  A free node that finds
  // no candidate is marked dead (mate -2): candidate edges are fixed and free
  // nodes only get matched, so it will not find one later, and its row is
  // not walked again.  Every reader of mate takes a negative value as
  // unmatched; no neighbour can select a dead node (that edge would be a
  // free candidate of the dead node).
  //
  // A free node whose proposal of the last round is still free proposes it
  // again without walking its row: the free nodes only shrink, so the
  // earliest candidate of a set stays the earliest of any subset holding it.
  // Only the nodes whose proposal got matched (and the first round, prop
  // -1) walk their rows.  The decision is the same on the G lanes of a node.
  //
  // The loads go out in three waves: mate and the last proposal; then, for a
  // free node, the proposal's mate together with the node's record and row
  // bounds (read for nothing when it proposes again); then the row.
  const int32_t mi = i < n ? mate[i] : 0;
  const int32_t pj = i < n ? prop[i] : -1;
  bool walk = false;
  NodeSt si{};
  int32_t kb = 0, k1 = 0;
  if (i < n && mi == -1) {
    si = ns[i];
    kb = grp[i];
    k1 = grp[i + 1];
    if (pj >= 0 && mate[pj] < 0)
      best = pj;
    else
      walk = true;
  }
  if (walk) row_best<G>(i, sub, si.mx, kb, k1, gci, gw, ns, salt, bnum, bden, best, bk);
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    if (!walk) break;  // uniform over the node's lanes
    EdgeKey o;
    const int32_t ob = __shfl_xor(best, off, G);
    o.rank = __shfl_xor(bk.rank, off, G);
    o.first = __shfl_xor(bk.first, off, G);
    o.w = __shfl_xor(bk.w, off, G);
    o.lo = __shfl_xor(bk.lo, off, G);
    o.hi = __shfl_xor(bk.hi, off, G);
    if (ob >= 0 && (best < 0 || key_before(o, bk, salt))) {
      bk = o;
      best = ob;
    }
  }
  // prop changes only where a node walks (a node proposing again finds its
  // proposal there) and once where a node got matched: its proposal, which
  // names its mate, is cleared so that the accept pass can skip it
  const bool proposed = i < n && sub == 0 && best >= 0;
  if (walk && sub == 0) {
    prop[i] = best;
    if (best < 0) mate[i] = -2;
  }
  if (i < n && sub == 0 && mi >= 0 && pj >= 0) prop[i] = -1;
  return proposed;
}

template <int G>
__global__ void __launch_bounds__(TPB) k_propose(int64_t n, const int32_t* __restrict__ grp,
                                                 const int32_t* __restrict__ gci, const int32_t* __restrict__ gw,
                                                 int32_t* __restrict__ mate, const NodeSt* __restrict__ ns,
                                                 uint64_t salt, int32_t bnum, int32_t bden,
                                                 int32_t* __restrict__ prop, int32_t* count) {
  // XCD-contiguous node ranges: the records of a row's neighbours are then
  // mostly in the XCD's own L2
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t i = t / G;
  const int sub = (int)(t - i * G);
  const bool proposed = propose_node<G>(i, sub, n, grp, gci, gw, mate, ns, salt, bnum, bden, prop);
  // "some node proposed": set once; most wavefronts see the flag already set
  // and skip the atomic (same-address atomics from every wavefront serialize)
  const unsigned long long ballot = __ballot(proposed);
  if ((threadIdx.x & 63) == 0 && ballot && __atomic_load_n(count, __ATOMIC_RELAXED) == 0) atomicOr(count, 1);
}


// The round on the levels whose rows are short (8-30 entries).  A wavefront
// pays for a row walk when any of its lanes walks, which most do for ten
// rounds while a fifth to a third of the nodes walk; so, as in
// k_propose_grid, the workgroup lists its walkers in LDS (with the record
// and row bounds loaded beside the last proposal's mate) and then walks
// them PK_G lanes per walker, PK_U slots per lane at a time, the lanes'
// keys merged by a butterfly.  A walker's lanes read consecutive slots of
// its row, so a row load of a wavefront touches a few cache lines per
// walker instead of one line per lane (one lane per walker took 1.7 ms more
// per step at 256^3: the loads of 64 different rows per instruction are what
// such a round waits on).  The decisions are those of propose_node.
constexpr int PK_G = 4, PK_U = 4;
__global__ void __launch_bounds__(TPB) k_propose_packed(int64_t n, const int32_t* __restrict__ grp,
                                                        const int32_t* __restrict__ gci,
                                                        const int32_t* __restrict__ gw, int32_t* __restrict__ mate,
                                                        const NodeSt* __restrict__ ns, uint64_t salt, int32_t bnum,
                                                        int32_t bden, int32_t* __restrict__ prop, int32_t* count) {
  __shared__ int4 s_walk[TPB];  // node, largest weight, row start, row end
  __shared__ int s_nw;
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  if (threadIdx.x == 0) s_nw = 0;
  __syncthreads();
  bool proposed = false;
  if (i < n) {
    const int32_t mi = mate[i], pj = prop[i];
    if (mi >= 0 && pj >= 0) prop[i] = -1;  // matched in the last round
    if (mi == -1) {
      const NodeSt si = ns[i];
      const int32_t kb = grp[i], k1 = grp[i + 1];
      if (pj >= 0 && mate[pj] < 0)
        proposed = true;
      else
        s_walk[atomicAdd(&s_nw, 1)] = make_int4((int32_t)i, si.mx, kb, k1);
    }
  }
  __syncthreads();
  const int nw = s_nw;
  const int sub = (int)threadIdx.x % PK_G;
  // the same trip count on every thread: the butterfly's shuffles run on all
  // lanes, a lane group without a walker holds no candidate
  for (int t0 = 0; t0 < nw; t0 += TPB / PK_G) {
    const int t = t0 + (int)threadIdx.x / PK_G;
    const bool act = t < nw;  // the same on a walker's lanes
    const int4 wk = act ? s_walk[t] : make_int4(0, 0, 0, 0);
    int32_t best = -1;
    EdgeKey bk{};
    if (act) row_best<PK_G, PK_U>(wk.x, sub, wk.y, wk.z, wk.w, gci, gw, ns, salt, bnum, bden, best, bk);
#pragma unroll
    for (int off = 1; off < PK_G; off <<= 1) {
      EdgeKey o;
      const int32_t ob = __shfl_xor(best, off, PK_G);
      o.rank = __shfl_xor(bk.rank, off, PK_G);
      o.first = __shfl_xor(bk.first, off, PK_G);
      o.w = __shfl_xor(bk.w, off, PK_G);
      o.lo = __shfl_xor(bk.lo, off, PK_G);
      o.hi = __shfl_xor(bk.hi, off, PK_G);
      if (ob >= 0 && (best < 0 || key_before(o, bk, salt))) {
        bk = o;
        best = ob;
      }
    }
    if (act && sub == 0) {
      prop[wk.x] = best;
      if (best < 0) mate[wk.x] = -2;
      proposed = proposed || best >= 0;
    }
  }
  const unsigned long long ballot = __ballot(proposed);
  if ((threadIdx.x & 63) == 0 && ballot && __atomic_load_n(count, __ATOMIC_RELAXED) == 0) atomicOr(count, 1);
}

// The grid pass and the accept pass give a thread RN nodes (a workgroup
// TPB x RN), their loads in flight together: the rounds wait on dependent
// loads, and more of them in flight per thread hides more of that wait
// (k_propose_packed, whose walk holds more registers, measured best at one
// node per thread).
constexpr int RN = 4;

// The same round on the grid graph itself (the first pass of the grid level):
// its rows are the grid neighbours in ascending order, every weight is 1, so
// every node's largest weight is 1 (a grid of one node has no row), and a
// node's visiting rank is node_rank of its index.  A walk then reads only
// the neighbours' 4-byte mates: neighbours and ranks are computed, not
// loaded.  mate stands in for the record's copy of it: the two differ only
// where a dead node (no candidate) holds -2, and both are negative there.
// The decisions are those of propose_node on the stored grid graph.
//
// The walk is arithmetic (the coordinates, the key comparisons) and a
// wavefront pays for it when any of its lanes walks, which most do for ten
// rounds while only a fifth to a third of the nodes walk.  So the workgroup
// first sorts its nodes out: matched and dead nodes stop, a node whose last
// proposal is still free proposes it again (prop already holds it), and the
// rest are listed in LDS and walked by the workgroup's first threads.  The
// ranks are read from rank[] (node_rank of every node, written once per
// pass): seven hashes per walk cost more than seven loads.
// Round one (first != 0) finds every node free with nothing proposed, loads
// no mates and writes both prop and mate of every node: no initialisation
// pass is needed.
__device__ inline int grid_nbrs32(unsigned nx, unsigned ny, unsigned nz, unsigned p, unsigned* nb) {
  const unsigned nxy = nx * ny;
  const unsigned k = p / nxy, r = p - k * nxy;
  const unsigned j = r / nx, i = r - j * nx;
  int c = 0;
  if (k > 0) nb[c++] = p - nxy;
  if (j > 0) nb[c++] = p - nx;
  if (i > 0) nb[c++] = p - 1;
  if (i + 1 < nx) nb[c++] = p + 1;
  if (j + 1 < ny) nb[c++] = p + nx;
  if (k + 1 < nz) nb[c++] = p + nxy;
  return c;
}

__global__ void __launch_bounds__(TPB) k_propose_grid(int nx, int ny, int nz, int32_t* __restrict__ mate,
                                                      const uint64_t* __restrict__ rank, uint64_t salt,
                                                      int32_t bnum, int32_t bden, int32_t* __restrict__ prop,
                                                      int32_t* count, int first) {
  __shared__ unsigned s_walk[TPB * RN];
  __shared__ int s_nw;
  const unsigned N = (unsigned)nx * ny * nz;
  const unsigned i0 = xcd_block(blockIdx.x, gridDim.x) * (TPB * RN) + threadIdx.x;
  if (threadIdx.x == 0) s_nw = 0;
  __syncthreads();
  bool proposed = false;
  int32_t mi[RN], pj[RN], mp[RN];
#pragma unroll
  for (int k = 0; k < RN; ++k) {
    const unsigned i = i0 + k * TPB;
    mi[k] = (i < N && !first) ? mate[i] : -1;
    pj[k] = (i < N && !first) ? prop[i] : -1;
  }
#pragma unroll
  for (int k = 0; k < RN; ++k) mp[k] = (i0 + k * TPB < N && mi[k] == -1 && pj[k] >= 0) ? mate[pj[k]] : 0;
#pragma unroll
  for (int k = 0; k < RN; ++k) {
    const unsigned i = i0 + k * TPB;
    if (i >= N) continue;
    bool walk = first != 0;
    if (!walk) {
      if (mi[k] >= 0 && pj[k] >= 0) prop[i] = -1;  // matched in the last round
      if (mi[k] == -1) {
        if (pj[k] >= 0 && mp[k] < 0)
          proposed = true;
        else
          walk = true;
      }
    }
    if (walk) s_walk[atomicAdd(&s_nw, 1)] = i;
  }
  __syncthreads();
  const int nw = s_nw;
  for (int t = threadIdx.x; t < nw; t += TPB) {
    const unsigned w = s_walk[t];
    unsigned nb[6];
    const int c = grid_nbrs32(nx, ny, nz, w, nb);
    int32_t mj[6];
    uint64_t rr[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      mj[u] = (u < c && !first) ? mate[nb[u]] : -1;
      rr[u] = rank[u < c ? nb[u] : w];
    }
    const uint64_t ri = rank[w];
    int32_t best = -1;
    EdgeKey bk{};
    uint64_t bh = 0;
    bool bhv = false;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      if (u >= c || mj[u] >= 0) continue;
      if ((int64_t)bden < (int64_t)bnum) continue;  // weight 1 against the largest weight 1
      const int32_t j = (int32_t)nb[u];
      const uint64_t rj = rr[u];
      const bool wfirst = ri != rj ? ri < rj : w < (unsigned)j;
      EdgeKey e;
      e.rank = wfirst ? ri : rj;
      e.first = wfirst ? (int32_t)w : j;
      e.w = 1;
      e.lo = min((int32_t)w, j);
      e.hi = max((int32_t)w, j);
      uint64_t eh = 0;
      bool ehv = false;
      if (best < 0 || key_before_h(e, eh, ehv, bk, bh, bhv, salt)) {
        bk = e;
        bh = eh;
        bhv = ehv;
        best = j;
      }
    }
    prop[w] = best;
    if (best < 0)
      mate[w] = -2;
    else if (first)
      mate[w] = -1;
    proposed = proposed || best >= 0;
  }
  const unsigned long long ballot = __ballot(proposed);
  if ((threadIdx.x & 63) == 0 && ballot && __atomic_load_n(count, __ATOMIC_RELAXED) == 0) atomicOr(count, 1);
}

// Every handshake round of a small level in one workgroup (MATCH_T threads,
// G lanes per node): there the launches of the rounds cost more than their
// work.  The rounds are those of k_propose / k_accept: within a round the
// passes over the nodes read no state another pass of the round changes
// (a dead mark only turns -1 into -2).  A round with a proposal matches at
// least the earliest free candidate edge (both of its ends propose it), so
// at most n/2 + 1 rounds run; past n rounds the flag bit is raised.
constexpr int MATCH_T = 1024;
template <int G>
__global__ void __launch_bounds__(MATCH_T) k_match_small(int64_t n, const int32_t* __restrict__ grp,
                                                         const int32_t* __restrict__ gci,
                                                         const int32_t* __restrict__ gw, int32_t* __restrict__ mate,
                                                         NodeSt* __restrict__ ns, uint64_t salt, int32_t bnum,
                                                         int32_t bden, int32_t* __restrict__ prop, int32_t* flag,
                                                         int32_t bit) {
  __shared__ int32_t s_any;
  const int tid = (int)threadIdx.x;
  const int sub = tid % G;
  for (int64_t r = 0;; ++r) {
    if (tid == 0) s_any = 0;
    __syncthreads();
    bool any = false;
    for (int64_t i0 = 0; i0 < n; i0 += MATCH_T / G) {
      const bool pr = propose_node<G>(i0 + tid / G, sub, n, grp, gci, gw, mate, ns, salt, bnum, bden, prop);
      any = any || pr;
    }
    if (any) s_any = 1;
    __syncthreads();  // the round's proposals are visible to the workgroup
    if (s_any == 0) break;
    if (r > n) {
      if (tid == 0) atomicOr(flag, bit);
      break;
    }
    for (int64_t i = tid; i < n; i += MATCH_T) {
      if (mate[i] != -1) continue;
      const int32_t pi = prop[i];
      if (pi >= 0 && prop[pi] == (int32_t)i) {
        mate[i] = pi;
        ns[i].mate = pi;
      }
    }
    __syncthreads();
  }
}

// Only prop is read: dead nodes hold -1 there, and the proposal round after
// a match clears the matched nodes' proposals.  ns is null on the grid pass,
// whose proposal rounds read no records.
__global__ void k_accept(int64_t n, const int32_t* prop, int32_t* mate, NodeSt* ns) {
  const int64_t i0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (TPB * RN) + threadIdx.x;
  int32_t p[RN], q[RN];
#pragma unroll
  for (int k = 0; k < RN; ++k) p[k] = i0 + k * TPB < n ? prop[i0 + k * TPB] : -1;
#pragma unroll
  for (int k = 0; k < RN; ++k) q[k] = p[k] >= 0 ? prop[p[k]] : -1;
#pragma unroll
  for (int k = 0; k < RN; ++k) {
    const int64_t i = i0 + k * TPB;
    if (p[k] >= 0 && q[k] == (int32_t)i) {
      mate[i] = p[k];
      if (ns) ns[i].mate = p[k];
    }
  }
}

__global__ void k_match_init(int64_t n, const int32_t* grp, const int32_t* gw, uint64_t salt, NodeSt* ns,
                             int32_t* mate, int32_t* prop) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t m = 0;
  for (int32_t k = grp[i]; k < grp[i + 1]; ++k) m = max(m, gw[k]);
  NodeSt r;
  r.mx = m;
  r.mate = -1;
  ns[i] = r;
  mate[i] = -1;
  prop[i] = -1;
}

__global__ void k_leader_flag(int64_t n, const int32_t* mate, int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t m = mate[i];
  flag[i] = (m < 0 || (int32_t)i < m) ? 1 : 0;
}

// Aggregates are numbered by their smallest member (ascending scan order).
__global__ void k_assign(int64_t n, const int32_t* mate, const int32_t* id, int32_t* agg,
                         int32_t* lead) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t m = mate[i];
  const bool leader = m < 0 || (int32_t)i < m;
  const int32_t L = leader ? (int32_t)i : m;
  const int32_t a = id[L];
  agg[i] = a;
  if (leader) lead[a] = (int32_t)i;
}

__global__ void k_cg_count(int64_t nc, const int32_t* lead, const int32_t* mate, const int32_t* grp,
                           int32_t* cnt) {
  int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t a = lead[I], b = mate[a];
  int32_t c = grp[a + 1] - grp[a];
  if (b >= 0) c += grp[b + 1] - grp[b];
  cnt[I] = c;
}

// Coarse graph row I: (agg(j), w) over the rows of the (one or two) members,
// sorted by coarse column, duplicates summed, the diagonal dropped.
//
// G lanes take a row: they read the members' rows with contiguous loads and
// insert the candidates into a hash table of T slots in LDS (open
// addressing; equal columns meet in one slot, whose integer weight sums
// them, so the order of the insertions does not matter).  The table's
// entries are compacted and each is written at its rank among them, which
// sorts the row.  A row has 10-30 candidates and 8-27 entries on the grid
// hierarchies; a row of more than T candidates (none there) is counted and
// then written in order by its first lane from the rows themselves.
//
// A workgroup's R rows (a tile) are written end to end from the start of
// the tile's room for candidates (cptr of its first row): nrp[I] receives
// row I's offset in the tile and ttot[tile] the tile's length.  After an
// exclusive scan of ttot, k_cg_copy moves each tile to its place with
// contiguous loads and stores and turns nrp into the row pointers.
// The entries of row I in ascending column order, for a row of more than T
// candidates: with emit, written at out/ow; returns their number.
__device__ int32_t cg_row_select(int32_t I, int32_t ka, int32_t na, int32_t kb, int32_t nb,
                                 const int32_t* __restrict__ gci, const int32_t* __restrict__ gw,
                                 const int32_t* __restrict__ agg, bool emit, int32_t* out, int32_t* ow,
                                 int32_t* mx) {
  const int32_t c = na + nb;
  auto col = [&](int32_t e) { return agg[gci[e < na ? ka + e : kb + (e - na)]]; };
  auto wgt = [&](int32_t e) { return gw[e < na ? ka + e : kb + (e - na)]; };
  int32_t u = 0, last = -1;
  for (;;) {
    int32_t m = 0x7fffffff, w = 0;
    for (int32_t e = 0; e < c; ++e) {
      const int32_t J = col(e);
      if (J == I || J <= last) continue;
      if (J < m) {
        m = J;
        w = wgt(e);
      } else if (J == m) {
        w += wgt(e);
      }
    }
    if (m == 0x7fffffff) break;
    if (emit) {
      out[u] = m;
      ow[u] = w;
    }
    *mx = max(*mx, w);
    last = m;
    ++u;
  }
  return u;
}

// The t-th grid neighbour of node v, in the order of grid_nbrs32.
__device__ inline unsigned grid_nbr_at(unsigned nx, unsigned ny, unsigned nz, unsigned v, int t) {
  unsigned nb[6];
  const int c = grid_nbrs32(nx, ny, nz, v, nb);
  unsigned r = nb[0];
#pragma unroll
  for (int u = 1; u < 6; ++u)
    if (u < c && u == t) r = nb[u];
  return r;
}

// GRID: the first pass of the grid level, whose graph is the grid graph
// (weights 1): the members' neighbours are computed from the grid sizes
// instead of read from the stored rows.
template <int G, int T, bool GRID>
__global__ void __launch_bounds__(TPB) k_cg_fill(int64_t nc, const int32_t* __restrict__ lead,
                                                 const int32_t* __restrict__ mate, const int32_t* __restrict__ grp,
                                                 const int32_t* __restrict__ gci, const int32_t* __restrict__ gw,
                                                 const int32_t* __restrict__ agg, const int32_t* __restrict__ cptr,
                                                 int32_t* cj, int32_t* cw, int32_t* nrp, int32_t* ttot, int nx,
                                                 int ny, int nz, NodeSt* nsn, int32_t* maten, int32_t* propn) {
  static_assert(TPB % G == 0 && T % G == 0 && (T & (T - 1)) == 0, "table shape");
  constexpr int R = TPB / G;   // rows per workgroup
  constexpr int PS = T / G;    // table slots per lane
  constexpr int TB = __builtin_ctz(T);
  __shared__ int32_t s_key[R * T];
  __shared__ int32_t s_wt[R * T];
  __shared__ int2 s_ent[R * T];
  __shared__ int32_t s_len[R], s_off[R];
  static_assert(R <= 64, "one wavefront scans the tile's rows");
  const int tid = (int)threadIdx.x;
  const int r = tid / G, lane = tid % G;
  const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t I = tile * R + r;
  int32_t* key = s_key + r * T;
  int32_t* wt = s_wt + r * T;
  int2* ent = s_ent + r * T;
#pragma unroll
  for (int q = 0; q < PS; ++q) {
    key[lane * PS + q] = -1;
    wt[lane * PS + q] = 0;
  }
  int32_t a = 0, b = -1, ka = 0, na = 0, kb = 0, nb = 0;
  if (I < nc) {
    a = lead[I];
    b = mate[a];
    ka = grp[a];
    na = grp[a + 1] - ka;
    if (b >= 0) {
      kb = grp[b];
      nb = grp[b + 1] - kb;
    }
  }
  const int32_t c = na + nb;
  const bool small = I < nc && c <= T;  // the same on the row's lanes
  __syncthreads();
  if (small) {
    for (int32_t e = lane; e < c; e += G) {
      int32_t J, w;
      if constexpr (GRID) {
        J = agg[grid_nbr_at(nx, ny, nz, e < na ? a : b, e < na ? e : e - na)];
        w = 1;
      } else {
        const int32_t k = e < na ? ka + e : kb + (e - na);
        J = agg[gci[k]];
        w = gw[k];
      }
      if (J == (int32_t)I) continue;
      unsigned h = ((unsigned)J * 0x9E3779B1u) >> (32 - TB);
      // at most c <= T distinct columns: a free slot or J's own is found
      for (;;) {
        const int32_t old = atomicCAS(&key[h], -1, J);
        if (old == -1 || old == J) {
          atomicAdd(&wt[h], w);
          break;
        }
        h = (h + 1) & (T - 1);
      }
    }
  }
  __syncthreads();
  // compact the occupied slots (each lane holds PS consecutive ones)
  int32_t kk[PS], ww[PS];
  int cl = 0;
#pragma unroll
  for (int q = 0; q < PS; ++q) {
    kk[q] = key[lane * PS + q];
    ww[q] = wt[lane * PS + q];
    cl += kk[q] != -1;
  }
  int incl = cl;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const int v = __shfl_up(incl, off, G);
    if (lane >= off) incl += v;
  }
  int32_t u = __shfl(incl, G - 1, G);
  int pos = incl - cl;
#pragma unroll
  for (int q = 0; q < PS; ++q)
    if (kk[q] != -1) ent[pos++] = make_int2(kk[q], ww[q]);
  int32_t mx = 0;  // the row's largest weight
  if (!small) {
    if (I < nc && lane == 0) u = cg_row_select((int32_t)I, ka, na, kb, nb, gci, gw, agg, false, nullptr, nullptr, &mx);
    u = __shfl(u, 0, G);
  }
  if (I >= nc) u = 0;
  if (lane == 0) s_len[r] = u;
  __syncthreads();
  // the rows' offsets in the tile, and the tile's length
  if (tid < 64) {
    const int32_t v = tid < R ? s_len[tid] : 0;
    int32_t sc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t w = __shfl_up(sc, off, 64);
      if (tid >= off) sc += w;
    }
    if (tid < R) s_off[tid] = sc - v;
    if (tid == 63) ttot[tile] = sc;
  }
  __syncthreads();
  if (I < nc) {
    const int32_t o = cptr[tile * R] + s_off[r];
    if (small) {
      // columns are distinct: an entry's rank is its place in the sorted row
      for (int t = lane; t < u; t += G) {
        const int2 v = ent[t];
        int rk = 0;
        for (int x = 0; x < u; ++x) rk += ent[x].x < v.x;
        cj[o + rk] = v.x;
        cw[o + rk] = v.y;
        mx = max(mx, v.y);
      }
    } else if (lane == 0) {
      (void)cg_row_select((int32_t)I, ka, na, kb, nb, gci, gw, agg, true, cj + o, cw + o, &mx);
    }
    if (lane == 0) nrp[I] = s_off[r];
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) mx = max(mx, __shfl_xor(mx, off, G));
  // the next pass's matching state of node I (what k_match_init writes)
  if (nsn && I < nc && lane == 0) {
    nsn[I] = NodeSt{mx, -1};
    maten[I] = -1;
    propn[I] = -1;
  }
}

// Tile t's rows moved from cj/cw[cptr[t R]...] to nci/nw[tbase[t]...] (tbase:
// the exclusive scan of the tile lengths, the total at tbase[nt]); nrp[I]
// turns from the row's offset in its tile into the row pointer.
__global__ void k_cg_copy(int64_t nc, int R, const int32_t* __restrict__ cptr, const int32_t* __restrict__ cj,
                          const int32_t* __restrict__ cw, const int32_t* __restrict__ tbase, int32_t* nrp,
                          int32_t* nci, int32_t* nw) {
  const int64_t t = blockIdx.x;
  const int64_t I0 = t * R;
  const int32_t src = cptr[I0], dst = tbase[t], len = tbase[t + 1] - dst;
  for (int32_t q = (int32_t)threadIdx.x; q < len; q += (int32_t)blockDim.x) {
    nci[dst + q] = cj[src + q];
    nw[dst + q] = cw[src + q];
  }
  const int64_t I = I0 + threadIdx.x;
  if ((int)threadIdx.x < R && I < nc) nrp[I] += dst;
  if (threadIdx.x == 0 && I0 + R >= nc) nrp[nc] = dst + len;
}

// Members of the composite aggregates, from the passes' own records: an
// aggregate of pass p is its leader (a node, or an aggregate of pass p - 1)
// and the leader's mate when it has one, so the fine nodes of a composite
// aggregate I are found by expanding I through the passes, last to first.
// The 2^NP slots of the expansion (absent members -1) are sorted, so the
// members come out ascending; the fill also writes the composite map acc.
struct PassMaps {
  const int32_t* lead[MAX_PASS];
  const int32_t* mate[MAX_PASS];
};

template <int NP>
__device__ inline int expand_members(int32_t I, const PassMaps& pm, int32_t (&m)[1 << NP]) {
  m[0] = I;
#pragma unroll
  for (int q = NP - 1; q >= 0; --q) {
    const int c = 1 << (NP - 1 - q);  // slots filled before pass q's expansion
#pragma unroll
    for (int x = (1 << NP) / 2 - 1; x >= 0; --x) {
      if (x >= c) continue;
      const int32_t A = m[x];
      int32_t L = -1, M = -1;
      if (A >= 0) {
        L = pm.lead[q][A];
        const int32_t mm = pm.mate[q][L];
        M = mm >= 0 ? mm : -1;
      }
      m[2 * x] = L;
      m[2 * x + 1] = M;
    }
  }
  int cnt = 0;
#pragma unroll
  for (int x = 0; x < (1 << NP); ++x) {
    cnt += m[x] >= 0;
    if (m[x] < 0) m[x] = 0x7fffffff;
  }
#pragma unroll
  for (int k = 2; k <= (1 << NP); k <<= 1) {
#pragma unroll
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
#pragma unroll
      for (int e = 0; e < (1 << NP); ++e) {
        const int f = e ^ jj;
        if (f > e) {
          const bool up = (e & k) == 0;
          const int32_t a = m[e], b = m[f];
          const bool sw = up ? a > b : a < b;
          m[e] = sw ? b : a;
          m[f] = sw ? a : b;
        }
      }
    }
  }
  return cnt;
}

template <int NP>
__global__ void k_member_count(int64_t nc, PassMaps pm, int32_t* cnt) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int32_t m[1 << NP];
  cnt[I] = expand_members<NP>((int32_t)I, pm, m);
}

template <int NP>
__global__ void k_member_fill(int64_t nc, PassMaps pm, const int32_t* mptr, int32_t* mem, int32_t* acc) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int32_t m[1 << NP];
  const int c = expand_members<NP>((int32_t)I, pm, m);
  const int32_t o = mptr[I];
#pragma unroll
  for (int x = 0; x < (1 << NP); ++x) {
    if (x < c) {
      mem[o + x] = m[x];
      acc[m[x]] = (int32_t)I;
    }
  }
}

// ---------------------------------------------------------------- colouring
// Colour classes for the multicolour Gauss-Seidel smoother (Sec. 3).
// Level 0: parity of i + j + k (the grid graph is bipartite).
__global__ void k_parity_colour(int nx, int ny, int nz, int32_t* col) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (p >= N) return;
  const int64_t i = p % nx, j = (p / nx) % ny, k = p / ((int64_t)nx * ny);
  col[p] = (int32_t)((i + j + k) & 1);
}

// One Jones-Plassmann round r on a coarse level: a node whose earlier
// neighbours (smaller (rank, id)) were all coloured in rounds before r takes
// the smallest colour none of them has.  That is the greedy colouring in
// ascending (rank, id) order: when a node is coloured, exactly its earlier
// neighbours are.  cround[v] = round that coloured v (INT32_MAX: not yet);
// a node coloured in this same round counts as not coloured, so the result
// and the number of rounds do not depend on the order of the threads.
// Colours >= 128 are not represented: such a node gets 128 (reported).
__global__ void k_jp_round(int64_t n, const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                           const uint64_t* __restrict__ rank, int32_t r, int32_t* cround, int32_t* col,
                           int32_t* pending) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool waiting = false;
  if (i < n && cround[i] == INT32_MAX) {
    const uint64_t ri = rank[i];
    uint64_t used0 = 0, used1 = 0;
    bool ready = true;
    for (int32_t k = grp[i]; k < grp[i + 1]; ++k) {
      const int32_t j = gci[k];
      const uint64_t rj = rank[j];
      if (!(rj < ri || (rj == ri && j < i))) continue;  // later neighbour
      if (cround[j] >= r) {
        ready = false;
        break;
      }
      const int32_t cj = col[j];
      if (cj < 64)
        used0 |= 1ull << cj;
      else if (cj < 128)
        used1 |= 1ull << (cj - 64);
    }
    if (ready) {
      int32_t c = used0 != ~0ull ? __builtin_ctzll(~used0) : (used1 != ~0ull ? 64 + __builtin_ctzll(~used1) : 128);
      col[i] = c;
      cround[i] = r;
    } else {
      waiting = true;
    }
  }
  const unsigned long long ballot = __ballot(waiting);
  if ((threadIdx.x & 63) == 0 && ballot && __atomic_load_n(pending, __ATOMIC_RELAXED) == 0) atomicOr(pending, 1);
}

// *ncol = 1 + largest colour (one atomic per wavefront)
__global__ void k_colour_max(int64_t n, const int32_t* col, int32_t* ncol) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t c = i < n ? col[i] + 1 : 0;
  for (int off = 32; off > 0; off >>= 1) c = max(c, __shfl_down(c, off, 64));
  if ((threadIdx.x & 63) == 0 && c > 0) atomicMax(ncol, c);
}

// Counting sort of the nodes by colour, stable: hist[c * nb + b] = nodes of
// colour c in block b (256 nodes per block); after an exclusive scan of hist,
// a node's place is hist[c * nb + b] + (earlier nodes of its block with colour c).
__global__ void k_colour_hist(int64_t n, const int32_t* col, int32_t ncol, int64_t nb, int32_t* hist) {
  __shared__ int32_t h[128];
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) h[c] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && col[i] >= 0 && col[i] < ncol) atomicAdd(&h[col[i]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) hist[(int64_t)c * nb + blockIdx.x] = h[c];
}

__global__ void k_colour_place(int64_t n, const int32_t* col, int32_t ncol, int64_t nb, const int32_t* hist,
                               int32_t* perm) {
  __shared__ int32_t cs[TPB];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t c = i < n ? col[i] : -1;
  cs[threadIdx.x] = c;
  __syncthreads();
  if (i >= n || c < 0 || c >= ncol) return;
  int32_t before = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) before += cs[t] == c;
  perm[hist[(int64_t)c * nb + blockIdx.x] + before] = (int32_t)i;
}

// Values of one colour class: row k of the class is level row rows[k]; its
// slot t holds the level's slot t of that row (same column).  The inverse
// diagonal block follows when dinv != NULL.
template <typename T>
__global__ void k_cls_gather(int64_t n, const int32_t* __restrict__ rows, const int32_t* __restrict__ sl,
                             const int32_t* __restrict__ col, const T* __restrict__ val, const T* __restrict__ dinv,
                             const int32_t* __restrict__ csl, T* __restrict__ cval, T* __restrict__ cdinv,
                             const T* __restrict__ fk) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t i = rows[k];
  const int64_t s = i / SL, l = i - s * SL;
  const int64_t cs = k / SL, cl = k - cs * SL;
  const int64_t src = 9 * (int64_t)sl[s], dst = 9 * (int64_t)csl[cs];
  const int w = (csl[cs + 1] - csl[cs]) / SL;
  const int wsrc = (sl[s + 1] - sl[s]) / SL;
  for (int t = 0; t < w; ++t) {
    if (fk) {  // factored grid level: identity on the diagonal, fk_i elsewhere
      const int32_t j = t < wsrc ? col[sl[s] + (int64_t)t * SL + l] : -1;
      for (int e = 0; e < 9; ++e)
        cval[dst + (int64_t)SL * (9 * t + e) + cl] =
            j < 0 ? T(0) : (j == i ? T((e == 0 || e == 4 || e == 8) ? 1 : 0) : fk[s * 9 * SL + e * SL + l]);
      continue;
    }
    for (int e = 0; e < 9; ++e)
      cval[dst + (int64_t)SL * (9 * t + e) + cl] = t < wsrc ? val[src + (int64_t)SL * (9 * t + e) + l] : T(0);
  }
  if (dinv)
    for (int e = 0; e < 9; ++e) cdinv[cs * 9 * SL + e * SL + cl] = dinv[s * 9 * SL + e * SL + l];
}

// One thread per node.  A_pq = dt L_pq M_p (+ I on the diagonal) in FP64;
// level-0 block D_p^{-1} A_pq with the diagonal stored as exactly I when
// left scaling is on; D_p^{-1} kept for the preconditioner input; b and the
// initial guess written alongside.
template <typename T>
__global__ void k_assemble(int nx, int ny, int nz, double inv_h2, const double* __restrict__ prm,
                           int left_scale, int x0_is_mn, const int32_t* __restrict__ sl_ptr,
                           const int32_t* __restrict__ col, double* __restrict__ Aval,
                           T* __restrict__ Lval, double* __restrict__ dinv0, T* __restrict__ ldinv,
                           double* __restrict__ b, double* __restrict__ u, int32_t* flag,
                           double* __restrict__ Mh, T* __restrict__ K, T* __restrict__ Knm,
                           double* __restrict__ mt_out, int fact) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (p >= N) return;
  const double alpha = prm[0], dt = prm[1];
  // the step's inputs, by address (the caller's buffers): m^n, m^{n-1} or
  // null, F or null
  const double* __restrict__ mn = (const double*)(uintptr_t)__double_as_longlong(prm[8]);
  const double* __restrict__ mprev = (const double*)(uintptr_t)__double_as_longlong(prm[9]);
  const double* __restrict__ F = (const double*)(uintptr_t)__double_as_longlong(prm[10]);
  // frozen field: m^n (BDF1) or 2 m^n - m^{n-1} (BDF2, mprev != NULL)
  double mt[3], bb[3];
  bool fin = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double a = mn[3 * p + c];
    fin = fin && isfinite(a);
    if (mprev) {
      const double q = mprev[3 * p + c];
      fin = fin && isfinite(q);
      mt[c] = 2.0 * a - q;
      bb[c] = (4.0 * a - q) / 3.0;
    } else {
      mt[c] = a;
      bb[c] = a;
    }
  }
  if (!fin) atomicOr(flag, 1);
  if (mt_out) {
#pragma unroll
    for (int c = 0; c < 3; ++c) mt_out[3 * p + c] = mt[c];
  }
  const double m1 = mt[0], m2 = mt[1], m3 = mt[2];
  int64_t nb[6];
  const int deg = grid_nbrs(nx, ny, nz, p, nb);
  double M[9];
  block_M(m1, m2, m3, alpha, M);
  const double s_off = dt * inv_h2;
  const double s_diag = dt * (-(double)deg * inv_h2);
  double D[9], Di[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double v = s_diag * M[e];
    if (e == 0 || e == 4 || e == 8) v = 1.0 + v;
    D[e] = v;
  }
  inv3(D, Di);
  const int64_t s = p / SL;
  const int l = (int)(p - s * SL);
  const int64_t cb = sl_ptr[s];
  const int w = fact ? 0 : (int)((sl_ptr[s + 1] - cb) / SL);
  if (fact) {
    // factored form: the off-diagonal block of the row and its scaled form,
    // the same values the sliced-ELL slots would hold
    double blk[9], sb[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) blk[e] = s_off * M[e];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        sb[3 * r + q] = (Di[3 * r] * blk[q] + Di[3 * r + 1] * blk[3 + q]) + Di[3 * r + 2] * blk[6 + q];
    const int64_t fb = s * 9 * SL + l;
    // (the sliced copies only where a reader needs them: the solve
    // recomputes the blocks from the frozen field)
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      if (Mh) Mh[fb + e * SL] = blk[e];
      if (K) K[fb + e * SL] = (T)sb[e];
      if (Knm) Knm[9 * p + e] = (T)sb[e];  // node-major copy for the Galerkin product
    }
  }
  for (int t = 0; t < w; ++t) {
    const int32_t c = col[cb + (int64_t)t * SL + l];
    if (c < 0) break;
    double blk[9], sb[9];
    if (c == p) {
#pragma unroll
      for (int e = 0; e < 9; ++e) blk[e] = D[e];
      if (left_scale) {
#pragma unroll
        for (int e = 0; e < 9; ++e) sb[e] = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
      } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) sb[e] = D[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) blk[e] = s_off * M[e];
      if (left_scale) {
        // D^{-1} A_pq, each entry summed over k = 0, 1, 2 in order
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            sb[3 * r + q] = (Di[3 * r] * blk[q] + Di[3 * r + 1] * blk[3 + q]) + Di[3 * r + 2] * blk[6 + q];
      } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) sb[e] = blk[e];
      }
    }
    const int64_t vb = cb * 9 + (int64_t)t * 9 * SL + l;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      Aval[vb + e * SL] = blk[e];
      Lval[vb + e * SL] = (T)sb[e];
    }
  }
  const int64_t db = s * 9 * SL + l;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    if (dinv0) dinv0[db + e * SL] = Di[e];
    if (!left_scale) ldinv[db + e * SL] = (T)Di[e];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    b[3 * p + c] = F ? bb[c] + prm[2] * F[3 * p + c] : bb[c];
    u[3 * p + c] = x0_is_mn ? mt[c] : 0.0;
  }
}

// The sliced per-node blocks of the factored grid level (Mh, in FP64, and
// K, in T) from the frozen field the assembly kept, for the callers that
// read them back: the same values the assembly computes (grid_blocks).
template <typename T>
__global__ void k_fact_blocks(int nx, int ny, int nz, double inv_h2, const double* __restrict__ prm,
                              const double* __restrict__ mt, double* __restrict__ Mh, T* __restrict__ K) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)nx * ny * nz) return;
  int64_t nb[6];
  const int deg = grid_nbrs(nx, ny, nz, p, nb);
  double blk[9], kb[9];
  grid_blocks(mt + 3 * p, prm[0], prm[1], inv_h2, deg, blk, nullptr, kb);
  const int64_t s = p / SL, l = p - s * SL;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Mh[s * 9 * SL + e * SL + l] = blk[e];
    K[s * 9 * SL + e * SL + l] = (T)kb[e];
  }
}

// ---------------------------------------------------------------- Galerkin
// The fine block (i, j) of a Galerkin sum, in FP64.  Factored grid level: the
// identity on the diagonal, else K_i, read from the node-major copy the
// assembly writes (nine contiguous values) or from fk.  Other levels: the
// slot-ordered copy (nine contiguous values) when there is one, else the
// sliced-ELL values.
template <typename T, bool FACT>
__device__ inline void fine_block(const GalSrc<T>& g, int32_t i, int32_t j, int64_t k, int64_t fs, int fl,
                                  int64_t fb, int u, double* f) {
  if (FACT) {
    if (j == i) {
#pragma unroll
      for (int e = 0; e < 9; ++e) f[e] = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
    } else if (g.knm) {
#pragma unroll
      for (int e = 0; e < 9; ++e) f[e] = (double)g.knm[9 * (int64_t)i + e];
    } else {
      const int64_t kb = fs * 9 * SL + fl;
#pragma unroll
      for (int e = 0; e < 9; ++e) f[e] = (double)g.fk[kb + e * SL];
    }
  } else if (g.fvt) {
#pragma unroll
    for (int e = 0; e < 9; ++e) f[e] = (double)g.fvt[k * 9 + e];
  } else {
    const int64_t vb = fb * 9 + (int64_t)u * 9 * SL + fl;
#pragma unroll
    for (int e = 0; e < 9; ++e) f[e] = (double)g.fval[vb + e * SL];
  }
}

// Large coarse levels: one workgroup per slice of the coarse matrix; a thread
// takes GC consecutive block slots (row l, slots t..t+GC-1) of the slice, so
// that one walk over the fine rows of the members serves GC coarse blocks.
// Block (I, J) is the sum, over the members i of aggregate I in ascending
// order and over the stored blocks (i, j) of row i in ascending j with
// agg(j) = J, of the fine block a_ij (eq. Ac_direct), accumulated in FP64
// starting from zero.  The inverse of a diagonal block is computed from the
// stored (rounded) block.
constexpr int GC = 4;
template <typename T, bool FACT>
__global__ void __launch_bounds__(TPB) k_galerkin_slices(int64_t nc, const int32_t* __restrict__ csl, const int32_t* __restrict__ ccol,
                           T* __restrict__ cval, T* __restrict__ cdinv, const int32_t* __restrict__ mptr,
                           const int32_t* __restrict__ mem, const int32_t* __restrict__ fsl,
                           const int32_t* __restrict__ fcol, const int32_t* __restrict__ agg, const GalSrc<T> g) {
  // XCD-contiguous slices: neighbouring aggregates read the same fine rows
  const int64_t s = xcd_block(blockIdx.x, gridDim.x);
  const int64_t cb = csl[s];
  const int width = (int)((csl[s + 1] - cb) / SL);
  const int nchunk = (width + GC - 1) / GC;
  // Grid level stored per node: the member rows of the slice's coarse rows
  // (up to GM members per row) are staged in LDS once, their entries'
  // aggregates, the diagonal's position and K_i, and every slot group of a
  // coarse row reads them there (a row's slot groups would otherwise gather
  // the same aggregates from L2 once each).
  constexpr int GM = 4;
  __shared__ int32_t s_aa[SL * GM * 8];
  __shared__ int32_t s_dp[SL * GM];
  __shared__ int32_t s_nm[SL];
  __shared__ T s_k[SL * GM * 9];
  if (FACT && g.knm) {
    for (int tt = threadIdx.x; tt < SL * GM; tt += blockDim.x) {
      const int lr = tt / GM, m = tt - lr * GM;
      const int64_t I = s * SL + lr;
      int32_t nm = 0;
      if (I < nc) {
        const int32_t q0 = mptr[I];
        nm = mptr[I + 1] - q0;
        if (m < nm && nm <= GM) {
          const int32_t i = mem[q0 + m];
          const int32_t k0 = g.frp[i], len = min(g.frp[i + 1] - k0, 8);
          int dp = -1;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int32_t j = k < len ? g.fci[k0 + k] : -1;
            s_aa[(lr * GM + m) * 8 + k] = j >= 0 ? agg[j] : -1;
            dp = j == i ? k : dp;
          }
          s_dp[lr * GM + m] = dp;
#pragma unroll
          for (int e = 0; e < 9; ++e) s_k[(lr * GM + m) * 9 + e] = g.knm[9 * (int64_t)i + e];
        }
      }
      if (m == 0) s_nm[lr] = nm;
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < nchunk * SL; k += blockDim.x) {
    const int c = k / SL, l = k - c * SL;
    const int64_t I = s * SL + l;
    if (I >= nc) continue;
    int32_t J[GC];
#pragma unroll
    for (int h = 0; h < GC; ++h) {
      const int t = c * GC + h;
      J[h] = t < width ? ccol[cb + (int64_t)t * SL + l] : -1;
    }
    bool any = false;
#pragma unroll
    for (int h = 0; h < GC; ++h) any = any || J[h] >= 0;
    if (!any) continue;  // padding only
    double acc[GC][9];
#pragma unroll
    for (int h = 0; h < GC; ++h)
#pragma unroll
      for (int e = 0; e < 9; ++e) acc[h][e] = 0.0;
    if (FACT && g.knm) {
      // Grid-level rows (at most 8 entries): every block of row i is K_i but
      // the diagonal one, I.  So the entries of the row that fall into slot h
      // are taken from a bit mask, in ascending order, and each costs one
      // block addition; the FP64 sums are those of the walk below.
      auto add_member = [&](const int32_t* aa, int dpos, const double* kd) {
#pragma unroll
        for (int h = 0; h < GC; ++h) {
          unsigned m = 0;
#pragma unroll
          for (int k = 0; k < 8; ++k) m |= (J[h] >= 0 && aa[k] == J[h]) ? 1u << k : 0u;
          while (m) {
            const int k = __ffs(m) - 1;
            m &= m - 1;
            const bool d = k == dpos;
#pragma unroll
            for (int e = 0; e < 9; ++e) acc[h][e] += d ? ((e == 0 || e == 4 || e == 8) ? 1.0 : 0.0) : kd[e];
          }
        }
      };
      const int nm = s_nm[l];
      if (nm <= GM) {
        for (int m = 0; m < nm; ++m) {
          const int b = l * GM + m;
          int32_t aa[8];
          double kd[9];
#pragma unroll
          for (int k = 0; k < 8; ++k) aa[k] = s_aa[b * 8 + k];
#pragma unroll
          for (int e = 0; e < 9; ++e) kd[e] = (double)s_k[b * 9 + e];
          add_member(aa, s_dp[b], kd);
        }
      } else {
        for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
          const int32_t i = mem[q];
          const int32_t k0 = g.frp[i], len = min(g.frp[i + 1] - k0, 8);
          int32_t aa[8];
          int dpos = -1;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int32_t j = k < len ? g.fci[k0 + k] : -1;
            aa[k] = j >= 0 ? agg[j] : -1;
            dpos = j == i ? k : dpos;
          }
          double kd[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) kd[e] = (double)g.knm[9 * (int64_t)i + e];
          add_member(aa, dpos, kd);
        }
      }
    } else {
      for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
        const int32_t i = mem[q];
        const int64_t fs = i / SL;
        const int fl = i - (int)(fs * SL);
        const int64_t fb = (FACT || g.fvt) ? 0 : fsl[fs];  // sliced fine values only
        // the member's row in CSR order (contiguous columns and, on coarse
        // levels, contiguous blocks), four at a time: their column and
        // aggregate loads are in flight together; the blocks are still added
        // in ascending column order
        const int32_t k0 = g.frp[i], k1 = g.frp[i + 1];
        for (int32_t kb = k0; kb < k1; kb += 4) {
          int32_t jj[4], aa[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) jj[k] = kb + k < k1 ? g.fci[kb + k] : -1;
#pragma unroll
          for (int k = 0; k < 4; ++k) aa[k] = jj[k] >= 0 ? agg[jj[k]] : -1;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            int hit = -1;
#pragma unroll
            for (int h = 0; h < GC; ++h) hit = aa[k] >= 0 && aa[k] == J[h] ? h : hit;
            if (hit < 0) continue;
            double f[9];
            fine_block<T, FACT>(g, i, jj[k], kb + k, fs, fl, fb, kb + k - k0, f);
#pragma unroll
            for (int h = 0; h < GC; ++h)
              if (h == hit)
#pragma unroll
                for (int e = 0; e < 9; ++e) acc[h][e] += f[e];
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < GC; ++h) {
      if (J[h] < 0) continue;
      const int t = c * GC + h;
      const int64_t vb = cb * 9 + (int64_t)t * 9 * SL + l;
      T stv[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) stv[e] = (T)acc[h][e];
      if (cval) {
#pragma unroll
        for (int e = 0; e < 9; ++e) cval[vb + e * SL] = stv[e];
      }
      if (g.cvt) {
        // CSR-ordered copy for the next level's product, which walks member rows
        const int64_t pos = (int64_t)g.crp[I] + t;
#pragma unroll
        for (int e = 0; e < 9; ++e) g.cvt[pos * 9 + e] = stv[e];
      }
      if (J[h] == (int32_t)I) {
        double D[9], Di[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) D[e] = (double)stv[e];
        inv3(D, Di);
        const int64_t db = s * 9 * SL + l;
#pragma unroll
        for (int e = 0; e < 9; ++e) cdinv[db + e * SL] = (T)Di[e];
      }
    }
  }
}

// Level 1 of a grid level stored per node, one thread per coarse block in
// the coarse level's CSR order: a workgroup takes a slice of 64 coarse rows,
// stages their members' rows once in LDS (each entry's aggregate, the
// diagonal's position and K_i; up to GM members per row, larger aggregates
// walk their rows from memory), and its threads take the slice's blocks in
// order, so the CSR-ordered copy is written by consecutive threads.  Block
// (I, J) sums, over the members of I in ascending order and over the entries
// of each member's row in ascending order whose aggregate is J, the fine
// block: the identity on the diagonal, K_i elsewhere (eq. Ac_direct), in
// FP64 from zero, as k_galerkin_slices does.
template <typename T>
__global__ void __launch_bounds__(TPB) k_galerkin_grid(int64_t nc, const int32_t* __restrict__ csl,
                                                       T* __restrict__ cval, T* __restrict__ cdinv,
                                                       const int32_t* __restrict__ mptr,
                                                       const int32_t* __restrict__ mem,
                                                       const int32_t* __restrict__ agg, const GalSrc<T> g) {
  const int64_t s = xcd_block(blockIdx.x, gridDim.x);
  constexpr int GM = 4;
  __shared__ int32_t s_aa[SL * GM * 8];
  __shared__ int32_t s_dp[SL * GM];
  __shared__ int32_t s_nm[SL];
  __shared__ T s_k[SL * GM * 9];
  __shared__ int32_t s_rs[SL + 1];
  for (int tt = threadIdx.x; tt < SL * GM; tt += blockDim.x) {
    const int lr = tt / GM, m = tt - lr * GM;
    const int64_t I = s * SL + lr;
    int32_t nm = 0;
    if (I < nc) {
      const int32_t q0 = mptr[I];
      nm = mptr[I + 1] - q0;
      if (m < nm && nm <= GM) {
        const int32_t i = mem[q0 + m];
        const int32_t k0 = g.frp[i], len = min(g.frp[i + 1] - k0, 8);
        int dp = -1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int32_t j = k < len ? g.fci[k0 + k] : -1;
          s_aa[(lr * GM + m) * 8 + k] = j >= 0 ? agg[j] : -1;
          dp = j == i ? k : dp;
        }
        s_dp[lr * GM + m] = dp;
#pragma unroll
        for (int e = 0; e < 9; ++e) s_k[(lr * GM + m) * 9 + e] = g.knm[9 * (int64_t)i + e];
      }
    }
    if (m == 0) s_nm[lr] = nm;
  }
  for (int tt = threadIdx.x; tt <= SL; tt += blockDim.x) s_rs[tt] = g.crp[min(s * SL + tt, nc)];
  __syncthreads();
  const int32_t p0 = s_rs[0], tot = s_rs[SL] - p0;
  const int64_t cb = csl[s];
  for (int q = threadIdx.x; q < tot; q += blockDim.x) {
    // the block's row: the last l with s_rs[l] <= p0 + q
    int lo = 0, hi = SL;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_rs[mid] <= p0 + q)
        lo = mid;
      else
        hi = mid;
    }
    const int l = lo;
    const int64_t I = s * SL + l;
    const int t = p0 + q - s_rs[l];
    const int32_t J = g.cci[p0 + q];
    double acc[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[e] = 0.0;
    auto add_row = [&](const int32_t* aa, int dpos, const double* kd) {
      unsigned msk = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) msk |= aa[k] == J ? 1u << k : 0u;
      while (msk) {
        const int k = __ffs(msk) - 1;
        msk &= msk - 1;
        const bool d = k == dpos;
#pragma unroll
        for (int e = 0; e < 9; ++e) acc[e] += d ? ((e == 0 || e == 4 || e == 8) ? 1.0 : 0.0) : kd[e];
      }
    };
    const int nm = s_nm[l];
    if (nm <= GM) {
      for (int m = 0; m < nm; ++m) {
        const int b = l * GM + m;
        int32_t aa[8];
        double kd[9];
#pragma unroll
        for (int k = 0; k < 8; ++k) aa[k] = s_aa[b * 8 + k];
#pragma unroll
        for (int e = 0; e < 9; ++e) kd[e] = (double)s_k[b * 9 + e];
        add_row(aa, s_dp[b], kd);
      }
    } else {
      for (int32_t qq = mptr[I]; qq < mptr[I + 1]; ++qq) {
        const int32_t i = mem[qq];
        const int32_t k0 = g.frp[i], len = min(g.frp[i + 1] - k0, 8);
        int32_t aa[8];
        int dpos = -1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int32_t j = k < len ? g.fci[k0 + k] : -1;
          aa[k] = j >= 0 ? agg[j] : -1;
          dpos = j == i ? k : dpos;
        }
        double kd[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) kd[e] = (double)g.knm[9 * (int64_t)i + e];
        add_row(aa, dpos, kd);
      }
    }
    T stv[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) stv[e] = (T)acc[e];
    const int64_t pos = (int64_t)p0 + q;
#pragma unroll
    for (int e = 0; e < 9; ++e) g.cvt[pos * 9 + e] = stv[e];
    if (cval) {
      const int64_t vb = cb * 9 + (int64_t)t * 9 * SL + l;
#pragma unroll
      for (int e = 0; e < 9; ++e) cval[vb + e * SL] = stv[e];
    }
    if (J == (int32_t)I) {
      double D[9], Di[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) D[e] = (double)stv[e];
      inv3(D, Di);
      const int64_t db = s * 9 * SL + l;
#pragma unroll
      for (int e = 0; e < 9; ++e) cdinv[db + e * SL] = (T)Di[e];
    }
  }
}

// Coarse levels of a coarse level, row by row: GR_L lanes share a
// coarse row I, lane t owning its slots t and t + GR_L (further passes for
// rows of more than 2 GR_L blocks).  The group walks the fine rows of I's
// members once: lane e loads entry e of a member row (its column's aggregate
// and its nine values, contiguous in the fine level's CSR-ordered copy), and
// the entries are handed round the group in row order; the lane owning the
// entry's aggregate adds it.  So every block (I, J) is the sum, over the
// members i of I in ascending order and over the stored blocks (i, j) of row i
// in ascending j with agg(j) = J, of a_ij (eq. Ac_direct), accumulated in FP64
// from zero, as in the other two kernels, while each fine row is read once per
// coarse row (not once per group of slots) and with contiguous loads.
constexpr int GR_L = 16;
template <typename T>
__global__ void __launch_bounds__(TPB) k_galerkin_rows(int64_t nc, const int32_t* __restrict__ csl,
                                                       T* __restrict__ cval, T* __restrict__ cdinv,
                                                       const int32_t* __restrict__ mptr,
                                                       const int32_t* __restrict__ mem,
                                                       const int32_t* __restrict__ agg, const GalSrc<T> g) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t I = blk * (TPB / GR_L) + threadIdx.x / GR_L;
  const int t = (int)(threadIdx.x % GR_L);
  if (I >= nc) return;  // a whole group
  const int32_t c0 = g.crp[I], w = g.crp[I + 1] - c0;
  const int32_t q0 = mptr[I], q1 = mptr[I + 1];
  const int64_t s = I / SL, l = I - s * SL;
  for (int sp = 0; sp < w; sp += 2 * GR_L) {
    const int s0 = sp + t, s1 = sp + GR_L + t;
    const int32_t J0 = s0 < w ? g.cci[c0 + s0] : -1, J1 = s1 < w ? g.cci[c0 + s1] : -1;
    double a0[9], a1[9];
#pragma unroll
    for (int x = 0; x < 9; ++x) a0[x] = a1[x] = 0.0;
    for (int32_t q = q0; q < q1; ++q) {
      const int32_t i = mem[q];
      const int32_t k0 = g.frp[i], len = g.frp[i + 1] - k0;
      for (int b = 0; b < len; b += GR_L) {
        const int e = b + t;
        int32_t a = -1;
        T v[9];
#pragma unroll
        for (int x = 0; x < 9; ++x) v[x] = T(0);
        if (e < len) {
          a = agg[g.fci[k0 + e]];
#pragma unroll
          for (int x = 0; x < 9; ++x) v[x] = g.fvt[(int64_t)(k0 + e) * 9 + x];
        }
        // the entries of this stretch that fall into each of the lane's two
        // slots, as bit masks; then their blocks are fetched from their
        // lanes in ascending order, as many passes as the wavefront's fullest
        // mask (every lane takes part in each pass, so every source lane of
        // a shuffle is active)
        const int n = min(GR_L, len - b);
        unsigned m0 = 0, m1 = 0;
        for (int u = 0; u < n; ++u) {
          const int32_t A = __shfl(a, u, GR_L);
          m0 |= (J0 >= 0 && A == J0) ? 1u << u : 0u;
          m1 |= (J1 >= 0 && A == J1) ? 1u << u : 0u;
        }
        while (__any(m0 != 0)) {
          const int u = m0 ? __ffs(m0) - 1 : 0;
          double f[9];
#pragma unroll
          for (int x = 0; x < 9; ++x) f[x] = (double)__shfl(v[x], u, GR_L);
          if (m0) {
#pragma unroll
            for (int x = 0; x < 9; ++x) a0[x] += f[x];
            m0 &= m0 - 1;
          }
        }
        while (__any(m1 != 0)) {
          const int u = m1 ? __ffs(m1) - 1 : 0;
          double f[9];
#pragma unroll
          for (int x = 0; x < 9; ++x) f[x] = (double)__shfl(v[x], u, GR_L);
          if (m1) {
#pragma unroll
            for (int x = 0; x < 9; ++x) a1[x] += f[x];
            m1 &= m1 - 1;
          }
        }
      }
    }
    // slot s0 (then s1): stored in T, the inverse of a diagonal block from the stored block
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t J = h ? J1 : J0;
      if (J < 0) continue;
      const int so = h ? s1 : s0;
      T stv[9];
#pragma unroll
      for (int x = 0; x < 9; ++x) stv[x] = (T)(h ? a1[x] : a0[x]);
      if (cval) {
        const int64_t vb = (int64_t)csl[s] * 9 + (int64_t)so * 9 * SL + l;
#pragma unroll
        for (int x = 0; x < 9; ++x) cval[vb + x * SL] = stv[x];
      }
      if (g.cvt) {
        const int64_t pos = (int64_t)c0 + so;
#pragma unroll
        for (int x = 0; x < 9; ++x) g.cvt[pos * 9 + x] = stv[x];
      }
      if (J == (int32_t)I) {
        double D[9], Di[9];
#pragma unroll
        for (int x = 0; x < 9; ++x) D[x] = (double)stv[x];
        inv3(D, Di);
        const int64_t db = s * 9 * SL + l;
#pragma unroll
        for (int x = 0; x < 9; ++x) cdinv[db + x * SL] = (T)Di[x];
      }
    }
  }
}

// Small coarse levels (few slices): one thread per block slot (I, J), its
// slice found by bisection.  The block is the sum, over the
// members i of aggregate I in ascending order and over the stored blocks
// (i, j) of row i in ascending j with agg(j) = J, of the fine block a_ij
// (eq. Ac_direct), accumulated in FP64 starting from zero.  The inverse of a
// diagonal block is computed from the stored (rounded) block.
template <typename T, bool FACT>
__global__ void k_galerkin_slots(int64_t nc, int64_t ns, const int32_t* __restrict__ csl,
                           const int32_t* __restrict__ ccol, T* __restrict__ cval, T* __restrict__ cdinv,
                           const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                           const int32_t* __restrict__ fsl, const int32_t* __restrict__ fcol,
                           const int32_t* __restrict__ agg, const GalSrc<T> g) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= csl[ns]) return;
  // slice of slot p: the last s with csl[s] <= p
  int64_t lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (csl[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t s = lo, cb = csl[s];
  const int t = (int)((p - cb) / SL), l = (int)((p - cb) % SL);
  const int64_t I = s * SL + l;
  const int32_t J = ccol[p];
  if (J < 0 || I >= nc) return;
  double acc[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) acc[e] = 0.0;
  for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
    const int32_t i = mem[q];
    const int64_t fs = i / SL;
    const int fl = i - (int)(fs * SL);
    const int64_t fb = (FACT || g.fvt) ? 0 : fsl[fs];  // sliced fine values only
    const int32_t k0 = g.frp[i], k1 = g.frp[i + 1];
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t j = g.fci[k];
      if (agg[j] != J) continue;
      double f[9];
      fine_block<T, FACT>(g, i, j, k, fs, fl, fb, k - k0, f);
#pragma unroll
      for (int e = 0; e < 9; ++e) acc[e] += f[e];
    }
  }
  const int64_t vb = cb * 9 + (int64_t)t * 9 * SL + l;
  T st[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) st[e] = (T)acc[e];
  if (cval) {
#pragma unroll
    for (int e = 0; e < 9; ++e) cval[vb + e * SL] = st[e];
  }
  if (g.cvt) {
    const int64_t pos = (int64_t)g.crp[I] + t;
#pragma unroll
    for (int e = 0; e < 9; ++e) g.cvt[pos * 9 + e] = st[e];
  }
  if (J == (int32_t)I) {
    double D[9], Di[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) D[e] = (double)st[e];
    inv3(D, Di);
    const int64_t db = s * 9 * SL + l;
#pragma unroll
    for (int e = 0; e < 9; ++e) cdinv[db + e * SL] = (T)Di[e];
  }
}

// ---------------------------------------------------------------- coarsest
template <typename T>
__global__ void k_dense_scatter(int64_t n, const int32_t* __restrict__ sl, const int32_t* __restrict__ col,
                                const T* __restrict__ val, double* __restrict__ dense) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n) return;
  const int64_t s = I / SL;
  const int l = (int)(I - s * SL);
  const int64_t cb = sl[s];
  const int w = (int)((sl[s + 1] - cb) / SL);
  const int64_t nd = 3 * n;
  for (int t = 0; t < w; ++t) {
    const int32_t J = col[cb + (int64_t)t * SL + l];
    if (J < 0) break;
    const int64_t vb = cb * 9 + (int64_t)t * 9 * SL + l;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) dense[(3 * I + r) * nd + 3 * J + c] = (double)val[vb + (3 * r + c) * SL];
  }
}

// In-place Gauss-Jordan inversion with partial pivoting (first largest
// magnitude in the pivot column), one workgroup.  Row interchanges are undone
// at the end by swapping columns in reverse order.  The matrix lives in LDS
// when it fits (a != dense), else in global memory.
constexpr int GJ_T = 1024;

__device__ void gauss_jordan(int64_t nd, double* a, int32_t* piv, int32_t* flag, double* colk,
                             double* redv, int32_t* redi) {
  const int t = threadIdx.x;
  for (int64_t k = 0; k < nd; ++k) {
    // pivot search: first row of largest |a_ik|, i >= k
    double best = -1.0;
    int32_t bi = (int32_t)nd;
    for (int64_t i = k + t; i < nd; i += GJ_T) {
      const double v = fabs(a[i * nd + k]);
      if (v > best) {
        best = v;
        bi = (int32_t)i;
      }
    }
    redv[t] = best;
    redi[t] = bi;
    __syncthreads();
    for (int off = GJ_T / 2; off > 0; off >>= 1) {
      if (t < off) {
        const double v2 = redv[t + off];
        const int32_t i2 = redi[t + off];
        if (v2 > redv[t] || (v2 == redv[t] && i2 < redi[t])) {
          redv[t] = v2;
          redi[t] = i2;
        }
      }
      __syncthreads();
    }
    // no usable pivot (zero or NaN column): keep row k and report singular
    const int32_t p = (redi[0] < nd && redv[0] > 0.0) ? redi[0] : (int32_t)k;
    if (t == 0) {
      piv[k] = p;
      if (!(redv[0] > 0.0)) atomicOr(flag, 2);
    }
    __syncthreads();
    if (p != k) {
      for (int64_t j = t; j < nd; j += GJ_T) {
        const double x = a[k * nd + j];
        a[k * nd + j] = a[(int64_t)p * nd + j];
        a[(int64_t)p * nd + j] = x;
      }
      __syncthreads();
    }
    for (int64_t i = t; i < nd; i += GJ_T) colk[i] = a[i * nd + k];
    __syncthreads();
    const double pv = colk[k];
    for (int64_t j = t; j < nd; j += GJ_T) a[k * nd + j] = (j == k ? 1.0 : a[k * nd + j]) / pv;
    __syncthreads();
    for (int64_t e = t; e < nd * nd; e += GJ_T) {
      const int64_t i = e / nd, j = e - i * nd;
      if (i == k) continue;
      const double f = colk[i];
      if (j == k)
        a[e] = -f * a[k * nd + k];
      else
        a[e] -= f * a[k * nd + j];
    }
    __syncthreads();
  }
  for (int64_t k = nd - 1; k >= 0; --k) {
    const int32_t p = piv[k];
    if (p != k) {
      for (int64_t i = t; i < nd; i += GJ_T) {
        const double x = a[i * nd + k];
        a[i * nd + k] = a[i * nd + p];
        a[i * nd + p] = x;
      }
    }
    __syncthreads();
  }
}

constexpr int64_t GJ_LDS_MAX = 136;  // 136^2 doubles + work arrays fit in 160 KB LDS

// The same inversion with the matrix in LDS, in three barriers per pivot
// step: the first wavefront finds the pivot (shuffles, the same rule); then
// rows k and p are exchanged, row k normalised (also into rowk) and the
// pivot column kept in colk; then every other row is eliminated.  The
// values are those of gauss_jordan (the same operations on the same
// operands).  The column interchanges are applied as one permutation when
// the inverse is written back.
__global__ void __launch_bounds__(GJ_T) k_gauss_jordan_lds(int64_t nd64, double* dense, int32_t* piv,
                                                           int32_t* flag) {
  extern __shared__ double lds[];
  const int nd = (int)nd64;
  double* a = lds;
  double* colk = a + nd * nd;
  double* rowk = colk + nd;
  int32_t* perm = (int32_t*)(rowk + nd);
  __shared__ int s_p;
  __shared__ double s_pk, s_kk;
  const int t = (int)threadIdx.x;
  for (int e = t; e < nd * nd; e += GJ_T) a[e] = dense[e];
  __syncthreads();
  for (int k = 0; k < nd; ++k) {
    if (t < 64) {
      // first row of largest |a_ik|, i >= k
      double best = -1.0;
      int bi = nd;
      for (int i = k + t; i < nd; i += 64) {
        const double v = fabs(a[i * nd + k]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double v2 = __shfl_xor(best, off, 64);
        const int i2 = __shfl_xor(bi, off, 64);
        if (v2 > best || (v2 == best && i2 < bi)) {
          best = v2;
          bi = i2;
        }
      }
      if (t == 0) {
        // no usable pivot (zero or NaN column): keep row k and report singular
        const int p = (bi < nd && best > 0.0) ? bi : k;
        s_p = p;
        s_pk = a[p * nd + k];
        s_kk = a[k * nd + k];
        piv[k] = p;
        if (!(best > 0.0)) atomicOr(flag, 2);
      }
    }
    __syncthreads();
    const int p = s_p;
    const double pv = s_pk;
    for (int j = t; j < nd; j += GJ_T) {
      const double xk = a[k * nd + j], xp = a[p * nd + j];
      const double r = (j == k ? 1.0 : xp) / pv;
      if (p != k) a[p * nd + j] = xk;
      a[k * nd + j] = r;
      rowk[j] = r;
    }
    for (int i = t; i < nd; i += GJ_T) colk[i] = i == k ? s_pk : i == p ? s_kk : a[i * nd + k];
    __syncthreads();
    for (int e = t; e < nd * nd; e += GJ_T) {
      const int i = e / nd, j = e - i * nd;
      if (i == k) continue;
      const double f = colk[i];
      if (j == k)
        a[e] = -f * rowk[k];
      else
        a[e] -= f * rowk[j];
    }
    __syncthreads();
  }
  // the column interchanges, last to first, as one permutation: position j
  // of the inverse holds column perm[j] of a
  if (t == 0) {
    for (int j = 0; j < nd; ++j) perm[j] = j;
    for (int k = nd - 1; k >= 0; --k) {
      const int q = piv[k];
      const int32_t x = perm[k];
      perm[k] = perm[q];
      perm[q] = x;
    }
  }
  __syncthreads();
  for (int e = t; e < nd * nd; e += GJ_T) {
    const int i = e / nd, j = e - i * nd;
    dense[e] = a[i * nd + perm[j]];
  }
}

__global__ void __launch_bounds__(GJ_T) k_gauss_jordan_global(int64_t nd, double* dense, int32_t* piv,
                                                              int32_t* flag, double* colk) {
  __shared__ double redv[GJ_T];
  __shared__ int32_t redi[GJ_T];
  gauss_jordan(nd, dense, piv, flag, colk, redv, redi);
}

template <typename T>
__global__ void k_dense_apply(int64_t nd, const double* __restrict__ inv, const T* __restrict__ b,
                              T* __restrict__ x) {
  extern __shared__ double sb[];
  for (int64_t i = threadIdx.x; i < nd; i += blockDim.x) sb[i] = (double)b[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * nw + wv; r < nd; r += (int64_t)gridDim.x * nw) {
    double s = 0.0;
    for (int64_t c = lane; c < nd; c += 64) s += inv[r * nd + c] * sb[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) x[r] = (T)s;
  }
}

// The restriction to the coarsest level and its exact solve in one
// workgroup: bc_I = sum of r_i over the members of aggregate I (ascending, in
// the level's precision, as the restriction does), then x = A_c^{-1} bc.
template <typename T>
__global__ void k_restrict_dense(int64_t nc, const int32_t* __restrict__ mptr, const int32_t* __restrict__ mem,
                                 const T* __restrict__ r, const double* __restrict__ inv, T* __restrict__ x) {
  extern __shared__ double sb[];
  for (int64_t I = threadIdx.x; I < nc; I += blockDim.x) {
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
      const int64_t i = mem[q];
      a0 += r[3 * i];
      a1 += r[3 * i + 1];
      a2 += r[3 * i + 2];
    }
    sb[3 * I] = (double)a0;
    sb[3 * I + 1] = (double)a1;
    sb[3 * I + 2] = (double)a2;
  }
  __syncthreads();
  const int64_t nd = 3 * nc;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int64_t row = wv; row < nd; row += nw) {
    double s = 0.0;
    for (int64_t c = lane; c < nd; c += 64) s += inv[row * nd + c] * sb[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) x[row] = (T)s;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
void launch_fill_i32(hipStream_t st, int32_t* p, int64_t n, int32_t v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n)), dim3(TPB), 0, st, p, n, v);
}
void launch_fill_f64(hipStream_t st, double* p, int64_t n, double v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(nblk(n)), dim3(TPB), 0, st, p, n, v);
}

int64_t scan_tmp_ints(int64_t n) { return ceil_div(n > 0 ? n : 1, SCAN_CHUNK) + 1; }

void launch_scan_excl(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                      int32_t* tmp) {
  const int64_t nb = ceil_div(n > 0 ? n : 1, SCAN_CHUNK);
  if (n <= 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, st, total, 1, 0);
    return;
  }
  if (n <= (int64_t)SCAN1_T * SCAN1_ITEMS) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN1_T), 0, st, in, out, n, total);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, st, tmp, nb, total);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, out, n, tmp);
}

void launch_check_eq(hipStream_t st, const int32_t* a, int32_t expect, int32_t* flag, int32_t bit) {
  hipLaunchKernelGGL(k_check_eq, dim3(1), dim3(64), 0, st, a, expect, flag, bit);
}
void launch_check_many(hipStream_t st, const int32_t* const* p, const int32_t* v, int n, int32_t* flag, int32_t bit) {
  CountChecks c{};
  for (int k = 0; k < n && k < CHECK_BATCH; ++k) {
    c.p[k] = p[k];
    c.v[k] = v[k];
  }
  c.n = n < CHECK_BATCH ? n : CHECK_BATCH;
  if (c.n > 0) hipLaunchKernelGGL(k_check_many, dim3(1), dim3(CHECK_BATCH), 0, st, c, flag, bit);
}

void launch_grid_degree(hipStream_t st, int nx, int ny, int nz, int32_t* deg) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(k_grid_degree, dim3(nblk(N)), dim3(TPB), 0, st, nx, ny, nz, deg);
}
void launch_grid_graph(hipStream_t st, int nx, int ny, int nz, const int32_t* grp, int32_t* gci,
                       int32_t* gw) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(k_grid_graph, dim3(nblk(N)), dim3(TPB), 0, st, nx, ny, nz, grp, gci, gw);
}
void launch_pattern_rp(hipStream_t st, int64_t n, const int32_t* grp, int32_t* brp) {
  hipLaunchKernelGGL(k_pattern_rp, dim3(nblk(n + 1)), dim3(TPB), 0, st, n, grp, brp);
}
void launch_pattern_cols(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci,
                         const int32_t* brp, int32_t* bci) {
  if (n > 0) hipLaunchKernelGGL(k_pattern_cols, dim3(nblk(n * PC_L)), dim3(TPB), 0, st, n, grp, gci, brp, bci);
}
void launch_slice_width(hipStream_t st, int64_t n, const int32_t* rows, const int32_t* brp, int32_t* wslots) {
  const int64_t ns = ceil_div(n, SL);
  if (ns > 0) hipLaunchKernelGGL(k_slice_width, dim3(nblk(ns)), dim3(TPB), 0, st, n, rows, brp, wslots);
}
void launch_sell_cols(hipStream_t st, int64_t n, const int32_t* rows, const int32_t* brp, const int32_t* bci,
                      const int32_t* sl_ptr, int32_t* col) {
  const int64_t ns = ceil_div(n, SL);
  if (ns > 0)
    hipLaunchKernelGGL(k_sell_cols, dim3(nblk(ns * SL)), dim3(TPB), 0, st, n, rows, brp, bci, sl_ptr, col);
}
void launch_node_rank(hipStream_t st, int64_t n, uint64_t salt, uint64_t* rank) {
  if (n > 0) hipLaunchKernelGGL(k_node_rank, dim3(nblk(n)), dim3(TPB), 0, st, n, salt, rank);
}
void launch_propose(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci, const int32_t* gw,
                    int32_t* mate, const NodeSt* ns, uint64_t salt, int32_t bnum, int32_t bden, int32_t* prop,
                    int32_t* count, int G) {
  if (n <= 0) return;
#define LLG_PR(GG)                                                                                         \
  hipLaunchKernelGGL((k_propose<GG>), dim3(nblk(n * GG)), dim3(TPB), 0, st, n, grp, gci, gw, mate, ns, salt, \
                     bnum, bden, prop, count)
  if (G >= 16)
    LLG_PR(16);
  else if (G == 8)
    LLG_PR(8);
  else if (G == 4)
    LLG_PR(4);
  else if (G == 2)
    LLG_PR(2);
  else
    hipLaunchKernelGGL(k_propose_packed, dim3(nblk(n)), dim3(TPB), 0, st, n, grp, gci, gw, mate, ns, salt, bnum,
                       bden, prop, count);
#undef LLG_PR
}
void launch_propose_grid(hipStream_t st, int nx, int ny, int nz, int32_t* mate, const uint64_t* rank,
                         uint64_t salt, int32_t bnum, int32_t bden, int32_t* prop, int32_t* count, bool first) {
  const int64_t N = (int64_t)nx * ny * nz;
  if (N > 0)
    hipLaunchKernelGGL(k_propose_grid, dim3(nblk(N, TPB * RN)), dim3(TPB), 0, st, nx, ny, nz, mate, rank, salt, bnum,
                       bden, prop, count, first ? 1 : 0);
}
void launch_match_small(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci, const int32_t* gw,
                        int32_t* mate, NodeSt* ns, uint64_t salt, int32_t bnum, int32_t bden, int32_t* prop,
                        int32_t* flag, int32_t bit, int G) {
  if (n <= 0) return;
  if (G >= 2)
    hipLaunchKernelGGL(k_match_small<2>, dim3(1), dim3(MATCH_T), 0, st, n, grp, gci, gw, mate, ns, salt, bnum, bden,
                       prop, flag, bit);
  else
    hipLaunchKernelGGL(k_match_small<1>, dim3(1), dim3(MATCH_T), 0, st, n, grp, gci, gw, mate, ns, salt, bnum, bden,
                       prop, flag, bit);
}
void launch_accept(hipStream_t st, int64_t n, const int32_t* prop, int32_t* mate, NodeSt* ns) {
  if (n > 0) hipLaunchKernelGGL(k_accept, dim3(nblk(n, TPB * RN)), dim3(TPB), 0, st, n, prop, mate, ns);
}
void launch_match_init(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gw, uint64_t salt,
                       NodeSt* ns, int32_t* mate, int32_t* prop) {
  if (n > 0) hipLaunchKernelGGL(k_match_init, dim3(nblk(n)), dim3(TPB), 0, st, n, grp, gw, salt, ns, mate, prop);
}
void launch_leader_flag(hipStream_t st, int64_t n, const int32_t* mate, int32_t* flag) {
  if (n > 0) hipLaunchKernelGGL(k_leader_flag, dim3(nblk(n)), dim3(TPB), 0, st, n, mate, flag);
}
void launch_assign(hipStream_t st, int64_t n, const int32_t* mate, const int32_t* id, int32_t* agg,
                   int32_t* lead) {
  if (n > 0) hipLaunchKernelGGL(k_assign, dim3(nblk(n)), dim3(TPB), 0, st, n, mate, id, agg, lead);
}
void launch_cg_count(hipStream_t st, int64_t nc, const int32_t* lead, const int32_t* mate,
                     const int32_t* grp, int32_t* cnt) {
  if (nc > 0) hipLaunchKernelGGL(k_cg_count, dim3(nblk(nc)), dim3(TPB), 0, st, nc, lead, mate, grp, cnt);
}
int cg_tile_rows(int shape) { return shape == 1 ? TPB / 16 : shape == 2 ? TPB / 4 : TPB / 8; }

void launch_cg_fill(hipStream_t st, int64_t nc, const int32_t* lead, const int32_t* mate,
                    const int32_t* grp, const int32_t* gci, const int32_t* gw, const int32_t* agg,
                    const int32_t* cptr, int32_t* cj, int32_t* cw, int32_t* nrp, int32_t* ttot, bool wide,
                    const int* grid, NodeSt* nsn, int32_t* maten, int32_t* propn) {
  if (nc <= 0) return;
  const dim3 gr(nblk(nc, cg_tile_rows(wide ? 1 : grid ? 2 : 0)));
  // the rows of the grid graph have at most twelve candidates: four lanes
  // and 16 slots (eight lanes and 32 slots took 0.45 ms more per step at
  // 256^3); the grid level's second pass, and all rows in 2D, up to about
  // 20: eight lanes and 32 slots; the coarse levels of 3D grids up to
  // about 50: sixteen lanes and 64 slots
  if (wide)
    hipLaunchKernelGGL((k_cg_fill<16, 64, false>), gr, dim3(TPB), 0, st, nc, lead, mate, grp, gci, gw, agg, cptr, cj,
                       cw, nrp, ttot, 0, 0, 0, nsn, maten, propn);
  else if (grid)
    hipLaunchKernelGGL((k_cg_fill<4, 16, true>), gr, dim3(TPB), 0, st, nc, lead, mate, grp, gci, gw, agg, cptr, cj,
                       cw, nrp, ttot, grid[0], grid[1], grid[2], nsn, maten, propn);
  else
    hipLaunchKernelGGL((k_cg_fill<8, 32, false>), gr, dim3(TPB), 0, st, nc, lead, mate, grp, gci, gw, agg, cptr, cj,
                       cw, nrp, ttot, 0, 0, 0, nsn, maten, propn);
}
void launch_cg_copy(hipStream_t st, int64_t nc, int shape, const int32_t* cptr, const int32_t* cj,
                    const int32_t* cw, const int32_t* tbase, int32_t* nrp, int32_t* nci, int32_t* nw) {
  if (nc <= 0) return;
  const int R = cg_tile_rows(shape);
  hipLaunchKernelGGL(k_cg_copy, dim3(nblk(nc, R)), dim3(TPB), 0, st, nc, R, cptr, cj, cw, tbase, nrp, nci, nw);
}
static PassMaps pass_maps(int np, const int32_t* const* lead, const int32_t* const* mate) {
  PassMaps pm{};
  for (int q = 0; q < np; ++q) {
    pm.lead[q] = lead[q];
    pm.mate[q] = mate[q];
  }
  return pm;
}
void launch_member_count(hipStream_t st, int64_t nc, int np, const int32_t* const* lead,
                         const int32_t* const* mate, int32_t* cnt) {
  if (nc <= 0) return;
  const PassMaps pm = pass_maps(np, lead, mate);
  if (np == 1)
    hipLaunchKernelGGL(k_member_count<1>, dim3(nblk(nc)), dim3(TPB), 0, st, nc, pm, cnt);
  else if (np == 2)
    hipLaunchKernelGGL(k_member_count<2>, dim3(nblk(nc)), dim3(TPB), 0, st, nc, pm, cnt);
  else
    hipLaunchKernelGGL(k_member_count<3>, dim3(nblk(nc)), dim3(TPB), 0, st, nc, pm, cnt);
}
void launch_member_fill(hipStream_t st, int64_t nc, int np, const int32_t* const* lead,
                        const int32_t* const* mate, const int32_t* mptr, int32_t* mem, int32_t* acc) {
  if (nc <= 0) return;
  const PassMaps pm = pass_maps(np, lead, mate);
  if (np == 1)
    hipLaunchKernelGGL(k_member_fill<1>, dim3(nblk(nc)), dim3(TPB), 0, st, nc, pm, mptr, mem, acc);
  else if (np == 2)
    hipLaunchKernelGGL(k_member_fill<2>, dim3(nblk(nc)), dim3(TPB), 0, st, nc, pm, mptr, mem, acc);
  else
    hipLaunchKernelGGL(k_member_fill<3>, dim3(nblk(nc)), dim3(TPB), 0, st, nc, pm, mptr, mem, acc);
}

template <typename T>
void launch_assemble(hipStream_t st, int nx, int ny, int nz, double inv_h2, const double* prm,
                     int left_scale, int x0_is_mn, Sell A, double* Aval, T* Lval, double* dinv0, T* ldinv,
                     double* b, double* u, int32_t* flag, bool fact, double* Mh, T* K, T* Knm, double* mt_out) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL((k_assemble<T>), dim3(nblk(N)), dim3(TPB), 0, st, nx, ny, nz, inv_h2, prm,
                     left_scale, x0_is_mn, A.sl_ptr, A.col, Aval, Lval, dinv0, ldinv, b, u, flag, Mh,
                     K, Knm, mt_out, fact ? 1 : 0);
}
template void launch_assemble<double>(hipStream_t, int, int, int, double, const double*, int, int, Sell,
                                      double*, double*, double*, double*, double*, double*, int32_t*, bool,
                                      double*, double*, double*, double*);
template void launch_assemble<float>(hipStream_t, int, int, int, double, const double*, int, int, Sell,
                                     double*, float*, double*, float*, double*, double*, int32_t*, bool,
                                     double*, float*, float*, double*);
template <typename T>
void launch_fact_blocks(hipStream_t st, int nx, int ny, int nz, double inv_h2, const double* prm, const double* mt,
                        double* Mh, T* K) {
  const int64_t N = (int64_t)nx * ny * nz;
  if (N > 0)
    hipLaunchKernelGGL((k_fact_blocks<T>), dim3(nblk(N)), dim3(TPB), 0, st, nx, ny, nz, inv_h2, prm, mt, Mh, K);
}
template void launch_fact_blocks<double>(hipStream_t, int, int, int, double, const double*, const double*, double*,
                                         double*);
template void launch_fact_blocks<float>(hipStream_t, int, int, int, double, const double*, const double*, double*,
                                        float*);

void init_kernel_attributes() {
  const size_t lds_max = (size_t)(GJ_LDS_MAX * GJ_LDS_MAX + 2 * GJ_LDS_MAX) * sizeof(double) +
                         GJ_LDS_MAX * sizeof(int32_t);
  (void)hipFuncSetAttribute((const void*)k_gauss_jordan_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_max);
  (void)hipGetLastError();
}

template <typename T>
void launch_galerkin(hipStream_t st, Sell C, T* cval, T* cdinv, const int32_t* mptr, const int32_t* mem, Sell F,
                     const int32_t* agg, const GalSrc<T>& g) {
  if (C.n <= 0) return;
#define LLG_GAL(FACT)                                                                                          \
  if (C.nslices >= 1024)                                                                                       \
    hipLaunchKernelGGL((k_galerkin_slices<T, FACT>), dim3((unsigned)C.nslices), dim3(TPB), 0, st, C.n, C.sl_ptr, \
                       C.col, cval, cdinv, mptr, mem, F.sl_ptr, F.col, agg, g);                                  \
  else                                                                                                         \
    hipLaunchKernelGGL((k_galerkin_slots<T, FACT>), dim3(nblk(C.nslots)), dim3(TPB), 0, st, C.n, C.nslices,      \
                       C.sl_ptr, C.col, cval, cdinv, mptr, mem, F.sl_ptr, F.col, agg, g)
  // the coarse levels of a coarse level row by row, from its CSR-ordered copy
  // (also the small ones: 24-71 us against 50-310 us by slot, one thread and
  // one slice bisection each, at 1,000-32,000 rows).  Level 1 of a grid level
  // stored per node block by block, a thread per block in CSR order (row by
  // row it measured 5.2 ms at 256^3, by slot groups 2.31 ms, block by block
  // 1.78 ms: its blocks come from K_i, one load per member).
  const bool rows = g.crp && g.cci && !g.fk && g.fvt != nullptr;
  const dim3 rg(nblk(C.n, TPB / GR_L)), rt(TPB);
  if (rows) {
    hipLaunchKernelGGL((k_galerkin_rows<T>), rg, rt, 0, st, C.n, C.sl_ptr, cval, cdinv, mptr, mem, agg, g);
  } else if (g.fk && g.knm && g.crp && g.cci && g.cvt) {
    // level 1 of the per-node grid level, block by block in CSR order
    hipLaunchKernelGGL((k_galerkin_grid<T>), dim3((unsigned)C.nslices), rt, 0, st, C.n, C.sl_ptr, cval, cdinv, mptr,
                       mem, agg, g);
  } else if (g.fk) {
    LLG_GAL(true);
  } else {
    LLG_GAL(false);
  }
#undef LLG_GAL
}
template void launch_galerkin<double>(hipStream_t, Sell, double*, double*, const int32_t*, const int32_t*, Sell,
                                      const int32_t*, const GalSrc<double>&);
template void launch_galerkin<float>(hipStream_t, Sell, float*, float*, const int32_t*, const int32_t*, Sell,
                                     const int32_t*, const GalSrc<float>&);

template <typename T>
void launch_dense_scatter(hipStream_t st, Sell C, const T* cval, double* dense) {
  const int64_t nd = 3 * C.n;
  launch_fill_f64(st, dense, nd * nd, 0.0);
  if (C.n > 0)
    hipLaunchKernelGGL((k_dense_scatter<T>), dim3(nblk(C.n)), dim3(TPB), 0, st, C.n, C.sl_ptr, C.col,
                       cval, dense);
}
template void launch_dense_scatter<double>(hipStream_t, Sell, const double*, double*);
template void launch_dense_scatter<float>(hipStream_t, Sell, const float*, double*);

void launch_parity_colour(hipStream_t st, int nx, int ny, int nz, int32_t* col) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(k_parity_colour, dim3(nblk(N)), dim3(TPB), 0, st, nx, ny, nz, col);
}
void launch_jp_round(hipStream_t st, int64_t n, const int32_t* grp, const int32_t* gci, const uint64_t* rank,
                     int32_t r, int32_t* cround, int32_t* col, int32_t* pending) {
  if (n > 0)
    hipLaunchKernelGGL(k_jp_round, dim3(nblk(n)), dim3(TPB), 0, st, n, grp, gci, rank, r, cround, col, pending);
}
void launch_colour_max(hipStream_t st, int64_t n, const int32_t* col, int32_t* ncol) {
  if (n > 0) hipLaunchKernelGGL(k_colour_max, dim3(nblk(n)), dim3(TPB), 0, st, n, col, ncol);
}
int64_t colour_blocks(int64_t n) { return (int64_t)nblk(n); }
void launch_colour_hist(hipStream_t st, int64_t n, const int32_t* col, int32_t ncol, int32_t* hist) {
  const int64_t nb = colour_blocks(n);
  hipLaunchKernelGGL(k_colour_hist, dim3((unsigned)nb), dim3(TPB), 0, st, n, col, ncol, nb, hist);
}
void launch_colour_place(hipStream_t st, int64_t n, const int32_t* col, int32_t ncol, const int32_t* hist,
                         int32_t* perm) {
  const int64_t nb = colour_blocks(n);
  hipLaunchKernelGGL(k_colour_place, dim3((unsigned)nb), dim3(TPB), 0, st, n, col, ncol, nb, hist, perm);
}
template <typename T>
void launch_cls_gather(hipStream_t st, int64_t n, const int32_t* rows, Sell A, const T* val, const T* dinv,
                       Sell C, T* cval, T* cdinv, const T* fk) {
  if (n > 0)
    hipLaunchKernelGGL((k_cls_gather<T>), dim3(nblk(n)), dim3(TPB), 0, st, n, rows, A.sl_ptr, A.col, val, dinv,
                       C.sl_ptr, cval, cdinv, fk);
}
template void launch_cls_gather<double>(hipStream_t, int64_t, const int32_t*, Sell, const double*, const double*,
                                        Sell, double*, double*, const double*);
template void launch_cls_gather<float>(hipStream_t, int64_t, const int32_t*, Sell, const float*, const float*,
                                       Sell, float*, float*, const float*);

void launch_gauss_jordan(hipStream_t st, int64_t nd, double* dense, int32_t* piv, int32_t* flag) {
  static int lds_ok = -1;
  const size_t lds_max = (size_t)(GJ_LDS_MAX * GJ_LDS_MAX + 2 * GJ_LDS_MAX) * sizeof(double) +
                         GJ_LDS_MAX * sizeof(int32_t);
  if (lds_ok < 0)
    lds_ok = hipFuncSetAttribute((const void*)k_gauss_jordan_lds,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max) == hipSuccess;
  if (nd <= GJ_LDS_MAX && lds_ok) {
    const size_t lds = (size_t)(nd * nd + 2 * nd) * sizeof(double) + nd * sizeof(int32_t);
    hipLaunchKernelGGL(k_gauss_jordan_lds, dim3(1), dim3(GJ_T), lds, st, nd, dense, piv, flag);
  } else {
    // the pivot column is staged after the pivot indices: callers size the
    // pivot buffer for nd ints plus nd doubles
    double* colk = (double*)(piv + ((nd + 1) & ~(int64_t)1));
    hipLaunchKernelGGL(k_gauss_jordan_global, dim3(1), dim3(GJ_T), 0, st, nd, dense, piv, flag, colk);
  }
}

template <typename T>
void launch_dense_apply(hipStream_t st, int64_t nd, const double* inv, const T* b, T* x) {
  const int wpb = 16;
  const unsigned nb = (unsigned)std::min<int64_t>(ceil_div(nd, wpb), 64);
  hipLaunchKernelGGL((k_dense_apply<T>), dim3(nb), dim3(64 * wpb), nd * sizeof(double), st, nd, inv, b, x);
}
template void launch_dense_apply<double>(hipStream_t, int64_t, const double*, const double*, double*);
template void launch_dense_apply<float>(hipStream_t, int64_t, const double*, const float*, float*);

template <typename T>
void launch_restrict_dense(hipStream_t st, int64_t nc, const int32_t* mptr, const int32_t* mem, const T* r,
                           const double* inv, T* x) {
  if (nc <= 0) return;
  hipLaunchKernelGGL((k_restrict_dense<T>), dim3(1), dim3(1024), 3 * nc * sizeof(double), st, nc, mptr, mem, r, inv,
                     x);
}
template void launch_restrict_dense<double>(hipStream_t, int64_t, const int32_t*, const int32_t*, const double*,
                                            const double*, double*);
template void launch_restrict_dense<float>(hipStream_t, int64_t, const int32_t*, const int32_t*, const float*,
                                           const double*, float*);

}  // namespace llg
