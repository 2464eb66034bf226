// llgo.cpp -- FP64 CPU oracle for one semi-implicit BDF1 Landau-Lifshitz step.
//
// TEST INFRASTRUCTURE ONLY (see llgo.h).  Plain, single-threaded, double
// precision, no blocking or fusion: each function follows one passage of the
// paper, cited in its comment, or the reading of it recorded in the design
// notes when the paper is silent.
#include "llgo.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

struct Graph {  // integer-weighted undirected graph, CSR, no self loops
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<int64_t> w;
};

struct Bsr {  // 3x3 block CSR
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;  // 9 per block, row-major
  int64_t nnzb() const { return (int64_t)ci.size(); }
};

struct Level {
  Bsr A;
  std::vector<double> dinv;  // 9 per node: inverse of the diagonal block
  std::vector<int32_t> agg;  // node -> aggregate on the next level (empty at the coarsest)
  int64_t nc = 0;
  std::vector<int32_t> colour;  // multicolour Gauss-Seidel: colour class of every node
  int32_t ncol = 0;
};

struct Hier {
  llgo_grid g;
  llgo_opts o;
  double omega = 0;
  Bsr A;                      // unscaled fine operator
  std::vector<double> dinv0;  // inverse diagonal blocks of A
  std::vector<Level> lv;
  // dense LU of the coarsest matrix
  int64_t nd = 0;
  std::vector<double> lu;
  std::vector<int64_t> piv;
};

// ---------------------------------------------------------------- grid (O1)
// Cell-centred grid, homogeneous Neumann boundary by mirrored ghosts: a missing
// neighbour is replaced by the node itself, so its term cancels and the row of
// the Laplacian is L_ij = 1/h^2 per in-grid neighbour, L_ii = -deg_i/h^2.
int64_t num_nodes(const llgo_grid& g) { return (int64_t)g.n[0] * g.n[1] * g.n[2]; }

// Neighbours of node p in ascending index order (k-1, j-1, i-1, i+1, j+1, k+1).
int neighbours(const llgo_grid& g, int64_t p, int64_t* nb) {
  const int64_t nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
  int c = 0;
  if (k > 0) nb[c++] = p - nx * ny;
  if (j > 0) nb[c++] = p - nx;
  if (i > 0) nb[c++] = p - 1;
  if (i < nx - 1) nb[c++] = p + 1;
  if (j < ny - 1) nb[c++] = p + nx;
  if (k < nz - 1) nb[c++] = p + nx * ny;
  return c;
}

bool grid_ok(const llgo_grid* g) {
  if (!g) return false;
  if (g->dim != 2 && g->dim != 3) return false;
  if (g->n[0] < 2 || g->n[1] < 2) return false;
  if (g->dim == 2 && g->n[2] != 1) return false;
  if (g->dim == 3 && g->n[2] < 2) return false;
  if (!(g->h > 0) || !std::isfinite(g->h)) return false;
  return true;
}

// --------------------------------------------------- block assembly (O3, Sec. 2.1)
// The damped component-wise system of Sec. 2.1 reads, for node i with frozen
// m = (m1, m2, m3), u + dt * M_i (Delta_h u)_i = m^n, where row r of M_i holds
// the coefficients of (Delta_h u_1, Delta_h u_2, Delta_h u_3) in equation r.
void block_M(const double* m, double a, double* M) {
  const double m1 = m[0], m2 = m[1], m3 = m[2];
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

void assemble(const llgo_grid& g, const double* m, double alpha, double dt, Bsr& A) {
  const int64_t N = num_nodes(g);
  const double inv_h2 = 1.0 / (g.h * g.h);
  A.n = N;
  A.rp.assign(N + 1, 0);
  A.ci.clear();
  A.v.clear();
  int64_t nb[6];
  for (int64_t p = 0; p < N; ++p) {
    const int deg = neighbours(g, p, nb);
    double M[9];
    block_M(m + 3 * p, alpha, M);
    const double s_off = dt * inv_h2;
    const double s_diag = dt * (-(double)deg * inv_h2);
    // columns ascending: neighbours below p, p itself, neighbours above p
    std::vector<int64_t> cols(nb, nb + deg);
    cols.push_back(p);
    std::sort(cols.begin(), cols.end());
    for (int64_t q : cols) {
      A.ci.push_back((int32_t)q);
      for (int e = 0; e < 9; ++e) {
        if (q == p) {
          double val = s_diag * M[e];
          if (e == 0 || e == 4 || e == 8) val = 1.0 + val;
          A.v.push_back(val);
        } else {
          A.v.push_back(s_off * M[e]);
        }
      }
    }
    A.rp[p + 1] = (int64_t)A.ci.size();
  }
}

// -------------------------------------------------- 3x3 inverse (O4)
// Inverse of a 3x3 block by the adjugate divided by the determinant.
void inv3(const double* D, double* R) {
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
  for (int k = 0; k < 9; ++k) R[k] = adj[k] * rdet;
}

// C = X * Y for 3x3 blocks, each entry summed over k = 0, 1, 2 in order.
void mul3(const double* X, const double* Y, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = (X[3 * r + 0] * Y[0 * 3 + c] + X[3 * r + 1] * Y[1 * 3 + c]) +
                     X[3 * r + 2] * Y[2 * 3 + c];
}

void diag_inverses(const Bsr& A, std::vector<double>& dinv) {
  dinv.assign(9 * A.n, 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) inv3(&A.v[9 * k], &dinv[9 * i]);
}

// Left scaling: row i of A multiplied by D_i^{-1}; the diagonal block becomes
// the identity and is stored as exactly I.
void left_scale(const Bsr& A, const std::vector<double>& dinv, Bsr& S) {
  S.n = A.n;
  S.rp = A.rp;
  S.ci = A.ci;
  S.v.assign(A.v.size(), 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      if (A.ci[k] == i) {
        for (int e = 0; e < 9; ++e) S.v[9 * k + e] = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
      } else {
        mul3(&dinv[9 * i], &A.v[9 * k], &S.v[9 * k]);
      }
    }
}

// ------------------------------------------------------ aggregation (O5, Sec. 3.1)
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct Edge {
  int64_t w;
  uint64_t rank;  // visiting rank of the endpoint that is visited first
  int32_t first;  // that endpoint
  uint64_t h;     // edge hash
  int32_t i, j;   // i < j
};

// Visiting rank of node v in a pass: a hash of v, ties broken by v.
uint64_t node_rank(int64_t v, uint64_t salt) {
  return splitmix64((((uint64_t)v) << 32 | (uint64_t)v) ^ salt);
}

bool visited_before(uint64_t ra, int64_t a, uint64_t rb, int64_t b) {
  return ra != rb ? ra < rb : a < b;
}

// Strict total order on edges: by the visiting rank of the first-visited
// endpoint, then larger weight, then larger edge hash, then smaller (i, j).
bool edge_before(const Edge& x, const Edge& y) {
  if (x.rank != y.rank) return x.rank < y.rank;
  if (x.first != y.first) return x.first < y.first;
  if (x.w != y.w) return x.w > y.w;
  if (x.h != y.h) return x.h > y.h;
  if (x.i != y.i) return x.i < y.i;
  return x.j < y.j;
}

// One pass of pairwise matching favouring the strongest couplings (Sec. 3.1,
// Sec. 3.1.1).  Nodes are visited in a hashed order; a node that is still
// free when visited pairs with its strongest free neighbour among those whose
// coupling reaches beta times the node's largest coupling, and otherwise stays
// a singleton.  Written here as the equivalent greedy scan over edges sorted by
// (visit rank of the first-visited endpoint, weight, hash), an edge being a
// candidate when it is strong for that first-visited endpoint.
void match_pass(const Graph& G, uint64_t salt, int bnum, int bden, std::vector<int32_t>& agg,
                std::vector<int32_t>& mate, int64_t& nc) {
  const int64_t n = G.n;
  std::vector<int64_t> mx(n, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = G.rp[i]; k < G.rp[i + 1]; ++k) mx[i] = std::max(mx[i], G.w[k]);
  std::vector<Edge> E;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      const int64_t j = G.ci[k];
      if (!(i < j)) continue;
      const int64_t w = G.w[k];
      const uint64_t ri = node_rank(i, salt), rj = node_rank(j, salt);
      const int64_t f = visited_before(ri, i, rj, j) ? i : j;
      if (!((int64_t)bden * w >= (int64_t)bnum * mx[f])) continue;
      const uint64_t key = ((uint64_t)i << 32) | (uint64_t)j;
      E.push_back(Edge{w, f == i ? ri : rj, (int32_t)f, splitmix64(key ^ salt), (int32_t)i, (int32_t)j});
    }
  std::sort(E.begin(), E.end(), edge_before);
  mate.assign(n, -1);
  for (const Edge& e : E)
    if (mate[e.i] < 0 && mate[e.j] < 0) {
      mate[e.i] = e.j;
      mate[e.j] = e.i;
    }
  // numbering: scan nodes in ascending order; an unassigned node opens the
  // next aggregate and its partner joins it
  agg.assign(n, -1);
  nc = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = (int32_t)nc;
    if (mate[i] >= 0) agg[mate[i]] = (int32_t)nc;
    ++nc;
  }
}

// Coarse graph P^T G P with the diagonal dropped; weights are summed.
void coarse_graph(const Graph& G, const std::vector<int32_t>& agg, int64_t nc, Graph& C) {
  std::vector<std::vector<std::pair<int32_t, int64_t>>> rows(nc);
  for (int64_t i = 0; i < G.n; ++i)
    for (int64_t k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      const int32_t I = agg[i], J = agg[G.ci[k]];
      if (I != J) rows[I].push_back({J, G.w[k]});
    }
  C.n = nc;
  C.rp.assign(nc + 1, 0);
  C.ci.clear();
  C.w.clear();
  for (int64_t I = 0; I < nc; ++I) {
    auto& r = rows[I];
    std::sort(r.begin(), r.end());
    for (size_t t = 0; t < r.size(); ++t) {
      if (t > 0 && r[t].first == r[t - 1].first) {
        C.w.back() += r[t].second;
      } else {
        C.ci.push_back(r[t].first);
        C.w.push_back(r[t].second);
      }
    }
    C.rp[I + 1] = (int64_t)C.ci.size();
  }
}

void grid_graph(const llgo_grid& g, Graph& G) {
  const int64_t N = num_nodes(g);
  G.n = N;
  G.rp.assign(N + 1, 0);
  G.ci.clear();
  G.w.clear();
  int64_t nb[6];
  for (int64_t p = 0; p < N; ++p) {
    const int d = neighbours(g, p, nb);
    for (int t = 0; t < d; ++t) {
      G.ci.push_back((int32_t)nb[t]);
      G.w.push_back(1);
    }
    G.rp[p + 1] = (int64_t)G.ci.size();
  }
}

// ------------------------------------------------------ Galerkin (O6, eq. Ac_direct)
// (A_c)_{IJ} = sum over fine rows i in aggregate I (ascending i) and stored
// blocks (i, j) (ascending j) with agg(j) = J of the block a_ij.
void galerkin(const Bsr& A, const std::vector<int32_t>& agg, int64_t nc, Bsr& C) {
  // members of each aggregate in ascending order
  std::vector<std::vector<int64_t>> mem(nc);
  for (int64_t i = 0; i < A.n; ++i) mem[agg[i]].push_back(i);
  C.n = nc;
  C.rp.assign(nc + 1, 0);
  C.ci.clear();
  C.v.clear();
  for (int64_t I = 0; I < nc; ++I) {
    std::vector<int32_t> cols;
    for (int64_t i : mem[I])
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) cols.push_back(agg[A.ci[k]]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    const int64_t base = (int64_t)C.ci.size();
    for (int32_t J : cols) C.ci.push_back(J);
    C.v.resize(9 * C.ci.size(), 0.0);
    for (int64_t i : mem[I])
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int32_t J = agg[A.ci[k]];
        const int64_t s = base + (std::lower_bound(cols.begin(), cols.end(), J) - cols.begin());
        for (int e = 0; e < 9; ++e) C.v[9 * s + e] += A.v[9 * k + e];
      }
    C.rp[I + 1] = (int64_t)C.ci.size();
  }
}

// -------------------------------------------------- dense LU (O8)
// Partial pivoting: the pivot is the first entry of largest magnitude.
void dense_from_bsr(const Bsr& A, std::vector<double>& D) {
  const int64_t m = 3 * A.n;
  D.assign(m * m, 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int64_t j = A.ci[k];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) D[(3 * i + r) * m + 3 * j + c] = A.v[9 * k + 3 * r + c];
    }
}

void lu_factor(int64_t m, std::vector<double>& a, std::vector<int64_t>& piv) {
  piv.assign(m, 0);
  for (int64_t k = 0; k < m; ++k) {
    int64_t p = k;
    double best = std::fabs(a[k * m + k]);
    for (int64_t i = k + 1; i < m; ++i)
      if (std::fabs(a[i * m + k]) > best) {
        best = std::fabs(a[i * m + k]);
        p = i;
      }
    piv[k] = p;
    if (p != k)
      for (int64_t j = 0; j < m; ++j) std::swap(a[k * m + j], a[p * m + j]);
    for (int64_t i = k + 1; i < m; ++i) {
      const double l = a[i * m + k] / a[k * m + k];
      a[i * m + k] = l;
      for (int64_t j = k + 1; j < m; ++j) a[i * m + j] -= l * a[k * m + j];
    }
  }
}

void lu_solve(int64_t m, const std::vector<double>& a, const std::vector<int64_t>& piv, double* x) {
  for (int64_t k = 0; k < m; ++k)
    if (piv[k] != k) std::swap(x[k], x[piv[k]]);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < i; ++j) x[i] -= a[i * m + j] * x[j];
  for (int64_t i = m - 1; i >= 0; --i) {
    for (int64_t j = i + 1; j < m; ++j) x[i] -= a[i * m + j] * x[j];
    x[i] /= a[i * m + i];
  }
}

// ------------------------------------------------------ vectors
void spmv(const Bsr& A, const double* x, double* y) {
  for (int64_t i = 0; i < A.n; ++i) {
    double s[3] = {0, 0, 0};
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const double* b = &A.v[9 * k];
      const double* xj = x + 3 * (int64_t)A.ci[k];
      for (int r = 0; r < 3; ++r) s[r] += b[3 * r] * xj[0] + b[3 * r + 1] * xj[1] + b[3 * r + 2] * xj[2];
    }
    y[3 * i] = s[0];
    y[3 * i + 1] = s[1];
    y[3 * i + 2] = s[2];
  }
}

void apply_blocks(const std::vector<double>& B, int64_t n, const double* x, double* y) {
  for (int64_t i = 0; i < n; ++i) {
    const double* b = &B[9 * i];
    const double* xi = x + 3 * i;
    for (int r = 0; r < 3; ++r) y[3 * i + r] = b[3 * r] * xi[0] + b[3 * r + 1] * xi[1] + b[3 * r + 2] * xi[2];
  }
}

double dot(int64_t m, const double* x, const double* y) {
  double s = 0;
  for (int64_t i = 0; i < m; ++i) s += x[i] * y[i];
  return s;
}

double nrm2(int64_t m, const double* x) { return std::sqrt(dot(m, x, x)); }

// ------------------------------------------------------ multicolour Gauss-Seidel (Sec. 3)
// Colour classes are independent sets of the level's graph, so one block
// Gauss-Seidel sweep taken class by class is the sequential sweep over the rows
// sorted by class.
// Level 0: the 5-/7-point grid graph is bipartite; the class is the parity of
// i + j + k.
void parity_colouring(const llgo_grid& g, std::vector<int32_t>& col, int32_t& ncol) {
  const int64_t nx = g.n[0], ny = g.n[1], N = num_nodes(g);
  col.assign(N, 0);
  for (int64_t p = 0; p < N; ++p) {
    const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
    col[p] = (int32_t)((i + j + k) & 1);
  }
  ncol = 2;
}

// Coarse levels: greedy colouring in priority order.  Nodes are taken by
// ascending (node_rank(v, salt), v); each takes the smallest colour that no
// already coloured neighbour has.
void greedy_colouring(const Graph& G, uint64_t salt, std::vector<int32_t>& col, int32_t& ncol) {
  const int64_t n = G.n;
  std::vector<int64_t> order(n);
  for (int64_t v = 0; v < n; ++v) order[v] = v;
  std::vector<uint64_t> rk(n);
  for (int64_t v = 0; v < n; ++v) rk[v] = node_rank(v, salt);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return rk[a] != rk[b] ? rk[a] < rk[b] : a < b;
  });
  col.assign(n, -1);
  ncol = 0;
  std::vector<char> used;
  for (int64_t v : order) {
    used.assign((size_t)ncol + 1, 0);
    for (int64_t k = G.rp[v]; k < G.rp[v + 1]; ++k) {
      const int32_t c = col[G.ci[k]];
      if (c >= 0) used[c] = 1;
    }
    int32_t c = 0;
    while (used[c]) ++c;
    col[v] = c;
    ncol = std::max(ncol, c + 1);
  }
}

// One block Gauss-Seidel sweep, class by class (ascending classes when
// forward, descending otherwise): every row i of the class takes
// x_i += D_i^{-1} (b_i - sum_j A_ij x_j) with the current x.
void gs_sweep(const Level& L, const double* b, double* x, bool forward) {
  for (int32_t q = 0; q < L.ncol; ++q) {
    const int32_t c = forward ? q : L.ncol - 1 - q;
    for (int64_t i = 0; i < L.A.n; ++i) {
      if (L.colour[i] != c) continue;
      double r[3] = {b[3 * i], b[3 * i + 1], b[3 * i + 2]};
      for (int64_t k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k) {
        const double* blk = &L.A.v[9 * k];
        const double* xj = x + 3 * (int64_t)L.A.ci[k];
        for (int t = 0; t < 3; ++t) r[t] -= blk[3 * t] * xj[0] + blk[3 * t + 1] * xj[1] + blk[3 * t + 2] * xj[2];
      }
      const double* d = &L.dinv[9 * i];
      for (int t = 0; t < 3; ++t) x[3 * i + t] += d[3 * t] * r[0] + d[3 * t + 1] * r[1] + d[3 * t + 2] * r[2];
    }
  }
}

// ------------------------------------------------------ V-cycle / K-cycle (Sec. 3, Sec. 3.1)
// Multigrid = smoothing + coarse grid correction; damped block Jacobi with
// nu_pre / nu_post sweeps, restriction P^T, prolongation P, exact solve at the
// coarsest level.  With kcycle_depth > 0 the coarse residual equation of
// levels 1..depth is solved by two steps of minimal-residual (GCR)
// acceleration preconditioned by the cycle of that level (the K-cycle that
// Sec. 3.1 describes as Krylov acceleration at each level).
void cycle(const Hier& H, size_t l, const double* b, double* x);

void spmv_level(const Hier& H, size_t l, const double* x, double* y) { spmv(H.lv[l].A, x, y); }

// e ~ A_lc^{-1} r: two GCR steps, search directions v1 = B r, v2 = B rho.
void kcycle_correction(const Hier& H, size_t lc, const double* r, double* e) {
  const int64_t m = 3 * H.lv[lc].A.n;
  std::vector<double> v1(m), w1(m), rho(m), v2(m), w2(m), w2p(m);
  cycle(H, lc, r, v1.data());
  spmv_level(H, lc, v1.data(), w1.data());
  const double a1 = dot(m, w1.data(), r) / dot(m, w1.data(), w1.data());
  for (int64_t i = 0; i < m; ++i) rho[i] = r[i] - a1 * w1[i];
  cycle(H, lc, rho.data(), v2.data());
  spmv_level(H, lc, v2.data(), w2.data());
  const double gamma = dot(m, w1.data(), w2.data()) / dot(m, w1.data(), w1.data());
  for (int64_t i = 0; i < m; ++i) w2p[i] = w2[i] - gamma * w1[i];
  const double a2 = dot(m, w2p.data(), rho.data()) / dot(m, w2p.data(), w2p.data());
  // e = a1 v1 + a2 (v2 - gamma v1)
  for (int64_t i = 0; i < m; ++i) e[i] = a1 * v1[i] + a2 * (v2[i] - gamma * v1[i]);
}

void cycle(const Hier& H, size_t l, const double* b, double* x) {
  const Level& L = H.lv[l];
  const int64_t n = L.A.n, m = 3 * n;
  if (l + 1 == H.lv.size()) {
    std::copy(b, b + m, x);
    lu_solve(H.nd, H.lu, H.piv, x);
    return;
  }
  std::vector<double> r(m), t(m);
  std::fill(x, x + m, 0.0);
  const bool gs = H.o.smoother == 1;
  for (int s = 0; s < H.o.nu_pre; ++s) {  // x += omega D^{-1} (b - A x)
    if (gs) {
      gs_sweep(L, b, x, true);
      continue;
    }
    spmv(L.A, x, t.data());
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - t[i];
    apply_blocks(L.dinv, n, r.data(), t.data());
    for (int64_t i = 0; i < m; ++i) x[i] += H.omega * t[i];
  }
  spmv(L.A, x, t.data());
  for (int64_t i = 0; i < m; ++i) r[i] = b[i] - t[i];
  const int64_t nc = L.nc;
  std::vector<double> bc(3 * nc, 0.0), xc(3 * nc, 0.0);
  for (int64_t i = 0; i < n; ++i)  // restriction: P^T r
    for (int c = 0; c < 3; ++c) bc[3 * (int64_t)L.agg[i] + c] += r[3 * i + c];
  const size_t lc = l + 1;
  if (lc + 1 < H.lv.size() && (int)lc <= H.o.kcycle_depth)
    kcycle_correction(H, lc, bc.data(), xc.data());
  else
    cycle(H, lc, bc.data(), xc.data());
  for (int64_t i = 0; i < n; ++i)  // prolongation: x += P e
    for (int c = 0; c < 3; ++c) x[3 * i + c] += xc[3 * (int64_t)L.agg[i] + c];
  for (int s = 0; s < H.o.nu_post; ++s) {
    if (gs) {  // backward classes: the post-sweep mirrors the pre-sweep
      gs_sweep(L, b, x, false);
      continue;
    }
    spmv(L.A, x, t.data());
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - t[i];
    apply_blocks(L.dinv, n, r.data(), t.data());
    for (int64_t i = 0; i < m; ++i) x[i] += H.omega * t[i];
  }
}

// Preconditioner B(v) = V(0, D^{-1} v) when the hierarchy is built on D^{-1} A.
void precond(const Hier& H, const double* v, double* z) {
  const int64_t m = 3 * H.A.n;
  if (H.o.left_scale) {
    std::vector<double> s(m);
    apply_blocks(H.dinv0, H.A.n, v, s.data());
    cycle(H, 0, s.data(), z);
  } else {
    cycle(H, 0, v, z);
  }
}

// ------------------------------------------------------ FGMRES (O10)
// Right-preconditioned flexible GMRES with modified Gram-Schmidt Arnoldi and
// Givens rotations (Saad 1993); it replaces the GCR of Algorithm 1, to which it
// is equivalent for a fixed linear preconditioner.
int fgmres(const Hier& H, const double* b, const double* u0, double* u, llgo_stats* st) {
  const int64_t m = 3 * H.A.n;
  const int R = H.o.restart;
  std::vector<double> V((size_t)(R + 1) * m), Z((size_t)R * m), w(m), r(m);
  std::vector<double> Hm((size_t)(R + 1) * R, 0.0), cs(R), sn(R), g(R + 1);
  std::copy(u0, u0 + m, u);
  const double bnorm = nrm2(m, b);
  const double target = H.o.rtol * bnorm;
  int total = 0, restarts = 0;
  double est = 0, truer = 0;
  spmv(H.A, u, w.data());
  for (int64_t i = 0; i < m; ++i) r[i] = b[i] - w[i];
  double beta = nrm2(m, r.data());
  truer = beta;
  if (bnorm == 0.0 || beta <= target) {
    if (st) *st = llgo_stats{0, 0, (int32_t)H.lv.size(), 1, bnorm > 0 ? beta / bnorm : 0, bnorm > 0 ? beta / bnorm : 0};
    return LLGO_OK;
  }
  bool converged = false;
  while (!converged && total < H.o.max_iters) {
    for (int64_t i = 0; i < m; ++i) V[i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    for (; j < R && total < H.o.max_iters; ++j) {
      double* vj = &V[(size_t)j * m];
      double* zj = &Z[(size_t)j * m];
      if (H.o.krylov == 2)  // unpreconditioned GMRES: z_j = v_j
        std::copy(vj, vj + m, zj);
      else
        precond(H, vj, zj);
      spmv(H.A, zj, w.data());
      const double wnorm0 = nrm2(m, w.data());
      for (int i = 0; i <= j; ++i) {
        const double* vi = &V[(size_t)i * m];
        const double hij = dot(m, vi, w.data());
        Hm[(size_t)i * R + j] = hij;
        for (int64_t q = 0; q < m; ++q) w[q] -= hij * vi[q];
      }
      const double hn = nrm2(m, w.data());
      Hm[(size_t)(j + 1) * R + j] = hn;
      const bool breakdown = hn <= 1e-14 * wnorm0;
      if (!breakdown) {
        double* vn = &V[(size_t)(j + 1) * m];
        for (int64_t q = 0; q < m; ++q) vn[q] = w[q] / hn;
      }
      for (int i = 0; i < j; ++i) {  // previous rotations on column j
        const double a = Hm[(size_t)i * R + j], c = Hm[(size_t)(i + 1) * R + j];
        Hm[(size_t)i * R + j] = cs[i] * a + sn[i] * c;
        Hm[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = Hm[(size_t)j * R + j], c = Hm[(size_t)(j + 1) * R + j];
      const double rho = std::hypot(a, c);
      cs[j] = a / rho;
      sn[j] = c / rho;
      Hm[(size_t)j * R + j] = rho;
      Hm[(size_t)(j + 1) * R + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      est = std::fabs(g[j + 1]);
      if (est <= target || breakdown) {
        ++j;
        break;
      }
    }
    // y = H^{-1} g (upper triangular j x j); u += Z y
    std::vector<double> y(j);
    for (int i = j - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < j; ++k) s -= Hm[(size_t)i * R + k] * y[k];
      y[i] = s / Hm[(size_t)i * R + i];
    }
    for (int k = 0; k < j; ++k) {
      const double* zk = &Z[(size_t)k * m];
      for (int64_t q = 0; q < m; ++q) u[q] += y[k] * zk[q];
    }
    spmv(H.A, u, w.data());
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - w[i];
    beta = nrm2(m, r.data());
    truer = beta;
    converged = beta <= target;
    if (!converged) ++restarts;
  }
  if (st) *st = llgo_stats{total, restarts, (int32_t)H.lv.size(), converged ? 1 : 0, est / bnorm, truer / bnorm};
  return converged ? LLGO_OK : LLGO_ERR_NOT_CONVERGED;
}

// ------------------------------------------------------ GCR (Algorithm 1)
// Preconditioned GCR: z_j from the preconditioner applied to the current
// residual, c_j = A z_j orthogonalized against the previous c_i and
// normalized, residual update along c_j, and the solution assembled once at
// the end from Z (Gamma^{-1} a).  Restarted after `restart` iterations.
int gcr(const Hier& H, const double* b, const double* u0, double* u, llgo_stats* st) {
  const int64_t m = 3 * H.A.n;
  const int R = H.o.restart;
  std::vector<double> Z((size_t)R * m), C((size_t)R * m), r(m), w(m);
  std::vector<double> G((size_t)R * R, 0.0), al(R);
  std::copy(u0, u0 + m, u);
  const double bnorm = nrm2(m, b);
  const double target = H.o.rtol * bnorm;
  spmv(H.A, u, w.data());
  for (int64_t i = 0; i < m; ++i) r[i] = b[i] - w[i];
  double rn = nrm2(m, r.data());
  int total = 0, restarts = 0;
  bool converged = bnorm == 0.0 || rn <= target;
  double est = bnorm > 0 ? rn / bnorm : 0;
  while (!converged && total < H.o.max_iters) {
    int j = 0;
    for (; j < R && total < H.o.max_iters; ++j) {
      double* zj = &Z[(size_t)j * m];
      double* cj = &C[(size_t)j * m];
      precond(H, r.data(), zj);
      spmv(H.A, zj, cj);
      for (int i = 0; i < j; ++i) {
        const double* ci = &C[(size_t)i * m];
        const double gij = dot(m, ci, cj);
        G[(size_t)i * R + j] = gij;
        for (int64_t q = 0; q < m; ++q) cj[q] -= gij * ci[q];
      }
      const double gjj = nrm2(m, cj);
      G[(size_t)j * R + j] = gjj;
      for (int64_t q = 0; q < m; ++q) cj[q] /= gjj;
      al[j] = dot(m, cj, r.data());
      for (int64_t q = 0; q < m; ++q) r[q] -= al[j] * cj[q];
      ++total;
      rn = nrm2(m, r.data());
      est = rn / bnorm;
      if (rn < target) {
        ++j;
        break;
      }
    }
    std::vector<double> y(j);  // Gamma y = a, Gamma upper triangular
    for (int i = j - 1; i >= 0; --i) {
      double s = al[i];
      for (int k = i + 1; k < j; ++k) s -= G[(size_t)i * R + k] * y[k];
      y[i] = s / G[(size_t)i * R + i];
    }
    for (int k = 0; k < j; ++k) {
      const double* zk = &Z[(size_t)k * m];
      for (int64_t q = 0; q < m; ++q) u[q] += y[k] * zk[q];
    }
    spmv(H.A, u, w.data());
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - w[i];
    rn = nrm2(m, r.data());
    converged = rn <= target;
    if (!converged) ++restarts;
  }
  if (st) *st = llgo_stats{total, restarts, (int32_t)H.lv.size(), converged ? 1 : 0, est, bnorm > 0 ? rn / bnorm : 0};
  return converged ? LLGO_OK : LLGO_ERR_NOT_CONVERGED;
}

// ------------------------------------------------------ Krylov baselines
// The unpreconditioned solvers the paper compares against (GMRES above with
// z_j = v_j; BiCGstab; TFQMR), on the unscaled operator A.  Converged when
// the true residual satisfies ||b - A u|| <= rtol ||b||; when the recurrence
// says so and the true residual does not, or on a breakdown, the method
// restarts from the current iterate.  Iterations count matrix-vector pairs
// (two products each).

// Bi-CGSTAB (van der Vorst 1992), shadow vector r^ = r_0 of each start.
int bicgstab(const Hier& H, const double* b, const double* u0, double* u, llgo_stats* st) {
  const int64_t m = 3 * H.A.n;
  std::copy(u0, u0 + m, u);
  std::vector<double> r(m), rh(m), p(m), v(m), s(m), t(m);
  const double bnorm = nrm2(m, b);
  const double target = H.o.rtol * bnorm;
  int total = 0, restarts = 0;
  double rn = 0, est = 0;
  bool converged = false, restarting = false;
  for (;;) {
    spmv(H.A, u, v.data());
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - v[i];
    rn = nrm2(m, r.data());
    if (bnorm == 0.0 || rn <= target) {
      converged = true;
      break;
    }
    if (total >= H.o.max_iters) break;
    if (restarting) ++restarts;
    std::copy(r.begin(), r.end(), rh.begin());
    std::copy(r.begin(), r.end(), p.begin());
    double rho = dot(m, r.data(), rh.data());
    const int before = total;
    while (total < H.o.max_iters) {
      spmv(H.A, p.data(), v.data());
      const double vr = dot(m, v.data(), rh.data());
      const double alpha = rho / vr;
      if (vr == 0.0 || !std::isfinite(alpha)) break;  // breakdown: restart
      for (int64_t i = 0; i < m; ++i) s[i] = r[i] - alpha * v[i];
      spmv(H.A, s.data(), t.data());
      const double tt = dot(m, t.data(), t.data());
      const double omega = tt > 0.0 ? dot(m, t.data(), s.data()) / tt : 0.0;
      if (!std::isfinite(omega)) break;
      for (int64_t i = 0; i < m; ++i) u[i] += alpha * p[i] + omega * s[i];
      for (int64_t i = 0; i < m; ++i) r[i] = s[i] - omega * t[i];
      ++total;
      est = nrm2(m, r.data());
      if (est <= target || omega == 0.0) break;
      const double rho1 = dot(m, r.data(), rh.data());
      const double beta = (rho1 / rho) * (alpha / omega);
      if (rho1 == 0.0 || !std::isfinite(beta)) break;
      rho = rho1;
      for (int64_t i = 0; i < m; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    }
    if (total == before) break;  // no progress from this start
    restarting = true;
  }
  if (st) *st = llgo_stats{total, restarts, (int32_t)H.lv.size(), converged ? 1 : 0, bnorm > 0 ? est / bnorm : 0,
                           bnorm > 0 ? rn / bnorm : 0};
  return converged ? LLGO_OK : LLGO_ERR_NOT_CONVERGED;
}

// TFQMR (Freund 1993), in the two half-steps per iteration of its usual
// statement: the quasi-residual bound tau sqrt(m + 1) decides when the true
// residual is checked.
int tfqmr(const Hier& H, const double* b, const double* u0, double* u, llgo_stats* st) {
  const int64_t m = 3 * H.A.n;
  std::copy(u0, u0 + m, u);
  std::vector<double> r(m), rs(m), w(m), ue(m), uo(m), v(m), d(m), aue(m), auo(m);
  const double bnorm = nrm2(m, b);
  const double target = H.o.rtol * bnorm;
  int total = 0, restarts = 0;
  double rn = 0, est = 0;
  bool converged = false, restarting = false;
  for (;;) {
    spmv(H.A, u, v.data());
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - v[i];
    rn = nrm2(m, r.data());
    if (bnorm == 0.0 || rn <= target) {
      converged = true;
      break;
    }
    if (total >= H.o.max_iters) break;
    if (restarting) ++restarts;
    // w = u_even = r_0, A u_even, v = A u_even, d = 0, tau = |r_0|, theta = eta = 0
    std::copy(r.begin(), r.end(), rs.begin());
    std::copy(r.begin(), r.end(), w.begin());
    std::copy(r.begin(), r.end(), ue.begin());
    spmv(H.A, ue.data(), aue.data());
    std::copy(aue.begin(), aue.end(), v.begin());
    std::fill(d.begin(), d.end(), 0.0);
    double tau = rn, theta = 0.0, eta = 0.0;
    double rho = dot(m, r.data(), rs.data());
    int half = 0;
    const int before = total;
    while (total < H.o.max_iters) {
      const double vr = dot(m, v.data(), rs.data());
      const double alpha = rho / vr;
      if (vr == 0.0 || rho == 0.0 || !std::isfinite(alpha)) break;  // breakdown: restart
      for (int64_t i = 0; i < m; ++i) uo[i] = ue[i] - alpha * v[i];
      spmv(H.A, uo.data(), auo.data());
      bool check = false;
      for (int step = 0; step < 2; ++step) {  // the even half-step uses u_even, the odd one u_odd
        const double* um = step == 0 ? ue.data() : uo.data();
        const double* aum = step == 0 ? aue.data() : auo.data();
        for (int64_t i = 0; i < m; ++i) w[i] -= alpha * aum[i];
        const double f = (theta * theta / alpha) * eta;
        for (int64_t i = 0; i < m; ++i) d[i] = um[i] + f * d[i];
        theta = nrm2(m, w.data()) / tau;
        const double c = 1.0 / std::sqrt(1.0 + theta * theta);
        tau = tau * theta * c;
        eta = c * c * alpha;
        for (int64_t i = 0; i < m; ++i) u[i] += eta * d[i];
        ++half;
        if (tau * std::sqrt((double)half + 1.0) <= target) check = true;
      }
      ++total;
      est = tau;
      if (check) break;
      const double rho1 = dot(m, w.data(), rs.data());
      const double beta = rho1 / rho;
      if (!std::isfinite(beta)) break;
      rho = rho1;
      for (int64_t i = 0; i < m; ++i) ue[i] = w[i] + beta * uo[i];
      spmv(H.A, ue.data(), aue.data());
      for (int64_t i = 0; i < m; ++i) v[i] = aue[i] + beta * (auo[i] + beta * v[i]);
    }
    if (total == before) break;  // no progress from this start
    restarting = true;
  }
  if (st) *st = llgo_stats{total, restarts, (int32_t)H.lv.size(), converged ? 1 : 0, bnorm > 0 ? est / bnorm : 0,
                           bnorm > 0 ? rn / bnorm : 0};
  return converged ? LLGO_OK : LLGO_ERR_NOT_CONVERGED;
}

// ------------------------------------------------------ setup// ------------------------------------------------------ setup
// The aggregation hierarchy of the grid graph (O5, Sec. 3.1.1), which does
// not depend on the field: per level, npass passes of pairwise matching on
// the current integer graph, the composite aggregate map, and the coarse
// graph P^T G P.  Coarsening stops at <= max_coarse nodes, at max_levels, or
// when a level would keep more than `stagnation` of its nodes.  visit(l, G,
// agg, nc) is called for every level l that gets a next level, with G the
// graph of level l.  Returns the number of levels.
template <typename Visit>
int aggregate_levels(const llgo_grid& g, const llgo_opts& o, Visit visit) {
  Graph G;
  grid_graph(g, G);
  for (int l = 0;; ++l) {
    const int64_t N = G.n;
    if (N <= o.max_coarse || l + 1 >= o.max_levels) return l + 1;
    // npass passes of pairwise matching; the composite aggregate map is the
    // composition of the per-pass maps
    std::vector<int32_t> agg(N);
    for (int64_t i = 0; i < N; ++i) agg[i] = (int32_t)i;
    Graph cur = G;
    int64_t nc = N;
    for (int p = 0; p < o.npass; ++p) {
      std::vector<int32_t> a, mate;
      int64_t c = 0;
      const uint64_t salt = o.agg_salt ^ (((uint64_t)l << 8) | (uint64_t)p);
      match_pass(cur, salt, o.beta_num, o.beta_den, a, mate, c);
      Graph nxt;
      coarse_graph(cur, a, c, nxt);
      for (int64_t i = 0; i < N; ++i) agg[i] = a[agg[i]];
      cur = std::move(nxt);
      nc = c;
    }
    if ((double)nc > o.stagnation * (double)N) return l + 1;
    visit(l, G, agg, nc);
    G = std::move(cur);
  }
}

int build(Hier& H, const double* m_tilde, double alpha, double dt) {
  const llgo_grid& g = H.g;
  const llgo_opts& o = H.o;
  H.omega = o.omega > 0 ? o.omega : (g.dim == 2 ? 4.0 / 5.0 : 6.0 / 7.0);
  assemble(g, m_tilde, alpha, dt, H.A);
  diag_inverses(H.A, H.dinv0);
  H.lv.clear();
  H.lv.emplace_back();
  if (o.left_scale)
    left_scale(H.A, H.dinv0, H.lv[0].A);
  else
    H.lv[0].A = H.A;
  aggregate_levels(g, o, [&](int l, const Graph& G, const std::vector<int32_t>& agg, int64_t nc) {
    Level& L = H.lv[l];
    L.agg = agg;
    L.nc = nc;
    if (o.smoother == 1) {
      if (l == 0)
        parity_colouring(g, L.colour, L.ncol);
      else
        greedy_colouring(G, o.agg_salt ^ (((uint64_t)l << 8) | 0x80u), L.colour, L.ncol);
    }
    Level next;
    galerkin(L.A, L.agg, nc, next.A);
    H.lv.push_back(std::move(next));
  });
  for (Level& L : H.lv) diag_inverses(L.A, L.dinv);
  const Level& C = H.lv.back();
  if (C.A.n > o.max_dense) return LLGO_ERR_UNSUPPORTED;
  H.nd = 3 * C.A.n;
  dense_from_bsr(C.A, H.lu);
  lu_factor(H.nd, H.lu, H.piv);
  return LLGO_OK;
}

bool opts_ok(const llgo_opts* o) {
  return o && o->rtol >= 0 && o->restart >= 1 && o->max_iters >= 1 && o->nu_pre >= 0 &&
         o->nu_post >= 0 && o->npass >= 1 && o->beta_num >= 0 && o->beta_den >= 1 &&
         o->max_coarse >= 1 && o->max_levels >= 1 && o->max_dense >= 1 && o->kcycle_depth >= 0 &&
         (o->smoother == 0 || o->smoother == 1) && o->krylov >= 0 && o->krylov <= 4;
}

}  // namespace

extern "C" {

void llgo_default_opts(llgo_opts* o) {
  o->rtol = 1e-10;
  o->restart = 30;
  o->max_iters = 1000;
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
  o->krylov = 0;
  o->kcycle_depth = 0;
  o->smoother = 0;
}

int llgo_aggregate_levels(const llgo_grid* g, const llgo_opts* o, int32_t* levels, int64_t* level_nodes,
                          int32_t* agg, int64_t cap) {
  if (!grid_ok(g) || !opts_ok(o) || !levels || !level_nodes || cap < 0 || (cap > 0 && !agg)) return LLGO_ERR_ARG;
  int64_t off = 0;
  bool fits = true;
  const int L = aggregate_levels(*g, *o, [&](int l, const Graph& G, const std::vector<int32_t>& a, int64_t nc) {
    level_nodes[l] = G.n;
    level_nodes[l + 1] = nc;
    if (off + G.n > cap) fits = false;
    if (fits) std::copy(a.begin(), a.end(), agg + off);
    off += G.n;
  });
  if (L == 1) level_nodes[0] = num_nodes(*g);
  *levels = L;
  return fits ? LLGO_OK : LLGO_ERR_ARG;
}

uint64_t llgo_splitmix64(uint64_t x) { return splitmix64(x); }

int llgo_match_pass(int64_t n, const int64_t* rp, const int32_t* ci, const int64_t* w,
                    uint64_t salt, int32_t beta_num, int32_t beta_den, int32_t* agg,
                    int32_t* mate, int64_t* nc) {
  if (n < 0 || !rp || !agg || !nc || beta_den < 1) return LLGO_ERR_ARG;
  Graph G;
  G.n = n;
  G.rp.assign(rp, rp + n + 1);
  G.ci.assign(ci, ci + rp[n]);
  G.w.assign(w, w + rp[n]);
  std::vector<int32_t> a, mt;
  match_pass(G, salt, beta_num, beta_den, a, mt, *nc);
  std::copy(a.begin(), a.end(), agg);
  if (mate) std::copy(mt.begin(), mt.end(), mate);
  return LLGO_OK;
}

int llgo_galerkin(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                  const int32_t* agg, int64_t nc, int64_t* nnzb_c, int64_t* rp_c, int32_t* ci_c,
                  double* val_c) {
  if (n < 0 || nc < 0 || !rp || !agg || !nnzb_c) return LLGO_ERR_ARG;
  Bsr A;
  A.n = n;
  A.rp.assign(rp, rp + n + 1);
  A.ci.assign(ci, ci + rp[n]);
  A.v.assign(val, val + 9 * rp[n]);
  std::vector<int32_t> ag(agg, agg + n);
  Bsr C;
  galerkin(A, ag, nc, C);
  *nnzb_c = C.nnzb();
  if (rp_c) std::copy(C.rp.begin(), C.rp.end(), rp_c);
  if (ci_c) std::copy(C.ci.begin(), C.ci.end(), ci_c);
  if (val_c) std::copy(C.v.begin(), C.v.end(), val_c);
  return LLGO_OK;
}

int llgo_assemble_nnzb(const llgo_grid* g, int64_t* nnzb) {
  if (!grid_ok(g) || !nnzb) return LLGO_ERR_ARG;
  int64_t s = 0, nb[6];
  for (int64_t p = 0; p < num_nodes(*g); ++p) s += 1 + neighbours(*g, p, nb);
  *nnzb = s;
  return LLGO_OK;
}

int llgo_assemble(const llgo_grid* g, const double* m_tilde, double alpha, double dt, int64_t* rp,
                  int32_t* ci, double* val) {
  if (!grid_ok(g) || !m_tilde || !rp || !ci || !val) return LLGO_ERR_ARG;
  Bsr A;
  assemble(*g, m_tilde, alpha, dt, A);
  std::copy(A.rp.begin(), A.rp.end(), rp);
  std::copy(A.ci.begin(), A.ci.end(), ci);
  std::copy(A.v.begin(), A.v.end(), val);
  return LLGO_OK;
}

void* llgo_setup(const llgo_grid* g, const llgo_opts* o, const double* m_tilde, double alpha,
                 double dt, int* status) {
  int s = LLGO_OK;
  Hier* H = nullptr;
  if (!grid_ok(g) || !opts_ok(o) || !m_tilde || !(dt > 0) || !(alpha >= 0) || !std::isfinite(dt) ||
      !std::isfinite(alpha)) {
    s = LLGO_ERR_ARG;
  } else {
    H = new Hier();
    H->g = *g;
    H->o = *o;
    s = build(*H, m_tilde, alpha, dt);
    if (s != LLGO_OK) {
      delete H;
      H = nullptr;
    }
  }
  if (status) *status = s;
  return H;
}

void llgo_free(void* h) { delete (Hier*)h; }

int llgo_num_levels(void* h) { return h ? (int)((Hier*)h)->lv.size() : LLGO_ERR_ARG; }

static const Bsr* level_bsr(Hier* H, int level) {
  if (level == -1) return &H->A;
  if (level < 0 || level >= (int)H->lv.size()) return nullptr;
  return &H->lv[level].A;
}

int llgo_level_info(void* h, int level, int64_t* n, int64_t* nnzb) {
  if (!h) return LLGO_ERR_ARG;
  const Bsr* A = level_bsr((Hier*)h, level);
  if (!A) return LLGO_ERR_ARG;
  if (n) *n = A->n;
  if (nnzb) *nnzb = A->nnzb();
  return LLGO_OK;
}

int llgo_level_matrix(void* h, int level, int64_t* rp, int32_t* ci, double* val) {
  if (!h) return LLGO_ERR_ARG;
  const Bsr* A = level_bsr((Hier*)h, level);
  if (!A) return LLGO_ERR_ARG;
  if (rp) std::copy(A->rp.begin(), A->rp.end(), rp);
  if (ci) std::copy(A->ci.begin(), A->ci.end(), ci);
  if (val) std::copy(A->v.begin(), A->v.end(), val);
  return LLGO_OK;
}

int llgo_level_dinv(void* h, int level, double* dinv) {
  Hier* H = (Hier*)h;
  if (!H || !dinv) return LLGO_ERR_ARG;
  if (level == -1) {
    std::copy(H->dinv0.begin(), H->dinv0.end(), dinv);
    return LLGO_OK;
  }
  if (level < 0 || level >= (int)H->lv.size()) return LLGO_ERR_ARG;
  std::copy(H->lv[level].dinv.begin(), H->lv[level].dinv.end(), dinv);
  return LLGO_OK;
}

int llgo_level_agg(void* h, int level, int32_t* agg) {
  Hier* H = (Hier*)h;
  if (!H || !agg || level < 0 || level + 1 >= (int)H->lv.size()) return LLGO_ERR_ARG;
  std::copy(H->lv[level].agg.begin(), H->lv[level].agg.end(), agg);
  return LLGO_OK;
}

int llgo_level_colour(void* h, int level, int32_t* colour, int32_t* ncol) {
  Hier* H = (Hier*)h;
  if (!H || level < 0 || level >= (int)H->lv.size() || !colour || !ncol) return LLGO_ERR_ARG;
  const Level& L = H->lv[level];
  if (L.colour.empty()) return LLGO_ERR_ARG;
  std::copy(L.colour.begin(), L.colour.end(), colour);
  *ncol = L.ncol;
  return LLGO_OK;
}

int llgo_apply_A(void* h, const double* x, double* y) {
  if (!h || !x || !y) return LLGO_ERR_ARG;
  spmv(((Hier*)h)->A, x, y);
  return LLGO_OK;
}

int llgo_precond(void* h, const double* v, double* z) {
  if (!h || !v || !z) return LLGO_ERR_ARG;
  precond(*(Hier*)h, v, z);
  return LLGO_OK;
}

int llgo_solve(void* h, const double* b, const double* u0, double* u, llgo_stats* st) {
  if (!h || !b || !u0 || !u) return LLGO_ERR_ARG;
  Hier* H = (Hier*)h;
  switch (H->o.krylov) {
    case 1: return gcr(*H, b, u0, u, st);
    case 3: return bicgstab(*H, b, u0, u, st);
    case 4: return tfqmr(*H, b, u0, u, st);
    default: return fgmres(*H, b, u0, u, st);  // 0: AMG-preconditioned, 2: unpreconditioned
  }
}

// One semi-implicit step (Sec. 2.1): m~ = m^n, b = m^n + dt F, solve, project
// (Sec. 4.3).
}  // extern "C"

namespace {
// Solve the system frozen at m_tilde with time-step factor dt_eff for the
// right-hand side b, starting from m_tilde (x0_is_mn) or zero, then project
// (Sec. 4.3) or copy.
int solve_and_project(const llgo_grid* g, const llgo_opts* o, const double* m_tilde, double alpha,
                      double dt_eff, const std::vector<double>& b, double* m_np1, llgo_stats* st) {
  const int64_t N = num_nodes(*g), m = 3 * N;
  int s = LLGO_OK;
  Hier* H = (Hier*)llgo_setup(g, o, m_tilde, alpha, dt_eff, &s);
  if (!H) return s;
  std::vector<double> u0(m, 0.0), u(m);
  if (o->x0_is_mn) std::copy(m_tilde, m_tilde + m, u0.begin());
  s = llgo_solve(H, b.data(), u0.data(), u.data(), st);
  delete H;
  if (s != LLGO_OK && s != LLGO_ERR_NOT_CONVERGED) return s;
  if (o->project) {
    for (int64_t p = 0; p < N; ++p) {
      const double* x = &u[3 * p];
      const double nrm = std::sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
      if (!(nrm > 0) || !std::isfinite(nrm)) return LLGO_ERR_NONFINITE;
      for (int c = 0; c < 3; ++c) m_np1[3 * p + c] = x[c] / nrm;
    }
  } else {
    std::copy(u.begin(), u.end(), m_np1);
  }
  return s;
}
}  // namespace

extern "C" {

// BDF1 (Sec. 2.1): u + dt m^n x Delta_h u + alpha dt m^n x (m^n x Delta_h u)
// = m^n (+ dt F), m^{n+1} = u / |u|.
int llgo_step(const llgo_grid* g, const llgo_opts* o, const double* m_n, double alpha, double dt,
              const double* F, double* m_np1, llgo_stats* st) {
  if (!grid_ok(g) || !opts_ok(o) || !m_n || !m_np1) return LLGO_ERR_ARG;
  const int64_t N = num_nodes(*g), m = 3 * N;
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(m_n[i])) return LLGO_ERR_NONFINITE;
  std::vector<double> b(m);
  for (int64_t i = 0; i < m; ++i) b[i] = F ? m_n[i] + dt * F[i] : m_n[i];
  return solve_and_project(g, o, m_n, alpha, dt, b, m_np1, st);
}

// BDF2 with second-order extrapolation: (3 u - 4 m^n + m^{n-1}) / (2 dt)
// = -m~ x Delta_h u - alpha m~ x (m~ x Delta_h u) + F, m~ = 2 m^n - m^{n-1}.
// Times 2 dt / 3 this is the BDF1 system frozen at m~ (not of unit length)
// with dt' = 2 dt / 3 and right-hand side (4 m^n - m^{n-1}) / 3 + dt' F.
int llgo_step2(const llgo_grid* g, const llgo_opts* o, const double* m_n, const double* m_nm1, double alpha,
               double dt, const double* F, double* m_np1, llgo_stats* st) {
  if (!grid_ok(g) || !opts_ok(o) || !m_n || !m_nm1 || !m_np1) return LLGO_ERR_ARG;
  const int64_t N = num_nodes(*g), m = 3 * N;
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(m_n[i]) || !std::isfinite(m_nm1[i])) return LLGO_ERR_NONFINITE;
  const double dtp = (2.0 * dt) / 3.0;
  std::vector<double> mt(m), b(m);
  for (int64_t i = 0; i < m; ++i) {
    mt[i] = 2.0 * m_n[i] - m_nm1[i];
    b[i] = (4.0 * m_n[i] - m_nm1[i]) / 3.0;
    if (F) b[i] = b[i] + dtp * F[i];
  }
  return solve_and_project(g, o, mt.data(), alpha, dtp, b, m_np1, st);
}

}  // extern "C"

// ------------------------------------------------------ full field (Sec. 2)
namespace {
// Newell, Williams and Dunlop (1993): the generating functions of the
// diagonal (f) and off-diagonal (g) cell-averaged demagnetizing tensor.
// Terms whose prefactor vanishes are dropped (their limits are zero).
// The tensor is the 27-point second difference of f or g, whose terms grow
// like |r|^3 while the tensor falls like |r|^-3: near the 16-cell switch to
// the dipole the difference cancels about eight digits.  The functions and
// the difference are therefore evaluated in long double (64-bit significand
// on x86-64), which leaves the rounded double result within a few units of
// the last place of the exact cell average.
using ld = long double;
const ld PI_L = 3.141592653589793238462643383279502884L;

ld newell_f(ld x, ld y, ld z) {
  x = std::fabs(x);
  y = std::fabs(y);
  z = std::fabs(z);
  const ld x2 = x * x, y2 = y * y, z2 = z * z;
  const ld R = std::sqrt(x2 + y2 + z2);
  if (R == 0.0L) return 0.0L;
  ld r = 0.0L;
  if (y > 0.0L && z2 != x2) r += 0.5L * y * (z2 - x2) * std::asinh(y / std::sqrt(x2 + z2));
  if (z > 0.0L && y2 != x2) r += 0.5L * z * (y2 - x2) * std::asinh(z / std::sqrt(x2 + y2));
  if (x > 0.0L && y > 0.0L && z > 0.0L) r -= x * y * z * std::atan(y * z / (x * R));
  r += (2.0L * x2 - y2 - z2) * R / 6.0L;
  return r;
}

ld newell_g(ld x, ld y, ld z) {
  const ld sgn = (x > 0 ? 1.0L : (x < 0 ? -1.0L : 0.0L)) * (y > 0 ? 1.0L : (y < 0 ? -1.0L : 0.0L));
  if (sgn == 0.0L) return 0.0L;
  x = std::fabs(x);
  y = std::fabs(y);
  z = std::fabs(z);
  const ld x2 = x * x, y2 = y * y, z2 = z * z;
  const ld R = std::sqrt(x2 + y2 + z2);
  ld r = 0.0L;
  if (z > 0.0L) r += x * y * z * std::asinh(z / std::sqrt(x2 + y2));
  r += (y / 6.0L) * (3.0L * z2 - y2) * std::asinh(x / std::sqrt(y2 + z2));
  r += (x / 6.0L) * (3.0L * z2 - x2) * std::asinh(y / std::sqrt(x2 + z2));
  if (z > 0.0L) {
    r -= (z2 * z / 6.0L) * std::atan(x * y / (z * R));
    r -= (z * y2 / 2.0L) * std::atan(x * z / (y * R));
    r -= (z * x2 / 2.0L) * std::atan(y * z / (x * R));
  }
  r -= x * y * R / 3.0L;
  return sgn * r;
}

// the 27-point second difference (weights 2 at 0, -1 at +-1 per axis) of fun
// around (X, Y, Z) with spacings (a, b, c), over 4 pi a b c
template <typename Fn>
double newell_sum(Fn fun, ld X, ld Y, ld Z, ld a, ld b, ld c) {
  const ld w[3] = {-1.0L, 2.0L, -1.0L};
  ld acc = 0.0L;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        acc += w[i] * w[j] * w[k] * fun(X + (i - 1) * a, Y + (j - 1) * b, Z + (k - 1) * c);
  return (double)(acc / (4.0L * PI_L * a * b * c));
}

void demag(double X, double Y, double Z, double dx, double dy, double dz, double* N) {
  const double far = std::max(std::fabs(X) / dx, std::max(std::fabs(Y) / dy, std::fabs(Z) / dz));
  if (far > 16.0) {
    const ld x = X, y = Y, z = Z, r2 = x * x + y * y + z * z, r = std::sqrt(r2);
    const ld k = -((ld)dx * dy * dz) / (4.0L * PI_L * r2 * r);
    N[0] = (double)(k * (3.0L * x * x / r2 - 1.0L));
    N[1] = (double)(k * (3.0L * y * y / r2 - 1.0L));
    N[2] = (double)(k * (3.0L * z * z / r2 - 1.0L));
    N[3] = (double)(k * 3.0L * x * y / r2);
    N[4] = (double)(k * 3.0L * x * z / r2);
    N[5] = (double)(k * 3.0L * y * z / r2);
    return;
  }
  N[0] = newell_sum(newell_f, X, Y, Z, dx, dy, dz);
  N[1] = newell_sum(newell_f, Y, X, Z, dy, dx, dz);
  N[2] = newell_sum(newell_f, Z, Y, X, dz, dy, dx);
  N[3] = newell_sum(newell_g, X, Y, Z, dx, dy, dz);
  N[4] = newell_sum(newell_g, X, Z, Y, dx, dz, dy);
  N[5] = newell_sum(newell_g, Y, Z, X, dy, dz, dx);
}

// h_i = -sum_j N(x_i - x_j) m_j, the tensor tabulated once per offset
void stray(const llgo_grid& g, const double* m, double* h) {
  const int64_t nx = g.n[0], ny = g.n[1], nz = g.n[2], N = num_nodes(g);
  const int64_t ox = 2 * nx - 1, oy = 2 * ny - 1, oz = 2 * nz - 1;
  std::vector<double> T((size_t)(ox * oy * oz) * 6);
  for (int64_t c = 0; c < oz; ++c)
    for (int64_t b = 0; b < oy; ++b)
      for (int64_t a = 0; a < ox; ++a)
        demag((double)(a - (nx - 1)) * g.h, (double)(b - (ny - 1)) * g.h, (double)(c - (nz - 1)) * g.h, g.h, g.h,
              g.h, &T[6 * (size_t)(a + ox * (b + oy * c))]);
  for (int64_t p = 0; p < N; ++p) {
    const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t q = 0; q < N; ++q) {
      const int64_t i2 = q % nx, j2 = (q / nx) % ny, k2 = q / (nx * ny);
      const double* t = &T[6 * (size_t)((i - i2 + nx - 1) + ox * ((j - j2 + ny - 1) + oy * (k - k2 + nz - 1)))];
      const double* mq = m + 3 * q;
      s[0] += t[0] * mq[0] + t[3] * mq[1] + t[4] * mq[2];
      s[1] += t[3] * mq[0] + t[1] * mq[1] + t[5] * mq[2];
      s[2] += t[4] * mq[0] + t[5] * mq[1] + t[2] * mq[2];
    }
    for (int c = 0; c < 3; ++c) h[3 * p + c] = -s[c];
  }
}
}  // namespace

extern "C" {

void llgo_demag_tensor(double X, double Y, double Z, double dx, double dy, double dz, double* N) {
  demag(X, Y, Z, dx, dy, dz, N);
}

int llgo_stray_field(const llgo_grid* g, const double* m, double* h) {
  if (!grid_ok(g) || !m || !h) return LLGO_ERR_ARG;
  stray(*g, m, h);
  return LLGO_OK;
}

int llgo_stray_field_at(const llgo_grid* g, const double* m, const int64_t* cells, int64_t count, double* h) {
  if (!grid_ok(g) || !m || (count > 0 && (!cells || !h)) || count < 0) return LLGO_ERR_ARG;
  const int64_t nx = g->n[0], ny = g->n[1], N = num_nodes(*g);
  for (int64_t s = 0; s < count; ++s) {
    const int64_t p = cells[s];
    if (p < 0 || p >= N) return LLGO_ERR_ARG;
    const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
    double acc[3] = {0.0, 0.0, 0.0}, t[6];
    for (int64_t q = 0; q < N; ++q) {
      const int64_t i2 = q % nx, j2 = (q / nx) % ny, k2 = q / (nx * ny);
      demag((double)(i - i2) * g->h, (double)(j - j2) * g->h, (double)(k - k2) * g->h, g->h, g->h, g->h, t);
      const double* mq = m + 3 * q;
      acc[0] += t[0] * mq[0] + t[3] * mq[1] + t[4] * mq[2];
      acc[1] += t[3] * mq[0] + t[1] * mq[1] + t[5] * mq[2];
      acc[2] += t[4] * mq[0] + t[5] * mq[1] + t[2] * mq[2];
    }
    for (int c = 0; c < 3; ++c) h[3 * s + c] = -acc[c];
  }
  return LLGO_OK;
}

int llgo_step_field(const llgo_grid* g, const llgo_opts* o, const double* m_n, const double* m_nm1, double alpha,
                    double dt, const llgo_field* fld, const double* F, double* m_np1, llgo_stats* st) {
  if (!grid_ok(g) || !opts_ok(o) || !m_n || !m_np1 || !fld) return LLGO_ERR_ARG;
  const int64_t N = num_nodes(*g), m = 3 * N;
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(m_n[i]) || (m_nm1 && !std::isfinite(m_nm1[i]))) return LLGO_ERR_NONFINITE;
  const double dtp = m_nm1 ? (2.0 * dt) / 3.0 : dt;
  std::vector<double> mt(m), b(m), f(m, 0.0);
  for (int64_t i = 0; i < m; ++i) {
    mt[i] = m_nm1 ? 2.0 * m_n[i] - m_nm1[i] : m_n[i];
    b[i] = m_nm1 ? (4.0 * m_n[i] - m_nm1[i]) / 3.0 : m_n[i];
    if (F) b[i] = b[i] + dtp * F[i];
  }
  if (fld->stray) stray(*g, mt.data(), f.data());
  for (int64_t p = 0; p < N; ++p) {
    const double* x = &mt[3 * p];
    double fp[3] = {f[3 * p] + fld->h_ext[0], (f[3 * p + 1] + fld->h_ext[1]) - fld->q * x[1],
                    (f[3 * p + 2] + fld->h_ext[2]) - fld->q * x[2]};
    // c1 = m~ x f, c2 = m~ x c1, b -= dt' (c1 + alpha c2)
    const double c1[3] = {x[1] * fp[2] - x[2] * fp[1], x[2] * fp[0] - x[0] * fp[2], x[0] * fp[1] - x[1] * fp[0]};
    const double c2[3] = {x[1] * c1[2] - x[2] * c1[1], x[2] * c1[0] - x[0] * c1[2], x[0] * c1[1] - x[1] * c1[0]};
    for (int c = 0; c < 3; ++c) b[3 * p + c] = b[3 * p + c] - dtp * (c1[c] + alpha * c2[c]);
  }
  return solve_and_project(g, o, mt.data(), alpha, dtp * fld->eps, b, m_np1, st);
}

}  // extern "C"
