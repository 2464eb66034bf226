"""Pins for the oracle's pairwise matching and Galerkin coarsening (Sec. 3.1.1).

The oracle's matching is a greedy scan over edges sorted by a strict total
order.  Two independent pure-Python formulations must give the same pairs:
the node-driven description (visit nodes in hashed order, each free node takes
its strongest free unvisited neighbour among the strong ones) and parallel
handshake rounds (each free node proposes its best available edge; mutual
proposals are matched).  SplitMix64 is pinned to its published test vectors.
Galerkin block sums (eq. Ac_direct) are checked against explicit products
(P kron I3)^T A (P kron I3) with scipy.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import llg_inputs as I
from helpers import GOLDEN, MASK, bsr_to_dense, bsr_to_scipy, grid_graph_csr, sm64


def test_splitmix64_published_vectors(orc):
    # the published sequence for seed 1234567
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    for k, e in enumerate(expect):
        x = (1234567 + k * GOLDEN) & MASK
        assert sm64(x) == e
        assert orc.splitmix64(x) == e


def _rank(v, salt):
    return (sm64((((v << 32) | v) ^ salt) & MASK), v)


def _edge_hash(i, j, salt):
    a, b = min(i, j), max(i, j)
    return sm64((((a << 32) | b) ^ salt) & MASK)


def node_visit_matching(G, salt, beta=(1, 4)):
    n = G.shape[0]
    mx = np.zeros(n, np.int64)
    for i in range(n):
        row = G.data[G.indptr[i]:G.indptr[i + 1]]
        mx[i] = row.max() if len(row) else 0
    order = sorted(range(n), key=lambda v: _rank(v, salt))
    visited = np.zeros(n, bool)
    mate = -np.ones(n, np.int64)
    for v in order:
        visited[v] = True
        if mate[v] >= 0:
            continue
        best = None
        for k in range(G.indptr[v], G.indptr[v + 1]):
            j, w = int(G.indices[k]), int(G.data[k])
            if visited[j] or mate[j] >= 0:
                continue
            if beta[1] * w < beta[0] * mx[v]:
                continue
            key = (-w, -_edge_hash(v, j, salt), min(v, j), max(v, j))
            if best is None or key < best[0]:
                best = (key, j)
        if best is not None:
            mate[v] = best[1]
            mate[best[1]] = v
    return mate


def handshake_matching(G, salt, beta=(1, 4)):
    n = G.shape[0]
    mx = np.zeros(n, np.int64)
    for i in range(n):
        row = G.data[G.indptr[i]:G.indptr[i + 1]]
        mx[i] = row.max() if len(row) else 0
    rk = [_rank(v, salt) for v in range(n)]
    mate = -np.ones(n, np.int64)
    rounds = 0
    while True:
        prop = -np.ones(n, np.int64)
        any_prop = False
        for i in range(n):
            if mate[i] >= 0:
                continue
            best = None
            for k in range(G.indptr[i], G.indptr[i + 1]):
                j, w = int(G.indices[k]), int(G.data[k])
                if mate[j] >= 0:
                    continue
                f = i if rk[i] < rk[j] else j
                if beta[1] * w < beta[0] * mx[f]:
                    continue
                key = (rk[f], -w, -_edge_hash(i, j, salt), min(i, j), max(i, j))
                if best is None or key < best[0]:
                    best = (key, j)
            if best is not None:
                prop[i] = best[1]
                any_prop = True
        if not any_prop:
            break
        for i in range(n):
            if prop[i] >= 0 and prop[prop[i]] == i:
                mate[i] = prop[i]
        rounds += 1
        assert rounds < n + 2
    return mate


def random_graph(n, deg, seed, wmax=5):
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n, n * deg)
    c = rng.integers(0, n, n * deg)
    keep = r != c
    r, c = r[keep], c[keep]
    w = rng.integers(1, wmax + 1, len(r))
    G = sp.csr_matrix((np.concatenate([w, w]), (np.concatenate([r, c]), np.concatenate([c, r]))), shape=(n, n))
    G.sum_duplicates()
    G.sort_indices()
    return G


def _graphs():
    yield "grid2d", grid_graph_csr(2, 17)
    yield "grid3d", grid_graph_csr(3, 7)
    yield "rect2d", grid_graph_csr(2, (23, 5))
    for s in range(3):
        yield "random%d" % s, random_graph(150, 3, s)
    # a coarse graph with varied weights: grid after one oracle pass
    import oracle
    G = grid_graph_csr(2, 20)
    agg, _, nc = oracle.match_pass(G.indptr, G.indices, G.data, 0)
    P = sp.csr_matrix((np.ones(400, np.int64), (np.arange(400), agg)), shape=(400, nc))
    C = (P.T @ G @ P).tocsr()
    C.setdiag(0)
    C.eliminate_zeros()
    C.sort_indices()
    yield "coarse2d", C


@pytest.mark.parametrize("salt", [0, 0x1234, (3 << 8) | 1])
def test_matching_three_formulations_agree(orc, salt):
    for name, G in _graphs():
        agg, mate, nc = orc.match_pass(G.indptr, G.indices, G.data, salt)
        m1 = node_visit_matching(G, salt)
        m2 = handshake_matching(G, salt)
        assert np.array_equal(mate, m1), name
        assert np.array_equal(mate, m2), name


def _check_partition(agg, nc, maxsize):
    n = len(agg)
    assert agg.min() >= 0 and agg.max() == nc - 1
    sizes = np.bincount(agg, minlength=nc)
    assert sizes.min() >= 1 and sizes.max() <= maxsize
    # aggregate ids are ordered by their smallest member
    first = np.full(nc, n)
    for i in range(n - 1, -1, -1):
        first[agg[i]] = i
    assert np.all(np.diff(first) > 0)


def test_matching_partition_invariants(orc):
    for name, G in _graphs():
        agg, mate, nc = orc.match_pass(G.indptr, G.indices, G.data, 7)
        _check_partition(agg, nc, 2)
        for i in range(len(agg)):
            if mate[i] >= 0:
                assert mate[mate[i]] == i and agg[i] == agg[mate[i]]
                assert G[i, mate[i]] > 0  # partners are neighbours


def test_hierarchy_aggregates_compose_two_passes(orc):
    dim, n = 2, 40
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=2)
    H = orc.Hierarchy(g, orc.default_opts(), m, 0.1, 1e-3)
    G = grid_graph_csr(dim, n)
    for l in range(H.num_levels - 1):
        L = H.level(l)
        nn = G.shape[0]
        comp = np.arange(nn)
        cur = G
        for p in range(2):
            agg, _, nc = orc.match_pass(cur.indptr, cur.indices, cur.data, (l << 8) | p)
            P = sp.csr_matrix((np.ones(cur.shape[0], np.int64), (np.arange(cur.shape[0]), agg)),
                              shape=(cur.shape[0], nc))
            nxt = (P.T @ cur @ P).tocsr()
            nxt.setdiag(0)
            nxt.eliminate_zeros()
            nxt.sort_indices()
            comp = agg[comp]
            cur = nxt
        assert np.array_equal(L.agg, comp)
        _check_partition(L.agg, comp.max() + 1, 4)
        # the coarse block pattern is the coarse graph plus the diagonal
        nxtL = H.level(l + 1)
        pat = (cur + sp.identity(cur.shape[0], format="csr", dtype=np.int64)).tocsr()
        pat.sort_indices()
        assert np.array_equal(nxtL.rp, pat.indptr) and np.array_equal(nxtL.ci, pat.indices)
        G = cur


def _random_bsr(n, deg, seed, integer):
    rng = np.random.default_rng(seed)
    G = random_graph(n, deg, seed)
    G = (G + sp.identity(n, format="csr", dtype=np.int64)).tocsr()
    G.sort_indices()
    nz = G.nnz
    if integer:
        val = rng.integers(-9, 10, (nz, 3, 3)).astype(np.float64)
    else:
        val = rng.standard_normal((nz, 3, 3))
    return G.indptr.astype(np.int64), G.indices.astype(np.int32), val


@pytest.mark.parametrize("integer", [True, False])
def test_galerkin_block_sums(orc, integer):
    n = 120
    rp, ci, val = _random_bsr(n, 3, 5, integer)
    rng = np.random.default_rng(1)
    agg = rng.integers(0, 37, n).astype(np.int32)
    agg = np.unique(agg, return_inverse=True)[1].astype(np.int32)  # dense ids
    nc = int(agg.max()) + 1
    rpc, cic, vc = orc.galerkin(rp, ci, val, agg, nc)
    A = bsr_to_scipy(rp, ci, val).toarray()
    P = np.zeros((n, nc))
    P[np.arange(n), agg] = 1.0
    P3 = np.kron(P, np.eye(3))
    ref = P3.T @ A @ P3
    got = bsr_to_dense(rpc, cic, vc)
    if integer:
        assert np.array_equal(got, ref)
    else:
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    # pattern = {(agg i, agg j)} over stored blocks, sorted per row
    pat = set()
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            pat.add((agg[i], agg[ci[k]]))
    got_pat = {(I_, int(cic[k])) for I_ in range(nc) for k in range(rpc[I_], rpc[I_ + 1])}
    assert got_pat == pat
    for I_ in range(nc):
        row = cic[rpc[I_]:rpc[I_ + 1]]
        assert list(row) == sorted(row)


def test_hierarchy_levels_are_galerkin_of_scaled_operator(orc):
    dim, n = 3, 9
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=6)
    H = orc.Hierarchy(g, orc.default_opts(max_coarse=10), m, 0.1, 2e-3)
    assert H.num_levels >= 3
    A = H.level(-1)
    D = np.array([A.val[k] for i in range(len(A.rp) - 1) for k in range(A.rp[i], A.rp[i + 1]) if A.ci[k] == i])
    Dinv = np.linalg.inv(D)
    assert np.abs(A.dinv - Dinv).max() <= 1e-13 * np.abs(Dinv).max()
    L0 = H.level(0)
    for i in range(len(A.rp) - 1):
        for k in range(A.rp[i], A.rp[i + 1]):
            if A.ci[k] == i:
                assert np.array_equal(L0.val[k], np.eye(3))
            else:
                ref = Dinv[i] @ A.val[k]
                assert np.abs(L0.val[k] - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    for l in range(H.num_levels - 1):
        Ll, Ln = H.level(l), H.level(l + 1)
        nl, nc = len(Ll.rp) - 1, len(Ln.rp) - 1
        P = np.zeros((nl, nc))
        P[np.arange(nl), Ll.agg] = 1.0
        P3 = np.kron(P, np.eye(3))
        ref = P3.T @ bsr_to_dense(Ll.rp, Ll.ci, Ll.val) @ P3
        got = bsr_to_dense(Ln.rp, Ln.ci, Ln.val)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
        Dl = np.array([Ln.val[k] for i in range(nc) for k in range(Ln.rp[i], Ln.rp[i + 1]) if Ln.ci[k] == i])
        assert np.abs(Ln.dinv - np.linalg.inv(Dl)).max() <= 1e-12 * np.abs(Ln.dinv).max()


def test_coarsening_rate(orc):
    """Two pairwise passes per level shrink the grid by a factor close to
    (slightly less than) four per level."""
    dim, n = 2, 128
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=2)
    H = orc.Hierarchy(g, orc.default_opts(), m, 0.1, 1e-3)
    sizes = [len(H.level(l).rp) - 1 for l in range(H.num_levels)]
    assert sizes[-1] <= 256
    for a, b in zip(sizes, sizes[1:]):
        assert 0.2 < b / a < 0.4


@pytest.mark.parametrize("dim,n", [(2, 45), (3, 14)])
def test_aggregate_levels_alone_equals_hierarchy(orc, dim, n):
    """The graph-only hierarchy (used at sizes where the full oracle
    hierarchy does not fit a test) gives the hierarchy's maps and sizes."""
    g = orc.make_grid(dim, n)
    o = orc.default_opts()
    sizes, maps = orc.aggregate_levels(g, o)
    m = I.smooth_unit_field(dim, n, seed=4)
    H = orc.Hierarchy(g, o, m, 0.1, 1e-3)
    assert len(sizes) == H.num_levels
    for l in range(H.num_levels):
        assert sizes[l] == len(H.level(l).rp) - 1
    for l in range(H.num_levels - 1):
        assert np.array_equal(maps[l], H.level(l).agg)
