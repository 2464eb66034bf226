"""Independent constructions used to pin the oracle (numpy / scipy only)."""
import numpy as np
import scipy.sparse as sp

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def sm64(x):
    """SplitMix64 output for state x (Steele, Lea, Flood, OOPSLA 2014)."""
    z = (x + GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def lap1d(n: int, h: float) -> sp.csr_matrix:
    """1D cell-centred Neumann Laplacian: mirrored ghost cells cancel the
    missing neighbour, so the end rows are (-1, 1)/h^2."""
    main = -2.0 * np.ones(n)
    main[0] = main[-1] = -1.0
    off = np.ones(n - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)


def laplacian(dim: int, n, h: float) -> sp.csr_matrix:
    """Tensor-product Laplacian in node order p = i + nx (j + ny k)."""
    if isinstance(n, int):
        n = (n,) * dim
    mats = [lap1d(k, h) for k in n]
    eye = [sp.identity(k, format="csr") for k in n]
    if dim == 2:
        L = (sp.kron(eye[1], mats[0]) + sp.kron(mats[1], eye[0])).tocsr()
    else:
        L = (sp.kron(sp.kron(eye[2], eye[1]), mats[0]) + sp.kron(sp.kron(eye[2], mats[1]), eye[0])
             + sp.kron(sp.kron(mats[2], eye[1]), eye[0])).tocsr()
    L.eliminate_zeros()
    L.sort_indices()
    return L


def apply_scheme(L, m, alpha, dt, u):
    """u + dt m x (L u) + alpha dt m x (m x (L u)), node-wise cross products."""
    Lu = (L @ u)
    mxl = np.cross(m, Lu)
    return u + dt * mxl + alpha * dt * np.cross(m, mxl)


def dense_scheme_matrix(L, m, alpha, dt):
    N = m.shape[0]
    A = np.zeros((3 * N, 3 * N))
    for c in range(3 * N):
        e = np.zeros(3 * N)
        e[c] = 1.0
        A[:, c] = apply_scheme(L, m, alpha, dt, e.reshape(N, 3)).ravel()
    return A


def bsr_to_dense(rp, ci, val, ncols=None):
    n = len(rp) - 1
    ncols = n if ncols is None else ncols
    D = np.zeros((3 * n, 3 * ncols))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            D[3 * i:3 * i + 3, 3 * ci[k]:3 * ci[k] + 3] += val[k]
    return D


def bsr_to_scipy(rp, ci, val, ncols=None):
    n = len(rp) - 1
    ncols = n if ncols is None else ncols
    return sp.bsr_matrix((np.asarray(val), np.asarray(ci), np.asarray(rp)), shape=(3 * n, 3 * ncols))


def grid_graph_csr(dim: int, n):
    """Grid graph with unit weights, CSR with sorted columns."""
    if isinstance(n, int):
        n = (n,) * dim
    N = int(np.prod(n))
    idx = np.arange(N).reshape(tuple(reversed(n)))
    rows, cols = [], []
    for ax in range(dim):
        k = idx.shape[ax]
        a = np.take(idx, range(0, k - 1), axis=ax).ravel()
        b = np.take(idx, range(1, k), axis=ax).ravel()
        rows += [a, b]
        cols += [b, a]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    G = sp.csr_matrix((np.ones(len(r), np.int64), (r, c)), shape=(N, N))
    G.sort_indices()
    return G
