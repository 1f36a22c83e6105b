"""Seeded synthetic KKT inputs.

This module only draws random problem data. It holds none of the solver's
arithmetic and is shared by the CPU oracle (tests) and the GPU library, which
otherwise share no code.

A system is the 2x2 block form of Sec. 3, eq. (linsys2x2), with m_d = 0:

    [ H + D_x + delta*I   J^T ] [x]   [r1]
    [ J                   0   ] [y] = [r2]

H is symmetric; only its lower triangle (diagonal included) is emitted, as a
sorted CSR. J is m x n_x CSR with sorted columns. D_x > 0 is diagonal.

The paper's test matrices (Ipopt/MA57 optimal-power-flow sequences, Table
tab:descr) are not available; these generators stand in for them with the
shapes the paper describes: very sparse, near-planar power-grid-like graphs
(Sec. 1), nnz(K)/N of a few, and a factor density of tens per column
(Table tab:ldlcomp).

Generators
----------
gen_dense_like  : H = B^T B, B with 3 N(0,1) entries per row at random
                  columns; J row i has a unit at column 2i plus 3 N(0,1)
                  entries at other random columns. Fill is heavy (the factor
                  keeps roughly a quarter of its lower triangle), so large
                  dense supernodes dominate.
gen_grid_like   : planar, connected "power grid" graph on random points in
                  the unit square (Euclidean minimum spanning tree plus n/2
                  random Delaunay edges, average degree 3). H is its weighted
                  Laplacian (weights U[0.1,10]) plus 1e-6*I; J row i has a
                  unit at column 2i plus 4..6 N(0,1) entries at the graph
                  neighbours of node 2i (grown breadth first when the node
                  has too few).
gen_rgg_literal : the literal random geometric graph (radius giving average
                  degree 3, which is below the percolation threshold and
                  therefore many tiny components), same H and J recipe.

Seeds: instance b of workload k uses numpy PCG64 with seed 1000*k + b.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Pattern:
    n_x: int
    m: int
    H_rowptr: np.ndarray  # int64 [n_x+1], tril(H) CSR, sorted, diagonal present
    H_col: np.ndarray     # int32
    J_rowptr: np.ndarray  # int64 [m+1]
    J_col: np.ndarray     # int32, sorted per row

    @property
    def nnz_h(self) -> int:
        return int(self.H_rowptr[-1])

    @property
    def nnz_j(self) -> int:
        return int(self.J_rowptr[-1])


@dataclasses.dataclass
class Batch:
    """nb instances on one shared pattern; value arrays are batch-major."""
    pattern: Pattern
    H_val: np.ndarray   # [nb, nnz_h] float64
    J_val: np.ndarray   # [nb, nnz_j]
    D_x: np.ndarray     # [nb, n_x]
    delta: np.ndarray   # [nb]
    gamma: np.ndarray   # [nb]
    r1: np.ndarray      # [nb, n_x]
    r2: np.ndarray      # [nb, m]

    @property
    def nb(self) -> int:
        return int(self.H_val.shape[0])

    def instance(self, b: int) -> "Batch":
        s = slice(b, b + 1)
        return Batch(self.pattern, self.H_val[s], self.J_val[s], self.D_x[s],
                     self.delta[s], self.gamma[s], self.r1[s], self.r2[s])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _loguniform(rng, lo_exp, hi_exp, size):
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size)


def _tril_csr(A: sp.spmatrix):
    """Lower triangle (diagonal kept) as sorted CSR arrays, with the diagonal
    forced present (explicit zero where the matrix has none)."""
    n = A.shape[0]
    L = sp.tril(A, format="coo")
    rows = np.concatenate([L.row, np.arange(n)])
    cols = np.concatenate([L.col, np.arange(n)])
    vals = np.concatenate([L.data, np.zeros(n)])
    T = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))  # sums duplicates
    T.sort_indices()
    return (T.indptr.astype(np.int64), T.indices.astype(np.int32),
            T.data.astype(np.float64))


def _csr_arrays(A: sp.csr_matrix):
    A = A.tocsr()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32),
            A.data.astype(np.float64))


# --------------------------------------------------------------------------
# dense-like generator (H = B^T B, random J)
# --------------------------------------------------------------------------

def _distinct_cols(rng, nrows, ncols, k, forbid=None):
    """k distinct uniform columns per row, optionally excluding forbid[row]."""
    out = np.empty((nrows, k), dtype=np.int64)
    todo = np.arange(nrows)
    while todo.size:
        c = rng.integers(0, ncols, size=(todo.size, k))
        ok = np.ones(todo.size, dtype=bool)
        cs = np.sort(c, axis=1)
        ok &= np.all(cs[:, 1:] != cs[:, :-1], axis=1)
        if forbid is not None:
            ok &= np.all(c != forbid[todo][:, None], axis=1)
        out[todo[ok]] = c[ok]
        todo = todo[~ok]
    return out


def dense_like_pattern_and_values(n_x: int, m: int, rng):
    if m * 2 > n_x:
        raise ValueError("dense_like needs 2*m <= n_x (unit entry at column 2i)")
    bc = _distinct_cols(rng, n_x, n_x, 3)
    bv = rng.standard_normal((n_x, 3))
    B = sp.csr_matrix((bv.ravel(), (np.repeat(np.arange(n_x), 3), bc.ravel())),
                      shape=(n_x, n_x))
    H = (B.T @ B).tocsr()
    Hp, Hc, Hv = _tril_csr(H)
    unit = 2 * np.arange(m)
    jc = _distinct_cols(rng, m, n_x, 3, forbid=unit)
    jv = rng.standard_normal((m, 3))
    rows = np.repeat(np.arange(m), 4)
    cols = np.concatenate([unit[:, None], jc], axis=1).ravel()
    vals = np.concatenate([np.ones((m, 1)), jv], axis=1).ravel()
    J = sp.csr_matrix((vals, (rows, cols)), shape=(m, n_x))
    Jp, Jc, Jv = _csr_arrays(J)
    return Pattern(n_x, m, Hp, Hc, Jp, Jc), Hv, Jv


# --------------------------------------------------------------------------
# grid-like generators (planar graph Laplacian, neighbour J)
# --------------------------------------------------------------------------

def _grid_edges_connected(n: int, rng):
    """EMST of random points plus n/2 random extra Delaunay edges."""
    from scipy.spatial import Delaunay
    from scipy.sparse.csgraph import minimum_spanning_tree
    pts = rng.random((n, 2))
    tri = Delaunay(pts)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    d = np.linalg.norm(pts[e[:, 0]] - pts[e[:, 1]], axis=1)
    G = sp.csr_matrix((d, (e[:, 0], e[:, 1])), shape=(n, n))
    T = minimum_spanning_tree(G).tocoo()
    tree = np.sort(np.stack([T.row, T.col], axis=1), axis=1)
    key_all = e[:, 0].astype(np.int64) * n + e[:, 1]
    key_tree = tree[:, 0].astype(np.int64) * n + tree[:, 1]
    rest = e[~np.isin(key_all, key_tree)]
    extra = rest[rng.choice(rest.shape[0], size=min(n // 2, rest.shape[0]),
                            replace=False)]
    edges = np.concatenate([tree, extra])
    return edges


def _rgg_edges_literal(n: int, rng):
    from scipy.spatial import cKDTree
    pts = rng.random((n, 2))
    r = np.sqrt(3.0 / (np.pi * n))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    return np.sort(pairs.astype(np.int64), axis=1)


def _neighbour_lists(n, edges):
    A = sp.csr_matrix((np.ones(edges.shape[0] * 2),
                       (np.concatenate([edges[:, 0], edges[:, 1]]),
                        np.concatenate([edges[:, 1], edges[:, 0]]))),
                      shape=(n, n))
    A.sort_indices()
    return A.indptr, A.indices


def _grid_J_pattern(n_x, m, edges, rng):
    """Row i: unit entry at 2i plus k in U{4..6} columns taken from the
    breadth-first neighbourhood of node 2i (fewer if its component is
    smaller)."""
    ptr, adj = _neighbour_lists(n_x, edges)
    ks = rng.integers(4, 7, size=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    cols = []
    for i in range(m):
        c0 = 2 * i
        k = int(ks[i])
        seen = {c0}
        frontier = [c0]
        picked = []
        while frontier and len(picked) < k:
            nxt = []
            for u in frontier:
                nb = adj[ptr[u]:ptr[u + 1]]
                nb = [int(v) for v in nb if v not in seen]
                if len(picked) + len(nb) > k:
                    nb = list(rng.permutation(np.array(nb, dtype=np.int64)))
                for v in nb:
                    if len(picked) >= k:
                        break
                    seen.add(v)
                    picked.append(v)
                    nxt.append(v)
                if len(picked) >= k:
                    break
            frontier = nxt
        row = sorted([c0] + picked)
        cols.extend(row)
        rowptr[i + 1] = rowptr[i] + len(row)
    return rowptr, np.asarray(cols, dtype=np.int32)


def grid_like_pattern(n_x: int, m: int, rng, literal: bool = False):
    if m * 2 > n_x:
        raise ValueError("grid_like needs 2*m <= n_x (unit entry at column 2i)")
    edges = _rgg_edges_literal(n_x, rng) if literal else _grid_edges_connected(n_x, rng)
    # tril(H) pattern: diagonal + one entry per edge
    rows = np.concatenate([np.arange(n_x), edges[:, 1]])
    cols = np.concatenate([np.arange(n_x), edges[:, 0]])
    P = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n_x, n_x))
    P.sort_indices()
    Hp = P.indptr.astype(np.int64)
    Hc = P.indices.astype(np.int32)
    Jp, Jc = _grid_J_pattern(n_x, m, edges, rng)
    return Pattern(n_x, m, Hp, Hc, Jp, Jc), edges


def grid_like_values(pat: Pattern, edges: np.ndarray, rng):
    """Weighted Laplacian (w ~ U[0.1,10]) + 1e-6 I in the tril(H) pattern,
    and J values: 1 at column 2i, N(0,1) elsewhere."""
    n = pat.n_x
    w = rng.uniform(0.1, 10.0, size=edges.shape[0])
    deg = np.zeros(n)
    np.add.at(deg, edges[:, 0], w)
    np.add.at(deg, edges[:, 1], w)
    rows = np.concatenate([np.arange(n), edges[:, 1]])
    cols = np.concatenate([np.arange(n), edges[:, 0]])
    vals = np.concatenate([deg + 1e-6, -w])
    Hm = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    Hm.sort_indices()
    assert np.array_equal(Hm.indptr, pat.H_rowptr) and np.array_equal(Hm.indices, pat.H_col)
    Hv = Hm.data.astype(np.float64)
    Jv = rng.standard_normal(pat.nnz_j)
    rows_j = np.repeat(np.arange(pat.m), np.diff(pat.J_rowptr))
    Jv[pat.J_col == 2 * rows_j] = 1.0
    return Hv, Jv


# --------------------------------------------------------------------------
# public entry points
# --------------------------------------------------------------------------

def _rhs_and_diag(rng, n_x, m, dx_exp):
    D = _loguniform(rng, -dx_exp, dx_exp, n_x)
    r1 = rng.standard_normal(n_x)
    r2 = rng.standard_normal(m)
    return D, r1, r2


def _stack(pat, rows):
    H, J, D, de, ga, r1, r2 = zip(*rows)
    return Batch(pat, np.stack(H), np.stack(J), np.stack(D),
                 np.asarray(de, dtype=np.float64), np.asarray(ga, dtype=np.float64),
                 np.stack(r1), np.stack(r2))


def dense_like(n_x: int, m: int | None = None, seed: int = 1000, delta: float = 1e-8,
               gamma: float = 1e4, dx_exp: float = 6.0) -> Batch:
    """One instance of the dense-like generator (its own pattern)."""
    m = n_x // 2 if m is None else m
    rng = _rng(seed)
    pat, Hv, Jv = dense_like_pattern_and_values(n_x, m, rng)
    D, r1, r2 = _rhs_and_diag(rng, n_x, m, dx_exp)
    return _stack(pat, [(Hv, Jv, D, delta, gamma, r1, r2)])


def grid_like(n_x: int, m: int | None = None, nb: int = 1, seed: int = 2000,
              delta: float = 1e-8, gammas=(1e4,), dx_exp: float = 8.0,
              literal: bool = False) -> Batch:
    """nb instances of the grid-like generator on one shared pattern.

    The pattern is drawn from PCG64(seed); instance b draws its values from
    PCG64(seed + b): Laplacian weights, J values, D_x = 10^U(-dx_exp, dx_exp),
    gamma = gammas[b % len(gammas)] and the right-hand side."""
    m = n_x // 2 if m is None else m
    pat, edges = grid_like_pattern(n_x, m, _rng(seed), literal=literal)
    rows = []
    for b in range(nb):
        rng = _rng(seed + b + 1) if b else _rng(seed + 7919)
        Hv, Jv = grid_like_values(pat, edges, rng)
        D, r1, r2 = _rhs_and_diag(rng, n_x, m, dx_exp)
        rows.append((Hv, Jv, D, delta, float(gammas[b % len(gammas)]), r1, r2))
    return _stack(pat, rows)


def workload(k: int, nb: int | None = None, n_x: int | None = None) -> Batch:
    """The five workloads (sizes may be overridden for tests).

    1: dense-like, n_x=1200, m=600, D_x=10^U(-6,6), delta=1e-8, gamma=1e4.
    2: grid-like (connected reading), n_x=500k, m=250k, D_x=10^U(-8,8),
       gamma in {1e4,1e6,1e8} (one instance per gamma).
    3: grid-like, n_x=500k, m=250k, D_x=10^U(-6,6), gamma in {1e4,1e6,1e8}.
    4: grid-like, 256 instances of n_x=20k, m=10k on one pattern,
       D_x=10^U(-8,8), gamma alternating {1e4,1e6}.
    """
    if k == 1:
        return dense_like(n_x or 1200, seed=1000)
    if k == 2:
        return grid_like(n_x or 500_000, nb=nb or 3, seed=2000, gammas=(1e4, 1e6, 1e8),
                         dx_exp=8.0)
    if k == 3:
        return grid_like(n_x or 500_000, nb=nb or 3, seed=3000, gammas=(1e4, 1e6, 1e8),
                         dx_exp=6.0)
    if k == 4:
        return grid_like(n_x or 20_000, nb=nb or 256, seed=4000, gammas=(1e4, 1e6),
                         dx_exp=8.0)
    raise ValueError(f"unknown workload {k}")


def fresh_dx(n_x: int, seed: int, dx_exp: float = 8.0) -> np.ndarray:
    """A new D_x = 10^U(-dx_exp, dx_exp) from PCG64(seed) (the next interior
    iteration of a sequence on an unchanged pattern)."""
    return _loguniform(_rng(seed), -dx_exp, dx_exp, n_x)


def uneven_dense_like(nb: int = 64, lo: int = 2000, hi: int = 50_000, seed: int = 5000,
                      gamma: float = 1e4):
    """nb dense-like instances with n_x log-uniform in [lo, hi], m = n_x/2,
    each on its own pattern (instance b seeded with seed + b)."""
    sizes = np.round(10.0 ** _rng(seed).uniform(np.log10(lo), np.log10(hi), nb)).astype(int)
    sizes -= sizes % 2
    return [dense_like(int(n), seed=seed + 1 + b, gamma=gamma) for b, n in enumerate(sizes)]


@dataclasses.dataclass
class Inequalities:
    """Inequality block of the 4x4 system (Sec. 3): J_d (m_d x n_x, shared
    pattern), per instance J_d values, D_s = S^-1 Z_s (positive diagonal) and
    the right-hand side parts r_s, r_yd."""
    m_d: int
    Jd_rowptr: np.ndarray   # int64 [m_d+1]
    Jd_col: np.ndarray      # int32, sorted per row
    Jd_val: np.ndarray      # [nb, nnz]
    D_s: np.ndarray         # [nb, m_d]
    r_s: np.ndarray         # [nb, m_d]
    r_yd: np.ndarray        # [nb, m_d]


def inequalities(pattern, nb=1, seed=0, frac=0.25, per_row=3, ds_exp=6.0) -> Inequalities:
    """m_d = frac * n_x inequality rows, each with per_row N(0,1) entries at
    distinct random columns; D_s = 10^U(-ds_exp, ds_exp); r_s, r_yd ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    n = pattern.n_x
    md = max(1, int(frac * n))
    k = min(per_row, n)
    cols = np.sort(np.stack([rng.choice(n, size=k, replace=False) for _ in range(md)]), axis=1)
    rowptr = np.arange(md + 1, dtype=np.int64) * k
    colv = cols.reshape(-1).astype(np.int32)
    return Inequalities(md, rowptr, colv, rng.standard_normal((nb, md * k)),
                        10.0 ** rng.uniform(-ds_exp, ds_exp, (nb, md)), rng.standard_normal((nb, md)),
                        rng.standard_normal((nb, md)))
