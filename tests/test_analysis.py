"""Host symbolic analysis (no GPU): ordering, fill, supernodes, schedules,
pattern validation, and the exported C ABI."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2110_03636_amd import hkkt, synth
from tests import helpers as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(hkkt.LIB_PATH):
        from paper_2110_03636_amd import build
        build.build()


def _boolean_fill(S):
    n = S.shape[0]
    S = S.copy()
    for k in range(n):
        rows = np.nonzero(S[k + 1:, k])[0] + k + 1
        if rows.size:
            S[np.ix_(rows, rows)] = True
    return np.tril(S)


def _struct(b):
    n = b.pattern.n_x
    Hd = H.dense_H(b)
    J = H.dense_J(b)
    return (np.abs(Hd) + np.eye(n) + np.abs(J).T @ np.abs(J)) != 0


def _cases():
    return [H.tiny_grid_like(120, 1), H.tiny_dense_like(80, 2), H.tiny_grid_like(200, 3),
            H.tiny_dense_like(150, 4), H.tiny_grid_like(900, 5)]


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "hkkt.h")).read()
    declared = set(re.findall(r"\b(hkkt_[a-z0-9_]+)\s*\(", hdr))
    declared = {d for d in declared if not d.endswith("_t")}
    assert declared == set(hkkt.EXPORTS), declared ^ set(hkkt.EXPORTS)
    L = ctypes.CDLL(hkkt.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("k", range(5))
@pytest.mark.parametrize("relax,ordering", [(0, 0), (1, 0), (0, 2), (1, 2)])
def test_supernodal_structure_equals_fill(k, relax, ordering):
    b = _cases()[k]
    n = b.pattern.n_x
    sym = hkkt.Symbolic.from_pattern(b.pattern, relax=relax, ordering=ordering)
    perm = sym.perm()
    assert sorted(perm.tolist()) == list(range(n))
    fill = _boolean_fill(_struct(b)[np.ix_(perm, perm)])
    sn = sym.supernodes()
    st = sym.stats()
    assert st["nnz_L"] == int(fill.sum())
    first, rowptr, rows, parent = sn["first"], sn["rowptr"], sn["rows"], sn["parent"]
    ns = first.size - 1
    col2sn = np.repeat(np.arange(ns), np.diff(first))
    for s in range(ns):
        f, l = first[s], first[s + 1]
        r = rows[rowptr[s]:rowptr[s + 1]]
        assert np.array_equal(r[:l - f], np.arange(f, l))          # own columns first
        assert np.all(np.diff(r) > 0)                                # sorted
        for j in range(f, l):
            true_rows = np.nonzero(fill[:, j])[0]
            panel_rows = r[r >= j]
            assert set(true_rows) <= set(panel_rows)
            if relax == 0:
                assert np.array_equal(true_rows, panel_rows)
        # supernodal etree: parent owns the first row below the block
        if r.size > l - f:
            assert parent[s] == col2sn[r[l - f]]
            pr = set(rows[rowptr[parent[s]]:rowptr[parent[s] + 1]])
            assert set(r[l - f:]) <= pr                              # extend-add target exists
        else:
            assert parent[s] == -1


@pytest.mark.parametrize("k", range(4))
def test_level_schedule_is_topological(k):
    b = _cases()[k]
    sym = hkkt.Symbolic.from_pattern(b.pattern)
    sn = sym.supernodes()
    ns = sn["first"].size - 1
    lev = np.empty(ns, np.int64)
    lp, ls = sn["level_ptr"], sn["level_sn"]
    for l in range(lp.size - 1):
        lev[ls[lp[l]:lp[l + 1]]] = l
    assert sorted(ls.tolist()) == list(range(ns))
    for s in range(ns):
        p = sn["parent"][s]
        if p >= 0:
            assert lev[s] < lev[p]
            assert s < p                                             # postorder numbering


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_amd_fill_close_to_exact_min_degree(seed):
    for b in (H.tiny_grid_like(3000, seed, dx_exp=6.0), H.tiny_dense_like(600, seed)):
        sym = hkkt.Symbolic.from_pattern(b.pattern)
        o = oracle.System.from_batch(b)
        o.factor(o.order_mindeg())
        nnz_md = o.L()[0][-1]
        assert sym.stats()["nnz_L"] <= 1.25 * nnz_md, (sym.stats()["nnz_L"], nnz_md)


def test_given_permutation_is_postordered_equivalent():
    b = H.tiny_grid_like(300, 9)
    o = oracle.System.from_batch(b)
    pmd = o.order_mindeg()
    sym = hkkt.Symbolic.from_pattern(b.pattern, perm=pmd)
    o.factor(pmd)
    # a postorder of the same elimination tree has the same fill
    assert sym.stats()["nnz_L"] == o.L()[0][-1]


def test_natural_ordering_option():
    b = H.tiny_dense_like(50, 10)
    sym = hkkt.Symbolic.from_pattern(b.pattern, ordering=1, relax=0)
    o = oracle.System.from_batch(b)
    o.factor(None)
    assert sym.stats()["nnz_L"] == o.L()[0][-1]


def test_workload_sizes():
    b = synth.workload(1)
    s = hkkt.Symbolic.from_pattern(b.pattern).stats()
    assert s["n_x"] == 1200 and s["m"] == 600 and s["nnz_J"] == 2400
    assert 150_000 < s["nnz_L"] < 240_000


def _pat(b):
    p = b.pattern
    return [p.n_x, p.m, p.H_rowptr.copy(), p.H_col.copy(), p.J_rowptr.copy(), p.J_col.copy()]


def test_pattern_validation_errors():
    b = H.tiny_grid_like(40, 11)
    base = _pat(b)
    bad = []
    a = [x.copy() if isinstance(x, np.ndarray) else x for x in base]
    a[3][1], a[3][2] = a[3][2], a[3][1]                # unsorted H columns somewhere
    bad.append(a)
    a = [x.copy() if isinstance(x, np.ndarray) else x for x in base]
    a[5][0] = 40                                        # J column out of range
    bad.append(a)
    a = [x.copy() if isinstance(x, np.ndarray) else x for x in base]
    a[5][1] = a[5][0]                                   # duplicate J column
    bad.append(a)
    a = [x.copy() if isinstance(x, np.ndarray) else x for x in base]
    a[2][5] = a[2][4] - 1                               # non-monotone row pointers
    bad.append(a)
    a = [x.copy() if isinstance(x, np.ndarray) else x for x in base]
    i = int(np.nonzero(np.diff(a[2]) > 1)[0][0])
    a[3][a[2][i]] = i + 1                               # upper-triangle entry in tril(H)
    bad.append(a)
    for args in bad:
        with pytest.raises(hkkt.HKKTError) as e:
            hkkt.Symbolic(*args)
        assert e.value.code == hkkt.ERR_PATTERN
    with pytest.raises(hkkt.HKKTError) as e:
        hkkt.Symbolic(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(1, np.int64),
                      np.zeros(0, np.int32))
    assert e.value.code == hkkt.ERR_ARG
    with pytest.raises(hkkt.HKKTError) as e:
        hkkt.Symbolic(*base, perm=np.zeros(40, np.int32))
    assert e.value.code == hkkt.ERR_PATTERN


def test_edge_shapes_analyse():
    # m = 0, a diagonal-only H, a single variable
    for n, m in ((1, 0), (5, 0), (6, 3)):
        Hd = np.eye(n)
        J = np.zeros((m, n))
        for i in range(m):
            J[i, 2 * i] = 1.0
        b = H.batch_from_dense(Hd, np.ones(n), J, 0.0, 1.0, np.ones(n), np.ones(m))
        s = hkkt.Symbolic.from_pattern(b.pattern).stats()
        assert s["n_x"] == n and s["nnz_L"] >= n


# ---------------------------------------------------------------------------
# uneven groups: G systems of different sizes analysed as one block-diagonal
# system (one launch per kernel for all members)
# ---------------------------------------------------------------------------
def _group_members():
    return [H.tiny_grid_like(150, 31), H.tiny_dense_like(40, 32), H.tiny_grid_like(90, 33),
            H.tiny_dense_like(64, 34)]


@pytest.mark.parametrize("relax", [0, 1])
def test_group_keeps_members_apart(relax):
    mem = _group_members()
    g = hkkt.GroupPattern([b.pattern for b in mem])
    sym = hkkt.Symbolic.from_group(g, relax=relax)
    perm = sym.perm()
    xo = g.x_off
    # every member's pivots stay in the member's own range
    for k in range(g.G):
        seg = perm[xo[k]:xo[k + 1]]
        assert seg.min() >= xo[k] and seg.max() < xo[k + 1]
    # no supernode spans two members; the combined fill is the members' fill
    sn = sym.supernodes()
    owner = np.searchsorted(xo, np.arange(g.n_x), side="right") - 1
    for s in range(sn["first"].size - 1):
        rows = sn["rows"][sn["rowptr"][s]:sn["rowptr"][s + 1]]
        assert np.unique(owner[rows]).size == 1
    Sg = np.zeros((g.n_x, g.n_x), bool)
    for k, b in enumerate(mem):
        Sg[xo[k]:xo[k + 1], xo[k]:xo[k + 1]] = _struct(b)
    fill = _boolean_fill(Sg[np.ix_(perm, perm)])
    assert sym.stats()["nnz_L"] == int(fill.sum())


def test_group_natural_order_fill_is_sum_of_members():
    mem = _group_members()
    g = hkkt.GroupPattern([b.pattern for b in mem])
    tot = hkkt.Symbolic.from_group(g, ordering=1).stats()["nnz_L"]
    parts = sum(hkkt.Symbolic.from_pattern(b.pattern, ordering=1).stats()["nnz_L"] for b in mem)
    assert tot == parts


def test_group_single_member_equals_plain():
    b = H.tiny_grid_like(200, 35)
    g = hkkt.GroupPattern([b.pattern])
    a = hkkt.Symbolic.from_group(g)
    p = hkkt.Symbolic.from_pattern(b.pattern)
    assert a.stats() == p.stats()
    assert np.array_equal(a.perm(), p.perm())


def test_group_pattern_concat_layout():
    mem = _group_members()[:2]
    g = hkkt.GroupPattern([b.pattern for b in mem])
    assert g.n_x == sum(b.pattern.n_x for b in mem) and g.m == sum(b.pattern.m for b in mem)
    Hd = np.zeros((g.n_x, g.n_x))
    Hv = hkkt.GroupPattern.concat([b.H_val for b in mem])[0]
    rows = np.repeat(np.arange(g.n_x), np.diff(g.H_rowptr))
    Hd[rows, g.H_col] = Hv
    for k, b in enumerate(mem):
        sl = slice(g.x_off[k], g.x_off[k + 1])
        assert np.array_equal(Hd[sl, sl], np.tril(H.dense_H(b)))
    assert np.count_nonzero(Hd) == sum(np.count_nonzero(np.tril(H.dense_H(b))) for b in mem)


def test_group_argument_errors():
    mem = _group_members()[:2]
    g = hkkt.GroupPattern([b.pattern for b in mem])
    with pytest.raises(hkkt.HKKTError) as e:   # offsets do not cover n_x
        hkkt.Symbolic(g.n_x, g.m, g.H_rowptr, g.H_col, g.J_rowptr, g.J_col, x_off=[0, 5, g.n_x - 1],
                      y_off=g.y_off)
    assert e.value.code == hkkt.ERR_ARG
    with pytest.raises(hkkt.HKKTError) as e:   # empty member
        hkkt.Symbolic(g.n_x, g.m, g.H_rowptr, g.H_col, g.J_rowptr, g.J_col, x_off=[0, 0, g.n_x],
                      y_off=g.y_off)
    assert e.value.code == hkkt.ERR_ARG
    # a J row of member 0 reaching into member 1
    Jc = g.J_col.copy()
    r0 = g.J_rowptr[0]
    Jc[r0] = g.x_off[1]
    Jc[:g.J_rowptr[1]] = np.sort(Jc[:g.J_rowptr[1]])
    with pytest.raises(hkkt.HKKTError) as e:
        hkkt.Symbolic(g.n_x, g.m, g.H_rowptr, g.H_col, g.J_rowptr, Jc, x_off=g.x_off, y_off=g.y_off)
    assert e.value.code == hkkt.ERR_PATTERN and "outside its member" in str(e.value)
    # member boundaries that split a member's own coupling
    xo = g.x_off.copy()
    xo[1] -= 1
    with pytest.raises(hkkt.HKKTError) as e:
        hkkt.Symbolic(g.n_x, g.m, g.H_rowptr, g.H_col, g.J_rowptr, g.J_col, x_off=xo, y_off=g.y_off)
    assert e.value.code == hkkt.ERR_PATTERN and "member" in str(e.value)


@pytest.mark.parametrize("k", range(4))
def test_contribution_blocks_never_overlap_while_live(k):
    """The contribution block of supernode s is live from its level to its
    parent's level (inclusive); two blocks live at the same level must not
    share a workspace entry, and the workspace is at most the plain sum."""
    b = _cases()[k]
    sym = hkkt.Symbolic.from_pattern(b.pattern)
    sn = sym.supernodes()
    off = sym.cb_offsets()
    first, rowptr, parent, lp, lsn = sn["first"], sn["rowptr"], sn["parent"], sn["level_ptr"], sn["level_sn"]
    ns = first.size - 1
    lev = np.empty(ns, int)
    for l in range(lp.size - 1):
        lev[lsn[lp[l]:lp[l + 1]]] = l
    nc = (rowptr[1:] - rowptr[:-1]) - (first[1:] - first[:-1])
    size = nc.astype(np.int64) ** 2
    assert off[ns] == sym.stats()["cb_entries"] and off[ns] <= ((size + 63) // 64 * 64).sum()
    has = np.nonzero(size)[0]
    assert (off[has] + size[has] <= off[ns]).all() and (off[has] >= 0).all()
    for l in range(lp.size - 1):
        live = [q for q in has if lev[q] <= l <= lev[parent[q]]]
        iv = sorted((off[q], off[q] + size[q]) for q in live)
        for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
            assert a1 <= b0, (l, a0, a1, b0, b1)


def test_group_contribution_workspace_below_sum():
    """Reuse pays on the dense-like members: the workspace is well below the
    sum of the blocks."""
    mem = [H.tiny_dense_like(300, 36), H.tiny_dense_like(500, 37), H.tiny_grid_like(3000, 38)]
    g = hkkt.GroupPattern([b.pattern for b in mem])
    sym = hkkt.Symbolic.from_group(g)
    sn = sym.supernodes()
    nc = (sn["rowptr"][1:] - sn["rowptr"][:-1]) - (sn["first"][1:] - sn["first"][:-1])
    rounded = ((nc.astype(np.int64) ** 2 + 63) // 64 * 64).sum()
    assert sym.cb_offsets()[-1] < 0.9 * rounded


def test_nested_dissection_orders_every_part():
    """Nested dissection (ordering 2) on a grid-like pattern, a group of
    disconnected members and a dense-like pattern: a permutation, members
    kept apart, and on a connected pattern the last pivots form a separator
    whose removal disconnects the graph of H_gamma."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg
    b = H.tiny_grid_like(5000, 61, dx_exp=6.0)
    sym = hkkt.Symbolic.from_pattern(b.pattern, ordering=2)
    perm = sym.perm()
    assert sorted(perm.tolist()) == list(range(b.pattern.n_x))
    p = b.pattern
    n = p.n_x
    Hs = sp.csr_matrix((np.ones(p.H_col.size), p.H_col, p.H_rowptr), shape=(n, n))
    Js = sp.csr_matrix((np.ones(p.J_col.size), p.J_col, p.J_rowptr), shape=(p.m, n))
    A = ((Hs + Hs.T + Js.T @ Js) != 0).tocsr()
    # the top separator: the pivots of the root supernode's columns
    sn = sym.supernodes()
    root_cols = perm[sn["first"][-2]:sn["first"][-1]]
    keep = np.setdiff1d(np.arange(b.pattern.n_x), root_cols)
    ncomp, _ = cg.connected_components(A[keep][:, keep], directed=False)
    assert ncomp >= 2
    mem = [H.tiny_grid_like(n, 62 + n) for n in (700, 400, 900)]
    g = hkkt.GroupPattern([m.pattern for m in mem])
    gs = hkkt.Symbolic.from_group(g, ordering=2)
    p = gs.perm()
    assert sorted(p.tolist()) == list(range(g.n_x))
    for k in range(3):   # member k's pivots are its own variables, in its range
        assert set(p[g.x_off[k]:g.x_off[k + 1]].tolist()) == set(range(g.x_off[k], g.x_off[k + 1]))
    d = H.tiny_dense_like(400, 63)
    ds = hkkt.Symbolic.from_pattern(d.pattern, ordering=2)
    assert sorted(ds.perm().tolist()) == list(range(400))
