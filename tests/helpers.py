"""Small shared helpers for the tests: dense views of generated systems,
tiny hand-made systems, and the oracle-side acceptance check of a GPU
solution. No solver arithmetic lives here."""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from paper_2110_03636_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def csr_from_dense_lower(Hd):
    """tril(H) CSR with the diagonal always present."""
    n = Hd.shape[0]
    rows, cols, vals = [], [], []
    for i in range(n):
        for j in range(i + 1):
            if Hd[i, j] != 0 or i == j:
                rows.append(i); cols.append(j); vals.append(float(Hd[i, j]))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    return np.cumsum(rp).astype(np.int64), np.asarray(cols, np.int32), np.asarray(vals)


def csr_from_dense(Jd):
    A = sp.csr_matrix(np.asarray(Jd, dtype=np.float64))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)


def batch_from_dense(Hd, Dx, Jd, delta, gamma, r1, r2):
    Hd = np.asarray(Hd, float); Jd = np.asarray(Jd, float).reshape(-1, Hd.shape[0])
    Hp, Hc, Hv = csr_from_dense_lower(Hd)
    if Jd.shape[0]:
        Jp, Jc, Jv = csr_from_dense(Jd)
    else:
        Jp, Jc, Jv = np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0)
    pat = synth.Pattern(Hd.shape[0], Jd.shape[0], Hp, Hc, Jp, Jc)
    return synth.Batch(pat, Hv[None], Jv[None], np.asarray(Dx, float)[None],
                       np.array([delta], float), np.array([gamma], float),
                       np.asarray(r1, float)[None], np.asarray(r2, float).reshape(1, -1))


def dense_H(batch, b=0):
    p = batch.pattern
    L = sp.csr_matrix((batch.H_val[b], p.H_col, p.H_rowptr), shape=(p.n_x, p.n_x)).toarray()
    return L + np.tril(L, -1).T


def dense_J(batch, b=0):
    p = batch.pattern
    return sp.csr_matrix((batch.J_val[b], p.J_col, p.J_rowptr), shape=(p.m, p.n_x)).toarray()


def dense_K(batch, b=0):
    p = batch.pattern
    n, m = p.n_x, p.m
    A = dense_H(batch, b) + np.diag(batch.D_x[b] + batch.delta[b])
    J = dense_J(batch, b)
    K = np.zeros((n + m, n + m))
    K[:n, :n] = A
    K[n:, :n] = J
    K[:n, n:] = J.T
    return K


def dense_Hgamma(batch, b=0):
    J = dense_J(batch, b)
    return dense_H(batch, b) + np.diag(batch.D_x[b] + batch.delta[b]) + batch.gamma[b] * (J.T @ J)


def csc_to_dense_lower(cp, ri, v, n):
    return sp.csc_matrix((v, ri, cp), shape=(n, n)).toarray()


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def frac_array(lst):
    return np.array([float(Fraction(s)) for s in lst])


def tiny_dense_like(n_x, seed, gamma=1e4, dx_exp=1.0, delta=1e-8):
    b = synth.dense_like(n_x, seed=seed, gamma=gamma, dx_exp=dx_exp, delta=delta)
    return b


def tiny_grid_like(n_x, seed, gamma=1e4, dx_exp=1.0, nb=1):
    return synth.grid_like(n_x, nb=nb, seed=seed, gammas=(gamma,), dx_exp=dx_exp)


def with_gamma(batch, gamma):
    import dataclasses
    return dataclasses.replace(batch, gamma=np.full_like(batch.gamma, gamma))


def rounded_solution_rr(o, r1, r2):
    """RR of the exact solution rounded to FP64, computed by the oracle
    (solve, then refinement with a double-double iterate): the least RR an
    FP64 z can be expected to reach."""
    o.factor(o.order_mindeg())
    xo, yo, io = o.solve(r1, r2)
    xr, yr, hist = o.refine_dd(r1, r2, xo, yo)
    assert hist[-1] < 1e-20, hist
    return o.metrics(r1, r2, xr, yr)[0]


def check_gpu_solution(o, r1, r2, x, y, info, tol):
    """Accept a GPU solution by the oracle's compensated residual: status 0
    and RR <= tol; or, only where the exact solution rounded to FP64 itself
    misses tol, status NOT_CONVERGED (3) with RR within 2x of that rounded
    solution's. The library's own RR (also compensated) must equal the
    oracle's to 1e-8 relative. Returns (rr, rr of the rounded solution or
    None)."""
    rr, be, fl = o.metrics(r1, r2, x, y)
    assert abs(info["rr"] - rr) <= 1e-8 * rr, (info["rr"], rr)
    if info["status"] == 0:
        assert rr <= tol, (rr, fl, info)
        return rr, None
    assert info["status"] == 3, info
    rr_round = rounded_solution_rr(o, r1, r2)
    assert rr_round > tol and rr <= 2 * rr_round, (rr, rr_round, fl)
    return rr, rr_round


def cg_count_tol(oracle_per_pass, gpu_passes):
    """Bound on |GPU CG iterations - oracle CG iterations| for one solve.
    Both run the same unpreconditioned CG with the same stopping rule, but
    their triangular solves and dot products round in different orders, and
    in floating point the iteration at which the recurrence residual crosses
    the tolerance shifts with the rounding (loss of orthogonality delays
    convergence by an amount that depends on the rounding errors, more so the
    longer the run). Per pass: 2 iterations, or 3% of the oracle's count for
    that pass when larger; 2 more for every pass the GPU runs beyond the
    oracle's, and 2 overall."""
    tol = sum(max(2, int(np.ceil(0.03 * k))) for k in oracle_per_pass)
    return tol + 2 + 2 * max(0, gpu_passes - len(oracle_per_pass))


def dense_Jd(ineq, n, b=0):
    Jd = np.zeros((ineq.m_d, n))
    rows = np.repeat(np.arange(ineq.m_d), np.diff(ineq.Jd_rowptr))
    Jd[rows, ineq.Jd_col] = ineq.Jd_val[b]
    return Jd


def dense_K4(batch, ineq, b=0):
    """K4 = [H + D_x + delta I, 0, J^T, J_d^T; 0, D_s, 0, -I; J, 0, 0, 0;
    J_d, -I, 0, 0] (Sec. 3, eq. linsys4x4 with delta in the (1,1) block)."""
    n, m, md = batch.pattern.n_x, batch.pattern.m, ineq.m_d
    Hd = dense_H(batch, b) + np.diag(batch.D_x[b] + batch.delta[b])
    J = dense_J(batch, b)
    Jd = dense_Jd(ineq, n, b)
    N = n + md + m + md
    K = np.zeros((N, N))
    o1, o2, o3 = n, n + md, n + md + m
    K[:n, :n] = Hd
    K[:n, o2:o3] = J.T
    K[:n, o3:] = Jd.T
    K[o1:o2, o1:o2] = np.diag(ineq.D_s[b])
    K[o1:o2, o3:] = -np.eye(md)
    K[o2:o3, :n] = J
    K[o3:, :n] = Jd
    K[o3:, o1:o2] = -np.eye(md)
    return K
