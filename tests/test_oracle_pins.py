"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: dense LAPACK
factorizations and solves, eigenvalue counts, closed forms (Theorem 1,
Theorem 4, the CG bound of Sec. 5.1), hand-solved systems, and invariances of
the exact solution. A plausible mistake in the oracle (a dropped gamma*J^T J
term, a transposed J, a wrong sign in the Schur right-hand side, a missing
delta) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2110_03636_amd import synth
from tests import helpers as H


def _sys(batch, b=0):
    return oracle.System.from_batch(batch, b)


# --------------------------------------------------------------------------
# assembly: H_gamma = H + D_x + delta I + gamma J^T J   (eq. eq:gamma)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gen,seed", [("dense", 11), ("grid", 12), ("dense", 13)])
def test_assembly_equals_dense_definition(gen, seed):
    b = H.tiny_dense_like(40, seed) if gen == "dense" else H.tiny_grid_like(50, seed)
    s = _sys(b)
    cp, ri, v = s.hgamma()
    got = H.csc_to_dense_lower(cp, ri, v, b.pattern.n_x)
    want = np.tril(H.dense_Hgamma(b))
    assert np.all(ri >= np.repeat(np.arange(b.pattern.n_x), np.diff(cp)))  # lower only
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-14 * np.abs(want).max())


# --------------------------------------------------------------------------
# Cholesky P H_gamma P^T = L L^T (left-looking, no pivoting, Sec. 3)
# --------------------------------------------------------------------------

def test_cholesky_equals_lapack_workload1():
    b = synth.workload(1)
    s = _sys(b)
    perm = s.order_mindeg()
    assert sorted(perm.tolist()) == list(range(b.pattern.n_x))
    st, fc = s.factor(perm)
    assert st == 0 and fc == -1
    cp, ri, v = s.L()
    n = b.pattern.n_x
    Ld = H.csc_to_dense_lower(cp, ri, v, n)
    A = H.dense_Hgamma(b)[np.ix_(perm, perm)]
    Lref = np.linalg.cholesky(A)
    colnorm = np.linalg.norm(Lref, axis=0)
    err = np.abs(Ld - Lref).max(axis=0) / colnorm
    assert err.max() < 1e-10, err.max()
    # the stored pattern is exactly the structural fill of the permuted matrix
    assert np.all(np.abs(Lref[np.abs(Ld) == 0]) < 1e-9 * colnorm.max())


def _boolean_fill(A):
    """Structural Cholesky fill by dense boolean elimination."""
    n = A.shape[0]
    S = A != 0
    for k in range(n):
        rows = np.nonzero(S[k + 1:, k])[0] + k + 1
        if rows.size:
            S[np.ix_(rows, rows)] = True
    return np.tril(S)


@pytest.mark.parametrize("seed", [1, 2])
def test_factor_pattern_equals_boolean_fill(seed):
    b = H.tiny_grid_like(60, seed)
    s = _sys(b)
    perm = s.order_mindeg()
    s.factor(perm)
    cp, ri, v = s.L()
    n = b.pattern.n_x
    got = np.zeros((n, n), bool)
    for j in range(n):
        got[ri[cp[j]:cp[j + 1]], j] = True
    A = H.dense_Hgamma(b)[np.ix_(perm, perm)]
    # structural pattern: the union of the patterns of H, D, J^T J
    Pt = (np.abs(H.dense_H(b)) + np.eye(n) + np.abs(H.dense_J(b)).T @ np.abs(H.dense_J(b))) != 0
    want = _boolean_fill(Pt[np.ix_(perm, perm)].astype(float))
    assert np.array_equal(got, want)


def test_cholesky_reconstruction_grid():
    b = H.tiny_grid_like(400, 5, dx_exp=8.0)
    s = _sys(b)
    perm = s.order_mindeg()
    assert s.factor(perm)[0] == 0
    cp, ri, v = s.L()
    n = b.pattern.n_x
    Ld = H.csc_to_dense_lower(cp, ri, v, n)
    A = H.dense_Hgamma(b)[np.ix_(perm, perm)]
    assert np.linalg.norm(A - Ld @ Ld.T) / np.linalg.norm(A) < 1e-13


def test_natural_order_equals_lapack():
    b = H.tiny_dense_like(30, 3)
    s = _sys(b)
    assert s.factor(None)[0] == 0
    cp, ri, v = s.L()
    Ld = H.csc_to_dense_lower(cp, ri, v, 30)
    np.testing.assert_allclose(Ld, np.linalg.cholesky(H.dense_Hgamma(b)), rtol=0,
                               atol=1e-12 * np.abs(Ld).max())


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_not_spd_column_equals_lapack(seed):
    # indefinite H: one strongly negative diagonal entry in H (not PD on null(J)
    # when gamma is small), the first failing pivot in elimination order must be
    # the one LAPACK's potrf reports on the same permuted dense matrix.
    b = H.tiny_grid_like(50, seed, gamma=1.0)
    rng = np.random.default_rng(seed)
    victim = int(rng.integers(0, 50))
    p = b.pattern
    diag_pos = [k for k in range(p.H_rowptr[victim], p.H_rowptr[victim + 1]) if p.H_col[k] == victim][0]
    b.H_val[0, diag_pos] -= 1e4
    s = _sys(b)
    perm = s.order_mindeg()
    st, fc = s.factor(perm)
    A = H.dense_Hgamma(b)[np.ix_(perm, perm)]
    _, info = sla.lapack.dpotrf(A, lower=1)
    assert info > 0 and st == 1
    assert fc == perm[info - 1]


# --------------------------------------------------------------------------
# triangular solves: x = H_gamma^{-1} b
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gen", ["dense", "grid"])
def test_hsolve_backward_error(gen):
    b = synth.workload(1) if gen == "dense" else H.tiny_grid_like(2000, 4, dx_exp=8.0)
    s = _sys(b)
    s.factor(s.order_mindeg())
    rng = np.random.default_rng(0)
    rhs = rng.standard_normal(b.pattern.n_x)
    x = s.hsolve(rhs)
    A = H.dense_Hgamma(b)
    be = np.linalg.norm(A @ x - rhs) / (np.linalg.norm(A, np.inf) * np.linalg.norm(x) + np.linalg.norm(rhs))
    assert be < 1e-15


def test_hsolve_equals_cho_solve_tiny():
    b = H.tiny_dense_like(40, 7)
    s = _sys(b)
    s.factor(s.order_mindeg())
    rhs = np.random.default_rng(1).standard_normal(40)
    want = sla.cho_solve(sla.cho_factor(H.dense_Hgamma(b)), rhs)
    np.testing.assert_allclose(s.hsolve(rhs), want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


# --------------------------------------------------------------------------
# the full hybrid solve (Algorithm 1 solve phase + refinement)
# --------------------------------------------------------------------------

def test_golden_hand_solved():
    g = H.load_golden("hand_kkt.json")
    for c in g["cases"]:
        b = H.batch_from_dense(c["H_dense"], c["D_x"], c["J_dense"], c["delta"], 1e2,
                               c["r1"], c["r2"])
        s = _sys(b)
        s.factor(None)
        x, y, info = s.solve(b.r1[0], b.r2[0])
        np.testing.assert_allclose(x, H.frac_array(c["x"]), atol=1e-13)
        np.testing.assert_allclose(y, H.frac_array(c["y"]), atol=1e-13)
        assert info["status"] == 0


def test_golden_schur_closed_form():
    c = H.load_golden("hand_kkt.json")["cases"][0]
    for g, Sstr in zip(c["schur"]["gammas"], c["schur"]["S"]):
        b = H.batch_from_dense(c["H_dense"], c["D_x"], c["J_dense"], c["delta"], g, c["r1"], c["r2"])
        s = _sys(b)
        s.factor(None)
        J = np.asarray(c["J_dense"], float)
        S = J @ s.hsolve(J[0])
        np.testing.assert_allclose(S, H.frac_array([Sstr]), rtol=1e-14)


@pytest.mark.parametrize("gen,seed", [("dense", 31), ("grid", 32), ("dense", 33), ("grid", 34)])
def test_hybrid_equals_dense_solve_and_ldl(gen, seed):
    b = H.tiny_dense_like(40, seed) if gen == "dense" else H.tiny_grid_like(60, seed)
    s = _sys(b)
    s.factor(s.order_mindeg())
    x, y, info = s.solve(b.r1[0], b.r2[0])
    K = H.dense_K(b)
    r = np.concatenate([b.r1[0], b.r2[0]])
    z_np = np.linalg.solve(K, r)
    lu, d, pp = sla.ldl(K, lower=True)
    # solve with the Bunch-Kaufman factors: K = lu d lu^T
    z_ldl = np.linalg.solve(lu.T, np.linalg.solve(d, np.linalg.solve(lu, r)))
    kap = np.linalg.cond(K)
    z = np.concatenate([x, y])
    tol = max(1e-11, kap * 1e-15)
    assert np.linalg.norm(z - z_np) / np.linalg.norm(z_np) < tol
    assert np.linalg.norm(z - z_ldl) / np.linalg.norm(z_ldl) < tol
    assert info["rr"] <= 1e-10


@pytest.mark.parametrize("seed", [41, 42])
def test_gamma_invariance(seed):
    # eq. linsys2x2mod is an exact transform: z does not depend on gamma;
    # gamma = 0 is plain Uzawa, valid because D_x > 0 makes H_delta SPD.
    base = H.tiny_dense_like(40, seed)
    zs = []
    for g in (0.0, 1.0, 1e2, 1e4):
        b = H.with_gamma(base, g)
        s = _sys(b)
        s.factor(s.order_mindeg())
        x, y, info = s.solve(b.r1[0], b.r2[0])
        assert info["rr"] <= 1e-10
        zs.append(np.concatenate([x, y]))
    for z in zs[1:]:
        assert np.linalg.norm(z - zs[0]) / np.linalg.norm(zs[0]) < 1e-8


def test_m_zero_is_plain_cholesky_solve():
    rng = np.random.default_rng(3)
    n = 20
    B = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.2)
    Hd = B.T @ B
    Dx = 10 ** rng.uniform(-1, 1, n)
    r1 = rng.standard_normal(n)
    b = H.batch_from_dense(Hd, Dx, np.zeros((0, n)), 1e-8, 1e4, r1, np.zeros(0))
    s = _sys(b)
    s.factor(s.order_mindeg())
    x, y, info = s.solve(b.r1[0], b.r2[0])
    want = np.linalg.solve(Hd + np.diag(Dx + 1e-8), r1)
    np.testing.assert_allclose(x, want, rtol=1e-11)
    assert y.size == 0 and info["inertia"] == (n, 0, 0)


def test_J_identity_block_closed_form():
    # J = [I_m 0]: x1 = r2; A22 x2 = r1b - A21 r2; y = r1a - A11 r2 - A12 x2
    rng = np.random.default_rng(4)
    n, m = 12, 5
    B = rng.standard_normal((n, n))
    Hd = B.T @ B / n
    Dx = 10 ** rng.uniform(-1, 1, n)
    J = np.hstack([np.eye(m), np.zeros((m, n - m))])
    r1 = rng.standard_normal(n)
    r2 = rng.standard_normal(m)
    b = H.batch_from_dense(Hd, Dx, J, 0.0, 1e3, r1, r2)
    s = _sys(b)
    s.factor(None)
    x, y, info = s.solve(r1, r2)
    A = Hd + np.diag(Dx)
    x1 = r2
    x2 = np.linalg.solve(A[m:, m:], r1[m:] - A[m:, :m] @ r2)
    yy = r1[:m] - A[:m, :m] @ r2 - A[:m, m:] @ x2
    np.testing.assert_allclose(x, np.concatenate([x1, x2]), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(y, yy, rtol=1e-9, atol=1e-11)


# --------------------------------------------------------------------------
# Theorem 4: eig(gamma S) = 1/(1 + eig(C)), C = (1/gamma)(J Htilde^{-1} J^T)^{-1}
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gamma", [1e2, 1e4, 1e6])
def test_theorem4_spectrum(gamma):
    base = H.tiny_dense_like(40, 51)
    b = H.with_gamma(base, gamma)
    s = _sys(b)
    s.factor(s.order_mindeg())
    J = H.dense_J(b)
    S = np.stack([J @ s.hsolve(J[i]) for i in range(J.shape[0])], axis=1)
    Ht = H.dense_H(b) + np.diag(b.D_x[0] + b.delta[0])
    Cm = np.linalg.inv(J @ np.linalg.solve(Ht, J.T)) / gamma
    want = np.sort(1.0 / (1.0 + np.linalg.eigvals(Cm).real))
    got = np.sort(np.linalg.eigvalsh(gamma * (S + S.T) / 2))
    np.testing.assert_allclose(got, want, rtol=1e-8)
    # I - C is the first-order term of eq. (S3)
    if gamma >= 1e4:
        assert np.abs(got - 1.0).max() < 2 * np.abs(np.linalg.eigvals(Cm)).max() + 1e-12


# --------------------------------------------------------------------------
# CG behaviour: the bound of Sec. 5.1 and counts falling with gamma
# --------------------------------------------------------------------------

def test_cg_iterations_within_bound_workload1():
    b = synth.workload(1)
    s = _sys(b)
    s.factor(s.order_mindeg())
    x, y, it, brk = s.hybrid_once(b.r1[0], b.r2[0])
    assert not brk
    Hg = H.dense_Hgamma(b)
    J = H.dense_J(b)
    S = J @ np.linalg.solve(Hg, J.T)
    ev = np.linalg.eigvalsh((S + S.T) / 2)
    kap = ev[-1] / ev[0]
    rho = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    # ||r_k||/||r_0|| <= sqrt(kappa) * ||e_k||_A/||e_0||_A <= 2 sqrt(kappa) rho^k
    k_bound = int(np.ceil(np.log(1e-12 / (2 * np.sqrt(kap))) / np.log(rho)))
    assert it <= k_bound + 2, (it, k_bound, kap)


def test_cg_iterations_fall_with_gamma():
    its = []
    for g in (1e0, 1e2, 1e4, 1e6):
        tot = 0
        for seed in (61, 62, 63):
            b = H.with_gamma(H.tiny_grid_like(600, seed, dx_exp=6.0), g)
            s = _sys(b)
            s.factor(s.order_mindeg())
            _, _, it, brk = s.hybrid_once(b.r1[0], b.r2[0])
            assert not brk
            tot += it
        its.append(tot / 3)
    for a, c in zip(its, its[1:]):
        assert c <= a + 1, its
    assert its[-1] < its[0]


# --------------------------------------------------------------------------
# inertia (Theorem 3 and Theorem 1)
# --------------------------------------------------------------------------

def _sign_counts(ev, tol):
    return (int(np.sum(ev > tol)), int(np.sum(ev < -tol)), int(np.sum(np.abs(ev) <= tol)))


def _ldl_inertia(K):
    _, d, _ = sla.ldl(K, lower=True)
    ev = np.linalg.eigvalsh(d)
    return _sign_counts(ev, 1e-12 * np.abs(ev).max())


def test_inertia_full_rank_with_indefinite_H():
    # H indefinite but PD on null(J) (Theorem 1): H_gamma is SPD for large gamma
    rng = np.random.default_rng(71)
    n, m = 14, 6
    J = rng.standard_normal((m, n))
    Q, _ = np.linalg.qr(J.T, mode="complete")
    N = Q[:, m:]                                   # basis of null(J)
    Hd = N @ np.diag(rng.uniform(1, 2, n - m)) @ N.T - 3.0 * (Q[:, :m] @ Q[:, :m].T)
    Dx = np.full(n, 1e-3)
    r1 = rng.standard_normal(n); r2 = rng.standard_normal(m)
    b = H.batch_from_dense(Hd, Dx, J, 0.0, 1e3, r1, r2)
    assert np.linalg.eigvalsh(Hd + np.diag(Dx)).min() < 0
    s = _sys(b)
    assert s.factor(None)[0] == 0
    x, y, info = s.solve(r1, r2)
    K = H.dense_K(b)
    ev = np.linalg.eigvalsh(K)
    assert _sign_counts(ev, 1e-10 * np.abs(ev).max()) == (n, m, 0) == info["inertia"]
    assert _ldl_inertia(K) == (n, m, 0)
    assert info["rr"] <= 1e-10


def test_inertia_duplicate_row_reports_breakdown():
    rng = np.random.default_rng(72)
    n, m = 16, 5
    J = rng.standard_normal((m, n))
    J[3] = J[1]                                    # rank(J) = m - 1
    B = rng.standard_normal((n, n))
    Hd = B.T @ B / n
    Dx = 10 ** rng.uniform(-1, 1, n)
    r1 = rng.standard_normal(n); r2 = rng.standard_normal(m)
    b = H.batch_from_dense(Hd, Dx, J, 0.0, 1e2, r1, r2)
    s = _sys(b)
    assert s.factor(None)[0] == 0
    x, y, info = s.solve(r1, r2)
    K = H.dense_K(b)
    ev = np.linalg.eigvalsh(K)
    want = _sign_counts(ev, 1e-9 * np.abs(ev).max())
    assert want == (n, m - 1, 1)
    # the breakdown shows a zero eigenvalue but not how many: only the n_x
    # positive ones (Cholesky of H_gamma) are reported, the rest undetermined
    assert info["status"] == 2 and info["inertia"] == (n, -1, -1)
    assert info["inertia"][0] == want[0] and want[2] >= 1


def test_inertia_two_duplicate_rows_undetermined():
    # rank(J) = m - 2: K has two zero eigenvalues; a breakdown alone cannot
    # count them, so the oracle must not claim exactly one
    rng = np.random.default_rng(74)
    n, m = 18, 6
    J = rng.standard_normal((m, n))
    J[3] = J[1]
    J[5] = 2.0 * J[0]
    B = rng.standard_normal((n, n))
    Hd = B.T @ B / n
    Dx = 10 ** rng.uniform(-1, 1, n)
    r1 = rng.standard_normal(n); r2 = rng.standard_normal(m)
    b = H.batch_from_dense(Hd, Dx, J, 0.0, 1e2, r1, r2)
    s = _sys(b)
    assert s.factor(None)[0] == 0
    x, y, info = s.solve(r1, r2)
    ev = np.linalg.eigvalsh(H.dense_K(b))
    want = _sign_counts(ev, 1e-9 * np.abs(ev).max())
    assert want == (n, m - 2, 2)
    assert info["status"] == 2 and info["inertia"] == (n, -1, -1)


def test_theorem1_gamma_threshold():
    rng = np.random.default_rng(73)
    n, m = 12, 5
    J = rng.standard_normal((m, n))
    Q, _ = np.linalg.qr(J.T, mode="complete")
    N = Q[:, m:]
    Ht = N @ np.diag(rng.uniform(1, 2, n - m)) @ N.T - 2.0 * (Q[:, :m] @ Q[:, :m].T) \
        + 0.3 * np.outer(N[:, 0], Q[:, 0]) + 0.3 * np.outer(Q[:, 0], N[:, 0])
    lam_min = np.linalg.eigvalsh(Ht).min()
    JTJ = J.T @ J
    ev = np.linalg.eigvalsh(JTJ)
    lam_min_star = ev[ev > 1e-10 * ev.max()].min()
    gamma_min = -lam_min / lam_min_star
    lo, hi = 0.0, 10 * gamma_min
    for _ in range(80):
        mid = (lo + hi) / 2
        if np.linalg.eigvalsh(Ht + mid * JTJ).min() > 0:
            hi = mid
        else:
            lo = mid
    gstar = hi
    assert gstar <= gamma_min * (1 + 1e-12)
    r1 = np.ones(n); r2 = np.ones(m)
    Dx = np.zeros(n)
    for g, ok in ((gstar * 1.05, 0), (gstar * 0.95, 1)):
        b = H.batch_from_dense(Ht, Dx, J, 0.0, g, r1, r2)
        st, fc = _sys(b).factor(None)
        assert st == ok


# --------------------------------------------------------------------------
# metrics (Sec. 5.1) and refinement
# --------------------------------------------------------------------------

def test_metrics_equal_dense_definitions():
    b = H.tiny_grid_like(80, 81, dx_exp=4.0)
    s = _sys(b)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(80); y = rng.standard_normal(40)
    rr, be, fl = s.metrics(b.r1[0], b.r2[0], x, y)
    K = H.dense_K(b)
    r = np.concatenate([b.r1[0], b.r2[0]])
    z = np.concatenate([x, y])
    res = np.linalg.norm(K @ z - r)
    assert rr == pytest.approx(res / np.linalg.norm(r), rel=1e-12, abs=0)
    assert be == pytest.approx(res / (np.linalg.norm(K, np.inf) * np.linalg.norm(z) + np.linalg.norm(r)),
                               rel=1e-12, abs=0)
    o1, o2 = s.apply_K(x, y)
    np.testing.assert_allclose(np.concatenate([o1, o2]), K @ z, rtol=1e-13, atol=1e-13 * np.abs(K @ z).max())


def test_refinement_contracts():
    # a loose inner CG tolerance forces several refinement passes; the RR
    # history must fall monotonically to the target
    b = synth.workload(1)
    s = _sys(b)
    s.factor(s.order_mindeg())
    x, y, info = s.solve(b.r1[0], b.r2[0], cg_tol=1e-3, kkt_tol=1e-10)
    h = info["rr_hist"]
    assert info["passes"] >= 2 and info["rr"] <= 1e-10
    assert all(c < a for a, c in zip(h, h[1:])), h


@pytest.mark.parametrize("gen,seed", [("dense", 91), ("grid", 92)])
def test_single_pass_is_exact(gen, seed):
    # eqs. Schur1/Schur2 are an exact transform: one pass with an accurate CG
    # already gives z (refinement must not be what makes the answer right)
    b = H.tiny_dense_like(40, seed) if gen == "dense" else H.tiny_grid_like(60, seed)
    s = _sys(b)
    s.factor(s.order_mindeg())
    x, y, it, brk = s.hybrid_once(b.r1[0], b.r2[0])
    K = H.dense_K(b)
    r = np.concatenate([b.r1[0], b.r2[0]])
    z_np = np.linalg.solve(K, r)
    z = np.concatenate([x, y])
    assert not brk
    assert np.linalg.norm(z - z_np) / np.linalg.norm(z_np) < max(1e-10, np.linalg.cond(K) * 1e-15)
    assert np.linalg.norm(K @ z - r) / np.linalg.norm(r) < 1e-9
    xs, ys, info = s.solve(b.r1[0], b.r2[0])
    assert info["passes"] <= 2


# --------------------------------------------------------------------------
# compensated residual, evaluation floor and the rounded exact solution
# (Sec. 5.1 RR; Ogita-Rump-Oishi Dot2 for the residual)
# --------------------------------------------------------------------------

U = 2.0 ** -53


def _exact_residual(b, x, y):
    """r - K z in exact rational arithmetic on the FP64 inputs, with K's
    diagonal H_ii + D_i + delta summed exactly."""
    from fractions import Fraction as F
    p = b.pattern
    n, m = p.n_x, p.m
    X = [F(float(v)) for v in x]
    Y = [F(float(v)) for v in y]
    g1 = [F(float(v)) for v in b.r1[0]]
    g2 = [F(float(v)) for v in b.r2[0]]
    for i in range(n):
        for k in range(p.H_rowptr[i], p.H_rowptr[i + 1]):
            j = int(p.H_col[k])
            h = F(float(b.H_val[0, k]))
            g1[i] -= h * X[j]
            if j != i:
                g1[j] -= h * X[i]
        g1[i] -= (F(float(b.D_x[0, i])) + F(float(b.delta[0]))) * X[i]
    for r in range(m):
        for k in range(p.J_rowptr[r], p.J_rowptr[r + 1]):
            j = int(p.J_col[k])
            v = F(float(b.J_val[0, k]))
            g1[j] -= v * Y[r]
            g2[r] -= v * X[j]
    return g1, g2


def _row_terms(b):
    p = b.pattern
    nt = np.full(p.n_x, 3)                       # r_i, D_i x_i, delta x_i
    for i in range(p.n_x):
        for k in range(p.H_rowptr[i], p.H_rowptr[i + 1]):
            j = int(p.H_col[k])
            nt[i] += 1
            if j != i:
                nt[j] += 1
    for k in range(p.J_rowptr[-1]):
        nt[p.J_col[k]] += 1
    nt2 = np.diff(p.J_rowptr) + 1
    return nt, nt2


@pytest.mark.parametrize("gen,seed", [("grid", 101), ("dense", 102), ("grid", 103)])
def test_compensated_residual_equals_exact(gen, seed):
    # z = the oracle's own solution: r - K z cancels to ~1e-14 of the terms,
    # where a plain FP64 sum is wrong in its leading digits; Dot2 keeps
    # |res - exact| <= u |exact| + (k u)^2 sum|terms| (k terms in the row)
    b = H.tiny_dense_like(30, seed, dx_exp=6.0) if gen == "dense" else H.tiny_grid_like(40, seed, dx_exp=8.0)
    s = _sys(b)
    s.factor(s.order_mindeg())
    x, y, info = s.solve(b.r1[0], b.r2[0])
    g1, g2, t1, t2 = s.residual(b.r1[0], b.r2[0], x, y)
    e1, e2 = _exact_residual(b, x, y)
    nt1, nt2 = _row_terms(b)
    for got, ex, t, k in ((g1, e1, t1, nt1), (g2, e2, t2, nt2)):
        for i in range(len(got)):
            bound = 2 * U * abs(float(ex[i])) + 2 * (k[i] * U) ** 2 * t[i]
            assert abs(got[i] - float(ex[i])) <= bound, (i, got[i], float(ex[i]), t[i])
    # the cancellation is real: the plain FP64 residual would be off by far more
    K = H.dense_K(b)
    plain = np.concatenate([b.r1[0], b.r2[0]]) - K @ np.concatenate([x, y])
    exact = np.array([float(v) for v in e1 + e2])
    assert np.abs(plain - exact).max() > 1e3 * np.abs(np.concatenate([g1, g2]) - exact).max()


@pytest.mark.parametrize("gen,seed,spread", [("grid", 111, 0.0), ("dense", 112, 0.0), ("grid", 113, 4.0)])
def test_floor_equals_dense_definition(gen, seed, spread):
    # floor = 2^-53 || |K||z| + |r| ||_2 / ||r||_2 (diag(H) >= 0 here, so the
    # term-wise sums equal |K||z|), checked densely and in exact arithmetic;
    # spread 0 keeps both block rows of K of the same weight, so that a
    # dropped term of either shows
    from fractions import Fraction as F
    dx = 1.0 if spread == 0.0 else 8.0
    b = H.tiny_dense_like(24, seed, dx_exp=dx) if gen == "dense" else H.tiny_grid_like(30, seed, dx_exp=dx)
    assert np.all(np.diag(H.dense_H(b)) >= 0)
    rng = np.random.default_rng(seed)
    n, m = b.pattern.n_x, b.pattern.m
    x = rng.standard_normal(n) * 10 ** rng.uniform(-spread, spread, n)
    y = rng.standard_normal(m) * 10 ** rng.uniform(-spread, spread, m)
    s = _sys(b)
    rr, be, fl = s.metrics(b.r1[0], b.r2[0], x, y)
    K = H.dense_K(b)
    r = np.concatenate([b.r1[0], b.r2[0]])
    z = np.concatenate([x, y])
    t = np.abs(K) @ np.abs(z) + np.abs(r)
    assert fl == pytest.approx(U * np.linalg.norm(t) / np.linalg.norm(r), rel=1e-13, abs=0)
    _, _, t1, t2 = s.residual(b.r1[0], b.r2[0], x, y)
    np.testing.assert_allclose(np.concatenate([t1, t2]), t, rtol=1e-13)
    # exact: sum of squares in rationals, one square root in FP64 at the end
    Kf = [[F(float(v)) for v in row] for row in np.abs(K)]
    zf = [F(float(abs(v))) for v in z]
    tf = [sum(Kf[i][j] * zf[j] for j in range(n + m)) + F(float(abs(r[i]))) for i in range(n + m)]
    want = U * np.sqrt(float(sum(v * v for v in tf))) / np.sqrt(float(sum(F(float(v)) ** 2 for v in r)))
    assert fl == pytest.approx(want, rel=1e-14, abs=0)


def _exact_K(b):
    """K in rationals from the FP64 inputs (diagonal H_ii + D_i + delta exact)."""
    from fractions import Fraction as F
    n, m = b.pattern.n_x, b.pattern.m
    Hd, J = H.dense_H(b), H.dense_J(b)
    K = [[F(0)] * (n + m) for _ in range(n + m)]
    for i in range(n):
        for j in range(n):
            K[i][j] = F(float(Hd[i, j]))
        K[i][i] += F(float(b.D_x[0, i])) + F(float(b.delta[0]))
    for r in range(m):
        for j in range(n):
            K[n + r][j] = K[j][n + r] = F(float(J[r, j]))
    return K


def _exact_solve(K, r):
    """Gauss-Jordan elimination in rationals."""
    from fractions import Fraction as F
    N = len(K)
    A = [list(K[i]) + [F(float(r[i]))] for i in range(N)]
    for c in range(N):
        p = next(i for i in range(c, N) if A[i][c] != 0)
        A[c], A[p] = A[p], A[c]
        for i in range(N):
            if i != c and A[i][c] != 0:
                f = A[i][c] / A[c][c]
                A[i] = [a - f * bb for a, bb in zip(A[i], A[c])]
    return [A[i][N] / A[i][i] for i in range(N)]


@pytest.mark.parametrize("seed", [121, 122])
def test_refine_dd_rounds_the_exact_solution(seed):
    # a badly scaled system (D_x over 12 decades): the double-double
    # refinement must return the exact solution rounded to FP64, and the RR
    # it reports must be that of the rounded solution in exact arithmetic
    rng = np.random.default_rng(seed)
    n, m = 9, 4
    B = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.4)
    Hd = B.T @ B
    Dx = 10 ** rng.uniform(-6, 6, n)
    J = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.5)
    J[np.arange(m), 2 * np.arange(m)] = 1.0
    r1 = rng.standard_normal(n); r2 = rng.standard_normal(m)
    b = H.batch_from_dense(Hd, Dx, J, 1e-8, 1e4, r1, r2)
    s = _sys(b)
    s.factor(None)
    x, y, info = s.solve(r1, r2)
    xr, yr, hist = s.refine_dd(r1, r2, x, y)
    zs = _exact_solve(_exact_K(b), np.concatenate([r1, r2]))
    got = np.concatenate([xr, yr])
    want = np.array([float(v) for v in zs])       # correctly rounded
    ulps = np.abs(got - want) / np.spacing(np.abs(want))
    assert ulps.max() <= 1.0, ulps
    assert hist[-1] < 1e-25
    e1, e2 = _exact_residual(b, xr, yr)
    rr_exact = np.sqrt(float(sum(v * v for v in e1 + e2))) / np.linalg.norm(np.concatenate([r1, r2]))
    rr, _, _ = s.metrics(r1, r2, xr, yr)
    assert rr == pytest.approx(rr_exact, rel=1e-12, abs=0)


def _mindeg_bruteforce(A):
    """Minimum degree on the explicit elimination graph, ties to the smallest
    index, by sets (tiny inputs)."""
    n = A.shape[0]
    adj = [set(np.nonzero(A[i])[0].tolist()) - {i} for i in range(n)]
    alive = set(range(n))
    perm = []
    while alive:
        v = min(alive, key=lambda u: (len(adj[u]), u))
        nb = adj[v]
        for u in nb:
            adj[u] |= nb
            adj[u] -= {u, v}
        alive.remove(v)
        for u in range(n):
            adj[u].discard(v)
        perm.append(v)
    return perm


@pytest.mark.parametrize("gen,seed", [("grid", 131), ("dense", 132), ("grid", 133)])
def test_order_is_exact_minimum_degree(gen, seed):
    b = H.tiny_dense_like(40, seed) if gen == "dense" else H.tiny_grid_like(60, seed)
    s = _sys(b)
    cp, ri, v = s.hgamma()
    n = b.pattern.n_x
    A = H.csc_to_dense_lower(cp, ri, np.ones_like(v), n) != 0
    A = A | A.T
    assert s.order_mindeg().tolist() == _mindeg_bruteforce(A)


# --------------------------------------------------------------------------
# Algorithm 1's regularization (Sec. 4.1) and the gamma heuristic (Sec. 3)
# --------------------------------------------------------------------------

def _system_with_hgamma_spectrum(n, m, lam, gamma, seed):
    """A system whose assembled H_gamma = H + D_x + delta I + gamma J^T J is
    Q diag(lam) Q^T (Q random orthogonal): H is chosen to make it so."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    target = Q @ np.diag(lam) @ Q.T
    target = (target + target.T) / 2
    J = rng.standard_normal((m, n)) if m else np.zeros((0, n))
    Dx = 10 ** rng.uniform(-1, 0, n)
    Hd = target - np.diag(Dx) - gamma * J.T @ J
    return H.batch_from_dense(Hd, Dx, J, 0.0, gamma, rng.standard_normal(n), rng.standard_normal(m)), target


def _first_success(target, delta_min, delta_max):
    """Algorithm 1's delta1 sequence decided by the dense eigenvalues (and
    LAPACK's Cholesky): (succeeded, delta1, delta_min after)."""
    def spd(d):
        ok_eig = np.linalg.eigvalsh(target + d * np.eye(target.shape[0])).min() > 0
        try:
            sla.cholesky(target + d * np.eye(target.shape[0]), lower=True)
            ok_chol = True
        except np.linalg.LinAlgError:
            ok_chol = False
        assert ok_eig == ok_chol      # the cases keep a clear margin
        return ok_eig
    d1 = 0.0
    ok = spd(d1)
    while not ok and d1 <= delta_max / 2:
        if d1 == 0.0:
            d1 = delta_min
        else:
            delta_min *= 2
            d1 = delta_min
        ok = spd(d1)
    return ok, d1, delta_min


@pytest.mark.parametrize("n,m,lam_min,dmin,expect", [
    (9, 0, -3e-9, 1e-9, 4e-9),        # three doublings past delta_min
    (9, 3, -3e-9, 1e-9, 4e-9),        # the same through gamma J^T J
    (9, 3, -3e-9, 4e-9, 4e-9),        # delta_min carried from an earlier matrix: first retry succeeds
    (9, 3, 2.0, 1e-9, 0.0),           # already SPD: delta1 = 0
    (9, 3, -7e-7, 1e-9, 5.12e-7),     # beyond delta_max / 2: fails after 5.12e-7
])
def test_regularization_delta1_equals_dense_first_success(n, m, lam_min, dmin, expect):
    lam = np.concatenate([[lam_min], np.linspace(1.0, 3.0, n - 1)])
    b, target = _system_with_hgamma_spectrum(n, m, lam, 1e2, seed=91 + m)
    ok, d1_ref, dmin_ref = _first_success(target, dmin, 1e-6)
    assert d1_ref == pytest.approx(expect, rel=1e-12, abs=0)
    s = _sys(b)
    st, d1, dmin_out, fc = s.factor_regularized(None, delta_min=dmin, delta_max=1e-6)
    assert (st == 0) == ok
    assert d1 == d1_ref and dmin_out == dmin_ref
    if ok:   # the perturbed system is solved: its residual includes delta1
        # (S inherits H_delta's 1e-9 eigenvalue: CG needs more than m = 3
        # iterations in floating point)
        x, y, info = s.solve(b.r1[0], b.r2[0], max_cg=50)
        Kd = H.dense_K(b) + np.diag(np.r_[np.full(n, d1), np.zeros(m)])
        r = np.r_[b.r1[0], b.r2[0]]
        z = np.r_[x, y]
        # at most the residual the rounded exact solution can have (H_delta's
        # 1e-9 eigenvalue makes ||z|| ~ 1e9 ||r|| when m = 0)
        bound = max(1e-9, 10 * 2.0 ** -53 * np.linalg.norm(np.abs(Kd) @ np.abs(z)) / np.linalg.norm(r))
        assert np.linalg.norm(Kd @ z - r) / np.linalg.norm(r) < bound


def test_gamma_heuristic_equals_dense_norms():
    for gen, seed in (("dense", 95), ("grid", 96)):
        b = H.tiny_dense_like(60, seed) if gen == "dense" else H.tiny_grid_like(300, seed, dx_exp=3.0)
        Hd = H.dense_H(b) + np.diag(b.D_x[0] + b.delta[0])
        Jd = H.dense_J(b)
        want = np.abs(Hd).sum(1).max() / np.abs(Jd).sum(1).max() ** 2
        assert _sys(b).gamma_heuristic() == pytest.approx(want, rel=1e-13)


def test_delta2_restart_equals_dense_perturbed_schur():
    """After a breakdown (duplicate J row, inconsistent r2) CG restarts on
    S + delta2 I (Algorithm 1): the pass returns y = (S + delta2 I)^{-1} b,
    x = H_gamma^{-1}(rhat - J^T y), with S, b and rhat formed densely."""
    rng = np.random.default_rng(97)
    n, m = 16, 5
    J = rng.standard_normal((m, n))
    J[3] = J[1]
    B = rng.standard_normal((n, n))
    Hd = B.T @ B / n
    Dx = 10 ** rng.uniform(-1, 1, n)
    gamma, d2 = 1e2, 1e-6
    b = H.batch_from_dense(Hd, Dx, J, 0.0, gamma, rng.standard_normal(n), rng.standard_normal(m))
    s = _sys(b)
    s.factor(None)
    x, y, it, brk = s.hybrid_once(b.r1[0], b.r2[0], delta2=d2, max_cg=100)
    assert brk
    Hg = Hd + np.diag(Dx) + gamma * J.T @ J
    rhat = b.r1[0] + gamma * J.T @ b.r2[0]
    S = J @ np.linalg.solve(Hg, J.T)
    bv = J @ np.linalg.solve(Hg, rhat) - b.r2[0]
    ys = np.linalg.solve(S + d2 * np.eye(m), bv)
    xs = np.linalg.solve(Hg, rhat - J.T @ ys)
    # y is fixed up to kappa(S + delta2 I) ~ 1e6 times CG's tolerance: its
    # residual on the perturbed Schur system is the sharp check; x depends on
    # J^T y only, which the null direction of J^T does not move
    assert np.linalg.norm((S + d2 * np.eye(m)) @ y - bv) / np.linalg.norm(bv) < 1e-9
    assert np.linalg.norm(y - ys) / np.linalg.norm(ys) < 1e-4
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-7
    # the full solve stops after the pass that broke down
    x2, y2, info = s.solve(b.r1[0], b.r2[0], delta2=d2, max_cg=100)
    assert info["passes"] == 1 and info["status"] in (0, 3) and info["inertia"] == (n, -1, -1)


# --------------------------------------------------------------------------
# symmetrized Ruiz scaling (Sec. 4.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gen", ["grid", "dense"])
def test_ruiz_rows_of_scaled_K_converge_to_one(gen):
    """Every row of D K D (dense, numpy) has its largest magnitude near 1,
    the deviation shrinking about twofold per sweep (Ruiz 2001's rate for
    the inf-norm)."""
    b = H.tiny_grid_like(400, 84, dx_exp=8.0) if gen == "grid" else H.tiny_dense_like(150, 85, dx_exp=6.0)
    o = _sys(b)
    K = H.dense_K(b)
    devs = []
    for it in (10, 20, 40):
        d = o.ruiz(it)
        assert np.all(d > 0)
        r = np.abs(d[:, None] * K * d[None, :]).max(axis=1)
        devs.append(np.abs(r - 1).max())
    assert devs[0] < 2e-2 and devs[1] < 1e-4 and devs[2] < 1e-9, devs


@pytest.mark.parametrize("seed", [86, 87])
def test_scaled_solve_equals_dense_solution(seed):
    """Passes on D K D and refinement on K reach the exact solution of K (the
    scaling is a congruence: the solution and the inertia are those of K)."""
    b = H.tiny_dense_like(50, seed, dx_exp=4.0)
    o = _sys(b)
    d = o.ruiz(10)
    x, y, info = o.solve_scaled(b.r1[0], b.r2[0], d, o.order_mindeg())
    z = np.linalg.solve(H.dense_K(b), np.r_[b.r1[0], b.r2[0]])
    assert info["status"] == 0 and info["rr"] <= 1e-10
    assert np.linalg.norm(np.r_[x, y] - z) / np.linalg.norm(z) < 1e-8
    assert info["inertia"] == (b.pattern.n_x, b.pattern.m, 0)


def test_scaled_solve_needs_fewer_cg_iterations():
    """With gamma judged on the scaled system (Sec. 4.1) each J row's
    effective gamma is gamma * d_y^2: on a grid-like system with D_x spread
    over 16 decades the scaled solve needs fewer CG iterations in total."""
    b = H.tiny_grid_like(3000, 83, gamma=1e4, dx_exp=8.0)
    o = _sys(b)
    p = o.order_mindeg()
    o.factor(p)
    x, y, info = o.solve(b.r1[0], b.r2[0])
    xs, ys, infs = o.solve_scaled(b.r1[0], b.r2[0], o.ruiz(10), p)
    assert info["status"] == 0 and infs["status"] == 0
    assert sum(infs["cg_iters"]) < sum(info["cg_iters"]), (infs["cg_iters"], info["cg_iters"])


@pytest.mark.parametrize("scaled", [False, True])
def test_inexact_refinement_reaches_the_solution_with_fewer_iterations(scaled):
    """Refinement passes after the first stop CG at max(cg_tol, min(1e-2,
    0.1 kkt_tol / RR)): the iterate still reaches RR <= 1e-10 and, on a tiny
    system, numpy's solution of K; the later passes take fewer CG
    iterations than at the full tolerance."""
    b = H.tiny_dense_like(50, 88, dx_exp=4.0)
    o = _sys(b)
    z = np.linalg.solve(H.dense_K(b), np.r_[b.r1[0], b.r2[0]])
    if scaled:
        x, y, info = o.solve_scaled(b.r1[0], b.r2[0], o.ruiz(10), o.order_mindeg(), inexact=1)
    else:
        o.factor(o.order_mindeg())
        x, y, info = o.solve(b.r1[0], b.r2[0], inexact=1)
    assert info["status"] == 0 and info["rr"] <= 1e-10
    assert np.linalg.norm(np.r_[x, y] - z) / np.linalg.norm(z) < 1e-8
    g = H.tiny_grid_like(3000, 89, gamma=1e4, dx_exp=8.0)
    og = _sys(g)
    p = og.order_mindeg()
    og.factor(p)
    d = og.ruiz(10)
    run = (lambda **kw: og.solve_scaled(g.r1[0], g.r2[0], d, p, **kw)) if scaled else \
        (lambda **kw: og.solve(g.r1[0], g.r2[0], **kw))
    _, _, full = run(inexact=0)
    _, _, inex = run(inexact=1)
    assert inex["status"] == 0 and inex["rr"] <= 1e-10
    assert inex["cg_iters"][0] == full["cg_iters"][0]          # the first pass is the paper's
    if full["passes"] > 1:
        assert sum(inex["cg_iters"][1:]) < sum(full["cg_iters"][1:]), (inex["cg_iters"], full["cg_iters"])


# --------------------------------------------------------------------------
# the 4x4 system (Sec. 3, eqs. linsys4x4 / linsys2x2) through the reduction
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,ds_exp", [(93, 2.0), (94, 6.0)])
def test_4x4_solve_equals_dense_solution(seed, ds_exp):
    b = H.tiny_dense_like(40, seed, dx_exp=2.0)
    q = synth.inequalities(b.pattern, 1, seed=seed + 1, frac=0.3, ds_exp=ds_exp)
    o4 = oracle.System4.from_batch(b, q)
    assert o4.factor(o4.two.order_mindeg())[0] == 0
    r = [b.r1[0], q.r_s[0], b.r2[0], q.r_yd[0]]
    x, sv, y, yd, info = o4.solve(*r)
    K4 = H.dense_K4(b, q)
    z = np.linalg.solve(K4, np.concatenate(r))
    got = np.concatenate([x, sv, y, yd])
    assert info["status"] == 0 and info["rr"] <= 1e-10
    assert np.linalg.norm(got - z) / np.linalg.norm(z) < 1e-8
    # RR and BE as defined in Sec. 5.1, on K4, at a point away from the
    # solution (so that the residual is not just rounding)
    zp = got + 1e-3 * np.random.default_rng(seed).standard_normal(got.size) * np.abs(got).max()
    n, md, m = b.pattern.n_x, q.m_d, b.pattern.m
    parts = np.split(zp, [n, n + md, n + md + m])
    res = np.linalg.norm(K4 @ zp - np.concatenate(r))
    rr, be = o4.metrics(*r, *parts)
    assert rr == pytest.approx(res / np.linalg.norm(np.concatenate(r)), rel=1e-10)
    kinf = np.abs(K4).sum(axis=1).max()
    assert be == pytest.approx(res / (kinf * np.linalg.norm(zp) + np.linalg.norm(np.concatenate(r))), rel=1e-10)


def test_4x4_reduced_matrix_and_no_inequalities():
    """The 2x2 system the reduction builds has Htilde = H + D_x + delta I +
    J_d^T D_s J_d (dense check of its H_gamma); with every D_s = 0 the
    reduction is still exact (dense solve)."""
    b = H.tiny_dense_like(30, 95, dx_exp=1.0)
    q = synth.inequalities(b.pattern, 1, seed=96, frac=0.3)
    o4 = oracle.System4.from_batch(b, q)
    cp, ri, v = o4.two.hgamma()
    got = np.zeros((30, 30))
    cols = np.repeat(np.arange(30), np.diff(cp))
    got[ri, cols] = v
    Jd = H.dense_Jd(q, 30)
    want = np.tril(H.dense_H(b) + np.diag(b.D_x[0] + b.delta[0]) + Jd.T @ np.diag(q.D_s[0]) @ Jd +
                   b.gamma[0] * H.dense_J(b).T @ H.dense_J(b))
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    import dataclasses
    q0 = dataclasses.replace(q, D_s=np.zeros_like(q.D_s))
    o0 = oracle.System4.from_batch(b, q0)
    o0.factor(None)
    r = [b.r1[0], q0.r_s[0], b.r2[0], q0.r_yd[0]]
    x, sv, y, yd, info = o0.solve(*r)
    z = np.linalg.solve(H.dense_K4(b, q0), np.concatenate(r))
    assert np.linalg.norm(np.concatenate([x, sv, y, yd]) - z) / np.linalg.norm(z) < 1e-8
