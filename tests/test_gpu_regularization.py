"""GPU parity of Algorithm 1's regularization and of the gamma heuristic
(Sec. 3 and 4.1) against the oracle, through the C ABI.

  - delta1 and delta_min after the loop: equal to the oracle's (the same
    sequence of Cholesky attempts, decided by each side's own factorization
    of the same matrices, with clear margins), and the solve of the
    perturbed system accepted by the oracle's compensated residual on K with
    delta + delta1;
  - the delta2 restart after a breakdown: status equal to the oracle's, x
    and J^T y equal to 1e-6 relative (y itself only up to kappa(S + delta2 I)
    times CG's tolerance), one pass;
  - gamma = ||H + D_x + delta I||_inf / ||J||_inf^2 equal to the oracle's to
    1e-14 relative (the same maxima of sums, in another order)."""
import numpy as np
import pytest

import oracle
from paper_2110_03636_amd import hkkt, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _dense_batch(specs, n, m, gamma, seed):
    """One batch whose instances share a full dense pattern; instance k has
    H_gamma = Q_k diag(lam_k) Q_k^T (its smallest eigenvalue lam_k[0])."""
    rng = np.random.default_rng(seed)
    J = rng.standard_normal((m, n))
    parts = []
    for lam_min in specs:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.concatenate([[lam_min], np.linspace(1.0, 3.0, n - 1)])
        target = Q @ np.diag(lam) @ Q.T
        target = (target + target.T) / 2
        Dx = 10 ** rng.uniform(-1, 0, n)
        Hd = target - np.diag(Dx) - gamma * J.T @ J
        parts.append(H.batch_from_dense(Hd, Dx, J, 0.0, gamma, rng.standard_normal(n), rng.standard_normal(m)))
    b0 = parts[0]
    import dataclasses
    return dataclasses.replace(b0, H_val=np.concatenate([p.H_val for p in parts]),
                               D_x=np.concatenate([p.D_x for p in parts]),
                               J_val=np.concatenate([p.J_val for p in parts]),
                               delta=np.concatenate([p.delta for p in parts]),
                               gamma=np.concatenate([p.gamma for p in parts]),
                               r1=np.concatenate([p.r1 for p in parts]), r2=np.concatenate([p.r2 for p in parts]))


# FP64 decides definiteness at FP64 resolution: the paper's delta_min = 1e-9
# scale. The FP32 factor of the mixed path (with its pivot test) resolves
# eigenvalues down to about n * u32 * ||H_gamma|| only, so its cases keep
# margins of that size (delta_min = 1e-4, delta_max = 1).
@pytest.mark.parametrize("precision,specs,dmin0,dmax", [
    ("fp64", [2.0, -3e-9, -3e-7, -7e-7, -1.5e-8], 1e-9, 1e-6),
    ("mixed", [2.0, -3e-4, -3e-2, -0.9, -1.5e-3], 1e-4, 1.0)])
def test_factor_regularized_equals_oracle(precision, specs, dmin0, dmax):
    b = _dense_batch(specs, 40, 12, 1e2, seed=301)
    s = hkkt.Solver(precision=precision, max_cg=100)
    s.analyze(b.pattern)
    rc, st, fc, d1, dmin = s.factor_regularized(b.H_val, b.D_x, b.J_val, b.delta, b.gamma,
                                                np.full(b.nb, dmin0), dmax)
    want = []
    for i in range(b.nb):
        o = oracle.System.from_batch(b, i)
        want.append(o.factor_regularized(s.perm(), dmin0, dmax))
    for i, (ost, od1, odmin, ofc) in enumerate(want):
        assert st[i] == ost and d1[i] == od1 and dmin[i] == odmin, (i, st[i], d1[i], dmin[i], want[i])
    assert list(st) == [0, 0, 0, 1, 0] and rc == hkkt.NOT_SPD
    rc, x, y, infos = s.solve(b.r1, b.r2)
    for i in range(b.nb):
        if st[i] != 0:
            assert infos[i]["status"] == hkkt.NOT_SPD
            continue
        o = oracle.System(b.pattern.n_x, b.pattern.m, b.pattern.H_rowptr, b.pattern.H_col, b.H_val[i], b.D_x[i],
                          b.pattern.J_rowptr, b.pattern.J_col, b.J_val[i], b.delta[i] + d1[i], b.gamma[i])
        H.check_gpu_solution(o, b.r1[i], b.r2[i], x[i], y[i], infos[i], 1e-10)


def test_factor_regularized_carries_delta_min_over_a_sequence():
    """Two matrices in a row (Algorithm 1's outer loop): the second starts
    from the delta_min the first left behind."""
    b = _dense_batch([-3e-9, -3e-9], 30, 8, 1e2, seed=302)
    s = hkkt.Solver(precision="fp64")
    s.analyze(b.pattern)
    dmin = np.array([1e-9])
    one = lambda i: [a[i:i + 1] for a in (b.H_val, b.D_x, b.J_val, b.delta, b.gamma)]
    rc, st, fc, d1, dmin = s.factor_regularized(*one(0), dmin, 1e-6)
    assert st[0] == 0 and d1[0] == 4e-9 and dmin[0] == 4e-9
    rc, st, fc, d1, dmin = s.factor_regularized(*one(1), dmin, 1e-6)
    assert st[0] == 0 and d1[0] == 4e-9 and dmin[0] == 4e-9


def test_delta2_restart_equals_oracle():
    rng = np.random.default_rng(303)
    n, m = 40, 12
    Bm = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.15)
    Hd = Bm.T @ Bm
    J = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.3)
    J[:, :m] += np.eye(m)
    J[5] = J[2]
    b = H.batch_from_dense(Hd, 10 ** rng.uniform(-1, 1, n), J, 0.0, 1e2, rng.standard_normal(n),
                           rng.standard_normal(m))
    s = hkkt.Solver(precision="fp64", delta2=1e-6, max_cg=200)
    s.analyze(b.pattern)
    assert s.factor_batch(b)[0] == 0
    rc, x, y, infos = s.solve(b.r1, b.r2)
    o = oracle.System.from_batch(b)
    o.factor(s.perm())
    xo, yo, io = o.solve(b.r1[0], b.r2[0], delta2=1e-6, max_cg=200)
    assert infos[0]["status"] == io["status"] and infos[0]["passes"] == io["passes"] == 1
    assert np.linalg.norm(x[0] - xo) / np.linalg.norm(xo) < 1e-6
    assert np.linalg.norm(J.T @ (y[0] - yo)) / np.linalg.norm(J.T @ yo) < 1e-6
    assert abs(infos[0]["cg_iters"] - sum(io["cg_iters"])) <= H.cg_count_tol(io["cg_iters"], infos[0]["passes"])
    assert s.inertia(0) == (n, -1, -1)


@pytest.mark.parametrize("case", ["dense", "grid", "batch"])
def test_gamma_heuristic_equals_oracle(case):
    b = {"dense": lambda: H.tiny_dense_like(300, 304),
         "grid": lambda: H.tiny_grid_like(4000, 305, dx_exp=6.0),
         "batch": lambda: synth.grid_like(3000, nb=4, seed=306, gammas=(1e4, 1e6), dx_exp=8.0)}[case]()
    s = hkkt.Solver(precision="fp64")
    s.analyze(b.pattern)
    g = s.gamma_heuristic(b.H_val, b.D_x, b.J_val, b.delta)
    for i in range(b.nb):
        assert g[i] == pytest.approx(oracle.System.from_batch(b, i).gamma_heuristic(), rel=1e-14)
