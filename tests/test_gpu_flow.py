"""GPU parity of the dataflow triangular solves (k_tri_flow: both sweeps over
all levels in one launch, every supernode task waiting only for its children
or parent) against the level-by-level launches and the oracle, through the C
ABI. Bars as for the other H_gamma^{-1} tests: FP64 backward error <= 1e-14
on the dense H_gamma and the two schedules' solutions equal to 1e-10
relative on well-conditioned systems (only the order of FP atomic additions
differs); FP32 backward error <= 1e-5; end-to-end solves accepted by the
oracle's compensated residual at 1e-10 with CG counts within the rounding
bound."""
import numpy as np
import pytest

import oracle
from paper_2110_03636_amd import hkkt, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _solver(b, precision, flow, **kw):
    s = hkkt.Solver(precision=precision, flow_live=flow, **kw)
    s.analyze(b.pattern)
    assert s.factor_batch(b)[0] == 0
    return s


def _be(b, i, x, rhs):
    A = H.dense_Hgamma(b, i)
    return np.linalg.norm(A @ x - rhs) / (np.linalg.norm(A, np.inf) * np.linalg.norm(x) + np.linalg.norm(rhs))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nb", [1, 5])
def test_flow_hsolve_equals_level_schedule(precision, nb):
    b = synth.grid_like(2500, nb=nb, seed=401 + nb, gammas=(10.0,), dx_exp=1.0)
    rhs = np.random.default_rng(nb).standard_normal((nb, b.pattern.n_x))
    ref = _solver(b, precision, 0).hsolve(rhs)
    s = _solver(b, precision, 1000)
    s.profile_begin()
    x = s.hsolve(rhs)
    prof = s.profile_end()
    assert prof["tri_flow"][1] == 1 and prof["fwd"][1] == 0 and prof["tri_tree_staged"][1] == 0, prof
    for i in range(nb):
        be = _be(b, i, x[i], rhs[i])
        rel = np.linalg.norm(x[i] - ref[i]) / np.linalg.norm(ref[i])
        if precision == "fp64":
            assert be < 1e-14 and rel < 1e-10, (i, be, rel)
        else:
            assert be < 1e-5 and rel < 1e-4, (i, be, rel)


def test_flow_repeated_applications_stay_exact():
    """Counters are cleared by the tasks themselves and flags carry a
    per-application token: twenty applications in a row on alternating
    instance subsets give the same result each time (FP64, every forward
    addition in a fixed order is not guaranteed, so to 1e-12)."""
    b = synth.grid_like(2000, nb=4, seed=410, gammas=(10.0,), dx_exp=1.0)
    s = _solver(b, "fp64", 1000)
    rhs = np.random.default_rng(3).standard_normal((4, b.pattern.n_x))
    first = s.hsolve(rhs)
    for _ in range(20):
        x = s.hsolve(rhs)
        assert np.abs(x - first).max() <= 1e-12 * np.abs(first).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_flow_cg_solve_equals_oracle(precision):
    """Every application of the CG loop through the dataflow launch."""
    b = synth.grid_like(3000, nb=6, seed=411, gammas=(1e4, 1e6), dx_exp=8.0)
    s = _solver(b, precision, 1000)
    s.profile_begin()
    rc, x, y, infos = s.solve(b.r1, b.r2)
    prof = s.profile_end()
    assert prof["tri_flow"][1] > 0
    for i in range(b.nb):
        o = oracle.System.from_batch(b, i)
        H.check_gpu_solution(o, b.r1[i], b.r2[i], x[i], y[i], infos[i], 1e-10)
        if precision == "fp64":
            o.factor(o.order_mindeg())
            xo, yo, io = o.solve(b.r1[i], b.r2[i])
            assert abs(infos[i]["cg_iters"] - sum(io["cg_iters"])) <= H.cg_count_tol(io["cg_iters"], infos[i]["passes"])


def test_flow_group_members_equal_oracle():
    """Uneven members in one group: the dataflow tasks of a finished member
    are skipped without blocking the others."""
    mem = [H.tiny_grid_like(n, 420 + n, gamma=g, dx_exp=6.0) for n, g in ((900, 1e4), (1500, 1e6), (400, 1e4))]
    g = hkkt.GroupPattern([m.pattern for m in mem])
    cat = hkkt.GroupPattern.concat
    s = hkkt.Solver(precision="fp64", flow_live=1000)
    s.analyze_group(g)
    delta = np.stack([m.delta for m in mem], axis=1)
    gamma = np.stack([m.gamma for m in mem], axis=1)
    rc, st, fc = s.factor(cat([m.H_val for m in mem]), cat([m.D_x for m in mem]), cat([m.J_val for m in mem]),
                          delta, gamma)
    assert rc == 0
    s.profile_begin()
    rc, x, y, infos = s.solve(cat([m.r1 for m in mem]), cat([m.r2 for m in mem]))
    assert s.profile_end()["tri_flow"][1] > 0
    xs, ys = g.split_x(x), g.split_y(y)
    for k, m in enumerate(mem):
        o = oracle.System.from_batch(m, 0)
        H.check_gpu_solution(o, m.r1[0], m.r2[0], xs[k][0], ys[k][0], infos[k], 1e-10)


def test_flow_not_used_for_wide_supernodes():
    """A dense-like pattern has supernodes beyond 128 rows: the level
    schedule runs instead, with the same result."""
    b = synth.workload(1)
    s = _solver(b, "fp64", 1000)
    s.profile_begin()
    rc, x, y, infos = s.solve(b.r1, b.r2)
    assert s.profile_end()["tri_flow"][1] == 0
    H.check_gpu_solution(oracle.System.from_batch(b, 0), b.r1[0], b.r2[0], x[0], y[0], infos[0], 1e-10)
