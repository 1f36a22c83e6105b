"""GPU parity of the 4x4 system of Sec. 3 (eq. linsys4x4, solved through the
2x2 reduction with refinement on the 4x4 residual) against the oracle's 4x4
solve, through the C ABI: each instance accepted when the oracle's own 4x4
residual of the GPU solution is at most 1e-10 (or within 10x of what the
oracle's solve reaches, where the plain FP64 residual of K4 with D_s up to
1e6 stops above it), status equal, solutions equal up to conditioning
(1e-6 relative)."""
import numpy as np
import pytest

import oracle
from paper_2110_03636_amd import hkkt, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,scaling", [("fp64", 0), ("mixed", 0), ("fp64", 1)])
def test_4x4_solve_equals_oracle(precision, scaling):
    b = synth.grid_like(3000, nb=4, seed=601, gammas=(1e4, 1e6), dx_exp=4.0)
    q = synth.inequalities(b.pattern, b.nb, seed=602, frac=0.25, ds_exp=4.0)
    s = hkkt.Solver(precision=precision, scaling=scaling, refine_inexact=1)
    s.analyze4(b.pattern, q)
    rc, st, fc = s.factor4(b, q)
    assert rc == 0
    rc, x, sv, y, yd, infos = s.solve4(b.r1, q.r_s, b.r2, q.r_yd)
    for i in range(b.nb):
        o4 = oracle.System4.from_batch(b, q, i)
        o4.factor(o4.two.order_mindeg())
        r = (b.r1[i], q.r_s[i], b.r2[i], q.r_yd[i])
        xo, so, yo, ydo, io = o4.solve(*r)
        rr, be = o4.metrics(*r, x[i], sv[i], y[i], yd[i])
        # both plain FP64 residuals of the same z: equal up to their rounding
        # (about u ||K4|| ||z|| / ||r||, near 1e-14 here)
        assert abs(infos[i]["rr"] - rr) <= 1e-3 * rr + 1e-12, (infos[i]["rr"], rr)
        assert rr <= max(1e-10, 10 * io["rr"]), (i, rr, io)
        assert infos[i]["status"] == io["status"] or (rr <= 1e-10 and infos[i]["status"] == 0)
        zg = np.concatenate([x[i], sv[i], y[i], yd[i]])
        zo = np.concatenate([xo, so, yo, ydo])
        assert np.linalg.norm(zg - zo) / np.linalg.norm(zo) < 1e-6


def test_4x4_dense_small_and_no_inequality_rows():
    """A dense-like system checked against numpy's solve of K4; and m_d = 0
    reduces to the 2x2 solve."""
    b = H.tiny_dense_like(60, 603, dx_exp=2.0)
    q = synth.inequalities(b.pattern, 1, seed=604, frac=0.3, ds_exp=2.0)
    s = hkkt.Solver(precision="fp64")
    s.analyze4(b.pattern, q)
    assert s.factor4(b, q)[0] == 0
    r = (b.r1[0], q.r_s[0], b.r2[0], q.r_yd[0])
    rc, x, sv, y, yd, infos = s.solve4(*[v[None] for v in r])
    z = np.linalg.solve(H.dense_K4(b, q), np.concatenate(r))
    assert infos[0]["status"] == 0 and infos[0]["rr"] <= 1e-10
    assert np.linalg.norm(np.concatenate([x[0], sv[0], y[0], yd[0]]) - z) / np.linalg.norm(z) < 1e-8
    q0 = synth.Inequalities(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros((1, 0)), np.zeros((1, 0)),
                            np.zeros((1, 0)), np.zeros((1, 0)))
    s0 = hkkt.Solver(precision="fp64")
    s0.analyze4(b.pattern, q0)
    assert s0.factor4(b, q0)[0] == 0
    rc, x0, _, y0, _, inf0 = s0.solve4(b.r1, np.zeros((1, 0)), b.r2, np.zeros((1, 0)))
    H.check_gpu_solution(oracle.System.from_batch(b), b.r1[0], b.r2[0], x0[0], y0[0],
                         dict(inf0[0], rr=oracle.System.from_batch(b).metrics(b.r1[0], b.r2[0], x0[0], y0[0])[0]),
                         1e-10)
