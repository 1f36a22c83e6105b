"""GPU parity of uneven groups: G KKT systems of different sizes and
patterns analysed as one block-diagonal system and run through every factor
and solve kernel together. Each member is checked against the oracle on its
own (the oracle's compensated residual of the member's KKT system: status 0
and RR <= kkt_tol, as in the single-pattern tests)."""
import numpy as np
import pytest

import oracle
from paper_2110_03636_amd import hkkt, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _members():
    # dense-like members of different sizes plus two grid-like ones
    dense = synth.uneven_dense_like(nb=3, lo=60, hi=400, seed=5100)
    return dense + [H.tiny_grid_like(2500, 41, dx_exp=8.0, gamma=1e6), H.tiny_grid_like(700, 42, dx_exp=4.0)]


def _group_values(mem, nb=1):
    """Combined [nb, ...] arrays of the members (every member has nb instances)."""
    cat = hkkt.GroupPattern.concat
    return dict(H=cat([b.H_val for b in mem]), Dx=cat([b.D_x for b in mem]), J=cat([b.J_val for b in mem]),
                delta=np.stack([b.delta for b in mem], axis=1), gamma=np.stack([b.gamma for b in mem], axis=1),
                r1=cat([b.r1 for b in mem]), r2=cat([b.r2 for b in mem]))


def _run(mem, precision, **kw):
    g = hkkt.GroupPattern([b.pattern for b in mem])
    v = _group_values(mem)
    s = hkkt.Solver(precision=precision, **kw).analyze_group(g)
    rc, st, fc = s.factor(v["H"], v["Dx"], v["J"], v["delta"], v["gamma"])
    out = s.solve(v["r1"], v["r2"])
    return g, s, (rc, st, fc), out


def _check_members(mem, g, x, y, infos, nb=1, kkt_tol=1e-10):
    xs, ys = g.split_x(x), g.split_y(y)
    for b in range(nb):
        for k, mb in enumerate(mem):
            o = oracle.System.from_batch(mb, b)
            rr, be, fl = o.metrics(mb.r1[b], mb.r2[b], xs[k][b], ys[k][b])
            inf = infos[b * g.G + k]
            assert inf["status"] == 0, (b, k, inf)
            assert rr <= kkt_tol, (b, k, rr, fl)
            assert abs(inf["rr"] - rr) <= 1e-8 * rr, (b, k, inf["rr"], rr)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_group_solve_each_member_equals_oracle(precision):
    mem = _members()
    g, s, (rc, st, fc), (rc2, x, y, infos) = _run(mem, precision)
    assert rc == 0 and list(st) == [0] * g.G and list(fc) == [-1] * g.G
    print("group", precision, [(i["cg_iters"], i["passes"], i["fp64_fallback"]) for i in infos])
    _check_members(mem, g, x, y, infos)
    for k, mb in enumerate(mem):
        assert s.inertia(k) == (mb.pattern.n_x, mb.pattern.m, 0)


def test_group_member_solution_matches_member_alone():
    """The same member solved alone and inside the group: the two solutions
    agree to the forward-error level RR allows (different elimination orders
    within the member are possible)."""
    mem = _members()
    g, s, _, (rc, x, y, infos) = _run(mem, "fp64")
    xs, ys = g.split_x(x), g.split_y(y)
    for k in (0, 3):
        mb = mem[k]
        s1 = hkkt.Solver().analyze(mb.pattern)
        s1.factor_batch(mb)
        _, x1, y1, _ = s1.solve(mb.r1, mb.r2)
        z = np.concatenate([xs[k][0], ys[k][0]])
        z1 = np.concatenate([x1[0], y1[0]])
        assert np.linalg.norm(z - z1) <= 1e-5 * np.linalg.norm(z1), k


def test_group_with_constraint_free_member_and_batch():
    """nb = 2 entries; one member without J rows (m = 0)."""
    rng = np.random.default_rng(43)
    n0 = 30
    Bm = rng.standard_normal((n0, n0)) * (rng.random((n0, n0)) < 0.3)
    Hd = Bm.T @ Bm + np.eye(n0)
    free = [H.batch_from_dense(Hd, 10 ** rng.uniform(-1, 1, n0), np.zeros((0, n0)), 1e-8, 1e4,
                               rng.standard_normal(n0), np.zeros(0)) for _ in range(2)]
    # stack the two instances of the constraint-free member
    f0, f1 = free
    import dataclasses
    fm = dataclasses.replace(f0, H_val=np.vstack([f0.H_val, f1.H_val]), J_val=np.zeros((2, 0)),
                             D_x=np.vstack([f0.D_x, f1.D_x]), delta=np.r_[f0.delta, f1.delta],
                             gamma=np.r_[f0.gamma, f1.gamma], r1=np.vstack([f0.r1, f1.r1]),
                             r2=np.zeros((2, 0)))
    grids = [synth.grid_like(1500, nb=2, seed=44, gammas=(1e4, 1e6), dx_exp=8.0),
             synth.grid_like(400, nb=2, seed=45, gammas=(1e2,), dx_exp=2.0)]
    mem = [grids[0], fm, grids[1]]
    g = hkkt.GroupPattern([b.pattern for b in mem])
    v = _group_values(mem, nb=2)
    for precision in ("fp64", "mixed"):
        s = hkkt.Solver(precision=precision).analyze_group(g)
        rc, st, fc = s.factor(v["H"], v["Dx"], v["J"], v["delta"], v["gamma"])
        assert rc == 0
        rc, x, y, infos = s.solve(v["r1"], v["r2"])
        _check_members(mem, g, x, y, infos, nb=2)
        assert infos[1]["cg_iters"] == 0 and infos[g.G + 1]["cg_iters"] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_group_not_spd_member_isolated(precision):
    """A member whose H_gamma is indefinite reports NOT_SPD with the oracle's
    column; the other members of the same entry still solve."""
    mem = _members()
    bad = 1
    p = mem[bad].pattern
    victim = 7
    diag = [q for q in range(p.H_rowptr[victim], p.H_rowptr[victim + 1]) if p.H_col[q] == victim][0]
    mem[bad].H_val[0, diag] -= 1e12
    g, s, (rc, st, fc), (rc2, x, y, infos) = _run(mem, precision)
    assert rc == hkkt.NOT_SPD
    assert [int(v) for v in st] == [hkkt.NOT_SPD if k == bad else 0 for k in range(g.G)]
    # the oracle factors the member in the group's elimination order
    perm = s.perm()[g.x_off[bad]:g.x_off[bad + 1]] - g.x_off[bad]
    ost, ofc = oracle.System.from_batch(mem[bad]).factor(perm)
    assert ost == 1 and fc[bad] - g.x_off[bad] == ofc
    assert infos[bad]["status"] == hkkt.NOT_SPD
    good = [k for k in range(g.G) if k != bad]
    xs, ys = g.split_x(x), g.split_y(y)
    for k in good:
        o = oracle.System.from_batch(mem[k])
        rr, be, fl = o.metrics(mem[k].r1[0], mem[k].r2[0], xs[k][0], ys[k][0])
        assert infos[k]["status"] == 0 and rr <= 1e-10, (k, rr, fl)


def test_group_hsolve_per_member():
    mem = _members()
    g = hkkt.GroupPattern([b.pattern for b in mem])
    v = _group_values(mem)
    s = hkkt.Solver().analyze_group(g)
    assert s.factor(v["H"], v["Dx"], v["J"], v["delta"], v["gamma"])[0] == 0
    rhs = np.random.default_rng(46).standard_normal((1, g.n_x))
    x = s.hsolve(rhs)
    for k, mb in enumerate(mem):
        o = oracle.System.from_batch(mb)
        o.factor(o.order_mindeg())
        sl = slice(g.x_off[k], g.x_off[k + 1])
        xo = o.hsolve(rhs[0, sl])
        assert np.linalg.norm(x[0, sl] - xo) <= 1e-6 * np.linalg.norm(xo), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_group_of_large_fronts_each_member_equals_oracle(precision):
    """Members of 2.5k–6k dense-like variables: each has fronts of thousands
    of rows (the blocked path: panel factorization launches with many
    work-groups per front, several fronts per level and launch, 128 x 128
    trailing updates). Every member's factor must succeed and its solution
    meet the oracle's bar; in particular each panel's factored diagonal
    block is stored only after every work-group of its front has read the
    unfactored one."""
    mem = synth.uneven_dense_like(nb=6, lo=2500, hi=6000, seed=5300)
    assert max(b.pattern.n_x for b in mem) > 4000
    g, s, (rc, st, fc), (rc2, x, y, infos) = _run(mem, precision)
    assert rc == 0 and list(st) == [0] * g.G, (rc, list(st), list(fc))
    assert s.stats()["max_width"] > 900
    _check_members(mem, g, x, y, infos)
