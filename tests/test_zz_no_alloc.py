"""The allocation-free triangular solve (hkkt_hsolve_noalloc) against the
allocating one (hkkt_hsolve) on the same factor, through the C ABI.

Bars (the ones the H_gamma^{-1} parity tests use):
  - deterministic forward solves (pull mode, fixed summation order): both
    entry points run the same kernels in the same order, so the solutions are
    bitwise equal;
  - FP atomics (push mode) in FP64: normwise backward error <= 1e-14 on the
    dense H_gamma, and the two solutions equal to 1e-10 relative on a
    well-conditioned H_gamma (they differ only in the order of the atomic
    additions);
  - the FP32 factor: backward error <= 1e-5 and the solutions within 1e-4.
Every case makes two calls in a row, the second with a smaller input, on the
one scratch array of the GPU; the device's free memory does not change
across the allocation-free calls."""
import numpy as np
import pytest

from paper_2110_03636_amd import hkkt
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _solver(b, precision, det):
    s = hkkt.Solver(precision=precision, device=True, deterministic=det)
    s.analyze(b.pattern)
    rc, st, fc = s.factor(_dev(b.H_val), _dev(b.D_x), _dev(b.J_val), b.delta, b.gamma)
    assert rc == 0
    return s


def _be(b, i, x, rhs):
    A = H.dense_Hgamma(b, i)
    return np.linalg.norm(A @ x - rhs) / (np.linalg.norm(A, np.inf) * np.linalg.norm(x) + np.linalg.norm(rhs))


def _call_noalloc(s, rhs, check_mem=True):
    """check_mem: the same kernels ran before in this process (the HIP
    runtime may reserve spill memory at a kernel's first launch)."""
    import torch
    x = torch.full_like(rhs, float("nan"))   # every entry must be written
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    s.hsolve_noalloc(rhs, x)
    torch.cuda.synchronize()
    if check_mem:
        assert torch.cuda.mem_get_info()[0] == free0
    return x


@pytest.mark.parametrize("precision,det", [("fp64", 1), ("fp64", 0), ("mixed", 0)])
def test_noalloc_equals_hsolve_two_calls(precision, det):
    import torch
    cases = [H.tiny_grid_like(3000, 51, dx_exp=1.0, gamma=10.0, nb=3),    # first call
             H.tiny_grid_like(1200, 52, dx_exp=1.0, gamma=10.0, nb=2)]    # second call: smaller input
    for b in cases:
        s = _solver(b, precision, det)
        rhs = _dev(np.random.default_rng(b.pattern.n_x).standard_normal((b.nb, b.pattern.n_x)))
        ref = s.hsolve(rhs)
        x = _call_noalloc(s, rhs)
        assert not torch.isnan(x).any()
        if det:
            assert torch.equal(x, ref)
            continue
        xr, xh, rh = x.cpu().numpy(), ref.cpu().numpy(), rhs.cpu().numpy()
        for i in range(b.nb):
            be = _be(b, i, xr[i], rh[i])
            rel = np.linalg.norm(xr[i] - xh[i]) / np.linalg.norm(xh[i])
            if precision == "fp64":
                assert be < 1e-14 and rel < 1e-10, (i, be, rel)
            else:
                assert be < 1e-5 and rel < 1e-4, (i, be, rel)


def test_noalloc_before_any_solve_uses_global_tree_kernel():
    """Without a staged panel copy built by an earlier solve of this
    factorization the levels of the staged kernel run in the global-memory
    tree kernel: same solution to the FP64 bar, and the later hsolve agrees."""
    b = H.tiny_grid_like(2500, 53, dx_exp=1.0, gamma=10.0, nb=2)
    s = _solver(b, "fp64", 0)
    rhs = _dev(np.random.default_rng(7).standard_normal((b.nb, b.pattern.n_x)))
    x = _call_noalloc(s, rhs, check_mem=False).cpu().numpy()
    ref = s.hsolve(rhs).cpu().numpy()
    rh = rhs.cpu().numpy()
    for i in range(b.nb):
        assert _be(b, i, x[i], rh[i]) < 1e-14
        assert np.linalg.norm(x[i] - ref[i]) / np.linalg.norm(ref[i]) < 1e-10


def test_noalloc_rejects_host_pointers_and_oversize():
    import torch
    b = H.tiny_grid_like(1000, 54, dx_exp=1.0, gamma=10.0)
    s = hkkt.Solver(precision="fp64", device=False)
    s.analyze(b.pattern)
    assert s.factor_batch(b)[0] == 0
    xh = np.zeros((1, b.pattern.n_x))
    with pytest.raises(hkkt.HKKTError) as e:
        hkkt._check(hkkt.lib().hkkt_hsolve_noalloc(s._ctx, 1, xh.ctypes.data, xh.ctypes.data), s._ctx)
    assert e.value.code == hkkt.ERR_ARG
    # 2100 instances x 2000 variables x (8 + 8) bytes > 64 MiB
    one = H.tiny_grid_like(2000, 55, dx_exp=1.0, gamma=10.0)
    nb = 2100
    sd = hkkt.Solver(precision="fp64", device=True)
    sd.analyze(one.pattern)
    rc, st, fc = sd.factor(_dev(np.repeat(one.H_val, nb, 0)), _dev(np.repeat(one.D_x, nb, 0)),
                           _dev(np.repeat(one.J_val, nb, 0)), np.repeat(one.delta, nb), np.repeat(one.gamma, nb))
    assert rc == 0
    rhs = torch.zeros((nb, one.pattern.n_x), dtype=torch.float64, device="cuda")
    with pytest.raises(hkkt.HKKTError) as e:
        sd.hsolve_noalloc(rhs, torch.empty_like(rhs))
    assert e.value.code == hkkt.ERR_ARG and "maximum" in str(e.value)


@pytest.mark.parametrize("precision,det", [("fp64", 1), ("mixed", 0)])
def test_noalloc_replayed_from_a_captured_graph(precision, det):
    """The allocation-free entry point launches kernels only (no allocation,
    copy, fill or synchronisation), so a caller can capture applications of
    H_gamma^{-1} in a hipGraph on the context's stream and replay them.
    Three applications (x1 = H^-1 b, x2 = H^-1 x1, x3 = H^-1 x2) captured
    once, replayed three times with eager work and synchronisations between
    the replays; every replay equals the eager chain (bitwise with
    deterministic solves, else to the parity bars)."""
    import torch
    b = H.tiny_grid_like(3000, 56, dx_exp=1.0, gamma=10.0, nb=3)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = _solver(b, precision, det)
        rhs = _dev(np.random.default_rng(9).standard_normal((b.nb, b.pattern.n_x)))
        x1, x2, x3 = (torch.empty_like(rhs) for _ in range(3))
        s.hsolve(rhs)                        # the staged tree kernel's panel copy of this factor
        s.hsolve_noalloc(rhs, x1)
        s.hsolve_noalloc(x1, x2)
        s.hsolve_noalloc(x2, x3)
        ref = [x1.clone(), x2.clone(), x3.clone()]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        s.hsolve_noalloc(rhs, x1)
        s.hsolve_noalloc(x1, x2)
        s.hsolve_noalloc(x2, x3)
    torch.cuda.synchronize()
    for rep in range(3):
        for x in (x1, x2, x3):
            x.fill_(float("nan"))
        eager = s.hsolve(rhs)                # eager work on the same context between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (x, r) in enumerate(zip((x1, x2, x3), ref)):
            assert not torch.isnan(x).any(), (rep, k)
            if det:
                assert torch.equal(x, r), (rep, k)
            else:
                rel = float((x - r).norm() / r.norm())
                assert rel < (1e-4 if precision == "mixed" else 1e-10), (rep, k, rel)
        assert float((eager - ref[0]).norm() / ref[0].norm()) < (1e-4 if precision == "mixed" else 1e-10)
