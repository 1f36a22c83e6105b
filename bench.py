#!/usr/bin/env python
"""Throughput benchmark of the hybrid direct-iterative KKT solve on one MI355X.

Metric: KKT solves per second at a relative KKT residual of 1e-10, for the
mixed-precision batched path, with the plain FP64 GPU path measured beside it.

Workload (one "step"): 256 instances of a grid-like KKT system with
n_x = 20,000, m = 10,000 sharing one sparsity pattern (per-instance values,
D_x = 10^U(-8,8), gamma alternating 1e4 / 1e6, delta = 1e-8), with every input
already resident in HBM. A step is one numeric factorization of all 256
instances plus one solve of all 256 to RR <= 1e-10 (FP32 factor and triangular
solves, FP64 refinement, FP64 refactor for instances whose refinement stalls).
The symbolic analysis is done once before timing (it is amortised over a
sequence of matrices).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def level_bytes(sym, s_elem):
    """Algorithmic bytes one instance moves per level of the supernodal tree,
    forward and backward solve: the structurally non-zero panel entries
    strictly below the diagonal (s_elem each), the reciprocal diagonal and
    the solution entries of the supernode's columns (read and written), the
    entries of the rows below (forward: read-modify-write of the ancestors'
    entries; backward: read) and their 4-byte row indices."""
    import numpy as np
    sn = sym.supernodes()
    first, rowptr, lp, lsn = sn["first"], sn["rowptr"], sn["level_ptr"], sn["level_sn"]
    fwd, bwd = [], []
    for l in range(len(lp) - 1):
        ids = lsn[lp[l]:lp[l + 1]]
        w = (first[ids + 1] - first[ids]).astype(np.int64)
        nr = (rowptr[ids + 1] - rowptr[ids]).astype(np.int64)
        nnz = nr * w - w * (w + 1) // 2
        below = nr - w
        fwd.append(int((s_elem * nnz + 3 * s_elem * w + 2 * s_elem * below + 4 * below).sum()))
        bwd.append(int((s_elem * nnz + 3 * s_elem * w + s_elem * below + 4 * below).sum()))
    return fwd, bwd


def per_instance_bytes(stats, s_elem):
    """Bytes one instance must move per kernel class and per application,
    per the layouts of the library (value bytes s_elem for the factor and
    the triangular-solve vector, 8 for FP64 values, 4 per index). Only
    structurally non-zero factor entries (nnz(L)) count; the padding the
    library stores in supernode panels does not."""
    n, m = stats["n_x"], stats["m"]
    nnzL, nnzJ = stats["nnz_L"], stats["nnz_J"]
    uv = stats["uv_entries"]
    rows = stats["sn_rows_total"]
    fwd = s_elem * nnzL + 2 * s_elem * n + 2 * s_elem * uv + 4 * uv
    bwd = s_elem * nnzL + 4 * rows + s_elem * (rows - n) + 2 * s_elem * n
    spmv = nnzJ * 12 + 8 * (m + n)
    return {"fwd": fwd, "bwd": bwd, "jt_spmv": spmv, "j_spmv": spmv}


def run_gpu(args):
    import numpy as np
    import torch
    from paper_2110_03636_amd import hkkt, synth

    torch.cuda.set_device(0)
    nb = args.nb
    b = synth.grid_like(args.n, nb=nb, seed=4000, gammas=(1e4, 1e6), dx_exp=8.0)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    H, D, J, R1, R2 = dev(b.H_val), dev(b.D_x), dev(b.J_val), dev(b.r1), dev(b.r2)

    tuned = {}
    given = {"mixed": args.schedule_mixed, "fp64": args.schedule_fp64}

    def make(prec, tune=False):
        s = hkkt.Solver(precision=prec, device=True, **solver_options(args))
        s.analyze(b.pattern)
        if given.get(prec):   # a schedule from an earlier autotuning (profiler runs)
            s.set_schedule(*[int(v) for v in given[prec].split(",")])
            tuned[prec] = dict(zip(("relax", "tree_width", "tree_staged"), s.schedule()), given=True)
        elif tune:   # once per pattern, outside the timed region (like the analysis)
            r = s.autotune(H, D, J, b.delta, b.gamma, R1, R2)
            tuned[prec] = {"relax": r["relax"], "tree_width": r["tree_width"], "tree_staged": r["tree_staged"]}
        return s

    def step(s, h=H, d=D, j=J, r1=R1, r2=R2, delta=b.delta, gamma=b.gamma):
        rc, st, fc = s.factor(h, d, j, delta, gamma)
        rc2, x, y, infos = s.solve(r1, r2)
        s.last_infos = infos
        s.last_xy = (x, y)
        return infos

    s = make("mixed", tune=not args.no_autotune)
    for _ in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    # one extra step with an event pair around every launch (an event pair
    # costs about as much as a short kernel, so the timed steps do not carry
    # them all): the per-class breakdown of a step; then one such step per
    # factor precision (the FP32 batch and the FP64 fallback batches run
    # kernels of the same classes with 4- and 8-byte elements)
    s.profile_select(None, 1)
    s.profile_begin()
    pinfos = step(s)
    prof = s.profile_end()                      # per step
    byprec = {}
    for prec, esz in (("mixed", 4), ("fp64", 8)):
        s.profile_precision(prec)
        s.profile_begin()
        pi = step(s)
        byprec[prec] = {"prof": s.profile_end(), "esz": esz, "infos": pi}
    s.profile_precision(None)
    stats = s.stats()
    nlev = len(level_bytes(s, 4)[0])
    # algorithmic bytes per (class, precision) over a profiled step:
    # per-instance bytes of one application of H_gamma^{-1} (J^T, J) times
    # the instance-applications run on factors of that precision. Each pass
    # applies H_gamma^{-1} once per CG iteration plus twice (w and the
    # primal recovery); J^T and J once per CG iteration plus twice / once.
    total, pprof, meta = {}, {}, {}
    for prec, d in byprec.items():
        pr, esz, pi = d["prof"], d["esz"], d["infos"]
        if prec == "fp64":
            cgk = [i["cg_iters_fp64"] for i in pi]; psk = [i["passes_fp64"] for i in pi]
        else:
            cgk = [i["cg_iters"] - i["cg_iters_fp64"] for i in pi]
            psk = [i["passes"] - i["passes_fp64"] for i in pi]
        apps = sum(cgk) + 2 * sum(psk)
        spmv_apps = 2 * sum(cgk) + 3 * sum(psk)
        lf, lb = level_bytes(s, esz)
        tk = tree_key(pr)
        lo = round(pr["bwd"][1] / pr[tk][1]) if pr[tk][1] else nlev
        per = per_instance_bytes(stats, esz)
        for cls, byt in (("fwd", sum(lf[:lo]) * apps), ("bwd", sum(lb[:lo]) * apps),
                         (tk, (sum(lf[lo:]) + sum(lb[lo:])) * apps),
                         ("jt_spmv", per["jt_spmv"] * spmv_apps / 2), ("j_spmv", per["j_spmv"] * spmv_apps / 2)):
            total[(cls, prec)] = byt
            pprof[(cls, prec)] = pr[cls]
        meta[prec] = {"lo": lo, "tk": tk, "apps": apps}
    best = max(total, key=lambda k: pprof[k][0])
    bcls, bprec = best
    # timed steps, with HIP events on the library's streams around every
    # PROF_EVERY-th launch of the dominant (class, precision) only: its
    # average launch duration over the timed region
    PROF_EVERY = 4
    s.profile_select([bcls], PROF_EVERY)
    s.profile_precision(bprec)
    s.profile_begin()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = step(s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    timed = s.profile_end()
    s.profile_select(None, 1)
    s.profile_precision(None)
    ok = sum(1 for i in infos if i["status"] == 0 and i["rr"] <= 1e-10)
    value = ok * args.steps / el
    xs, ys = s.last_xy
    launches = pprof[best][1]                   # per step
    avg_ms = timed[bcls][0] / max(timed[bcls][1], 1)
    per_launch = total[best] / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    # phases: all triangular-solve launches, and both SpMV kernels, both precisions
    phases = {}
    for name, classes in (("solve", ("fwd", "bwd", "tri_tree", "tri_tree_staged", "tri_wide")),
                          ("spmv", ("jt_spmv", "j_spmv"))):
        byt = sum(v for (c_, p_), v in total.items() if c_ in classes and pprof[(c_, p_)][1])
        ms = sum(byprec[p_]["prof"][c_][0] for p_ in byprec for c_ in classes)
        phases[name] = {"alg_GB": round(byt / 1e9, 3), "ms": round(ms, 3),
                        "GBps": round(byt / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                        "frac": round(byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None}
    phases["stream_copy_GBps"] = stream_copy_gbps()
    T = {"mixed": "float", "fp64": "double"}[bprec]
    kname = {"fwd": f"k_fwd_lvl<{T},true> (forward supernodal triangular solve, one launch per level)",
             "bwd": f"k_bwd_lvl<{T}> (backward supernodal triangular solve, one launch per level)",
             "tri_tree": f"k_tri_tree<{T},true,512> (one sweep over the thin top levels)",
             "tri_tree_staged": f"k_tri_tree2<{T},512,32> (one sweep over the thin top levels, "
                                "working set staged in LDS)",
             "jt_spmv": "k_jt", "j_spmv": "k_j"}[bcls]
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": int(per_launch),
                "launches_per_step": launches, "factor_precision": bprec,
                "per_level_launch_levels": meta[bprec]["lo"],
                "timing": f"HIP events around every {PROF_EVERY}th launch of this kernel on {bprec} factors "
                          f"over the {args.steps} timed steps ({timed[bcls][1]} launches timed); bytes and "
                          f"launches per step from one profiled step with events around every launch"}

    # plain FP64 comparators: batched (same steps as the mixed path, fewer of
    # them), and one instance at a time
    fp64_batched = fp64_plain = None
    if not args.no_comparators:
        s64 = make("fp64", tune=not args.no_autotune)
        step(s64)
        torch.cuda.synchronize()
        k64 = max(1, min(3, args.steps))
        t0 = time.perf_counter()
        for _ in range(k64):
            infos64 = step(s64)
        torch.cuda.synchronize()
        fp64_batched = sum(1 for i in infos64 if i["status"] == 0 and i["rr"] <= 1e-10) * k64 / (
            time.perf_counter() - t0)
        s1 = make("fp64")   # same scaling option as the batched solvers
        k1 = min(args.single, nb)
        step(s1, H[:1], D[:1], J[:1], R1[:1], R2[:1], b.delta[:1], b.gamma[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        good = 0
        for i in range(k1):
            sl = slice(i, i + 1)
            inf = step(s1, H[sl], D[sl], J[sl], R1[sl], R2[sl], b.delta[sl], b.gamma[sl])
            good += inf[0]["status"] == 0 and inf[0]["rr"] <= 1e-10
        torch.cuda.synchronize()
        fp64_plain = good / (time.perf_counter() - t0)

    cg = [i["cg_iters"] for i in infos]
    extra = {
        "fp64_batched_solves_per_s": round(fp64_batched, 2) if fp64_batched else None,
        "fp64_plain_solves_per_s": round(fp64_plain, 2) if fp64_plain else None,
        "fp64_plain_instances": min(args.single, nb),
        "speedup_vs_plain_fp64": round(value / fp64_plain, 2) if fp64_plain else None,
        "speedup_vs_fp64_batched": round(value / fp64_batched, 3) if fp64_batched else None,
        "converged": f"{ok}/{nb}",
        "not_converged": [{"rr": i["rr"], "floor": i["floor"], "fallback": i["fp64_fallback"]}
                          for i in infos if not (i["status"] == 0 and i["rr"] <= 1e-10)],
        "max_rr": max(i["rr"] for i in infos),
        "fp64_fallbacks": sum(i["fp64_fallback"] for i in infos),
        "cg_iters_mean": round(float(np.mean(cg)), 2),
        "passes_max": max(i["passes"] for i in infos),
        "profile_ms_per_step": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
        "profile_ms_per_step_by_factor_precision": {
            p_: {k: round(v[0], 3) for k, v in d["prof"].items() if v[1]} for p_, d in byprec.items()},
        "profile_note": "per-class kernel time of one extra step with an event pair around every launch",
        "phases": phases,
        "autotuned": tuned or None,
        "symbolic": {k: stats[k] for k in ("nnz_L", "L_storage", "supernodes", "levels", "etree_height")},
    }
    extra["_xy"] = (xs.cpu().numpy(), ys.cpu().numpy())
    return value, el, roofline, extra, b


# dense matrix-core peaks of MI355X (TFLOP/s)
MFMA_PEAK = {"mixed": 157.3, "fp64": 78.6}
LDS_FRONT_ROWS = {"mixed": 128, "fp64": 90}   # fronts above these row counts take the blocked MFMA path
FRONT_NB = 32                                 # columns per step of the blocked fronts


def big_front_flops(sym, lds_rows):
    """Flops of the trailing updates (C -= L21 L21^T over the lower triangle)
    of the fronts that take the blocked MFMA path, and of the whole
    factorization (sum over columns of c_j^2 multiply-adds, c_j = entries
    below the diagonal of column j)."""
    import numpy as np
    sn = sym.supernodes()
    first, rowptr = sn["first"], sn["rowptr"]
    upd = 0
    for q in range(first.size - 1):
        w = int(first[q + 1] - first[q])
        nr = int(rowptr[q + 1] - rowptr[q])
        if nr <= lds_rows:
            continue
        for kb in range(0, w, FRONT_NB):
            bw = min(FRONT_NB, w - kb)
            mt = nr - kb - bw
            upd += mt * (mt + 1) * bw          # lower triangle, 2 flops per multiply-add
    return upd, float(sym.stats()["flops_proxy"]) * 2


def solver_options(args):
    """Options every benchmark mode passes to its solvers (the headline's)."""
    extra = {} if args.mixed_pivot_tol is None else {"mixed_pivot_tol": args.mixed_pivot_tol}
    if args.cg_tol is not None:
        extra["cg_tol"] = args.cg_tol
    return dict(kkt_tol=1e-10, scaling=args.scaling, refine_inexact=args.refine_inexact,
                mixed_check=args.mixed_check, **extra)


def factor_mfma(args):
    """Numeric factorization of one dense-like system (the generator of the
    1200-variable configuration at a larger size), whose top supernodes are
    dense fronts of thousands of rows: achieved TFLOP/s of the blocked
    trailing updates (k_big_update, MFMA) against the matrix-core peak."""
    import torch
    from paper_2110_03636_amd import hkkt, synth
    b = synth.dense_like(args.factor_mfma, seed=1000 + args.factor_mfma)
    dev = lambda x: torch.as_tensor(x, device="cuda")
    H, D, J = dev(b.H_val), dev(b.D_x), dev(b.J_val)
    out = {}
    for prec in ("mixed", "fp64"):
        # the FP32 factor alone: no pivot test routing instances to an FP64 refactor
        s = hkkt.Solver(precision=prec, device=True, mixed_pivot_tol=0.0)
        s.analyze(b.pattern)
        s.factor(H, D, J, b.delta, b.gamma)
        torch.cuda.synchronize()
        s.profile_begin()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rc, st, fc = s.factor(H, D, J, b.delta, b.gamma)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        prof = s.profile_end()
        upd, total = big_front_flops(s, LDS_FRONT_ROWS[prec])
        big_ms = prof["front_big"][0] / args.steps
        out[prec] = {"factor_ms": round(el * 1e3, 3), "status": int(st[0]),
                     "big_front_ms": round(big_ms, 3), "big_front_update_gflop": round(upd / 1e9, 2),
                     "factor_gflop": round(total / 1e9, 2),
                     "big_front_tflops": round(upd / (big_ms * 1e-3) / 1e12, 2),
                     "factor_tflops": round(total / el / 1e12, 2),
                     "peak_tflops": MFMA_PEAK[prec],
                     "big_front_frac": round(upd / (big_ms * 1e-3) / 1e12 / MFMA_PEAK[prec], 4)}
    print(json.dumps({"workload": f"dense-like n_x={args.factor_mfma}, m={args.factor_mfma // 2}, one instance",
                      "symbolic": {k: s.stats()[k] for k in ("nnz_L", "L_storage", "max_width", "supernodes")},
                      **out}))


def uneven_group(args):
    """Uneven sizes in one launch: args.uneven dense-like systems (n_x
    log-uniform in [2000, 50000], m = n_x/2, each its own pattern) analysed as
    one group and factored and solved together in mixed precision."""
    import numpy as np
    import torch
    from paper_2110_03636_amd import hkkt, synth
    mem = synth.uneven_dense_like(nb=args.uneven, lo=2000, hi=args.uneven_hi, seed=5000)
    g = hkkt.GroupPattern([b.pattern for b in mem])
    cat = hkkt.GroupPattern.concat
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), device="cuda")
    H, D, J = dev(cat([b.H_val for b in mem])), dev(cat([b.D_x for b in mem])), dev(cat([b.J_val for b in mem]))
    R1, R2 = dev(cat([b.r1 for b in mem])), dev(cat([b.r2 for b in mem]))
    delta = np.stack([b.delta for b in mem], axis=1)
    gamma = np.stack([b.gamma for b in mem], axis=1)
    s = hkkt.Solver(precision="mixed", device=True, **solver_options(args))
    t0 = time.perf_counter()
    s.analyze_group(g)
    t_an = time.perf_counter() - t0
    print(f"uneven: analysed {g.G} members, n_x total {g.n_x} in {t_an:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st, fc = s.factor(H, D, J, delta, gamma)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    print(f"uneven: factor {t_f:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    rc2, x, y, infos = s.solve(R1, R2)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    ok = sum(1 for i in infos if i["status"] == 0 and i["rr"] <= 1e-10)
    statuses = {}
    for i in infos:
        statuses[str(i["status"])] = statuses.get(str(i["status"]), 0) + 1
    st_ = s.stats()
    print(json.dumps({"workload": f"{g.G} dense-like systems in one group, n_x log-uniform in [2000, {args.uneven_hi}] "
                                  f"(min {min(b.pattern.n_x for b in mem)}, max {max(b.pattern.n_x for b in mem)}, "
                                  f"total {g.n_x}), mixed precision, target RR<=1e-10",
                      "analyze_s": round(t_an, 2), "factor_s": round(t_f, 3), "solve_s": round(t_s, 3),
                      "solves_per_s": round(ok / (t_f + t_s), 3), "converged": f"{ok}/{g.G}", "status_counts": statuses,
                      "max_rr": float(np.nanmax([i["rr"] for i in infos])) if ok else None,
                      "fp64_fallbacks": sum(i["fp64_fallback"] for i in infos),
                      "cg_iters_max": max(i["cg_iters"] for i in infos), "passes_max": max(i["passes"] for i in infos),
                      "symbolic": {k: st_[k] for k in ("nnz_L", "L_storage", "cb_entries", "max_width", "levels")}}))


def large_single(args):
    """One large grid-like system (connected reading) in mixed precision,
    gamma = 1e6: sustained factor + solve cycles on a fixed pattern, each with
    a fresh D_x (the next interior iteration), after one autotuning."""
    import numpy as np
    import torch
    from paper_2110_03636_amd import hkkt, synth
    n = args.large
    t0 = time.perf_counter()
    b = synth.grid_like(n, nb=1, seed=5100, gammas=(1e6,), dx_exp=8.0)
    print(f"large: generated n_x={n} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), device="cuda")
    H, J, R1, R2 = dev(b.H_val), dev(b.J_val), dev(b.r1), dev(b.r2)
    dxs = [dev(synth.fresh_dx(n, 5200 + k)[None]) for k in range(args.cycles)]
    s = hkkt.Solver(precision="mixed", device=True, **solver_options(args))
    t0 = time.perf_counter()
    s.analyze(b.pattern)
    t_an = time.perf_counter() - t0
    print(f"large: analysed in {t_an:.1f} s", file=sys.stderr, flush=True)
    if args.schedule_mixed:   # a schedule from an earlier autotuning
        s.set_schedule(*[int(v) for v in args.schedule_mixed.split(",")])
        tune = dict(zip(("relax", "tree_width", "tree_staged"), s.schedule()), given=True)
    else:
        tune = s.autotune(H, dxs[0], J, b.delta, b.gamma)
    print(f"large: schedule {tune['relax']}/{tune['tree_width']}/{tune['tree_staged']}", file=sys.stderr, flush=True)
    s.factor(H, dxs[0], J, b.delta, b.gamma)
    s.solve(R1, R2)
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for k in range(args.cycles):
        s.factor(H, dxs[k], J, b.delta, b.gamma)
        rc, x, y, infos = s.solve(R1, R2)
        res.append(infos[0])
        print(f"large: cycle {k} rr={infos[0]['rr']:.2e} floor={infos[0]['floor']:.2e} cg={infos[0]['cg_iters']} "
              f"passes={infos[0]['passes']} fb={infos[0]['fp64_fallback']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ok = sum(1 for i in res if i["status"] == 0 and i["rr"] <= 1e-10)
    st = s.stats()
    print(json.dumps({"workload": f"grid-like n_x={n}, m={n // 2}, gamma=1e6, mixed precision, "
                                  f"{args.cycles} factor+solve cycles with fresh D_x, target RR<=1e-10",
                      "analyze_s": round(t_an, 2), "autotuned" if not tune.get("given") else "schedule_given":
                          {"relax": tune["relax"], "tree_width": tune["tree_width"], "tree_staged": tune["tree_staged"]},
                      "sustained_solves_per_s": round(ok / el, 3), "s_per_cycle": round(el / args.cycles, 3),
                      "converged": f"{ok}/{args.cycles}", "max_rr": max(i["rr"] for i in res),
                      "not_converged": [{"cycle": k, "rr": i["rr"], "floor": i["floor"], "status": i["status"]}
                                        for k, i in enumerate(res) if not (i["status"] == 0 and i["rr"] <= 1e-10)],
                      "fp64_fallbacks": sum(i["fp64_fallback"] for i in res),
                      "cg_iters_mean": round(float(np.mean([i["cg_iters"] for i in res])), 1),
                      "symbolic": {k: st[k] for k in ("nnz_L", "L_storage", "levels", "max_width")}}))


def solve_only(args):
    """Factor reuse across adjacent Newton steps (Sec. 2 reuse list): the
    256-instance batch is factored once, then solved for args.solve_only
    fresh right-hand sides in a row (the next Newton steps' residuals),
    each to RR <= 1e-10; solves/s beside the factor+solve rate of the same
    batch."""
    import numpy as np
    import torch
    from paper_2110_03636_amd import hkkt, synth
    b = synth.grid_like(args.n, nb=args.nb, seed=4000, gammas=(1e4, 1e6), dx_exp=8.0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    H, D, J = dev(b.H_val), dev(b.D_x), dev(b.J_val)
    rng = np.random.default_rng(4100)
    rhs = [(dev(rng.standard_normal((args.nb, args.n))), dev(rng.standard_normal((args.nb, args.n // 2))))
           for _ in range(args.solve_only)]
    s = hkkt.Solver(precision="mixed", device=True, **solver_options(args))
    s.analyze(b.pattern)
    if args.schedule_mixed:
        s.set_schedule(*[int(v) for v in args.schedule_mixed.split(",")])
    elif not args.no_autotune:
        s.autotune(H, D, J, b.delta, b.gamma, rhs[0][0], rhs[0][1])
    s.factor(H, D, J, b.delta, b.gamma)
    s.solve(*rhs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.factor(H, D, J, b.delta, b.gamma)
    rc, x, y, infos = s.solve(*rhs[0])
    torch.cuda.synchronize()
    t_fs = time.perf_counter() - t0
    ok_fs = sum(1 for i in infos if i["status"] == 0 and i["rr"] <= 1e-10)
    t0 = time.perf_counter()
    ok = 0
    for r1, r2 in rhs:
        rc, x, y, infos = s.solve(r1, r2)
        ok += sum(1 for i in infos if i["status"] == 0 and i["rr"] <= 1e-10)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"workload": f"batch of {args.nb} grid-like KKT systems, n_x={args.n}, one factorization, "
                                  f"{args.solve_only} right-hand sides in a row, mixed precision, target RR<=1e-10",
                      "solve_only_solves_per_s": round(ok / el, 2), "ms_per_solve_batch": round(el / args.solve_only * 1e3, 3),
                      "factor_plus_solve_solves_per_s": round(ok_fs / t_fs, 2),
                      "converged": f"{ok}/{args.nb * args.solve_only}"}))


def profile_hsolve(args):
    """Counter-collection driver: a 1 GiB device copy (calibration of the
    byte counters) followed by args.profile_hsolve applications of
    H_gamma^{-1} to all instances of the workload, on factors of precision
    args.profile_precision, with the schedule given for that precision (else
    the library default)."""
    import numpy as np
    import torch
    from paper_2110_03636_amd import hkkt, synth
    a = torch.empty(2**28, dtype=torch.float32, device="cuda").fill_(1.0)
    torch.empty_like(a).copy_(a)
    torch.cuda.synchronize()
    prec = args.profile_precision
    b = synth.grid_like(args.n, nb=args.nb, seed=4000, gammas=(1e4, 1e6), dx_exp=8.0)
    dev = lambda x: torch.as_tensor(x, device="cuda")
    # the FP32 factor of every instance (no pivot test sending some to FP64)
    s = hkkt.Solver(precision=prec, device=True, mixed_pivot_tol=0.0)
    s.analyze(b.pattern)
    sched = {"mixed": args.schedule_mixed, "fp64": args.schedule_fp64}[prec]
    if sched:
        s.set_schedule(*[int(v) for v in sched.split(",")])
    s.factor(dev(b.H_val), dev(b.D_x), dev(b.J_val), b.delta, b.gamma)
    rhs = dev(np.random.default_rng(0).standard_normal((args.nb, args.n)))
    s.profile_begin()
    for _ in range(args.profile_hsolve):
        s.hsolve(rhs)
    prof = s.profile_end()
    lf, lb = level_bytes(s, 4 if prec == "mixed" else 8)
    tk = tree_key(prof)
    lo = round(prof["bwd"][1] / prof[tk][1]) if prof[tk][1] else len(lf)
    print(json.dumps({"precision": prec, "schedule": list(s.schedule()), "levels": len(lf),
                      "per_level_launch_levels": lo, "tree_kernel": tk,
                      "alg_bytes_per_launch": {"fwd": sum(lf[:lo]) * args.nb / max(lo, 1),
                                               "bwd": sum(lb[:lo]) * args.nb / max(lo, 1),
                                               tk: (sum(lf[lo:]) + sum(lb[lo:])) * args.nb}}))


def tree_key(prof):
    """Profile class of the tree-traversal launches of a run (the staged
    kernel where the top levels fit it, else the global-memory one)."""
    return "tri_tree_staged" if prof.get("tri_tree_staged", (0, 0))[1] else "tri_tree"


def load_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, valid only while the kernel source is unchanged."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            t = json.load(f)
        src = open(os.path.join(ROOT, "paper_2110_03636_amd", "csrc", "kernels.inl"), "rb").read()
        if hashlib.sha256(src).hexdigest() != t.get("kernels_sha256"):
            return None
        return t
    except (OSError, ValueError):
        return None


def stream_copy_gbps():
    """Measured device-to-device copy bandwidth (1 GiB read + 1 GiB written),
    best of five, the practical HBM ceiling beside the 8 TB/s nominal peak."""
    import torch
    a = torch.empty(2**28, dtype=torch.float32, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    best = 0.0
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, c
    return round(best, 1)


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(b, budget_s, xy=None):
    """The oracle (plain FP64 C, one instance per thread) on the host cores:
    first a 1-thread run over the first instances for about budget_s / 3,
    then a pool of one thread per core (at most 16, the host share of one
    GPU) over the whole batch for up to budget_s. Ordering once per pattern,
    not timed (as on the GPU). Also the forward error of the GPU's solution
    against the oracle's, per instance the oracle solved."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    o0 = oracle.System.from_batch(b, 0)
    perm = o0.order_mindeg()
    zs = {}

    def one(i):
        o = oracle.System.from_batch(b, i)
        o.factor(perm)
        x, y, info = o.solve(b.r1[i], b.r2[i], kkt_tol=1e-10)
        zs[i] = (np.concatenate([x, y]), info)

    t0 = time.perf_counter()
    n1 = 0
    while n1 < max(1, b.nb // 4) and (time.perf_counter() - t0 < budget_s / 3 or n1 == 0):
        one(n1)
        n1 += 1
    rate1 = n1 / (time.perf_counter() - t0)
    model, avail = host_cpu()
    threads = max(1, min(16, avail))
    # every thread takes instances from a shared counter until the budget is
    # spent; the rate counts the instances finished in the pool's wall time
    import threading
    lock = threading.Lock()
    nxt = [n1]
    done = [0]
    t1 = time.perf_counter()

    def worker():
        while True:
            with lock:
                i = nxt[0]
                if i >= b.nb or time.perf_counter() - t1 > budget_s:
                    return
                nxt[0] += 1
            one(i)
            with lock:
                done[0] += 1

    with ThreadPoolExecutor(max_workers=threads) as ex:
        for f in [ex.submit(worker) for _ in range(threads)]:
            f.result()
    wall = time.perf_counter() - t1
    rate = done[0] / wall if wall > 0 else rate1
    out = {"value": round(rate, 3), "unit": "KKT solves/s", "cores": threads, "kind": "oracle",
           "one_core_value": round(rate1, 4), "cpu_model": model, "cpus_available": avail,
           "sample": f"{n1} instances on 1 thread ({rate1:.2f}/s), then {done[0]} more of the {b.nb} on "
                     f"{threads} threads in {wall:.1f} s; factor+solve to RR<=1e-10, ordering excluded"}
    if xy is not None:
        x, y = xy
        errs = {}
        for i, (z, info) in sorted(zs.items()):
            zg = np.concatenate([x[i], y[i]])
            errs[i] = float(np.linalg.norm(zg - z) / np.linalg.norm(z))
        v = np.array(list(errs.values()))
        g = np.array([b.gamma[i] for i in errs])
        out["fwd_err_vs_oracle"] = {
            "what": "||z_gpu - z_oracle||_2 / ||z_oracle||_2 per instance the oracle solved (index: error)",
            "max": float(v.max()), "median": float(np.median(v)),
            "by_gamma": {f"{gg:g}": {"max": float(v[g == gg].max()), "median": float(np.median(v[g == gg]))}
                         for gg in sorted(set(g.tolist()))},
            "per_instance": {str(i): float(f"{e:.2e}") for i, e in errs.items()}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--single", type=int, default=32, help="instances timed on the plain FP64 path")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--schedule-mixed", default="", help="relax,tree_width,staged for the mixed solver "
                    "(skips its autotuning; for profiler runs)")
    ap.add_argument("--schedule-fp64", default="", help="the same for the FP64 batched solver")
    ap.add_argument("--no-comparators", action="store_true",
                    help="skip the FP64 batched and plain FP64 runs (profiler runs of the mixed path)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed-check", type=int, default=0,
                    help="1: probe each FP32 factor at factor time and refactor in FP64 where it cannot drive "
                         "refinement")
    ap.add_argument("--mixed-pivot-tol", type=float, default=None,
                    help="FP32 pivot test threshold (library default 2^-12)")
    ap.add_argument("--cg-tol", type=float, default=None,
                    help="CG tolerance of the first hybrid pass (library default 1e-12)")
    ap.add_argument("--refine-inexact", type=int, default=1,
                    help="1 (default): refinement passes after the first stop CG at the accuracy the correction "
                         "needs; 0: every pass at the CG tolerance")
    ap.add_argument("--scaling", type=int, default=1,
                    help="1 (default): symmetrized Ruiz scaling of K before the hybrid method (Sec. 4.1), for the "
                         "batched and the plain solvers; 0: none")
    ap.add_argument("--no-autotune", action="store_true", help="library default schedule instead of the autotuner's")
    ap.add_argument("--uneven", type=int, default=0,
                    help="this many dense-like systems of uneven sizes in one group (factor + solve once)")
    ap.add_argument("--uneven-hi", type=int, default=50_000, help="largest n_x of --uneven")
    ap.add_argument("--large", type=int, default=0, help="one grid-like system of this n_x: sustained cycles")
    ap.add_argument("--cycles", type=int, default=20, help="factor + solve cycles of --large")
    ap.add_argument("--factor-mfma", type=int, default=0,
                    help="factorization of one dense-like system of this n_x (MFMA large-front measurement)")
    ap.add_argument("--solve-only", type=int, default=0,
                    help="factor once, then solve this many right-hand sides in a row (factor reuse)")
    ap.add_argument("--profile-precision", default="mixed", choices=("mixed", "fp64"),
                    help="factor precision of --profile-hsolve")
    ap.add_argument("--profile-hsolve", type=int, default=0,
                    help="counter-collection mode: calibration copy + this many H_gamma^{-1} applications")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(batches shard by instance across GPUs without communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if args.profile_hsolve:
        profile_hsolve(args)
        return
    if args.solve_only:
        solve_only(args)
        return
    if args.factor_mfma:
        factor_mfma(args)
        return
    if args.uneven:
        uneven_group(args)
        return
    if args.large:
        large_single(args)
        return
    value, el, roofline, extra, b = run_gpu(args)
    tr = load_traffic()
    ratio = None
    for k, r in (tr or {}).get("traffic_over_alg", {}).items():
        if roofline["kernel"].startswith(k):
            ratio = r
    if ratio is not None:
        # counter-measured HBM bytes per launch relative to the algorithmic
        # bytes of the same launches, applied to this run's launches
        roofline["traffic"] = int(ratio * roofline["bytes_per_launch"])
        roofline["traffic_over_alg"] = ratio
    xy = extra.pop("_xy", None)
    cpu = None if args.no_cpu else cpu_baseline(b, args.cpu_budget, xy)
    out = {
        "metric": "KKT solves/sec at 1e-10 rel. KKT residual: mixed-prec batched vs plain FP64",
        "value": round(value, 2),
        "unit": "KKT solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factor+triangular solves, f64 assembly/CG/residual/refinement",
        "data": "synthetic",
        "config": {"workload": f"batch of {args.nb} grid-like KKT systems, n_x={args.n}, m={args.n // 2}, "
                               f"shared pattern, mixed precision, target RR<=1e-10",
                   "global_batch": args.nb, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
