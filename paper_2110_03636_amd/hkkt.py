"""Thin ctypes binding of the C ABI in include/hkkt.h (argument marshalling
only; every step of the solve runs in the HIP library).

Host mode takes numpy arrays; device mode takes torch tensors on the GPU and
binds the context to torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhkkt.so")

OK, NOT_SPD, CG_BREAKDOWN, NOT_CONVERGED = 0, 1, 2, 3
ERR_ARG, ERR_PATTERN, ERR_STATE, ERR_DEVICE, ERR_OOM = -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
PTR_HOST, PTR_DEVICE = 0, 1

EXPORTS = [
    "hkkt_default_options", "hkkt_create", "hkkt_destroy", "hkkt_last_error", "hkkt_analyze",
    "hkkt_factor_batch", "hkkt_factor", "hkkt_solve_batch", "hkkt_solve", "hkkt_inertia",
    "hkkt_symbolic_create", "hkkt_symbolic_destroy", "hkkt_get_symbolic", "hkkt_symbolic_stats",
    "hkkt_symbolic_perm", "hkkt_symbolic_supernodes", "hkkt_get_factor", "hkkt_hsolve", "hkkt_timings",
    "hkkt_profile_begin", "hkkt_profile_end", "hkkt_analyze_group", "hkkt_symbolic_create_group", "hkkt_autotune",
    "hkkt_symbolic_cb_offsets", "hkkt_get_schedule", "hkkt_set_schedule", "hkkt_hsolve_noalloc",
    "hkkt_factor_regularized", "hkkt_gamma_heuristic", "hkkt_profile_select",
    "hkkt_analyze4", "hkkt_factor4_batch", "hkkt_solve4_batch", "hkkt_profile_precision",
]
PROF_NAMES = ["assemble", "front_lds", "front_big", "fwd", "bwd", "jt_spmv", "j_spmv", "cg_vec",
              "cg_scalar", "residual", "other", "tri_wide", "tri_tree", "tri_tree_staged",
              "tri_flow"]

i64p = C.POINTER(C.c_int64)
i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("pointer_mode", C.c_int), ("cg_tol", C.c_double),
                ("cg_tol_mixed", C.c_double), ("kkt_tol", C.c_double), ("quad_form_eps", C.c_double),
                ("delta2", C.c_double), ("max_cg", C.c_int), ("max_refine", C.c_int),
                ("ordering", C.c_int), ("relax", C.c_int), ("deterministic", C.c_int),
                ("mixed_check", C.c_int), ("mixed_check_tol", C.c_double), ("autotune_cache", C.c_int),
                ("scaling", C.c_int), ("flow_live", C.c_int), ("refine_inexact", C.c_int),
                ("mixed_pivot_tol", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("cg_iters", C.c_int), ("passes", C.c_int),
                ("fp64_fallback", C.c_int), ("cg_iters_fp64", C.c_int), ("passes_fp64", C.c_int),
                ("rr", C.c_double), ("be", C.c_double),
                ("floor", C.c_double), ("fail_col", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HKKTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hkkt error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the built library; fails loudly when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2110_03636_amd/build.py "
                               "(or __graft_entry__.build())")
        # Load torch's HIP runtime first when torch is present: the library's
        # libamdhip64.so.7 dependency then resolves to that same runtime, so a
        # process never holds two HIP/HSA runtimes (torch requests its copy by
        # an unversioned name and would otherwise load a second one).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        L.hkkt_default_options.argtypes = [C.POINTER(Options)]
        L.hkkt_create.argtypes = [C.POINTER(V), C.POINTER(Options), V]
        L.hkkt_destroy.argtypes = [V]
        L.hkkt_last_error.restype = C.c_char_p
        L.hkkt_last_error.argtypes = [V]
        L.hkkt_analyze.argtypes = [V, C.c_int64, C.c_int64, V, V, V, V, V]
        L.hkkt_analyze_group.argtypes = [V, C.c_int, V, V, C.c_int64, C.c_int64, V, V, V, V]
        L.hkkt_factor_batch.argtypes = [V, C.c_int, V, V, V, V, V, V, V]
        L.hkkt_autotune.argtypes = [V, C.c_int, V, V, V, V, V, V, V, V, V, C.c_int]
        L.hkkt_get_schedule.argtypes = [V, V]
        L.hkkt_set_schedule.argtypes = [V, V]
        L.hkkt_factor.argtypes = [V, V, V, V, C.c_double, C.c_double, V]
        L.hkkt_solve_batch.argtypes = [V, C.c_int, V, V, V, V, V]
        L.hkkt_solve.argtypes = [V, V, V, V, V, V]
        L.hkkt_inertia.argtypes = [V, C.c_int, V]
        L.hkkt_symbolic_create.argtypes = [C.POINTER(V), C.c_int64, C.c_int64, V, V, V, V, V, C.c_int,
                                           C.c_int, C.c_char_p, C.c_int]
        L.hkkt_symbolic_create_group.argtypes = [C.POINTER(V), C.c_int, V, V, C.c_int64, C.c_int64, V, V, V,
                                                 V, V, C.c_int, C.c_int, C.c_char_p, C.c_int]
        L.hkkt_symbolic_destroy.argtypes = [V]
        L.hkkt_get_symbolic.restype = V
        L.hkkt_get_symbolic.argtypes = [V]
        L.hkkt_symbolic_stats.argtypes = [V, V]
        L.hkkt_symbolic_perm.argtypes = [V, V]
        L.hkkt_symbolic_cb_offsets.argtypes = [V, V]
        L.hkkt_symbolic_supernodes.argtypes = [V, V, V, V, V, V, V]
        L.hkkt_get_factor.argtypes = [V, C.c_int, V, V, V]
        L.hkkt_hsolve.argtypes = [V, C.c_int, V, V]
        L.hkkt_hsolve_noalloc.argtypes = [V, C.c_int, V, V]
        L.hkkt_factor_regularized.argtypes = [V, C.c_int, V, V, V, V, V, V, C.c_double, V, V, V]
        L.hkkt_gamma_heuristic.argtypes = [V, C.c_int, V, V, V, V, V]
        L.hkkt_timings.argtypes = [V, V]
        L.hkkt_profile_begin.argtypes = [V]
        L.hkkt_profile_end.argtypes = [V, V, V]
        L.hkkt_profile_select.argtypes = [V, C.c_uint, C.c_int]
        L.hkkt_profile_precision.argtypes = [V, C.c_int]
        L.hkkt_analyze4.argtypes = [V, C.c_int64, C.c_int64, C.c_int64, V, V, V, V, V, V, V]
        L.hkkt_factor4_batch.argtypes = [V, C.c_int, V, V, V, V, V, V, V, V, V]
        L.hkkt_solve4_batch.argtypes = [V, C.c_int, V, V, V, V, V, V, V, V, V]
        _lib = L
    return _lib


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class GroupPattern:
    """Combined block-diagonal pattern of G member patterns (objects with
    n_x, m, H_rowptr, H_col, J_rowptr, J_col), in the layout
    hkkt_analyze_group takes: member k's variables at [x_off[k], x_off[k+1])
    and J rows at [y_off[k], y_off[k+1]). Index bookkeeping only."""

    def __init__(self, patterns):
        pats = list(patterns)
        if not pats:
            raise ValueError("empty group")
        self.G = len(pats)
        self.x_off = np.zeros(self.G + 1, np.int64)
        self.y_off = np.zeros(self.G + 1, np.int64)
        self.h_off = np.zeros(self.G + 1, np.int64)
        self.j_off = np.zeros(self.G + 1, np.int64)
        for k, p in enumerate(pats):
            self.x_off[k + 1] = self.x_off[k] + int(p.n_x)
            self.y_off[k + 1] = self.y_off[k] + int(p.m)
            self.h_off[k + 1] = self.h_off[k] + int(np.asarray(p.H_rowptr)[-1])
            self.j_off[k + 1] = self.j_off[k] + int(np.asarray(p.J_rowptr)[-1])
        self.n_x, self.m = int(self.x_off[-1]), int(self.y_off[-1])
        hp, hc, jp, jc = [np.zeros(1, np.int64)], [], [np.zeros(1, np.int64)], []
        for k, p in enumerate(pats):
            hp.append(np.asarray(p.H_rowptr, np.int64)[1:] + self.h_off[k])
            hc.append(np.asarray(p.H_col, np.int64) + self.x_off[k])
            jp.append(np.asarray(p.J_rowptr, np.int64)[1:] + self.j_off[k])
            jc.append(np.asarray(p.J_col, np.int64) + self.x_off[k])
        self.H_rowptr = np.concatenate(hp)
        self.H_col = np.concatenate(hc).astype(np.int32)
        self.J_rowptr = np.concatenate(jp)
        self.J_col = np.concatenate(jc).astype(np.int32)

    @staticmethod
    def concat(arrays):
        """[nb, len_k] per member -> [nb, sum len_k] (numpy or torch)."""
        arrays = list(arrays)
        if hasattr(arrays[0], "data_ptr"):
            import torch
            return torch.cat([a.reshape(a.shape[0], -1) for a in arrays], dim=1).contiguous()
        return np.concatenate([np.asarray(a).reshape(np.asarray(a).shape[0], -1) for a in arrays], axis=1)

    def split_x(self, x):
        """[nb, n_x] -> list of [nb, n_x_k]."""
        return [x[:, self.x_off[k]:self.x_off[k + 1]] for k in range(self.G)]

    def split_y(self, y):
        return [y[:, self.y_off[k]:self.y_off[k + 1]] for k in range(self.G)]


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


STAT_NAMES = ["n_x", "m", "nnz_A", "nnz_L", "L_storage", "supernodes", "levels", "flops_proxy",
              "max_width", "max_rows", "cb_entries", "etree_height", "uv_entries", "nnz_J",
              "L_lower_entries", "sn_rows_total"]


class _SymbolicView:
    """Accessors shared by the host-only analysis and a context's analysis."""

    def _h(self):
        raise NotImplementedError

    def stats(self):
        st = np.zeros(16, np.int64)
        _check(lib().hkkt_symbolic_stats(self._h(), st.ctypes.data), None)
        return dict(zip(STAT_NAMES, (int(v) for v in st)))

    def perm(self):
        n = self.stats()["n_x"]
        p = np.empty(n, np.int32)
        lib().hkkt_symbolic_perm(self._h(), p.ctypes.data)
        return p

    def cb_offsets(self):
        """Contribution-block offsets per supernode (+ workspace size)."""
        o = np.empty(self.stats()["supernodes"] + 1, np.int64)
        _check(lib().hkkt_symbolic_cb_offsets(self._h(), o.ctypes.data), None)
        return o

    def supernodes(self):
        s = self.stats()
        ns, nl = s["supernodes"], s["levels"]
        first = np.empty(ns + 1, np.int32)
        rowptr = np.empty(ns + 1, np.int64)
        rows = np.empty(s["sn_rows_total"], np.int32)
        parent = np.empty(ns, np.int32)
        lptr = np.empty(nl + 1, np.int32)
        lsn = np.empty(ns, np.int32)
        lib().hkkt_symbolic_supernodes(self._h(), first.ctypes.data, rowptr.ctypes.data, rows.ctypes.data,
                                       parent.ctypes.data, lptr.ctypes.data, lsn.ctypes.data)
        return dict(first=first, rowptr=rowptr, rows=rows, parent=parent, level_ptr=lptr, level_sn=lsn)


def _check(rc, ctx, what=""):
    if rc < 0:
        msg = lib().hkkt_last_error(ctx).decode() if ctx else what
        raise HKKTError(rc, msg)
    return rc


class Symbolic(_SymbolicView):
    """Host-only symbolic analysis (no GPU needed)."""

    def __init__(self, n_x, m, H_rowptr, H_col, J_rowptr, J_col, perm=None, ordering=0, relax=1, x_off=None,
                 y_off=None):
        self._keep = [_np(H_rowptr, np.int64), _np(H_col, np.int32), _np(J_rowptr, np.int64),
                      _np(J_col, np.int32)]
        pp = None if perm is None else _np(perm, np.int32)
        self._keep.append(pp)
        h = C.c_void_p()
        err = C.create_string_buffer(512)
        if x_off is None:
            rc = lib().hkkt_symbolic_create(C.byref(h), int(n_x), int(m), *[_ptr(a) for a in self._keep[:4]],
                                            _ptr(pp), ordering, relax, err, 512)
        else:
            xo, yo = _np(x_off, np.int64), _np(y_off, np.int64)
            self._keep += [xo, yo]
            rc = lib().hkkt_symbolic_create_group(C.byref(h), len(xo) - 1, _ptr(xo), _ptr(yo), int(n_x), int(m),
                                                  *[_ptr(a) for a in self._keep[:4]], _ptr(pp), ordering, relax,
                                                  err, 512)
        if rc != 0:
            raise HKKTError(rc, err.value.decode())
        self._handle = h

    @classmethod
    def from_pattern(cls, p, **kw):
        return cls(p.n_x, p.m, p.H_rowptr, p.H_col, p.J_rowptr, p.J_col, **kw)

    @classmethod
    def from_group(cls, g, **kw):
        return cls(g.n_x, g.m, g.H_rowptr, g.H_col, g.J_rowptr, g.J_col, x_off=g.x_off, y_off=g.y_off, **kw)

    def _h(self):
        return self._handle

    def __del__(self):
        try:
            if getattr(self, "_handle", None):
                lib().hkkt_symbolic_destroy(self._handle)
                self._handle = None
        except Exception:
            pass


class Solver(_SymbolicView):
    """One context: analyse a pattern, factor batches, solve.

    device=True: value/vector arguments are torch CUDA tensors (float64,
    contiguous, batch-major) and the context runs on torch's current stream.
    device=False: numpy arrays (host pointers)."""

    def __init__(self, precision="fp64", device=False, stream=None, **opts):
        o = Options()
        lib().hkkt_default_options(C.byref(o))
        o.precision = MIXED if precision in ("mixed", MIXED) else FP64
        o.pointer_mode = PTR_DEVICE if device else PTR_HOST
        for k, v in opts.items():
            setattr(o, k, v)
        self.device = device
        if device and stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(lib().hkkt_create(C.byref(h), C.byref(o), C.c_void_p(stream or 0)), None, "hkkt_create failed")
        self._ctx = h
        self.n = self.m = None
        self.nb = 0
        self.G = 1

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                lib().hkkt_destroy(self._ctx)
                self._ctx = None
        except Exception:
            pass

    def _h(self):
        h = lib().hkkt_get_symbolic(self._ctx)
        if not h:
            raise HKKTError(ERR_STATE, "not analysed")
        return h

    def analyze(self, pattern, perm=None):
        p = pattern
        keep = [_np(p.H_rowptr, np.int64), _np(p.H_col, np.int32), _np(p.J_rowptr, np.int64),
                _np(p.J_col, np.int32)]
        pp = None if perm is None else _np(perm, np.int32)
        _check(lib().hkkt_analyze(self._ctx, int(p.n_x), int(p.m), *[_ptr(a) for a in keep], _ptr(pp)),
               self._ctx)
        self.n, self.m = int(p.n_x), int(p.m)
        self.G = 1
        return self

    def analyze_group(self, group):
        """Analyse a GroupPattern (uneven systems in one launch). Afterwards
        factor() takes combined [nb, ...] values with delta, gamma of shape
        [nb, G]; statuses and infos are per (entry, member), flat index
        b * G + k."""
        g = group
        keep = [_np(g.x_off, np.int64), _np(g.y_off, np.int64), _np(g.H_rowptr, np.int64),
                _np(g.H_col, np.int32), _np(g.J_rowptr, np.int64), _np(g.J_col, np.int32)]
        _check(lib().hkkt_analyze_group(self._ctx, int(g.G), _ptr(keep[0]), _ptr(keep[1]), int(g.n_x), int(g.m),
                                        *[_ptr(a) for a in keep[2:]]), self._ctx)
        self.n, self.m, self.G = int(g.n_x), int(g.m), int(g.G)
        return self

    # -- values -------------------------------------------------------------
    def _arr(self, a, nb, width):
        if self.device:
            import torch
            t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))
            t = t.to(device="cuda", dtype=torch.float64).reshape(nb, width).contiguous()
            return t
        return _np(np.asarray(a, dtype=np.float64).reshape(nb, width), np.float64)

    def factor(self, H_val, D_x, J_val, delta, gamma):
        """Batch-major values ([nb, nnz] / [nb, n_x]); delta, gamma: [nb]
        ([nb, G] after analyze_group). Returns (rc, status[nb*G],
        fail_col[nb*G])."""
        delta = np.atleast_1d(np.asarray(delta, np.float64)).reshape(-1)
        gamma = np.atleast_1d(np.asarray(gamma, np.float64)).reshape(-1)
        if delta.shape != gamma.shape or delta.shape[0] % self.G:
            raise ValueError("delta and gamma need nb * G entries")
        nb = int(delta.shape[0]) // self.G
        if self.n is None:  # not analysed: let the library report the state error
            _check(lib().hkkt_factor_batch(self._ctx, nb, None, None, None, delta.ctypes.data,
                                           gamma.ctypes.data, None, None), self._ctx)
        Hv = self._arr(H_val, nb, -1)
        Dx = self._arr(D_x, nb, self.n)
        Jv = self._arr(J_val, nb, -1) if self.m > 0 else None
        if Jv is not None and Jv.shape[1] == 0:
            Jv = None
        self._keep_vals = (Hv, Dx, Jv)
        st = np.zeros(nb * self.G, np.int32)
        fc = np.zeros(nb * self.G, np.int64)
        rc = _check(lib().hkkt_factor_batch(self._ctx, nb, _ptr(Hv), _ptr(Dx), _ptr(Jv),
                                            _np(delta, np.float64).ctypes.data, _np(gamma, np.float64).ctypes.data,
                                            st.ctypes.data, fc.ctypes.data), self._ctx)
        self.nb = nb
        return rc, st, fc

    def autotune(self, H_val, D_x, J_val, delta, gamma, r1=None, r2=None):
        """Pick relax and the triangular-solve schedule (tree-kernel width,
        staged or global tree kernel) for the analysed pattern by timing
        candidates on these values, with trial solves of r1, r2 when given
        (see hkkt_autotune). Returns {"relax", "tree_width", "tree_staged",
        "cost_ms": [[relax, width, staged, ms], ...]}; the context is
        re-analysed and must be factored next."""
        delta = np.atleast_1d(np.asarray(delta, np.float64)).reshape(-1)
        gamma = np.atleast_1d(np.asarray(gamma, np.float64)).reshape(-1)
        nb = int(delta.shape[0]) // self.G
        Hv = self._arr(H_val, nb, -1)
        Dx = self._arr(D_x, nb, self.n)
        Jv = self._arr(J_val, nb, -1) if self.m > 0 else None
        if Jv is not None and Jv.shape[1] == 0:
            Jv = None
        R1 = self._arr(r1, nb, self.n) if r1 is not None else None
        R2 = self._arr(r2, nb, self.m) if (r1 is not None and r2 is not None and self.m > 0) else None
        choice = np.zeros(3, np.int32)
        cost = np.full(21, np.nan)
        _check(lib().hkkt_autotune(self._ctx, nb, _ptr(Hv), _ptr(Dx), _ptr(Jv), delta.ctypes.data,
                                   gamma.ctypes.data, _ptr(R1), _ptr(R2), choice.ctypes.data, cost.ctypes.data, 21),
               self._ctx)
        self.nb = 0   # re-analysed: factor next
        sched = [(0, 1)] + [(w, st) for w in (8, 32, 128) for st in (1, 0)]
        table = [[r, w, st, float(cost[i * 7 + j])] for i, r in enumerate((0, 1, 2)) for j, (w, st) in enumerate(sched)]
        return {"relax": int(choice[0]), "tree_width": int(choice[1]), "tree_staged": int(choice[2]),
                "cost_ms": table}

    def schedule(self):
        """(relax, tree_width, tree_staged) currently in use."""
        ch = np.zeros(3, np.int32)
        _check(lib().hkkt_get_schedule(self._ctx, ch.ctypes.data), self._ctx)
        return tuple(int(v) for v in ch)

    def set_schedule(self, relax, tree_width, tree_staged):
        """Apply a schedule (e.g. an earlier autotuner choice); a changed relax
        re-analyses the pattern, so factor next."""
        ch = np.array([relax, tree_width, tree_staged], np.int32)
        _check(lib().hkkt_set_schedule(self._ctx, ch.ctypes.data), self._ctx)
        self.nb = 0

    def factor_regularized(self, H_val, D_x, J_val, delta, gamma, delta_min, delta_max=1e-6):
        """Algorithm 1's delta1 loop around the factorization. delta_min:
        [nb*G] (or a scalar), updated as Algorithm 1 does. Returns (rc,
        status, fail_col, delta1, delta_min_after)."""
        delta = np.atleast_1d(np.asarray(delta, np.float64)).reshape(-1)
        gamma = np.atleast_1d(np.asarray(gamma, np.float64)).reshape(-1)
        nb = int(delta.shape[0]) // self.G
        dmin = np.array(np.broadcast_to(np.asarray(delta_min, np.float64), delta.shape), np.float64)
        d1 = np.zeros_like(delta)
        Hv = self._arr(H_val, nb, -1)
        Dx = self._arr(D_x, nb, self.n)
        Jv = self._arr(J_val, nb, -1) if self.m > 0 else None
        if Jv is not None and Jv.shape[1] == 0:
            Jv = None
        self._keep_vals = (Hv, Dx, Jv)
        st = np.zeros(nb * self.G, np.int32)
        fc = np.zeros(nb * self.G, np.int64)
        rc = _check(lib().hkkt_factor_regularized(self._ctx, nb, _ptr(Hv), _ptr(Dx), _ptr(Jv), delta.ctypes.data,
                                                  gamma.ctypes.data, dmin.ctypes.data, float(delta_max),
                                                  d1.ctypes.data, st.ctypes.data, fc.ctypes.data), self._ctx)
        self.nb = nb
        return rc, st, fc, d1, dmin

    def gamma_heuristic(self, H_val, D_x, J_val, delta):
        """||H + D_x + delta I||_inf / ||J||_inf^2 per (instance, member);
        drops the current factorization."""
        delta = np.atleast_1d(np.asarray(delta, np.float64)).reshape(-1)
        nb = int(delta.shape[0]) // self.G
        Hv = self._arr(H_val, nb, -1)
        Dx = self._arr(D_x, nb, self.n)
        Jv = self._arr(J_val, nb, -1) if self.m > 0 else None
        if Jv is not None and Jv.shape[1] == 0:
            Jv = None
        out = np.zeros(nb * self.G)
        _check(lib().hkkt_gamma_heuristic(self._ctx, nb, _ptr(Hv), _ptr(Dx), _ptr(Jv), delta.ctypes.data,
                                          out.ctypes.data), self._ctx)
        self.nb = 0
        return out

    # -- the 4x4 system of Sec. 3 ---------------------------------------------
    def analyze4(self, pattern, ineq, perm=None):
        p = pattern
        keep = [_np(p.H_rowptr, np.int64), _np(p.H_col, np.int32), _np(p.J_rowptr, np.int64),
                _np(p.J_col, np.int32), _np(ineq.Jd_rowptr, np.int64), _np(ineq.Jd_col, np.int32)]
        pp = None if perm is None else _np(perm, np.int32)
        _check(lib().hkkt_analyze4(self._ctx, int(p.n_x), int(p.m), int(ineq.m_d), *[_ptr(a) for a in keep],
                                   _ptr(pp)), self._ctx)
        self.n, self.m, self.md, self.G = int(p.n_x), int(p.m), int(ineq.m_d), 1
        return self

    def factor4(self, batch, ineq):
        nb = batch.nb
        delta = np.ascontiguousarray(batch.delta, np.float64)
        gamma = np.ascontiguousarray(batch.gamma, np.float64)
        vals = (self._arr(batch.H_val, nb, -1), self._arr(batch.D_x, nb, self.n),
                self._arr(batch.J_val, nb, -1) if self.m > 0 else None,
                self._arr(ineq.Jd_val, nb, -1) if self.md > 0 else None,
                self._arr(ineq.D_s, nb, self.md) if self.md > 0 else None)
        self._keep_vals = vals
        st = np.zeros(nb, np.int32)
        fc = np.zeros(nb, np.int64)
        rc = _check(lib().hkkt_factor4_batch(self._ctx, nb, *[_ptr(v) for v in vals], delta.ctypes.data,
                                             gamma.ctypes.data, st.ctypes.data, fc.ctypes.data), self._ctx)
        self.nb = nb
        return rc, st, fc

    def solve4(self, rx, rs, ry, ryd):
        """Returns (rc, dx, ds, dy, dyd, infos)."""
        nb = self.nb
        ins = [self._arr(rx, nb, self.n), self._arr(rs, nb, self.md) if self.md else None,
               self._arr(ry, nb, self.m) if self.m else None, self._arr(ryd, nb, self.md) if self.md else None]
        outs = [self._out(nb, self.n), self._out(nb, max(self.md, 0)), self._out(nb, max(self.m, 0)),
                self._out(nb, max(self.md, 0))]
        info = (Info * nb)()
        rc = _check(lib().hkkt_solve4_batch(self._ctx, nb, *[_ptr(a) for a in ins],
                                            _ptr(outs[0]), _ptr(outs[1]) if self.md else None,
                                            _ptr(outs[2]) if self.m else None, _ptr(outs[3]) if self.md else None,
                                            info), self._ctx)
        return (rc, *outs, [info[i].as_dict() for i in range(nb)])

    def factor_batch(self, batch):
        return self.factor(batch.H_val, batch.D_x, batch.J_val, batch.delta, batch.gamma)

    def _out(self, nb, width):
        if self.device:
            import torch
            return torch.empty((nb, width), dtype=torch.float64, device="cuda")
        return np.empty((nb, width), np.float64)

    def solve(self, r1, r2):
        """Returns (rc, x [nb, n_x], y [nb, m], infos: nb * G dicts, index
        b * G + k)."""
        nb = self.nb
        if not nb:   # nothing factored: let the library report the state error
            _check(lib().hkkt_solve_batch(self._ctx, 1, None, None, None, None, None), self._ctx)
        R1 = self._arr(r1, nb, self.n)
        R2 = self._arr(r2, nb, self.m) if self.m > 0 else None
        x = self._out(nb, self.n)
        y = self._out(nb, max(self.m, 0))
        info = (Info * (nb * self.G))()
        rc = _check(lib().hkkt_solve_batch(self._ctx, nb, _ptr(R1), _ptr(R2), _ptr(x),
                                           _ptr(y) if self.m > 0 else None, info), self._ctx)
        return rc, x, y, [info[i].as_dict() for i in range(nb * self.G)]

    def inertia(self, b=0):
        out = np.zeros(3, np.int64)
        _check(lib().hkkt_inertia(self._ctx, b, out.ctypes.data), self._ctx)
        return tuple(int(v) for v in out)

    def factor_csc(self, b=0):
        """L of instance b in the context's final order as (colptr, rowind, val)."""
        s = self.stats()
        nz = s["L_lower_entries"]
        cp = np.empty(self.n + 1, np.int64)
        ri = np.empty(nz, np.int32)
        v = np.empty(nz, np.float64)
        _check(lib().hkkt_get_factor(self._ctx, b, cp.ctypes.data, ri.ctypes.data, v.ctypes.data), self._ctx)
        return cp, ri, v

    def hsolve(self, bvec):
        """x = H_gamma^{-1} b for every instance ([nb, n_x], original order)."""
        B = self._arr(bvec, self.nb, self.n)
        x = self._out(self.nb, self.n)
        _check(lib().hkkt_hsolve(self._ctx, self.nb, _ptr(B), _ptr(x)), self._ctx)
        return x

    def hsolve_noalloc(self, bvec, x):
        """The allocation-free form of hsolve: bvec and x are caller-owned
        float64 CUDA tensors [nb, n_x] (device=True contexts only); x is
        written when the context's stream reaches the enqueued work."""
        _check(lib().hkkt_hsolve_noalloc(self._ctx, self.nb, _ptr(bvec), _ptr(x)), self._ctx)
        return x

    def timings(self):
        ms = np.zeros(8)
        lib().hkkt_timings(self._ctx, ms.ctypes.data)
        return dict(analyze=ms[0], factor=ms[1], solve=ms[2], fallback=ms[3])

    def profile_begin(self):
        _check(lib().hkkt_profile_begin(self._ctx), self._ctx)

    def profile_select(self, classes=None, every=1):
        """Record only the named classes (None: all), every `every`-th launch."""
        mask = 0xFFFFFFFF if classes is None else sum(1 << PROF_NAMES.index(k) for k in classes)
        _check(lib().hkkt_profile_select(self._ctx, mask, int(every)), self._ctx)

    def profile_precision(self, precision=None):
        """Record only launches on factors of this precision ("fp64" or
        "mixed"; None: all)."""
        if precision not in (None, "fp64", "mixed"):
            raise ValueError(f"precision must be None, 'fp64' or 'mixed', not {precision!r}")
        p = -1 if precision is None else {"fp64": FP64, "mixed": MIXED}[precision]
        _check(lib().hkkt_profile_precision(self._ctx, p), self._ctx)

    def profile_end(self):
        """{class: (total_ms, launches)} of the launches since profile_begin."""
        ms = np.zeros(len(PROF_NAMES))
        k = np.zeros(len(PROF_NAMES), np.int64)
        _check(lib().hkkt_profile_end(self._ctx, ms.ctypes.data, k.ctypes.data), self._ctx)
        return {PROF_NAMES[i]: (float(ms[i]), int(k[i])) for i in range(len(PROF_NAMES))}
