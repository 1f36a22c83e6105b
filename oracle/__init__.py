"""ctypes front end of the plain FP64 CPU oracle (oracle.c).

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline leg import this module; the product library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

i64p = C.POINTER(C.c_int64)
i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        # -ffp-contract=off: the compensated residual's error-free
        # transformations need every product and sum rounded on its own
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("cg_tol", C.c_double), ("kkt_tol", C.c_double), ("qf_eps", C.c_double),
                ("delta2", C.c_double), ("max_cg", C.c_int64), ("max_refine", C.c_int64),
                ("inexact", C.c_int64)]


class _Report(C.Structure):
    _fields_ = [("status", C.c_int64), ("passes", C.c_int64), ("cg_iters", C.c_int64 * 16),
                ("rr_hist", C.c_double * 16), ("rr", C.c_double), ("be", C.c_double),
                ("floor", C.c_double), ("inertia", C.c_int64 * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        L.orc_new.restype = C.c_void_p
        L.orc_new.argtypes = [C.c_int64, C.c_int64, i64p, i32p, f64p, f64p, i64p, i32p, f64p,
                              C.c_double, C.c_double]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_hgamma_nnz.restype = C.c_int64
        L.orc_hgamma_nnz.argtypes = [C.c_void_p]
        L.orc_hgamma.argtypes = [C.c_void_p, i64p, i32p, f64p]
        L.orc_order_mindeg.argtypes = [C.c_void_p, i32p]
        L.orc_factor.restype = C.c_int
        L.orc_factor.argtypes = [C.c_void_p, i32p, i64p]
        L.orc_L_nnz.restype = C.c_int64
        L.orc_L_nnz.argtypes = [C.c_void_p]
        L.orc_L.argtypes = [C.c_void_p, i64p, i32p, f64p]
        L.orc_hsolve.argtypes = [C.c_void_p, f64p, f64p]
        L.orc_metrics.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p, f64p]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [C.c_void_p, C.POINTER(_Opts), f64p, f64p, f64p, f64p, C.POINTER(_Report)]
        L.orc_hybrid_once.restype = C.c_int64
        L.orc_hybrid_once.argtypes = [C.c_void_p, C.POINTER(_Opts), f64p, f64p, f64p, f64p, C.POINTER(C.c_int)]
        L.orc_apply_K.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p]
        L.orc_residual.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p, f64p, f64p, f64p, f64p]
        L.orc_set_delta.argtypes = [C.c_void_p, C.c_double]
        L.orc_factor_regularized.restype = C.c_int
        L.orc_factor_regularized.argtypes = [C.c_void_p, i32p, f64p, C.c_double, f64p, i64p]
        L.orc_gamma_heuristic.restype = C.c_double
        L.orc_gamma_heuristic.argtypes = [C.c_void_p]
        L.orc_ruiz.argtypes = [C.c_void_p, C.c_int64, f64p]
        L.orc_solve_scaled.restype = C.c_int
        L.orc_solve_scaled.argtypes = [C.c_void_p, C.POINTER(_Opts), f64p, i32p, f64p, f64p, f64p, f64p,
                                       C.POINTER(_Report)]
        L.orc4_new.restype = C.c_void_p
        L.orc4_new.argtypes = [C.c_int64, C.c_int64, C.c_int64, i64p, i32p, f64p, f64p, i64p, i32p, f64p,
                               i64p, i32p, f64p, f64p, C.c_double, C.c_double]
        L.orc4_free.argtypes = [C.c_void_p]
        L.orc4_two.restype = C.c_void_p
        L.orc4_two.argtypes = [C.c_void_p]
        L.orc4_solve.argtypes = [C.c_void_p, C.POINTER(_Opts)] + [f64p] * 9
        L.orc4_metrics.argtypes = [C.c_void_p] + [f64p] * 9
        L.orc_refine_dd.restype = C.c_int64
        L.orc_refine_dd.argtypes = [C.c_void_p, C.POINTER(_Opts), f64p, f64p, f64p, f64p, C.c_int64, f64p]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class System:
    """One KKT system K = [H + D_x + delta I, J^T; J, 0] in FP64 on the CPU."""

    def __init__(self, n_x, m, H_rowptr, H_col, H_val, D_x, J_rowptr, J_col, J_val, delta, gamma):
        self.n, self.m = int(n_x), int(m)
        self._keep = [_c(H_rowptr, np.int64), _c(H_col, np.int32), _c(H_val, np.float64),
                      _c(D_x, np.float64), _c(J_rowptr, np.int64), _c(J_col, np.int32),
                      _c(J_val, np.float64)]
        k = self._keep
        self._h = lib().orc_new(self.n, self.m, _p(k[0], i64p), _p(k[1], i32p), _p(k[2], f64p),
                                _p(k[3], f64p), _p(k[4], i64p), _p(k[5], i32p), _p(k[6], f64p),
                                float(delta), float(gamma))
        self.perm = None

    @classmethod
    def from_batch(cls, batch, b=0):
        p = batch.pattern
        return cls(p.n_x, p.m, p.H_rowptr, p.H_col, batch.H_val[b], batch.D_x[b], p.J_rowptr,
                   p.J_col, batch.J_val[b], batch.delta[b], batch.gamma[b])

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().orc_free(self._h)
                self._h = None
        except Exception:
            pass

    def hgamma(self):
        """H_gamma lower triangle as (colptr, rowind, val), original order."""
        nz = lib().orc_hgamma_nnz(self._h)
        cp = np.empty(self.n + 1, np.int64)
        ri = np.empty(nz, np.int32)
        v = np.empty(nz, np.float64)
        lib().orc_hgamma(self._h, _p(cp, i64p), _p(ri, i32p), _p(v, f64p))
        return cp, ri, v

    def order_mindeg(self):
        perm = np.empty(self.n, np.int32)
        lib().orc_order_mindeg(self._h, _p(perm, i32p))
        return perm

    def factor(self, perm=None):
        """Returns (status, fail_col). perm[k] = original index of pivot k."""
        fc = np.zeros(1, np.int64)
        if perm is None:
            st = lib().orc_factor(self._h, None, _p(fc, i64p))
        else:
            pa = _c(perm, np.int32)
            st = lib().orc_factor(self._h, _p(pa, i32p), _p(fc, i64p))
        self.perm = None if perm is None else np.asarray(perm, np.int32)
        return int(st), int(fc[0])

    def factor_regularized(self, perm=None, delta_min=1e-9, delta_max=1e-6):
        """Algorithm 1's Cholesky attempts with delta1 regularization.
        Returns (status, delta1, delta_min after the loop, fail_col); the
        system keeps delta + delta1."""
        dm = np.array([delta_min], np.float64)
        d1 = np.zeros(1)
        fc = np.zeros(1, np.int64)
        pa = None if perm is None else _c(perm, np.int32)
        st = lib().orc_factor_regularized(self._h, None if pa is None else _p(pa, i32p), _p(dm, f64p),
                                          float(delta_max), _p(d1, f64p), _p(fc, i64p))
        self.perm = None if perm is None else np.asarray(perm, np.int32)
        return int(st), float(d1[0]), float(dm[0]), int(fc[0])

    def gamma_heuristic(self):
        """||H + D_x + delta I||_inf / ||J||_inf^2."""
        return float(lib().orc_gamma_heuristic(self._h))

    def L(self):
        nz = lib().orc_L_nnz(self._h)
        if nz < 0:
            raise RuntimeError("not factored")
        cp = np.empty(self.n + 1, np.int64)
        ri = np.empty(nz, np.int32)
        v = np.empty(nz, np.float64)
        lib().orc_L(self._h, _p(cp, i64p), _p(ri, i32p), _p(v, f64p))
        return cp, ri, v

    def hsolve(self, b):
        b = _c(b, np.float64)
        x = np.empty(self.n)
        lib().orc_hsolve(self._h, _p(b, f64p), _p(x, f64p))
        return x

    def metrics(self, r1, r2, x, y):
        """(RR, BE, floor) of z = (x, y) for K z = r."""
        a = [_c(v, np.float64) for v in (r1, r2, x, y)]
        out = np.empty(3)
        lib().orc_metrics(self._h, *[_p(v, f64p) for v in a], _p(out, f64p))
        return float(out[0]), float(out[1]), float(out[2])

    @staticmethod
    def _opts(cg_tol=1e-12, kkt_tol=1e-10, qf_eps=1e-14, delta2=0.0, max_cg=0, max_refine=10, inexact=0):
        return _Opts(cg_tol, kkt_tol, qf_eps, delta2, max_cg, max_refine, inexact)

    def solve(self, r1, r2, **kw):
        r1 = _c(r1, np.float64)
        r2 = _c(r2, np.float64)
        x = np.empty(self.n)
        y = np.empty(self.m)
        rep = _Report()
        o = self._opts(**kw)
        lib().orc_solve(self._h, C.byref(o), _p(r1, f64p), _p(r2, f64p), _p(x, f64p), _p(y, f64p),
                        C.byref(rep))
        info = dict(status=int(rep.status), passes=int(rep.passes),
                    cg_iters=[int(rep.cg_iters[i]) for i in range(rep.passes)],
                    rr_hist=[float(rep.rr_hist[i]) for i in range(rep.passes)],
                    rr=float(rep.rr), be=float(rep.be), floor=float(rep.floor),
                    inertia=tuple(int(v) for v in rep.inertia))
        return x, y, info

    def ruiz(self, iters=10):
        """Symmetrized Ruiz scaling vector d (n_x + m) of K."""
        d = np.empty(self.n + self.m)
        lib().orc_ruiz(self._h, int(iters), _p(d, f64p))
        return d

    def solve_scaled(self, r1, r2, d, perm=None, **kw):
        """Hybrid passes on D K D, refinement on K (orc_solve_scaled)."""
        r1 = _c(r1, np.float64)
        r2 = _c(r2, np.float64)
        d = _c(d, np.float64)
        x = np.empty(self.n)
        y = np.empty(self.m)
        rep = _Report()
        o = self._opts(**kw)
        pa = None if perm is None else _c(perm, np.int32)
        lib().orc_solve_scaled(self._h, C.byref(o), _p(d, f64p), None if pa is None else _p(pa, i32p),
                               _p(r1, f64p), _p(r2, f64p), _p(x, f64p), _p(y, f64p), C.byref(rep))
        info = dict(status=int(rep.status), passes=int(rep.passes),
                    cg_iters=[int(rep.cg_iters[i]) for i in range(rep.passes)],
                    rr_hist=[float(rep.rr_hist[i]) for i in range(rep.passes)],
                    rr=float(rep.rr), be=float(rep.be), floor=float(rep.floor),
                    inertia=tuple(int(v) for v in rep.inertia))
        return x, y, info

    def hybrid_once(self, r1, r2, **kw):
        r1 = _c(r1, np.float64)
        r2 = _c(r2, np.float64)
        x = np.empty(self.n)
        y = np.empty(self.m)
        brk = C.c_int(0)
        o = self._opts(**kw)
        it = lib().orc_hybrid_once(self._h, C.byref(o), _p(r1, f64p), _p(r2, f64p), _p(x, f64p),
                                   _p(y, f64p), C.byref(brk))
        return x, y, int(it), bool(brk.value)

    def residual(self, r1, r2, x, y):
        """Compensated r - K z and the per-row sums |r_i| + sum |term|."""
        a = [_c(v, np.float64) for v in (r1, r2, x, y)]
        g1, t1 = np.empty(self.n), np.empty(self.n)
        g2, t2 = np.empty(self.m), np.empty(self.m)
        lib().orc_residual(self._h, *[_p(v, f64p) for v in a], _p(g1, f64p), _p(g2, f64p), _p(t1, f64p),
                           _p(t2, f64p))
        return g1, g2, t1, t2

    def refine_dd(self, r1, r2, x, y, max_steps=8, **kw):
        """Refinement with a double-double iterate started at (x, y): returns
        (x, y) = the exact solution rounded to FP64 (to the accuracy reached)
        and the history of ||r - K z_dd|| / ||r||."""
        r1 = _c(r1, np.float64)
        r2 = _c(r2, np.float64)
        x = np.array(x, np.float64)
        y = np.array(y, np.float64)
        hist = np.zeros(max_steps + 1)
        o = self._opts(**kw)
        k = lib().orc_refine_dd(self._h, C.byref(o), _p(r1, f64p), _p(r2, f64p), _p(x, f64p), _p(y, f64p),
                                int(max_steps), _p(hist, f64p))
        return x, y, hist[:k + 1]

    def apply_K(self, x, y):
        x = _c(x, np.float64)
        y = _c(y, np.float64)
        o1 = np.empty(self.n)
        o2 = np.empty(self.m)
        lib().orc_apply_K(self._h, _p(x, f64p), _p(y, f64p), _p(o1, f64p), _p(o2, f64p))
        return o1, o2


class System4:
    """The 4x4 system of Sec. 3: K4 = [H + D_x + delta I, 0, J^T, J_d^T; 0, D_s,
    0, -I; J, 0, 0, 0; J_d, -I, 0, 0], solved through the 2x2 reduction."""

    def __init__(self, n_x, m, m_d, H_rowptr, H_col, H_val, D_x, J_rowptr, J_col, J_val, Jd_rowptr, Jd_col,
                 Jd_val, D_s, delta, gamma):
        self.n, self.m, self.md = int(n_x), int(m), int(m_d)
        k = self._keep = [_c(H_rowptr, np.int64), _c(H_col, np.int32), _c(H_val, np.float64), _c(D_x, np.float64),
                          _c(J_rowptr, np.int64), _c(J_col, np.int32), _c(J_val, np.float64),
                          _c(Jd_rowptr, np.int64), _c(Jd_col, np.int32), _c(Jd_val, np.float64),
                          _c(D_s, np.float64)]
        t = [i64p, i32p, f64p, f64p, i64p, i32p, f64p, i64p, i32p, f64p, f64p]
        self._h = lib().orc4_new(self.n, self.m, self.md, *[_p(a, tt) for a, tt in zip(k, t)],
                                 float(delta), float(gamma))
        self.two = System.__new__(System)        # view of the 2x2 system (owned here)
        self.two.n, self.two.m, self.two._h, self.two.perm = self.n, self.m, lib().orc4_two(self._h), None

    @classmethod
    def from_batch(cls, batch, ineq, b=0):
        p = batch.pattern
        return cls(p.n_x, p.m, ineq.m_d, p.H_rowptr, p.H_col, batch.H_val[b], batch.D_x[b], p.J_rowptr, p.J_col,
                   batch.J_val[b], ineq.Jd_rowptr, ineq.Jd_col, ineq.Jd_val[b], ineq.D_s[b], batch.delta[b],
                   batch.gamma[b])

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self.two._h = None
                lib().orc4_free(self._h)
                self._h = None
        except Exception:
            pass

    def factor(self, perm=None):
        return self.two.factor(perm)

    def solve(self, rx, rs, ry, ryd, **kw):
        a = [_c(v, np.float64) for v in (rx, rs, ry, ryd)]
        x, sv, y, yd = np.empty(self.n), np.empty(self.md), np.empty(self.m), np.empty(self.md)
        out = np.empty(5)
        o = System._opts(**kw)
        lib().orc4_solve(self._h, C.byref(o), *[_p(v, f64p) for v in a], *[_p(v, f64p) for v in (x, sv, y, yd)],
                         _p(out, f64p))
        return x, sv, y, yd, dict(rr=float(out[0]), be=float(out[1]), steps=int(out[2]), cg_iters=int(out[3]),
                                  status=int(out[4]))

    def metrics(self, rx, rs, ry, ryd, x, sv, y, yd):
        a = [_c(v, np.float64) for v in (rx, rs, ry, ryd, x, sv, y, yd)]
        out = np.empty(2)
        lib().orc4_metrics(self._h, *[_p(v, f64p) for v in a], _p(out, f64p))
        return float(out[0]), float(out[1])
