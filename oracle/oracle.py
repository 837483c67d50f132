"""ctypes binding of the C oracle (lpdec_oracle.c). Test infrastructure only.

Each wrapper marshals numpy arrays; every step of the computation runs in the C file,
which cites the paper's sections, equations and algorithms it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpdec_oracle.c")
_LIB = os.path.join(_HERE, "liblpdec_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("malp_mode", C.c_int), ("malp_max", C.c_int), ("ipm_max", C.c_int),
                ("tau_viol", C.c_double), ("tau_act", C.c_double), ("tau_int", C.c_double),
                ("sigma_c", C.c_double), ("eta", C.c_double), ("eps", C.c_double),
                ("eps_stall", C.c_double), ("tau_cost", C.c_double), ("box_clamp", C.c_int),
                ("cycle_stop", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("malp_iters", C.c_int), ("ipm_iters", C.c_int), ("p_max", C.c_int),
                ("p_final", C.c_int), ("status", C.c_int)]


@dataclass
class OracleOpts:
    malp_mode: int = 0
    malp_max: int = 200
    ipm_max: int = 100
    tau_viol: float = 1e-4
    tau_act: float = 1e-4
    tau_int: float = 1e-4
    sigma_c: float = 0.1
    eta: float = 0.9995
    eps: float = 1e-8
    eps_stall: float = 1e-7
    tau_cost: float = 1e-8
    box_clamp: int = 1
    cycle_stop: int = 1

    def c(self) -> _Opts:
        return _Opts(self.malp_mode, self.malp_max, self.ipm_max, self.tau_viol, self.tau_act,
                     self.tau_int, self.sigma_c, self.eta, self.eps, self.eps_stall, self.tau_cost,
                     self.box_clamp, self.cycle_stop)


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def find_cut(u, tau_viol=1e-6):
    """Algorithm 2 on one check: returns (violated, V mask, lhs)."""
    u = _f64(u)
    V = C.c_uint32(0)
    lhs = C.c_double(0)
    v = _L().orc_find_cut(C.c_int(u.size), _p(u), C.c_double(tau_viol), C.byref(V), C.byref(lhs))
    return bool(v), int(V.value), float(lhs.value)


@dataclass
class DecodeResult:
    u: np.ndarray
    xhat: np.ndarray
    flag: int
    objective: float
    malp_iters: int
    ipm_iters: int
    p_max: int
    p_final: int
    status: int
    trace_mask: np.ndarray | None = None  # [malp_iters, m] V masks after each cut update
    trace_obj: np.ndarray | None = None
    trace_p: np.ndarray | None = None
    trace_ipm: np.ndarray | None = None


def decode(code, gamma, opts: OracleOpts | None = None, trace: bool = False) -> DecodeResult:
    opts = opts or OracleOpts()
    gamma = _f64(gamma)
    m, n = code.m, code.n
    rp, cl = _i32(code.rowptr), _i32(code.col)
    u = np.zeros(n)
    xh = np.zeros(n, dtype=np.uint8)
    flag = C.c_int(0)
    obj = C.c_double(0)
    st = _Stats()
    o = opts.c()
    cap = opts.malp_max if trace else 0
    tm = np.zeros((max(cap, 1), m), dtype=np.uint32)
    to = np.zeros(max(cap, 1))
    tp = np.zeros(max(cap, 1), dtype=np.int32)
    ti = np.zeros(max(cap, 1), dtype=np.int32)
    _L().orc_decode(C.c_int(m), C.c_int(n), _p(rp), _p(cl), _p(gamma), C.byref(o), _p(u), _p(xh),
                    C.byref(flag), C.byref(obj), C.byref(st),
                    _p(tm) if trace else None, _p(to), _p(tp), _p(ti), C.c_int(cap))
    r = DecodeResult(u, xh, int(flag.value), float(obj.value), st.malp_iters, st.ipm_iters,
                     st.p_max, st.p_final, st.status)
    if trace:
        k = st.malp_iters
        r.trace_mask, r.trace_obj, r.trace_p, r.trace_ipm = tm[:k].copy(), to[:k].copy(), tp[:k].copy(), ti[:k].copy()
    return r


def lp_dense(code, gamma, mask):
    """Dense augmented-form LP (A, b, c) of a cut set (mask[j] = V bits, 0 = no cut)."""
    gamma = _f64(gamma)
    mask = np.ascontiguousarray(mask, dtype=np.uint32)
    p = int(np.count_nonzero(mask))
    q = code.n + p
    A = np.zeros((p, q))
    b = np.zeros(max(p, 1))
    c = np.zeros(q)
    _L().orc_lp_dense(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                      _p(gamma), _p(mask), _p(A), _p(b), _p(c))
    return A, b[:p], c


def ipm(code, gamma, mask, opts: OracleOpts | None = None):
    opts = opts or OracleOpts()
    gamma = _f64(gamma)
    mask = np.ascontiguousarray(mask, dtype=np.uint32)
    p = int(np.count_nonzero(mask))
    q = code.n + p
    x, z, y = np.zeros(q), np.zeros(q), np.zeros(max(p, 1))
    it = C.c_int(0)
    o = opts.c()
    rc = _L().orc_ipm(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                      _p(gamma), _p(mask), C.byref(o), _p(x), _p(y), _p(z), C.byref(it))
    return int(rc), x, y[:p], z, int(it.value)


def newton(code, gamma, mask, x, y, z, mu):
    gamma = _f64(gamma)
    mask = np.ascontiguousarray(mask, dtype=np.uint32)
    p = int(np.count_nonzero(mask))
    q = code.n + p
    dx, dz, dy = np.zeros(q), np.zeros(q), np.zeros(max(p, 1))
    x, y, z = _f64(x), _f64(np.resize(y, max(p, 1))), _f64(z)
    _L().orc_newton(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                    _p(gamma), _p(mask), _p(x), _p(y), _p(z), C.c_double(mu), _p(dx), _p(dy), _p(dz))
    return dx, dy[:p], dz


def mts(code, hascut, w):
    """Algorithm 7 with a binary heap. w: float32 weights, n+m entries (slack of check j at n+j).
    Returns (pair[m], order[p])."""
    hascut = np.ascontiguousarray(hascut, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float32)
    pair = np.full(code.m, -1, dtype=np.int32)
    order = np.zeros(code.m + 1, dtype=np.int32)
    p = _L().orc_mts(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                     _p(hascut), _p(w), _p(pair), _p(order))
    return pair, order[:p]


def mts_row(code, hascut, w, expand=0):
    """Algorithm 8 (row-wise greedy search) with the diagonal (expand=0) or the triangular
    (expand=1) expansion. w: float32 weights, n+m entries. Returns (pair[m], order[p]); with
    the diagonal expansion A_M is lower triangular in that order."""
    hascut = np.ascontiguousarray(hascut, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float32)
    pair = np.full(code.m, -1, dtype=np.int32)
    order = np.zeros(code.m + 1, dtype=np.int32)
    p = _L().orc_mts_row2(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                          _p(hascut), _p(w), C.c_int(expand), _p(pair), _p(order))
    return pair, order[:p]


def mts_levels_any(code, hascut, pair):
    """Levels of the two triangular solves for any triangular set (longest dependency chains)."""
    hascut = np.ascontiguousarray(hascut, dtype=np.uint8)
    lb = np.zeros(code.m, dtype=np.int32)
    lf = np.zeros(code.m, dtype=np.int32)
    _L().orc_mts_levels_any(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                            _p(hascut), _p(_i32(pair)), _p(lb), _p(lf))
    return lb, lf


def mts_levels(code, hascut, pair, order):
    hascut = np.ascontiguousarray(hascut, dtype=np.uint8)
    lb = np.zeros(code.m, dtype=np.int32)
    lf = np.zeros(code.m, dtype=np.int32)
    _L().orc_mts_levels(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                        _p(hascut), _p(_i32(pair)), _p(_i32(order)), C.c_int(len(order)), _p(lb), _p(lf))
    return lb, lf


def pcg(code, gamma, mask, d2, w, tol=1e-10, maxit=1000, precond=True, wkey=None):
    """FP64 PCG (Algorithm 4) with the Algorithm-7 preconditioner. Check-space vectors."""
    gamma = _f64(gamma)
    mask = np.ascontiguousarray(mask, dtype=np.uint32)
    d2 = _f64(d2)
    wkey = np.ascontiguousarray(d2.astype(np.float32) if wkey is None else wkey, dtype=np.float32)
    w = _f64(w)
    y = np.zeros(code.m)
    res = np.zeros(maxit + 1)
    it = _L().orc_pcg(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                      _p(gamma), _p(mask), _p(d2), _p(wkey), _p(w), C.c_double(tol), C.c_int(maxit),
                      C.c_int(1 if precond else 0), _p(y), _p(res))
    return y, int(it), res[:it + 1]


def normal_solve(code, gamma, mask, d2, w):
    gamma = _f64(gamma)
    mask = np.ascontiguousarray(mask, dtype=np.uint32)
    y = np.zeros(code.m)
    _L().orc_normal_solve(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                          _p(gamma), _p(mask), _p(_f64(d2)), _p(_f64(w)), _p(y))
    return y


def triangulate(code, hascut, inS):
    """Algorithm 5 (Triangulation Step) on the column set inS (n+m flags, slack of check j at
    n+j). Returns (matched, pair[m], order[matched]); success iff matched == inS.sum()."""
    hascut = np.ascontiguousarray(hascut, dtype=np.uint8)
    inS = np.ascontiguousarray(inS, dtype=np.uint8)
    pair = np.full(code.m, -1, dtype=np.int32)
    order = np.zeros(code.m + 1, dtype=np.int32)
    k = _L().orc_triangulate(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                             _p(hascut), _p(inS), _p(pair), _p(order))
    return int(k), pair, order[:k]


def mts_inc(code, hascut, w):
    """Algorithm 6 (incremental greedy search) with Algorithm 5. w: float32 weights, n+m
    entries. Returns (pair[m], order[p], triangulation calls); A_M is lower triangular in
    that order."""
    hascut = np.ascontiguousarray(hascut, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float32)
    pair = np.full(code.m, -1, dtype=np.int32)
    order = np.zeros(code.m + 1, dtype=np.int32)
    calls = C.c_int(0)
    p = _L().orc_mts_inc(C.c_int(code.m), C.c_int(code.n), _p(_i32(code.rowptr)), _p(_i32(code.col)),
                         _p(hascut), _p(w), _p(pair), _p(order), C.byref(calls))
    return pair, order[:p], int(calls.value)


@dataclass
class AlpResult(DecodeResult):
    cuts: np.ndarray | None = None     # [ncuts, 2]: check, V of every cut of the last LP


def alp_decode(code, gamma, opts: OracleOpts | None = None) -> AlpResult:
    """ALP decoding (Algorithm 1): every violated parity inequality is added and none removed.
    trace_p / trace_obj / trace_ipm: cuts, cost and IPM iterations of each LP."""
    opts = opts or OracleOpts()
    gamma = _f64(gamma)
    m, n = code.m, code.n
    u = np.zeros(n)
    xh = np.zeros(n, dtype=np.uint8)
    flag = C.c_int(0)
    obj = C.c_double(0)
    st = _Stats()
    o = opts.c()
    cap = opts.malp_max
    to = np.zeros(cap)
    tp = np.zeros(cap, dtype=np.int32)
    ti = np.zeros(cap, dtype=np.int32)
    ccap = 64 * m + 64
    cuts = np.zeros((ccap, 2), dtype=np.int32)
    nc = _L().orc_alp_decode(C.c_int(m), C.c_int(n), _p(_i32(code.rowptr)), _p(_i32(code.col)), _p(gamma),
                             C.byref(o), _p(u), _p(xh), C.byref(flag), C.byref(obj), C.byref(st),
                             _p(to), _p(tp), _p(ti), C.c_int(cap), _p(cuts), C.c_int(ccap))
    k = st.malp_iters
    return AlpResult(u, xh, int(flag.value), float(obj.value), st.malp_iters, st.ipm_iters, st.p_max,
                     st.p_final, st.status, None, to[:k].copy(), tp[:k].copy(), ti[:k].copy(),
                     cuts[:min(nc, ccap)].copy())
