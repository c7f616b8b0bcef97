"""ctypes marshalling for the FP64 oracle in ``nb6_oracle.c``.

Test infrastructure only (see the package docstring).  No arithmetic of the
method is done here: every function forwards numpy arrays to the C oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nb6_oracle.c")
_LIB = os.path.join(_HERE, "libnb6_oracle.so")

_lib = None


def lib_path() -> str:
    return _LIB


def build(src: str = _SRC, out: str = _LIB, extra: tuple[str, ...] = ()) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    cmd = [
        "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
        "-shared", "-fPIC", "-o", out, src, "-lm", *extra,
    ]
    subprocess.run(cmd, check=True)
    return out


def _load(path: str | None = None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
        ):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    d = ctypes.POINTER(ctypes.c_double)
    i32 = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.c_int64
    lib.nb6o_predict.argtypes = [i64, d, d, d, d, d, ctypes.c_double, d, d]
    lib.nb6o_predict.restype = None
    lib.nb6o_regular_force.argtypes = [
        i64, d, d, d, i64, i32, d, d, d, d, i32, i32, i64, d, d, d, ctypes.c_int,
    ]
    lib.nb6o_regular_force.restype = ctypes.c_int
    lib.nb6o_pair_terms.argtypes = [i64, i32, i32, d, d, d, d, d, d, d]
    lib.nb6o_pair_terms.restype = None
    lib.nb6o_irregular_force.argtypes = [
        i64, d, d, d, i64, i32, i32, i32, i64, d, d, d, d, d, ctypes.c_int,
    ]
    lib.nb6o_irregular_force.restype = ctypes.c_int
    lib.nb6o_regular_correct.argtypes = [
        i64, ctypes.c_double, d, d, d, d, d, d, d, d, d, d, i32, d,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.c_double, d, d, d, d, d, d,
    ]
    lib.nb6o_regular_correct.restype = ctypes.c_int
    lib.nb6o_max_threads.argtypes = []
    lib.nb6o_max_threads.restype = ctypes.c_int
    return lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def max_threads(lib=None) -> int:
    return int((lib or _load()).nb6o_max_threads())


def predict(x, v, a, jerk, t, tb, lib=None):
    """Cubic Taylor prediction of every particle to time ``tb``."""
    lib = lib or _load()
    n = len(t)
    x, v, a, jerk = (_f64(q, (n, 3)) for q in (x, v, a, jerk))
    t = _f64(t, (n,))
    xp = np.empty((n, 3))
    vp = np.empty((n, 3))
    lib.nb6o_predict(n, _pd(x), _pd(v), _pd(a), _pd(jerk), _pd(t),
                     float(tb), _pd(xp), _pd(vp))
    return xp, vp


@dataclass
class OracleResult:
    acc: np.ndarray      # [ni, 3]
    jerk: np.ndarray     # [ni, 3]
    nnb: np.ndarray      # [ni] true counts
    lists: list          # ni arrays of ascending j (complete when lcap >= nnb)
    sa: np.ndarray       # [ni] sum of m/r^2 over non-neighbours
    sj: np.ndarray       # [ni] jerk scale
    complete: bool       # every list fitted in lcap
    pot: np.ndarray = None  # [ni] regular potential -sum m/r over non-neighbours


def regular_force(m, xp, vp, idx, h2, dtr, lcap=1024, nthreads=0, lib=None):
    """Regular force, jerk and neighbour lists of the active set ``idx``."""
    lib = lib or _load()
    n = len(m)
    m = _f64(m, (n,))
    xp = _f64(xp, (n, 3))
    vp = _f64(vp, (n, 3))
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ni = len(idx)
    h2 = _f64(np.broadcast_to(h2, (ni,)), (ni,))
    dtr = _f64(np.broadcast_to(dtr, (ni,)), (ni,))
    acc = np.zeros((ni, 3))
    jrk = np.zeros((ni, 3))
    nnb = np.zeros(ni, dtype=np.int32)
    lst = np.full((ni, max(lcap, 1)), -1, dtype=np.int32)
    sa = np.zeros(ni)
    sj = np.zeros(ni)
    pot = np.zeros(ni)
    rc = lib.nb6o_regular_force(
        n, _pd(m), _pd(xp), _pd(vp), ni, _pi(idx), _pd(h2), _pd(dtr),
        _pd(acc), _pd(jrk), _pi(nnb), _pi(lst), int(lcap), _pd(sa), _pd(sj),
        _pd(pot), int(nthreads),
    )
    if rc != 0:
        raise ValueError(f"oracle rejected its input (code {rc})")
    lists = [lst[q, : min(int(nnb[q]), lcap)].copy() for q in range(ni)]
    return OracleResult(acc, jrk, nnb, lists, sa, sj,
                        bool(ni == 0 or nnb.max() <= lcap), pot)


def pair_terms(pi, pj, dtr, m, xp, vp, lib=None):
    """rmin and the (acc, jerk) contribution of each listed pair."""
    lib = lib or _load()
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    npair = len(pi)
    dtr = _f64(np.broadcast_to(dtr, (npair,)), (npair,))
    n = len(m)
    m = _f64(m, (n,))
    xp = _f64(xp, (n, 3))
    vp = _f64(vp, (n, 3))
    rmin = np.zeros(npair)
    dacc = np.zeros((npair, 3))
    djrk = np.zeros((npair, 3))
    lib.nb6o_pair_terms(npair, _pi(pi), _pi(pj), _pd(dtr), _pd(m), _pd(xp),
                        _pd(vp), _pd(rmin), _pd(dacc), _pd(djrk))
    return rmin, dacc, djrk


@dataclass
class IrregularResult:
    acc: np.ndarray      # [ni, 3]
    jerk: np.ndarray     # [ni, 3]
    sa: np.ndarray       # [ni] sum of m/r^2 over the list
    sj: np.ndarray       # [ni] jerk scale over the list
    pot: np.ndarray      # [ni] irregular potential -sum m/r over the list


def irregular_force(m, xp, vp, idx, lists, nthreads=0, lib=None):
    """Irregular force and its derivative of the active set ``idx`` over the
    neighbour lists ``lists`` (one integer sequence per active particle)."""
    lib = lib or _load()
    n = len(m)
    m = _f64(m, (n,))
    xp = _f64(xp, (n, 3))
    vp = _f64(vp, (n, 3))
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ni = len(idx)
    if len(lists) != ni:
        raise ValueError("one list per active particle")
    cnt = np.array([len(l) for l in lists], dtype=np.int32)
    lcap = max(1, int(cnt.max()) if ni else 1)
    lst = np.zeros((ni, lcap), dtype=np.int32)
    for q, l in enumerate(lists):
        lst[q, : len(l)] = l
    acc = np.zeros((ni, 3))
    jrk = np.zeros((ni, 3))
    sa = np.zeros(ni)
    sj = np.zeros(ni)
    pot = np.zeros(ni)
    rc = lib.nb6o_irregular_force(
        n, _pd(m), _pd(xp), _pd(vp), ni, _pi(idx), _pi(cnt), _pi(lst), lcap,
        _pd(acc), _pd(jrk), _pd(sa), _pd(sj), _pd(pot), int(nthreads),
    )
    if rc != 0:
        raise ValueError(f"oracle rejected its input (code {rc})")
    return IrregularResult(acc, jrk, sa, sj, pot)


@dataclass
class CorrectResult:
    df: np.ndarray       # [n, 3] regular force change over the step, fixed neighbour set
    dfd: np.ndarray      # [n, 3] the same for the derivative
    f2: np.ndarray       # [n, 3] second derivative of the regular force at t
    f3: np.ndarray       # [n, 3] third derivative
    dt_new: np.ndarray   # [n] next regular step
    h_new: np.ndarray    # [n] new neighbour radius


def regular_correct(t, t_old, f_old, fd_old, f_new, fd_new, g_old, gd_old, g_new, gd_new,
                    h_old, nnb, n_p, eta=0.02, dt_min=2.0 ** -20, dt_max=1.0,
                    f_lo=0.5, f_hi=1.25, lib=None):
    """Regular corrector of a block (see ``nb6o_regular_correct``)."""
    lib = lib or _load()
    t_old = _f64(np.atleast_1d(t_old))
    n = len(t_old)
    vecs = [_f64(q, (n, 3)) for q in (f_old, fd_old, f_new, fd_new, g_old, gd_old, g_new,
                                       gd_new)]
    h_old = _f64(np.broadcast_to(h_old, (n,)), (n,))
    n_p = _f64(np.broadcast_to(n_p, (n,)), (n,))
    nnb = np.ascontiguousarray(np.broadcast_to(nnb, (n,)), dtype=np.int32)
    out = [np.zeros((n, 3)) for _ in range(4)] + [np.zeros(n), np.zeros(n)]
    rc = lib.nb6o_regular_correct(
        n, float(t), _pd(t_old), *[_pd(v) for v in vecs], _pd(h_old), _pi(nnb), _pd(n_p),
        float(eta), float(dt_min), float(dt_max), float(f_lo), float(f_hi),
        *[_pd(o) for o in out])
    if rc != 0:
        raise ValueError(f"oracle rejected its input (code {rc})")
    return CorrectResult(*out)
