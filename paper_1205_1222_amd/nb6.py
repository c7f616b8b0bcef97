"""ctypes binding of ``libnb6.so`` (the C ABI of ``include/nb6.h``).

Argument marshalling only: every step of the regular-force path runs in the
HIP library.  The functions keep the C names.  Array arguments may be

* numpy arrays (host memory, ``NB6_MEM_HOST`` calls),
* torch tensors on the GPU (``NB6_MEM_DEVICE`` calls), or
* raw integer addresses.

Streams are ``torch.cuda.Stream`` objects, raw ``hipStream_t`` integers, or
``None`` for the null stream.

torch is imported before the library is loaded so that the process holds a
single HIP runtime (torch ships its own; the library binds to it by soname).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnb6.so")

NB6_OK = 0
NB6_WARN_NB_OVERFLOW = 1
NB6_PENDING = 2
NB6_ERR_ARG = -1
NB6_ERR_STATE = -2
NB6_ERR_NOMEM = -3
NB6_ERR_ADMISSION = -4
NB6_ERR_UNKNOWN_TICKET = -5
NB6_ERR_HIP = -6
NB6_ERR_DEVICE_INPUT = -7

NB6_MEM_HOST = 0
NB6_MEM_DEVICE = 1

NB6_DX_FF = 1
NB6_DX_FP64 = 2
NB6_DX_FP32 = 4
NB6_DX_LOCAL = 8
NB6_DX_ALL = 15
NB6_MAX_CAP = 1023
NB6_MAX_LIST_CAP = 8192
NB6_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTED = [
    "nb6_create", "nb6_destroy", "nb6_last_error", "nb6_load_particles",
    "nb6_predict_j", "nb6_regular_force", "nb6_sync_status", "nb6_last_slices",
    "nb6_last_plan",
    "nb6_get_predicted", "nb6_kernel_times", "nb6_submit", "nb6_poll",
    "nb6_set_lists", "nb6_irregular_force", "nb6_regular_correct",
    "nb6_regular_force_noalloc",
]

NB6_OPT_TIMING = 1
NB6_OPT_CALLER_ORDER = 2


class nb6_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("slice_hint", ctypes.c_int),
                ("hbm_budget", ctypes.c_int64), ("flags", ctypes.c_int),
                ("ipl_hint", ctypes.c_int), ("jl_hint", ctypes.c_int)]


class nb6_request(ctypes.Structure):
    _fields_ = [("cluster", ctypes.c_int), ("t_block", ctypes.c_double),
                ("dx_mode", ctypes.c_int), ("n_i", ctypes.c_int64),
                ("idx_i", ctypes.c_void_p), ("h2_i", ctypes.c_void_p),
                ("dtr_i", ctypes.c_void_p), ("acc", ctypes.c_void_p),
                ("jerk", ctypes.c_void_p), ("nnb", ctypes.c_void_p),
                ("list", ctypes.c_void_p), ("cap", ctypes.c_int32),
                ("mem_kind", ctypes.c_int)]


class nb6_ticket_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("slices", ctypes.c_int),
                ("batch_size", ctypes.c_int), ("submit_us", ctypes.c_double),
                ("admit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class nb6_corr_params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("dt_max", ctypes.c_double), ("f_lo", ctypes.c_double),
                ("f_hi", ctypes.c_double)]


class nb6_corr_block(ctypes.Structure):
    _fields_ = [("n_i", ctypes.c_int64), ("t", ctypes.c_double)] + [
        (name, ctypes.c_void_p) for name in (
            "t_old", "f_old", "fd_old", "f_new", "fd_new", "g_old", "gd_old", "g_new",
            "gd_new", "h_old", "nnb", "n_p", "df", "dfd", "f2", "f3", "dt_new", "h_new")]


class NB6Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nb6 error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1205_1222_amd.build` (there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.nb6_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(nb6_options)]
        L.nb6_destroy.argtypes = [vp]
        L.nb6_last_error.argtypes = [vp]
        L.nb6_last_error.restype = ctypes.c_char_p
        L.nb6_last_slices.argtypes = [vp]
        L.nb6_last_plan.argtypes = [vp, vp]
        L.nb6_load_particles.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, vp, vp, vp, vp,
                                         ctypes.c_int, vp]
        L.nb6_predict_j.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, vp]
        L.nb6_regular_force.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int,
                                        vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int, vp]
        L.nb6_regular_force_noalloc.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int,
                                                vp, vp, vp, vp, vp, ctypes.c_int32, vp]
        L.nb6_sync_status.argtypes = [vp, vp]
        L.nb6_kernel_times.argtypes = [vp, vp, vp]
        L.nb6_submit.argtypes = [vp, ctypes.POINTER(nb6_request), ctypes.POINTER(ctypes.c_uint64)]
        L.nb6_poll.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(nb6_ticket_info)]
        L.nb6_get_predicted.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp]
        L.nb6_set_lists.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int32,
                                    ctypes.c_int, vp]
        L.nb6_regular_correct.argtypes = [vp, ctypes.POINTER(nb6_corr_block),
                                          ctypes.POINTER(nb6_corr_params), ctypes.c_int, vp]
        L.nb6_irregular_force.argtypes = [vp, ctypes.c_int, ctypes.c_double, i64, vp, vp, vp,
                                          vp, ctypes.c_int, vp]
        for name in EXPORTED:
            if name != "nb6_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, dtype=None):
    """Address of a numpy array / torch tensor / int (None -> 0)."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        if dtype is not None and a.dtype != dtype:
            raise TypeError(f"expected {np.dtype(dtype)}, got {a.dtype}")
        return a.ctypes.data
    if isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if dtype is not None and a.dtype != _TORCH[np.dtype(dtype)]:
            raise TypeError(f"expected {np.dtype(dtype)}, got {a.dtype}")
        return a.data_ptr()
    raise TypeError(f"unsupported array type {type(a)}")


_TORCH = {np.dtype(np.float64): torch.float64, np.dtype(np.int32): torch.int32,
          np.dtype(np.float32): torch.float32}


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def check(ctx, rc, allow=(NB6_OK,)):
    if rc in allow:
        return rc
    msg = lib().nb6_last_error(ctx)
    raise NB6Error(rc, msg.decode() if msg else "")


# ---- the C entry points ---------------------------------------------------
def nb6_create(device=0, slice_hint=0, hbm_budget=0, flags=0, ipl_hint=0, jl_hint=0):
    h = ctypes.c_void_p()
    opt = nb6_options(device, slice_hint, hbm_budget, flags, ipl_hint, jl_hint)
    rc = lib().nb6_create(ctypes.byref(h), ctypes.byref(opt))
    if rc != NB6_OK:
        raise NB6Error(rc, "nb6_create failed")
    return h.value


def nb6_destroy(ctx):
    return lib().nb6_destroy(ctx)


def nb6_last_error(ctx):
    return lib().nb6_last_error(ctx).decode()


def nb6_last_slices(ctx):
    return lib().nb6_last_slices(ctx)


def nb6_last_plan(ctx):
    """(i per lane, lanes per i, slices, j per slice) of the last force call."""
    out = (ctypes.c_int * 4)()
    rc = lib().nb6_last_plan(ctx, out)
    if rc != NB6_OK:
        raise NB6Error(rc, "nb6_last_plan failed")
    return tuple(out)


def nb6_load_particles(ctx, cluster, n, m, x, v, a, jerk, t, idx=None,
                       mem_kind=NB6_MEM_HOST, stream=None):
    f = np.float64
    return lib().nb6_load_particles(
        ctx, cluster, n, _ptr(m, f), _ptr(x, f), _ptr(v, f), _ptr(a, f),
        _ptr(jerk, f), _ptr(t, f), _ptr(idx, np.int32), mem_kind, _stream(stream))


def nb6_predict_j(ctx, cluster, t_block, modes=0, stream=None):
    return lib().nb6_predict_j(ctx, cluster, float(t_block), modes, _stream(stream))


def nb6_regular_force(ctx, cluster, n_i, idx_i, h2_i, dtr_i, dx_mode, acc, jerk,
                      nnb, nblist, cap, mem_kind=NB6_MEM_HOST, stream=None, pot=None):
    """The C entry point; ``pot`` (optional) is its potential output, which the
    C signature takes after ``jerk``."""
    f = np.float64
    return lib().nb6_regular_force(
        ctx, cluster, n_i, _ptr(idx_i, np.int32), _ptr(h2_i, f), _ptr(dtr_i, f),
        dx_mode, _ptr(acc, f), _ptr(jerk, f), _ptr(pot, f), _ptr(nnb, np.int32),
        _ptr(nblist, np.int32), cap, mem_kind, _stream(stream))


def nb6_regular_force_noalloc(ctx, cluster, n_i, idx_i, h2_i, dtr_i, dx_mode, acc, jerk,
                              nnb, nblist, cap, stream=None, pot=None):
    """The C entry point (device arrays only); ``pot`` as in nb6_regular_force."""
    f = np.float64
    return lib().nb6_regular_force_noalloc(
        ctx, cluster, n_i, _ptr(idx_i, np.int32), _ptr(h2_i, f), _ptr(dtr_i, f),
        dx_mode, _ptr(acc, f), _ptr(jerk, f), _ptr(pot, f), _ptr(nnb, np.int32),
        _ptr(nblist, np.int32), cap, _stream(stream))


def nb6_set_lists(ctx, cluster, n_i, idx_i, nnb_i, nblist, cap, mem_kind=NB6_MEM_HOST,
                  stream=None):
    return lib().nb6_set_lists(ctx, cluster, n_i, _ptr(idx_i, np.int32), _ptr(nnb_i, np.int32),
                               _ptr(nblist, np.int32), cap, mem_kind, _stream(stream))


def nb6_irregular_force(ctx, cluster, t_block, n_i, idx_i, acc, jerk, mem_kind=NB6_MEM_HOST,
                        stream=None, pot=None):
    f = np.float64
    return lib().nb6_irregular_force(ctx, cluster, float(t_block), n_i, _ptr(idx_i, np.int32),
                                     _ptr(acc, f), _ptr(jerk, f), _ptr(pot, f), mem_kind,
                                     _stream(stream))


def nb6_get_predicted(ctx, cluster, dx_mode, x, v, mem_kind=NB6_MEM_HOST, stream=None):
    f = np.float64
    return lib().nb6_get_predicted(ctx, cluster, dx_mode, _ptr(x, f), _ptr(v, f), mem_kind,
                                   _stream(stream))


def nb6_kernel_times(ctx):
    """(ms[4], counts[4]) for predictor, force, finalize and irregular-force
    launches."""
    ms = np.zeros(4)
    counts = np.zeros(4, np.int64)
    rc = lib().nb6_kernel_times(ctx, ms.ctypes.data, counts.ctypes.data)
    check(ctx, rc)
    return ms, counts


def nb6_submit(ctx, cluster, t_block, dx_mode, n_i, idx_i, h2_i, dtr_i, acc, jerk, nnb,
               nblist, cap, mem_kind=NB6_MEM_HOST):
    """Queue one request; returns (status, ticket).  The arrays must stay alive
    until nb6_poll reports the request finished."""
    f = np.float64
    rq = nb6_request(cluster, float(t_block), dx_mode, n_i, _ptr(idx_i, np.int32),
                     _ptr(h2_i, f), _ptr(dtr_i, f), _ptr(acc, f), _ptr(jerk, f),
                     _ptr(nnb, np.int32), _ptr(nblist, np.int32), cap, mem_kind)
    t = ctypes.c_uint64(0)
    rc = lib().nb6_submit(ctx, ctypes.byref(rq), ctypes.byref(t))
    return rc, t.value


def nb6_poll(ctx, ticket, wait=0):
    """(status, info dict or None)."""
    info = nb6_ticket_info()
    rc = lib().nb6_poll(ctx, ticket, wait, ctypes.byref(info))
    if rc == NB6_PENDING or rc == NB6_ERR_UNKNOWN_TICKET:
        return rc, None
    return rc, {k: getattr(info, k) for k, _ in nb6_ticket_info._fields_}


def nb6_sync_status(ctx, stream=None):
    return lib().nb6_sync_status(ctx, _stream(stream))


# ---- convenience: allocate outputs, raise on errors ------------------------
def regular_force_host(ctx, cluster, idx_i, h2_i, dtr_i, dx_mode=NB6_DX_FF, cap=256,
                       with_pot=False):
    """Host-memory call; returns (acc, jerk, nnb, lists, status), and the
    potential as a sixth item when ``with_pot``."""
    idx_i = np.ascontiguousarray(idx_i, dtype=np.int32)
    ni = len(idx_i)
    h2_i = np.ascontiguousarray(np.broadcast_to(h2_i, (ni,)), dtype=np.float64)
    dtr_i = np.ascontiguousarray(np.broadcast_to(dtr_i, (ni,)), dtype=np.float64)
    acc = np.empty((ni, 3))
    jerk = np.empty((ni, 3))
    nnb = np.empty(ni, np.int32)
    lst = np.empty((ni, max(cap, 1)), np.int32)
    pot = np.empty(ni) if with_pot else None
    rc = nb6_regular_force(ctx, cluster, ni, idx_i, h2_i, dtr_i, dx_mode, acc, jerk,
                           nnb, lst if cap > 0 else None, cap, NB6_MEM_HOST, pot=pot)
    check(ctx, rc, (NB6_OK, NB6_WARN_NB_OVERFLOW))
    if with_pot:
        return acc, jerk, nnb, lst[:, :cap], rc, pot
    return acc, jerk, nnb, lst[:, :cap], rc


def set_lists_host(ctx, cluster, idx_i, nnb_i, nblist):
    """Host-memory nb6_set_lists: rows of ``nblist`` ([n_i, cap]) hold the first
    ``nnb_i`` entries of each list."""
    idx_i = np.ascontiguousarray(idx_i, dtype=np.int32)
    nnb_i = np.ascontiguousarray(nnb_i, dtype=np.int32)
    nblist = np.ascontiguousarray(nblist, dtype=np.int32)
    check(ctx, nb6_set_lists(ctx, cluster, len(idx_i), idx_i, nnb_i, nblist,
                             nblist.shape[1] if nblist.ndim == 2 else 1, NB6_MEM_HOST))


def irregular_force_host(ctx, cluster, t_block, idx_i, with_pot=False):
    """Host-memory nb6_irregular_force; returns (acc, jerk), and the potential
    as a third item when ``with_pot``."""
    idx_i = np.ascontiguousarray(idx_i, dtype=np.int32)
    ni = len(idx_i)
    acc = np.empty((ni, 3))
    jerk = np.empty((ni, 3))
    pot = np.empty(ni) if with_pot else None
    check(ctx, nb6_irregular_force(ctx, cluster, t_block, ni, idx_i, acc, jerk, NB6_MEM_HOST,
                                   pot=pot))
    return (acc, jerk, pot) if with_pot else (acc, jerk)


def nb6_regular_correct(ctx, n_i, t, arrays, params, mem_kind=NB6_MEM_HOST, stream=None):
    """``arrays``: dict of the nb6_corr_block arrays by field name (inputs and
    outputs); ``params``: (eta, dt_min, dt_max, f_lo, f_hi)."""
    f = np.float64
    blk = nb6_corr_block(n_i, float(t))
    for name, _ in nb6_corr_block._fields_[2:]:
        setattr(blk, name, _ptr(arrays[name], np.int32 if name == "nnb" else f))
    par = nb6_corr_params(*[float(x) for x in params])
    return lib().nb6_regular_correct(ctx, ctypes.byref(blk), ctypes.byref(par), mem_kind,
                                     _stream(stream))


def regular_correct_host(ctx, t, t_old, f_old, fd_old, f_new, fd_new, g_old, gd_old, g_new,
                         gd_new, h_old, nnb, n_p, eta=0.02, dt_min=2.0 ** -20, dt_max=1.0,
                         f_lo=0.5, f_hi=1.25):
    """Host-memory nb6_regular_correct; returns a dict of the outputs."""
    t_old = np.ascontiguousarray(np.atleast_1d(t_old), dtype=np.float64)
    n = len(t_old)
    arrays = {"t_old": t_old}
    for name, a in (("f_old", f_old), ("fd_old", fd_old), ("f_new", f_new), ("fd_new", fd_new),
                    ("g_old", g_old), ("gd_old", gd_old), ("g_new", g_new), ("gd_new", gd_new)):
        arrays[name] = np.ascontiguousarray(np.reshape(a, (n, 3)), dtype=np.float64)
    arrays["h_old"] = np.ascontiguousarray(np.broadcast_to(h_old, (n,)), dtype=np.float64)
    arrays["n_p"] = np.ascontiguousarray(np.broadcast_to(n_p, (n,)), dtype=np.float64)
    arrays["nnb"] = np.ascontiguousarray(np.broadcast_to(nnb, (n,)), dtype=np.int32)
    out = {k: np.empty((n, 3)) for k in ("df", "dfd", "f2", "f3")}
    out.update({k: np.empty(n) for k in ("dt_new", "h_new")})
    arrays.update(out)
    check(ctx, nb6_regular_correct(ctx, n, t, arrays, (eta, dt_min, dt_max, f_lo, f_hi)))
    return out
