"""Compare a GPU regular-force result with the oracle's (test infrastructure).

Rules (the readings behind them are listed in the repository's design notes):

* Neighbour lists must agree exactly, except for a pair whose end-point
  distance R_min lies within ``band`` (relative) of the neighbour radius:
  |R_min - h| <= band * h, evaluated in FP64 by the oracle.  Such a pair is
  "exempt" and may fall on either side.
* When an exempt pair falls on different sides, the oracle's sums are moved
  to the GPU's side of the boundary (its pair term is added or removed)
  before the forces are compared, so the force check measures arithmetic,
  not the boundary decision.
* Errors are reported per particle in two normalisations:
    e_i  = |da_i| / |a_i|      (relative to the net regular force), and
    es_i = |da_i| / S_i        (relative to S_i = sum over non-neighbours of
                                m_j / r^2, the scale of the summed terms);
  likewise for the jerk with S'_i = sum m_j (|V|/r^3 + 3|R.V|/r^4).
  Net values can cancel to a small fraction of the term scale, and the FP32
  rounding of each term (a few 1e-8 of the term) then dominates the error of
  the net value, so the relative error is bounded only for particles whose
  net value is at least ``floor_acc`` (``floor_jerk``) of its scale.  Random
  per-term rounding of FP32 arithmetic leaves a scaled error of at most about
  1e-7, so the relative bar of 1e-6 needs a net value of at least ~0.1 of
  the scale; the acceleration, whose terms add coherently towards the cluster
  centre, meets it down to 1e-3.  The scaled errors are bounded for every
  particle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import oracle as _o


@dataclass
class Comparison:
    n_i: int
    list_mismatch: int = 0          # disagreements outside the boundary band
    exempt_pairs: int = 0           # disagreements inside the band
    nnb_mismatch: int = 0           # count disagreements not explained by exempt pairs
    incomplete: int = 0             # i whose GPU list was truncated (nnb > cap)
    err: dict = field(default_factory=dict)
    mismatches: list = field(default_factory=list)

    def summary(self) -> dict:
        return dict(n_i=self.n_i, list_mismatch=self.list_mismatch,
                    exempt_pairs=self.exempt_pairs, nnb_mismatch=self.nnb_mismatch,
                    incomplete=self.incomplete, **self.err)


def _stats(prefix, e):
    if len(e) == 0:
        return {f"{prefix}_n": 0}
    return {f"{prefix}_median": float(np.median(e)),
            f"{prefix}_p99": float(np.quantile(e, 0.99)),
            f"{prefix}_max": float(np.max(e)),
            f"{prefix}_n": int(len(e))}


def compare(gpu_acc, gpu_jerk, gpu_nnb, gpu_lists, cap, ref, m, xp, vp, idx, h2, dtr,
            band=1e-6, floor_acc=1e-3, floor_jerk=0.1, lib=None) -> Comparison:
    """``ref`` is an ``OracleResult`` for the same (idx, h2, dtr) and state."""
    idx = np.asarray(idx)
    ni = len(idx)
    h2 = np.broadcast_to(np.asarray(h2, float), (ni,))
    dtr = np.broadcast_to(np.asarray(dtr, float), (ni,))
    c = Comparison(ni)
    acc_ref = ref.acc.copy()
    jerk_ref = ref.jerk.copy()
    nnb_ref = ref.nnb.astype(np.int64).copy()
    pi, pj, sign = [], [], []
    for q in range(ni):
        k = int(gpu_nnb[q])
        if k > cap:
            c.incomplete += 1
            continue
        g = gpu_lists[q][:k]
        o = ref.lists[q]
        if len(g) == len(o) and np.array_equal(g, o):
            continue
        gs, os_ = set(map(int, g)), set(map(int, o))
        if len(gs) != len(g) or list(g) != sorted(g):
            c.list_mismatch += 1
            c.mismatches.append((q, "unsorted-or-duplicate"))
            continue
        for j in gs - os_:
            pi.append(idx[q]); pj.append(j); sign.append((q, -1))
        for j in os_ - gs:
            pi.append(idx[q]); pj.append(j); sign.append((q, +1))
    if pi:
        qd = np.array([s[0] for s in sign])
        rmin, dacc, djrk = _o.pair_terms(pi, pj, dtr[qd], m, xp, vp, lib=lib)
        h = np.sqrt(h2[qd])
        exempt = np.abs(rmin - h) <= band * h
        for t, (q, sg) in enumerate(sign):
            if exempt[t]:
                c.exempt_pairs += 1
                # sg = -1: GPU listed j, oracle summed it -> remove from oracle sums
                acc_ref[q] += sg * dacc[t]
                jerk_ref[q] += sg * djrk[t]
                nnb_ref[q] -= sg
            else:
                c.list_mismatch += 1
                c.mismatches.append((int(q), int(pj[t]), float(rmin[t]), float(h[t])))
    ok = gpu_nnb <= cap
    c.nnb_mismatch = int(np.sum(ok & (gpu_nnb != nnb_ref)))

    da = np.linalg.norm(gpu_acc - acc_ref, axis=1)
    dj = np.linalg.norm(gpu_jerk - jerk_ref, axis=1)
    na = np.linalg.norm(acc_ref, axis=1)
    nj = np.linalg.norm(jerk_ref, axis=1)
    sa = np.maximum(ref.sa, 1e-300)
    sj = np.maximum(ref.sj, 1e-300)
    sel_a = na >= floor_acc * ref.sa
    sel_j = nj >= floor_jerk * ref.sj
    low_j = nj >= 1e-3 * ref.sj
    c.err.update(_stats("acc_rel", da[sel_a] / na[sel_a]))
    c.err.update(_stats("acc_scaled", da / sa))
    c.err.update(_stats("jerk_rel", dj[sel_j] / nj[sel_j]))
    c.err.update(_stats("jerk_scaled", dj / sj))
    c.err["acc_rel_excluded"] = int(ni - sel_a.sum())
    c.err["jerk_rel_excluded"] = int(ni - sel_j.sum())
    c.err.update(_stats("jerk_rel_floor1e-3", dj[low_j] / nj[low_j]))
    c.err["floors"] = {"acc": floor_acc, "jerk": floor_jerk}
    return c
