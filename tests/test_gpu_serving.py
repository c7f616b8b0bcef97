"""GPU tests of the serving queue (nb6_submit / nb6_poll) through the C ABI.

* every served result matches the FP64 oracle (same bars as the plain path);
* a request gives bit-identical results alone and fused with others;
* served results equal the plain call's when both use one i per lane, and
  under lanes per i (staged or not, forced lane counts, ragged slices);
* requests of C4's size (32768- and 65536-body clusters, blocks of up to all
  their particles) fused with small ones match the oracle on sampled rows;
* admission: a request larger than the HBM budget is refused; requests that
  only fit one at a time all complete;
* overflowed lists, unknown tickets, double polls.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle.compare import compare  # noqa: E402
from workloads import make_cluster  # noqa: E402


def _nb6():
    from paper_1205_1222_amd import nb6
    return nb6


SIZES = [2048, 3001, 4096, 6000]


@pytest.fixture(scope="module")
def clusters():
    return [make_cluster(n, 500 + k, masses="imf", k_nb=24) for k, n in enumerate(SIZES)]


def _load_all(nb6, ctx, cls):
    for c, cl in enumerate(cls):
        nb6.check(ctx, nb6.nb6_load_particles(ctx, c, cl.n, cl.m, cl.x, cl.v, cl.a,
                                              cl.jerk, cl.t))


def _requests(cls, seed=1, per_cluster=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for c, cl in enumerate(cls):
        for r in range(per_cluster):
            ni = int(rng.choice([1, 16, 64, 100, 257, 1024]))
            idx = np.sort(rng.choice(cl.n, ni, replace=False)).astype(np.int32)
            tb = cl.tb + r * 2.0 ** -12   # successive block times of the cluster
            out.append((c, tb, idx))
    return out


class Host:
    """Host buffers of one request (kept alive until polled)."""

    def __init__(self, ni, cap):
        self.acc = np.full((ni, 3), np.nan)
        self.jerk = np.full((ni, 3), np.nan)
        self.nnb = np.full(ni, -9, np.int32)
        self.lst = np.full((ni, max(cap, 1)), -9, np.int32)


def _submit(nb6, ctx, cl, c, tb, idx, cap, mode=1):
    h = Host(len(idx), cap)
    h.idx = np.ascontiguousarray(idx, np.int32)
    h.h2 = np.ascontiguousarray(cl.h2[idx])
    h.dtr = np.ascontiguousarray(cl.dtr[idx])
    rc, t = nb6.nb6_submit(ctx, c, tb, mode, len(idx), h.idx, h.h2, h.dtr, h.acc, h.jerk,
                           h.nnb, h.lst if cap > 0 else None, cap)
    nb6.check(ctx, rc)
    return t, h


@pytest.mark.parametrize("mode", [1, 8])
def test_served_results_match_oracle(clusters, mode):
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        cap = 256
        subs = []
        for c, tb, idx in _requests(clusters):
            subs.append((c, tb, idx) + _submit(nb6, ctx, clusters[c], c, tb, idx, cap, mode))
        sizes = []
        for c, tb, idx, t, h in subs:
            rc, info = nb6.nb6_poll(ctx, t, wait=1)
            assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW), rc
            sizes.append(info["batch_size"])
            assert info["submit_us"] <= info["admit_us"] <= info["done_us"]
            cl = clusters[c]
            xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, tb)
            ref = oracle.regular_force(cl.m, xp, vp, idx, cl.h2[idx], cl.dtr[idx], lcap=4096)
            cmp_ = compare(h.acc, h.jerk, h.nnb, h.lst, cap, ref, cl.m, xp, vp, idx,
                           cl.h2[idx], cl.dtr[idx])
            s = cmp_.summary()
            assert cmp_.list_mismatch == 0 and cmp_.nnb_mismatch == 0, s
            assert s["acc_scaled_max"] <= 1e-6 and s["jerk_scaled_max"] <= 1e-6, s
            assert s.get("acc_rel_max", 0) <= 1e-6 and s.get("jerk_rel_max", 0) <= 1e-6, s
        print("batch sizes", sizes, flush=True)
        assert max(sizes) > 1  # requests were fused
    finally:
        nb6.nb6_destroy(ctx)


@pytest.mark.parametrize("mode", [1, 8])
def test_alone_and_mixed_are_bit_identical(clusters, mode):
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        cap = 128
        reqs = _requests(clusters, seed=7, per_cluster=2)
        alone = []
        for c, tb, idx in reqs:  # one at a time
            t, h = _submit(nb6, ctx, clusters[c], c, tb, idx, cap, mode)
            rc, info = nb6.nb6_poll(ctx, t, wait=1)
            assert info["batch_size"] == 1
            alone.append(h)
        # all at once, in reverse order, mixed with other clusters' blocks
        mixed = [None] * len(reqs)
        tickets = []
        for k in reversed(range(len(reqs))):
            c, tb, idx = reqs[k]
            t, h = _submit(nb6, ctx, clusters[c], c, tb, idx, cap, mode)
            tickets.append((k, t, h))
        fused = 0
        for k, t, h in tickets:
            rc, info = nb6.nb6_poll(ctx, t, wait=1)
            fused = max(fused, info["batch_size"])
            mixed[k] = h
        assert fused > 1
        for a, m in zip(alone, mixed):
            np.testing.assert_array_equal(a.acc, m.acc)
            np.testing.assert_array_equal(a.jerk, m.jerk)
            np.testing.assert_array_equal(a.nnb, m.nnb)
            for q in range(len(a.nnb)):
                k = min(cap, a.nnb[q])
                np.testing.assert_array_equal(a.lst[q, :k], m.lst[q, :k])
    finally:
        nb6.nb6_destroy(ctx)


@pytest.mark.parametrize("hint,c,step,ni_max,mode", [(1, 2, 7, None, 1), (0, 3, 1, 4500, 1),
                                                     (2, 3, 1, 4500, 1), (0, 1, 1, 2000, 1),
                                                     (0, 0, 1, 20, 1), (0, 3, 1, 4500, 8),
                                                     (2, 3, 1, 4500, 8), (0, 0, 1, 20, 8)])
def test_served_equals_plain_call(clusters, hint, c, step, ni_max, mode):
    """A served request takes the plan a plain call on the same context takes
    (one i per lane, or two when the context asks for it; lanes per i for
    small blocks), hence the same bits."""
    nb6 = _nb6()
    ctx = nb6.nb6_create(0, ipl_hint=hint)
    try:
        _load_all(nb6, ctx, clusters)
        cl = clusters[c]
        idx = np.arange(0, cl.n, step, dtype=np.int32)[:ni_max]
        t, h = _submit(nb6, ctx, cl, c, cl.tb, idx, 64, mode)
        rc, _ = nb6.nb6_poll(ctx, t, wait=1)
        assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
        nb6.check(ctx, nb6.nb6_predict_j(ctx, c, cl.tb, mode))
        acc, jerk, nnb, lst, _ = nb6.regular_force_host(ctx, c, idx, cl.h2[idx], cl.dtr[idx],
                                                        mode, 64)
        print("plan", len(idx), nb6.nb6_last_plan(ctx), flush=True)
        np.testing.assert_array_equal(acc, h.acc)
        np.testing.assert_array_equal(jerk, h.jerk)
        np.testing.assert_array_equal(nnb, h.nnb)
        for q in range(len(idx)):
            k = min(64, nnb[q])
            np.testing.assert_array_equal(lst[q, :k], h.lst[q, :k])
    finally:
        nb6.nb6_destroy(ctx)


@pytest.mark.parametrize("jl", [2, 8, 32])
def test_served_lanes_items_forced_lane_counts(clusters, jl):
    """Lanes-class requests under forced lane counts and ragged slices, fused
    into one batch: the served workgroup items (staged through LDS, with idle
    waves when a request has fewer i-groups than the workgroup has waves)
    give the plain call's bits, whose single-wave workgroups read the
    vector cache and whose larger ones stage too."""
    nb6 = _nb6()
    ctx = nb6.nb6_create(0, jl_hint=jl, slice_hint=3)
    try:
        _load_all(nb6, ctx, clusters)
        rng = np.random.Generator(np.random.PCG64(jl))
        reqs = []
        for c, cl in enumerate(clusters):
            for ni, mode in ((5, 1), (70, 8), (200, 1)):
                idx = np.sort(rng.choice(cl.n, ni, replace=False)).astype(np.int32)
                reqs.append((c, idx, mode))
        subs = [_submit(nb6, ctx, clusters[c], c, clusters[c].tb, idx, 64, mode)
                for c, idx, mode in reqs]
        for t, h in subs:
            rc, _ = nb6.nb6_poll(ctx, t, wait=1)
            assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
        for (t, h), (c, idx, mode) in zip(subs, reqs):
            cl = clusters[c]
            nb6.check(ctx, nb6.nb6_predict_j(ctx, c, cl.tb, mode))
            acc, jerk, nnb, lst, _ = nb6.regular_force_host(ctx, c, idx, cl.h2[idx],
                                                            cl.dtr[idx], mode, 64)
            assert nb6.nb6_last_plan(ctx)[1] == jl
            np.testing.assert_array_equal(acc, h.acc)
            np.testing.assert_array_equal(jerk, h.jerk)
            np.testing.assert_array_equal(nnb, h.nnb)
            for q in range(len(idx)):
                k = min(64, nnb[q])
                np.testing.assert_array_equal(lst[q, :k], h.lst[q, :k])
    finally:
        nb6.nb6_destroy(ctx)


def test_plain_calls_after_serving(clusters):
    """A served request predicts its cluster to its own block time.  A plain
    call afterwards uses those float-float records (the same bits as the
    served result), and a mode whose records still hold the earlier block
    time is refused instead of being mixed with the newer one."""
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        c = 2
        cl = clusters[c]
        idx = np.arange(0, cl.n, 7, dtype=np.int32)
        nb6.check(ctx, nb6.nb6_predict_j(ctx, c, cl.tb, 0))     # every mode at tb
        tb2 = cl.tb + 2.0 ** -10
        t, h = _submit(nb6, ctx, cl, c, tb2, idx, 64)            # FF at tb2
        assert nb6.nb6_poll(ctx, t, wait=1)[0] in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
        acc, jerk, nnb, lst, _ = nb6.regular_force_host(ctx, c, idx, cl.h2[idx],
                                                        cl.dtr[idx], nb6.NB6_DX_FF, 64)
        np.testing.assert_array_equal(acc, h.acc)
        np.testing.assert_array_equal(jerk, h.jerk)
        np.testing.assert_array_equal(nnb, h.nnb)
        with pytest.raises(nb6.NB6Error) as e:
            nb6.regular_force_host(ctx, c, idx, cl.h2[idx], cl.dtr[idx], nb6.NB6_DX_FP64, 64)
        assert e.value.code == nb6.NB6_ERR_STATE
        # predicting another mode to tb2 makes it usable, and keeps FF current
        nb6.check(ctx, nb6.nb6_predict_j(ctx, c, tb2, nb6.NB6_DX_FP64))
        a64 = nb6.regular_force_host(ctx, c, idx, cl.h2[idx], cl.dtr[idx], nb6.NB6_DX_FP64,
                                     64)[0]
        assert np.max(np.abs(a64 - acc) / np.linalg.norm(acc, axis=1)[:, None]) < 1e-5
        aff = nb6.regular_force_host(ctx, c, idx, cl.h2[idx], cl.dtr[idx], nb6.NB6_DX_FF,
                                     64)[0]
        np.testing.assert_array_equal(aff, h.acc)
    finally:
        nb6.nb6_destroy(ctx)


def test_plain_calls_beside_the_queue(clusters):
    """Plain calls on some clusters while the queue serves others, on one
    context: every result equals the same computation done alone (the queue
    and the plain path keep separate scratch and status)."""
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        rng = np.random.Generator(np.random.PCG64(21))
        served = []
        for r in range(6):
            for c in (0, 1):
                cl = clusters[c]
                idx = np.sort(rng.choice(cl.n, int(rng.choice([16, 300, 1500])),
                                         replace=False)).astype(np.int32)
                served.append((c, cl.tb + r * 2.0 ** -12, idx))
        plain = [(c, np.arange(c, clusters[c].n, 5, dtype=np.int32)) for c in (2, 3)]

        def plain_call(c, idx):
            cl = clusters[c]
            nb6.check(ctx, nb6.nb6_predict_j(ctx, c, cl.tb, nb6.NB6_DX_FF))
            return nb6.regular_force_host(ctx, c, idx, cl.h2[idx], cl.dtr[idx],
                                          nb6.NB6_DX_FF, 64)[:3]

        alone_plain = [plain_call(c, idx) for c, idx in plain]
        alone_served = []
        for c, tb, idx in served:
            t, h = _submit(nb6, ctx, clusters[c], c, tb, idx, 64)
            assert nb6.nb6_poll(ctx, t, wait=1)[0] in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
            alone_served.append(h)
        # now all at once: the whole queue, then plain calls while it drains
        subs = [_submit(nb6, ctx, clusters[c], c, tb, idx, 64) for c, tb, idx in served]
        mixed_plain = [plain_call(c, idx) for c, idx in plain for _ in range(2)]
        for (t, h), ref in zip(subs, alone_served):
            assert nb6.nb6_poll(ctx, t, wait=1)[0] in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
            np.testing.assert_array_equal(h.acc, ref.acc)
            np.testing.assert_array_equal(h.jerk, ref.jerk)
            np.testing.assert_array_equal(h.nnb, ref.nnb)
        for k, got in enumerate(mixed_plain):
            ref = alone_plain[k // 2]
            for a, b in zip(got, ref):
                np.testing.assert_array_equal(a, b)
    finally:
        nb6.nb6_destroy(ctx)


def test_mixed_coordinate_modes(clusters):
    """Requests in all four coordinate modes fused into the same batches
    (one persistent launch per mode and work-partition class): each equals,
    bit for bit, the plain call in its mode at its block time.  Blocks of 200
    take 8 lanes per i, and blocks of 40 64 lanes per i: workgroups that
    share the j-records through LDS in the one case (a plain launch of
    several waves, a served workgroup item), lanes that read them from the
    vector cache in the other."""
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        modes = (nb6.NB6_DX_FF, nb6.NB6_DX_FP64, nb6.NB6_DX_FP32, nb6.NB6_DX_LOCAL)
        rng = np.random.Generator(np.random.PCG64(31))
        reqs = []
        for r in range(3):
            for c, cl in enumerate(clusters):
                ni = int(rng.choice([40, 200, 700]))
                idx = np.sort(rng.choice(cl.n, ni, replace=False)).astype(np.int32)
                reqs.append((c, cl.tb + r * 2.0 ** -12, idx, modes[(r + c) % 4]))
        subs = [_submit(nb6, ctx, clusters[c], c, tb, idx, 64, mode)
                for c, tb, idx, mode in reqs]
        fused = 0
        for (t, h), (c, tb, idx, mode) in zip(subs, reqs):
            rc, info = nb6.nb6_poll(ctx, t, wait=1)
            assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
            fused = max(fused, info["batch_size"])
        for (t, h), (c, tb, idx, mode) in zip(subs, reqs):
            cl = clusters[c]
            nb6.check(ctx, nb6.nb6_predict_j(ctx, c, tb, mode))
            acc, jerk, nnb, lst, _ = nb6.regular_force_host(ctx, c, idx, cl.h2[idx],
                                                            cl.dtr[idx], mode, 64)
            np.testing.assert_array_equal(acc, h.acc)
            np.testing.assert_array_equal(jerk, h.jerk)
            np.testing.assert_array_equal(nnb, h.nnb)
            for q in range(len(idx)):
                k = min(64, nnb[q])
                np.testing.assert_array_equal(lst[q, :k], h.lst[q, :k])
        assert fused > 1
    finally:
        nb6.nb6_destroy(ctx)


def test_admission_by_budget(clusters):
    nb6 = _nb6()
    budget = 6 << 20
    # one lane per i forced, so the 600-particle requests below keep their
    # slice counts (this cluster size would otherwise give them lanes per i
    # and fewer slices)
    ctx = nb6.nb6_create(0, hbm_budget=budget, jl_hint=1)
    try:
        _load_all(nb6, ctx, clusters)
        cl = clusters[3]
        # too big for the budget on its own: refused at submit
        big = np.arange(cl.n, dtype=np.int32)
        h = Host(len(big), 1023)
        rc, _ = nb6.nb6_submit(ctx, 3, cl.tb, 1, len(big), big, cl.h2[big].copy(),
                               cl.dtr[big].copy(), h.acc, h.jerk, h.nnb, h.lst, 1023)
        assert rc == nb6.NB6_ERR_ADMISSION
        # each fits alone (3.4 to 4.4 MB: lists, staging and 32 or 64 slices of
        # partials) but not two at once
        subs = []
        for c in range(4):
            cl = clusters[c]
            idx = np.arange(0, 600, dtype=np.int32)
            subs.append(_submit(nb6, ctx, cl, c, cl.tb, idx, 500))
        for t, h in subs:
            rc, info = nb6.nb6_poll(ctx, t, wait=1)
            assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
            assert info["batch_size"] == 1
            assert np.all(np.isfinite(h.acc))
    finally:
        nb6.nb6_destroy(ctx)


def test_overflow_unknown_and_double_poll(clusters):
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        cl = clusters[0]
        idx = np.array([3, 50, 900], np.int32)
        t_full, full = _submit(nb6, ctx, cl, 0, cl.tb, idx, 256)
        assert nb6.nb6_poll(ctx, t_full, wait=1)[0] == nb6.NB6_OK
        t, h = _submit(nb6, ctx, cl, 0, cl.tb, idx, 2)
        rc, _ = nb6.nb6_poll(ctx, t, wait=1)
        assert rc == nb6.NB6_WARN_NB_OVERFLOW
        np.testing.assert_array_equal(h.nnb, full.nnb)
        np.testing.assert_array_equal(h.lst[:, :2], full.lst[:, :2])
        assert nb6.nb6_poll(ctx, t, wait=0)[0] == nb6.NB6_ERR_UNKNOWN_TICKET
        assert nb6.nb6_poll(ctx, 987654, wait=0)[0] == nb6.NB6_ERR_UNKNOWN_TICKET
        # bad requests are refused at submit
        rc, _ = nb6.nb6_submit(ctx, 0, cl.tb, 3, 3, idx, cl.h2[idx].copy(), cl.dtr[idx].copy(),
                               h.acc, h.jerk, h.nnb, h.lst, 2)
        assert rc == nb6.NB6_ERR_ARG
        rc, _ = nb6.nb6_submit(ctx, 9, cl.tb, 1, 3, idx, cl.h2[idx].copy(), cl.dtr[idx].copy(),
                               h.acc, h.jerk, h.nnb, h.lst, 2)
        assert rc == nb6.NB6_ERR_STATE
    finally:
        nb6.nb6_destroy(ctx)


def test_device_mode_serving(clusters):
    import torch
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        cl = clusters[1]
        idx = np.arange(5, cl.n, 11, dtype=np.int32)
        t, h = _submit(nb6, ctx, cl, 1, cl.tb, idx, 128)
        assert nb6.nb6_poll(ctx, t, wait=1)[0] == nb6.NB6_OK
        dev = torch.device("cuda:0")
        ni = len(idx)
        ti = torch.from_numpy(idx).to(dev)
        th2 = torch.from_numpy(cl.h2[idx].copy()).to(dev)
        tdt = torch.from_numpy(cl.dtr[idx].copy()).to(dev)
        acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty_like(acc)
        nnb = torch.empty(ni, dtype=torch.int32, device=dev)
        lst = torch.empty((ni, 128), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        rc, t2 = nb6.nb6_submit(ctx, 1, cl.tb, 1, ni, ti, th2, tdt, acc, jerk, nnb, lst, 128,
                                nb6.NB6_MEM_DEVICE)
        nb6.check(ctx, rc)
        assert nb6.nb6_poll(ctx, t2, wait=1)[0] == nb6.NB6_OK
        np.testing.assert_array_equal(acc.cpu().numpy(), h.acc)
        np.testing.assert_array_equal(nnb.cpu().numpy(), h.nnb)
    finally:
        nb6.nb6_destroy(ctx)


def test_resize_refused_while_requests_are_queued(clusters):
    """A full load that would resize a cluster is refused while requests on
    it are queued or running, so no request is launched with buffers sized
    for another N.  Whichever way the race between the reload and the queue
    goes, every request ends with the results of the state it was submitted
    against, and the reload succeeds once the queue has drained."""
    nb6 = _nb6()
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, clusters)
        cl = clusters[3]
        idx = np.arange(cl.n, dtype=np.int32)
        subs = [_submit(nb6, ctx, cl, 3, cl.tb, idx, 64) for _ in range(4)]
        small = make_cluster(1500, 77, masses="equal", k_nb=16)
        rc = nb6.nb6_load_particles(ctx, 3, small.n, small.m, small.x, small.v, small.a,
                                    small.jerk, small.t)
        refused = rc == nb6.NB6_ERR_STATE
        assert rc in (nb6.NB6_OK, nb6.NB6_ERR_STATE), rc
        done = {}
        if not refused:  # accepted only after every request had finished
            for t, _ in subs:
                done[t] = nb6.nb6_poll(ctx, t, wait=0)[0]  # a final status releases t
                assert done[t] != nb6.NB6_PENDING
        first = None
        for t, h in subs:
            rc = done[t] if t in done else nb6.nb6_poll(ctx, t, wait=1)[0]
            assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW), rc
            if first is None:
                first = h
            np.testing.assert_array_equal(h.acc, first.acc)
            np.testing.assert_array_equal(h.nnb, first.nnb)
        xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
        si = idx[::97]
        ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
        c = compare(first.acc[si], first.jerk[si], first.nnb[si], first.lst[si], 64, ref,
                    cl.m, xp, vp, si, cl.h2[si], cl.dtr[si])
        assert c.list_mismatch == 0 and c.summary()["acc_scaled_max"] <= 1e-6, c.summary()
        print("reload refused while queued:", refused, flush=True)
        # the queue has drained: the resize is accepted and the cluster works
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 3, small.n, small.m, small.x, small.v,
                                              small.a, small.jerk, small.t))
        si = np.arange(0, small.n, 3, dtype=np.int32)
        t, h = _submit(nb6, ctx, small, 3, small.tb, si, 64)
        assert nb6.nb6_poll(ctx, t, wait=1)[0] in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
        xp, vp = oracle.predict(small.x, small.v, small.a, small.jerk, small.t, small.tb)
        ref = oracle.regular_force(small.m, xp, vp, si, small.h2[si], small.dtr[si], lcap=4096)
        c = compare(h.acc, h.jerk, h.nnb, h.lst, 64, ref, small.m, xp, vp, si, small.h2[si],
                    small.dtr[si])
        assert c.list_mismatch == 0 and c.summary()["acc_scaled_max"] <= 1e-6, c.summary()
    finally:
        nb6.nb6_destroy(ctx)


def test_large_clusters_fused_with_small_match_oracle():
    """Blocks of the serving trace's largest clusters (32768 and 65536 bodies,
    equal masses, ~50 neighbours; blocks of 4096 up to every particle) fused
    with small blocks of small clusters, in the float-float and local modes:
    every request completes, is fused with others, and 128 sampled rows of
    each (all rows of the small ones) meet the oracle bars."""
    nb6 = _nb6()
    sizes = [32768, 65536, 4096, 6000]
    cls = [make_cluster(n, 900 + k, masses="equal", k_nb=50) for k, n in enumerate(sizes)]
    ctx = nb6.nb6_create(0)
    try:
        _load_all(nb6, ctx, cls)
        rng = np.random.Generator(np.random.PCG64(77))
        reqs = []
        for mode in (nb6.NB6_DX_FF, nb6.NB6_DX_LOCAL):
            for c, ni in ((0, 32768), (1, 65536), (1, 4096), (0, 8192), (2, 16), (3, 300),
                          (2, 1024), (3, 64)):
                idx = (np.arange(cls[c].n, dtype=np.int32) if ni == cls[c].n else
                       np.sort(rng.choice(cls[c].n, ni, replace=False)).astype(np.int32))
                tb = cls[c].tb + len(reqs) * 2.0 ** -14
                reqs.append((c, tb, idx, mode))
        cap = 128
        subs = [_submit(nb6, ctx, cls[c], c, tb, idx, cap, mode) for c, tb, idx, mode in reqs]
        fused = 0
        for (t, h), (c, tb, idx, mode) in zip(subs, reqs):
            rc, info = nb6.nb6_poll(ctx, t, wait=1)
            assert rc in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW), rc
            fused = max(fused, info["batch_size"])
        assert fused > 1
        for (t, h), (c, tb, idx, mode) in zip(subs, reqs):
            cl = cls[c]
            samp = np.sort(rng.choice(len(idx), min(128, len(idx)), replace=False))
            si = idx[samp]
            xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, tb)
            ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
            cmp_ = compare(h.acc[samp], h.jerk[samp], h.nnb[samp], h.lst[samp], cap, ref, cl.m,
                           xp, vp, si, cl.h2[si], cl.dtr[si])
            s = cmp_.summary()
            print("C4-scale", cl.n, len(idx), mode, s["acc_rel_max"], s["jerk_rel_max"],
                  flush=True)
            assert cmp_.incomplete == 0
            assert cmp_.list_mismatch == 0 and cmp_.nnb_mismatch == 0, s
            assert s["acc_scaled_max"] <= 1e-6 and s["jerk_scaled_max"] <= 1e-6, s
            assert s.get("acc_rel_max", 0) <= 1e-6 and s.get("jerk_rel_max", 0) <= 1e-6, s
    finally:
        nb6.nb6_destroy(ctx)
