"""The force entry point that allocates nothing (nb6_regular_force_noalloc),
through the C ABI, against nb6_regular_force on the same context.

* Two calls in a row, the second smaller, whose plans fit the fixed scratch
  array: the same plan as the plain call, hence the same bits.
* A call whose plain plan does not fit: fewer j-slices, the same neighbour
  lists and counts, and forces within the oracle bars (both calls are
  checked against the FP64 oracle on sampled rows, and against each other
  scaled by the oracle's sum of term magnitudes).
* A block too large for one slice is refused with NB6_ERR_ARG.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle.compare import compare  # noqa: E402
from workloads import config  # noqa: E402


def _nb6():
    from paper_1205_1222_amd import nb6
    return nb6


def _call(nb6, ctx, noalloc, cl, idx, mode, cap, with_pot):
    import torch
    dev = torch.device("cuda:0")
    ni = len(idx)
    t_idx = torch.from_numpy(np.ascontiguousarray(idx, np.int32)).to(dev)
    t_h2 = torch.from_numpy(np.ascontiguousarray(cl.h2[idx])).to(dev)
    t_dtr = torch.from_numpy(np.ascontiguousarray(cl.dtr[idx])).to(dev)
    acc = torch.full((ni, 3), float("nan"), dtype=torch.float64, device=dev)
    jerk = torch.full((ni, 3), float("nan"), dtype=torch.float64, device=dev)
    nnb = torch.full((ni,), -9, dtype=torch.int32, device=dev)
    lst = torch.full((ni, max(cap, 1)), -9, dtype=torch.int32, device=dev)
    pot = torch.full((ni,), float("nan"), dtype=torch.float64, device=dev) if with_pot else None
    s = torch.cuda.current_stream()
    if noalloc:
        rc = nb6.nb6_regular_force_noalloc(ctx, 0, ni, t_idx, t_h2, t_dtr, mode, acc, jerk, nnb,
                                           lst, cap, s, pot=pot)
    else:
        rc = nb6.nb6_regular_force(ctx, 0, ni, t_idx, t_h2, t_dtr, mode, acc, jerk, nnb, lst,
                                   cap, nb6.NB6_MEM_DEVICE, s, pot=pot)
    nb6.check(ctx, rc)
    nb6.check(ctx, nb6.nb6_sync_status(ctx, s))
    plan = nb6.nb6_last_plan(ctx)
    out = [acc.cpu().numpy(), jerk.cpu().numpy(), nnb.cpu().numpy(), lst.cpu().numpy()]
    out.append(pot.cpu().numpy() if with_pot else None)
    return out, plan


def _lists_equal(a, b, cap):
    np.testing.assert_array_equal(a[2], b[2])
    for q in range(len(a[2])):
        k = min(cap, int(a[2][q]))
        np.testing.assert_array_equal(a[3][q, :k], b[3][q, :k])


def _check_oracle(cl, idx, out, cap, n_samp, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    samp = np.sort(rng.choice(len(idx), min(n_samp, len(idx)), replace=False))
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    si = idx[samp]
    ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
    c = compare(out[0][samp], out[1][samp], out[2][samp], out[3][samp], cap, ref, cl.m, xp, vp,
                si, cl.h2[si], cl.dtr[si])
    s = c.summary()
    assert c.incomplete == 0 and c.list_mismatch == 0 and c.nnb_mismatch == 0, s
    assert s["acc_scaled_max"] <= 1e-6 and s["jerk_scaled_max"] <= 1e-6, s
    assert s.get("acc_rel_max", 0.0) <= 1e-6 and s.get("jerk_rel_max", 0.0) <= 1e-6, s
    return samp, ref


def test_noalloc_two_calls_equal_the_plain_call():
    nb6 = _nb6()
    cfg = config(3)
    cl = cfg["cluster"]
    ctx = nb6.nb6_create(0)
    try:
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, cl.n, cl.m, cl.x, cl.v, cl.a, cl.jerk,
                                              cl.t))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, 0))
        big = (cfg["blocks"]["pow2_10"], nb6.NB6_DX_LOCAL, 256, True)
        small = (cfg["blocks"]["pow2_10"][::11], nb6.NB6_DX_FF, 200, False)
        got = [_call(nb6, ctx, True, cl, idx, mode, cap, pot) for idx, mode, cap, pot in
               (big, small)]
        want = [_call(nb6, ctx, False, cl, idx, mode, cap, pot) for idx, mode, cap, pot in
                (big, small)]
        for (g, gp), (w, wp), (idx, mode, cap, pot) in zip(got, want, (big, small)):
            print("noalloc plan", len(idx), gp, "plain plan", wp, flush=True)
            assert gp == wp
            for a, b in zip(g[:2], w[:2]):
                np.testing.assert_array_equal(a, b)
            _lists_equal(g, w, cap)
            if pot:
                np.testing.assert_array_equal(g[4], w[4])
            _check_oracle(cl, idx, g, cap, 128, 3)
    finally:
        nb6.nb6_destroy(ctx)


def test_noalloc_takes_fewer_slices_when_the_plan_does_not_fit():
    nb6 = _nb6()
    cfg = config(2, n=262144)
    cl = cfg["cluster"]
    ctx = nb6.nb6_create(0)
    try:
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, cl.n, cl.m, cl.x, cl.v, cl.a, cl.jerk,
                                              cl.t))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, nb6.NB6_DX_LOCAL))
        rng = np.random.Generator(np.random.PCG64(8))
        idx = np.sort(rng.choice(cl.n, 4096, replace=False)).astype(np.int32)
        cap = 256
        g, gp = _call(nb6, ctx, True, cl, idx, nb6.NB6_DX_LOCAL, cap, False)
        w, wp = _call(nb6, ctx, False, cl, idx, nb6.NB6_DX_LOCAL, cap, False)
        print("noalloc plan", gp, "plain plan", wp, flush=True)
        assert gp[2] < wp[2]
        part = 8 * 6 * gp[2] * 4096
        assert part + 4 * 4096 * (cap + 2) <= nb6.NB6_NOALLOC_SCRATCH_BYTES
        _lists_equal(g, w, cap)
        samp, ref = _check_oracle(cl, idx, g, cap, 128, 4)
        _check_oracle(cl, idx, w, cap, 128, 4)
        da = np.linalg.norm(g[0][samp] - w[0][samp], axis=1) / ref.sa
        dj = np.linalg.norm(g[1][samp] - w[1][samp], axis=1) / ref.sj
        assert da.max() <= 1e-6 and dj.max() <= 1e-6, (da.max(), dj.max())
        # a block too large for one slice is refused
        import torch
        dev = torch.device("cuda:0")
        n_big = 20000
        t = torch.zeros(n_big, dtype=torch.int32, device=dev)
        f = torch.ones(n_big, dtype=torch.float64, device=dev)
        o3 = torch.empty((n_big, 3), dtype=torch.float64, device=dev)
        lst = torch.empty((n_big, 1023), dtype=torch.int32, device=dev)
        rc = nb6.nb6_regular_force_noalloc(ctx, 0, n_big, t, f * 1e-4, f * 0.0,
                                           nb6.NB6_DX_LOCAL, o3, o3, t, lst, 1023,
                                           torch.cuda.current_stream())
        assert rc == nb6.NB6_ERR_ARG
        assert b"scratch" in nb6.lib().nb6_last_error(ctx)
    finally:
        nb6.nb6_destroy(ctx)
