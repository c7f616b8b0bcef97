"""GPU tests of the regular corrector of a block (nb6_regular_correct)
through the C ABI: the elementwise FP64 kernel against the oracle (the same
IEEE operations in the same order, so bit-identical except the cube root of
equation (1): the GPU's math library and the host's differ there by a few
units in the last place, 8 ulp of h_new allowed), a whole regular step built
from the library's own force calls, and argument errors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import config  # noqa: E402

PAR = dict(eta=0.02, dt_min=2.0 ** -20, dt_max=2.0 ** -2, f_lo=0.5, f_hi=1.25)


def _nb6():
    from paper_1205_1222_amd import nb6
    return nb6


@pytest.fixture(scope="module")
def ctx():
    nb6 = _nb6()
    c = nb6.nb6_create(0)
    yield c
    nb6.nb6_destroy(c)


def _compare(out, ref, name):
    for k in ("df", "dfd", "f2", "f3", "dt_new"):
        assert np.array_equal(out[k], getattr(ref, k)), (name, k)
    ulp = np.abs(out["h_new"] - ref.h_new) / np.spacing(ref.h_new)
    assert ulp.max() <= 8, (name, ulp.max())


def test_corrector_matches_oracle(ctx):
    nb6 = _nb6()
    rng = np.random.default_rng(61)
    n = 5000
    t = 0.75
    h = 2.0 ** -rng.integers(3, 12, n)
    t_old = t - h
    vec = lambda s: rng.normal(scale=s, size=(n, 3))  # noqa: E731
    f_old, fd_old = vec(1.0), vec(5.0)
    f_new = f_old + fd_old * h[:, None] + vec(1e-2)
    fd_new = fd_old + vec(0.5)
    g_old, gd_old = vec(10.0), vec(50.0)
    g_new = g_old + vec(1e-3)
    gd_new = gd_old + vec(1e-2)
    h_old = rng.uniform(0.01, 0.1, n)
    nnb = rng.integers(0, 120, n).astype(np.int32)
    n_p = rng.uniform(20, 80, n)
    args = (t, t_old, f_old, fd_old, f_new, fd_new, g_old, gd_old, g_new, gd_new, h_old, nnb,
            n_p)
    out = nb6.regular_correct_host(ctx, *args, **PAR)
    ref = oracle.regular_correct(*args, **PAR)
    _compare(out, ref, "random")
    print("dt_new values", np.unique(out["dt_new"]).size, flush=True)
    assert np.unique(out["dt_new"]).size > 3


def test_corrector_on_a_regular_step(ctx):
    """One regular step of a block of C2 built from the library's own calls:
    the regular force at t_old with the old radii, at t with new radii (new
    lists), the irregular force at t with the old and the new list.  The
    corrector's dF is the regular-force change over the old neighbour set,
    which the oracle gives as (full force - irregular over the old list) at t
    minus the regular force at t_old."""
    import torch  # noqa: F401
    nb6 = _nb6()
    cfg = config(2)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["random1024"][:300]
    ni = len(idx)
    t_old = cl.tb
    t = cl.tb + 2.0 ** -9
    h_old = np.sqrt(cl.h2[idx])
    h_new = h_old * 1.1
    dtr = cl.dtr[idx]
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, cl.n, cl.m, cl.x, cl.v, cl.a, cl.jerk,
                                          cl.t))
    cap = 512
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, t_old, nb6.NB6_DX_FF))
    f_old, fd_old, nnb_old, l_old, _ = nb6.regular_force_host(ctx, 0, idx, h_old ** 2, dtr,
                                                              nb6.NB6_DX_FF, cap)
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, t, nb6.NB6_DX_FF))
    f_new, fd_new, nnb_new, l_new, _ = nb6.regular_force_host(ctx, 0, idx, h_new ** 2, dtr,
                                                              nb6.NB6_DX_FF, cap)
    assert nnb_old.max() <= cap and nnb_new.max() <= cap
    assert np.any(nnb_new != nnb_old)
    nb6.set_lists_host(ctx, 0, idx, nnb_old, l_old)
    g_old, gd_old = nb6.irregular_force_host(ctx, 0, t, idx)
    nb6.set_lists_host(ctx, 0, idx, nnb_new, l_new)
    g_new, gd_new = nb6.irregular_force_host(ctx, 0, t, idx)
    args = (t, np.full(ni, t_old), f_old, fd_old, f_new, fd_new, g_old, gd_old, g_new, gd_new,
            h_old, nnb_new, 50.0)
    out = nb6.regular_correct_host(ctx, *args, **PAR)
    _compare(out, oracle.regular_correct(*args, **PAR), "step")
    # the fixed-list change, from the oracle
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, t)
    full = oracle.regular_force(cl.m, xp, vp, idx, 1e-300, 0.0, lcap=4)
    irr_old = oracle.irregular_force(cl.m, xp, vp, idx, [l_old[q, :nnb_old[q]] for q in range(ni)])
    xo, vo = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, t_old)
    reg_old = oracle.regular_force(cl.m, xo, vo, idx, h_old ** 2, dtr, lcap=4096)
    want = (full.acc - irr_old.acc) - reg_old.acc
    scale = full.sa
    err = np.linalg.norm(out["df"] - want, axis=1) / scale
    print("dF scaled error max %.3g" % err.max(), flush=True)
    assert err.max() <= 2e-6
    assert np.all(out["h_new"] > 0) and np.all(out["dt_new"] <= 2 * 2.0 ** -9)


def test_corrector_errors(ctx):
    import torch
    nb6 = _nb6()
    z = np.zeros((2, 3))
    good = (1.0, [0.5, 0.75], z, z, z, z, z, z, z, z, [0.1, 0.1], [10, 10], [10.0, 10.0])
    for bad in (dict(PAR, eta=0.0), dict(PAR, dt_min=3e-6), dict(PAR, dt_max=0.3),
                dict(PAR, dt_min=1.0, dt_max=0.5), dict(PAR, f_lo=0.0),
                dict(PAR, f_lo=2.0, f_hi=1.0)):
        with pytest.raises(nb6.NB6Error):
            nb6.regular_correct_host(ctx, *good, **bad)
    with pytest.raises(nb6.NB6Error):  # t_old not before t (HOST: refused)
        nb6.regular_correct_host(ctx, 1.0, [0.5, 1.0], *good[2:], **PAR)
    # DEVICE: the bad particle gets NaN and the status reports it
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    T = lambda a, dt=torch.float64: torch.as_tensor(np.asarray(a), dtype=dt, device=dev)  # noqa: E731
    arrays = {"t_old": T([0.5, 1.0])}
    for k in ("f_old", "fd_old", "f_new", "fd_new", "g_old", "gd_old", "g_new", "gd_new"):
        arrays[k] = T(np.ones((2, 3)))
    arrays.update(h_old=T([0.1, 0.1]), n_p=T([10.0, 10.0]), nnb=T([10, 10], torch.int32))
    for k in ("df", "dfd", "f2", "f3"):
        arrays[k] = torch.empty((2, 3), dtype=torch.float64, device=dev)
    arrays.update(dt_new=torch.empty(2, dtype=torch.float64, device=dev),
                  h_new=torch.empty(2, dtype=torch.float64, device=dev))
    params = (PAR["eta"], PAR["dt_min"], PAR["dt_max"], PAR["f_lo"], PAR["f_hi"])
    nb6.check(ctx, nb6.nb6_regular_correct(ctx, 2, 1.0, arrays, params, nb6.NB6_MEM_DEVICE, st))
    assert nb6.nb6_sync_status(ctx, st) == nb6.NB6_ERR_DEVICE_INPUT
    dt_new = arrays["dt_new"].cpu().numpy()
    assert np.isfinite(dt_new[0]) and np.isnan(dt_new[1])


def test_host_and_device_arrays_agree(ctx):
    """The corrector with host arrays (one pinned copy each way) and with
    device arrays gives the same bits, on a block large enough for several
    workgroups and a ragged tail."""
    import torch
    nb6 = _nb6()
    rng = np.random.default_rng(67)
    n = 70001
    t = 1.0
    h = 2.0 ** -rng.integers(3, 12, n)
    vec = lambda s: rng.normal(scale=s, size=(n, 3))  # noqa: E731
    arrays = {"t_old": t - h, "f_old": vec(1.0), "fd_old": vec(5.0), "f_new": vec(1.0),
              "fd_new": vec(5.0), "g_old": vec(10.0), "gd_old": vec(50.0), "g_new": vec(10.0),
              "gd_new": vec(50.0), "h_old": rng.uniform(0.01, 0.1, n),
              "nnb": rng.integers(0, 120, n).astype(np.int32), "n_p": rng.uniform(20, 80, n)}
    host = nb6.regular_correct_host(ctx, t, *[arrays[k] for k in (
        "t_old", "f_old", "fd_old", "f_new", "fd_new", "g_old", "gd_old", "g_new", "gd_new",
        "h_old", "nnb", "n_p")], **PAR)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0") for k, v in arrays.items()}
    for k in ("df", "dfd", "f2", "f3"):
        dev[k] = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
    for k in ("dt_new", "h_new"):
        dev[k] = torch.empty(n, dtype=torch.float64, device="cuda:0")
    par = (PAR["eta"], PAR["dt_min"], PAR["dt_max"], PAR["f_lo"], PAR["f_hi"])
    nb6.check(ctx, nb6.nb6_regular_correct(ctx, n, t, dev, par, nb6.NB6_MEM_DEVICE))
    torch.cuda.synchronize()
    nb6.check(ctx, nb6.nb6_sync_status(ctx))
    for k in ("df", "dfd", "f2", "f3", "dt_new", "h_new"):
        np.testing.assert_array_equal(host[k], dev[k].cpu().numpy(), err_msg=k)
