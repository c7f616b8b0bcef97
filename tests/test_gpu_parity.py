"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Bars (see the design notes for their derivation):
* neighbour lists: exact, except pairs within 1e-6 (relative) of the
  neighbour radius, which may fall on either side;
* FF, FP64 and local coordinate modes: per-particle force and jerk errors scaled by
  the sum of term magnitudes <= 1e-6; relative to the net value <= 1e-6
  wherever the net acceleration is at least 1e-3 of its scale and the net
  jerk at least 0.1 of its scale (below that, FP32 rounding of the individual
  terms, about 1e-7 of the scale, can exceed 1e-6 of the net value);
* FP32 coordinate mode (the paper's plain single precision): scaled errors
  <= 1e-4, list mismatches reported.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle.compare import compare  # noqa: E402
from workloads import config, make_cluster  # noqa: E402

MODES = {"ff": 1, "fp64": 2, "fp32": 4, "local": 8}
TOL_SCALED = {"ff": 1e-6, "fp64": 1e-6, "fp32": 1e-4, "local": 1e-6}
TOL_REL = {"ff": 1e-6, "fp64": 1e-6, "fp32": None, "local": 1e-6}
# File that collects one JSON line per parity case (unset: printed only).
OUT = os.environ.get("NB6_PARITY_LOG")


def _nb6():
    from paper_1205_1222_amd import nb6
    return nb6


@pytest.fixture(scope="module")
def ctx():
    nb6 = _nb6()
    c = nb6.nb6_create(0)
    yield c
    nb6.nb6_destroy(c)


def _record(name, summary):
    if OUT:
        os.makedirs(os.path.dirname(os.path.abspath(OUT)), exist_ok=True)
        with open(OUT, "a") as f:
            f.write(json.dumps({"case": name, **summary}) + "\n")
    print(name, json.dumps(summary), flush=True)


def load(ctx, cl, cluster=0):
    nb6 = _nb6()
    nb6.check(ctx, nb6.nb6_load_particles(ctx, cluster, cl.n, cl.m, cl.x, cl.v, cl.a,
                                          cl.jerk, cl.t))
    nb6.check(ctx, nb6.nb6_predict_j(ctx, cluster, cl.tb, 0))


def oracle_ref(cl, idx, lcap=4096):
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    ref = oracle.regular_force(cl.m, xp, vp, idx, cl.h2[idx], cl.dtr[idx], lcap=lcap)
    return xp, vp, ref


def check_mode(ctx, cl, idx, mode, name, cap=512, ref=None, cluster=0):
    nb6 = _nb6()
    if ref is None:
        ref = oracle_ref(cl, idx)
    xp, vp, r = ref
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, cluster, idx, cl.h2[idx],
                                                     cl.dtr[idx], MODES[mode], cap)
    c = compare(acc, jerk, nnb, lst, cap, r, cl.m, xp, vp, idx, cl.h2[idx], cl.dtr[idx])
    s = c.summary()
    s["mode"] = mode
    s["slices"] = nb6.nb6_last_slices(ctx)
    _record(name, s)
    assert c.incomplete == 0
    if mode != "fp32":
        assert c.list_mismatch == 0, c.mismatches[:10]
        assert c.nnb_mismatch == 0
    else:
        assert c.list_mismatch <= max(1, len(idx) // 100), c.mismatches[:10]
    assert s["acc_scaled_max"] <= TOL_SCALED[mode], s
    assert s["jerk_scaled_max"] <= TOL_SCALED[mode], s
    if TOL_REL[mode] is not None:
        assert s.get("acc_rel_max", 0.0) <= TOL_REL[mode], s
        assert s.get("jerk_rel_max", 0.0) <= TOL_REL[mode], s
    return acc, jerk, nnb, lst


# ---------------------------------------------------------------------------
def test_predict_matches_oracle(ctx):
    nb6 = _nb6()
    cl = config(2, n=4096)["cluster"]
    load(ctx, cl)
    xo, vo = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    for mode, tol_x in (("fp64", 1e-15), ("ff", 1e-14), ("fp32", 2.0 ** -23),
                        ("local", 1e-14)):
        x = np.empty((cl.n, 3))
        v = np.empty((cl.n, 3))
        nb6.check(ctx, nb6.nb6_get_predicted(ctx, 0, MODES[mode], x, v))
        scale = np.abs(cl.x) + np.abs(cl.v) + np.abs(cl.a) + np.abs(cl.jerk) + 1e-300
        ex = np.max(np.abs(x - xo) / scale)
        ev = np.max(np.abs(v - vo) / (np.abs(vo) + 1e-300))
        print(mode, "predict", ex, ev, flush=True)
        assert ex <= tol_x, (mode, ex)
        assert ev <= 2.0 ** -24, (mode, ev)


@pytest.mark.parametrize("mode", ["ff", "fp64", "fp32", "local"])
def test_config1_all_active(ctx, mode):
    cfg = config(1)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["all"]
    load(ctx, cl)
    check_mode(ctx, cl, idx, mode, f"C1_all_{mode}")


@pytest.mark.parametrize("mode", ["ff", "fp64", "local"])
def test_config2_random_block(ctx, mode):
    cfg = config(2)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["random1024"]
    load(ctx, cl)
    check_mode(ctx, cl, idx, mode, f"C2_random1024_{mode}")


@pytest.mark.parametrize("mode,offset", [("ff", (3.0, -2.0, 1.5)),
                                         ("ff", (1000.0, -500.0, 250.0)),
                                         ("fp64", (1000.0, -500.0, 250.0)),
                                         ("local", (3.0, -2.0, 1.5)),
                                         ("local", (1000.0, -500.0, 250.0))])
def test_offset_cluster(ctx, mode, offset):
    """A cluster far from the coordinate origin keeps the FF, FP64 and local
    bars: each cancels the large coordinates in full precision (the local
    mode against FP64 tile centres).  Differences of FP32 positions (the high
    parts alone) would be off by ~3e-5 of the force at the larger offset."""
    import dataclasses
    base = make_cluster(4096, 91, masses="imf", k_nb=32)
    cl = dataclasses.replace(base, x=base.x + np.array(offset))
    load(ctx, cl)
    idx = np.arange(0, cl.n, 3, dtype=np.int32)
    check_mode(ctx, cl, idx, mode, f"offset{int(offset[0])}_{mode}")


def test_ragged_sizes_and_slicings(ctx):
    nb6 = _nb6()
    cl = make_cluster(1003, 77, masses="imf", k_nb=20)
    load(ctx, cl)
    rng = np.random.Generator(np.random.PCG64(3))
    results = {}
    for ni in (1, 63, 65, 130, 1003):
        idx = np.sort(rng.choice(cl.n, ni, replace=False)).astype(np.int32)
        ref = oracle_ref(cl, idx)
        check_mode(ctx, cl, idx, "ff", f"ragged_n{ni}", ref=ref)
        check_mode(ctx, cl, idx, "local", f"ragged_n{ni}_local", ref=ref)
        results[ni] = (idx, ref)
    # force many slices (wavefront finalize) and a single slice
    for hint in (1, 3, 40):
        c2 = nb6.nb6_create(0, slice_hint=hint)
        try:
            load(c2, cl)
            idx, ref = results[130]
            check_mode(c2, cl, idx, "ff", f"ragged_hint{hint}", ref=ref)
            check_mode(c2, cl, idx, "local", f"ragged_hint{hint}_local", ref=ref)
            assert nb6.nb6_last_slices(c2) == min(hint, (cl.n + 255) // 256)
        finally:
            nb6.nb6_destroy(c2)


def test_lanes_per_i(ctx):
    """Small blocks give each i several lanes (j split across an i's lanes,
    butterfly sum at the end): automatic plans for blocks of 1..300 and
    forced lane counts on a ragged block and ragged slices."""
    nb6 = _nb6()
    cfg = config(2)
    cl = cfg["cluster"]
    load(ctx, cl)
    rng = np.random.Generator(np.random.PCG64(11))
    for ni in (1, 2, 3, 5, 31, 64, 100, 200, 300):
        idx = np.sort(rng.choice(cl.n, ni, replace=False)).astype(np.int32)
        ref = oracle_ref(cl, idx)
        check_mode(ctx, cl, idx, "ff", f"lanes_auto_n{ni}", ref=ref)
        check_mode(ctx, cl, idx, "local", f"lanes_auto_n{ni}_local", ref=ref)
        ipl, lanes, slices, slen = nb6.nb6_last_plan(ctx)
        print("plan", ni, ipl, lanes, slices, slen, flush=True)
        assert ipl == 1
        # up to 1024 i take 32, 16 or 8 lanes (by cluster size) where one
        # lane per i at 256-j slices would give fewer than 8 waves per CU
        import torch
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        thin = -(-ni // 64) * max(1, -(-cl.n // 256)) < 8 * cus
        mid = 32 if cl.n <= 2048 else 16 if cl.n <= 8192 else 8
        assert lanes == (64 if ni <= 64 else 16 if ni <= 128 else 8 if ni <= 256
                         else mid if ni <= 1024 and thin else 1)
        # each lane takes at least 32 j of a slice (16 for blocks of at most
        # 8 groups, whose few waves are latency-bound; the blocks of more than
        # 256 have slices of at least 256 j)
        groups = -(-ni // (64 // lanes))
        min_len = 256 if ni > 256 else (16 if groups <= 8 else 32) * lanes
        assert slen >= min(min_len, cl.n) and slices * slen >= cl.n
    idx = np.sort(rng.choice(cl.n, 3, replace=False)).astype(np.int32)
    for mode in ("fp64", "fp32"):
        check_mode(ctx, cl, idx, mode, f"lanes_auto_n3_{mode}")
    idx = np.sort(rng.choice(cl.n, 130, replace=False)).astype(np.int32)
    ref = oracle_ref(cl, idx)
    for jl, hint in ((2, 0), (16, 3), (64, 0), (64, 7)):
        c2 = nb6.nb6_create(0, jl_hint=jl, slice_hint=hint)
        try:
            load(c2, cl)
            check_mode(c2, cl, idx, "ff", f"lanes_forced{jl}_s{hint}", ref=ref)
            check_mode(c2, cl, idx, "local", f"lanes_forced{jl}_s{hint}_local", ref=ref)
            assert nb6.nb6_last_plan(c2)[1] == jl
            if jl == 16:  # staged through LDS: 48-byte and 32-byte records too
                for mode in ("fp64", "fp32"):
                    check_mode(c2, cl, idx, mode, f"lanes_forced{jl}_s{hint}_{mode}", ref=ref)
        finally:
            nb6.nb6_destroy(c2)
    for bad in ({"jl_hint": 3}, {"jl_hint": 128}, {"jl_hint": 4, "ipl_hint": 2}):
        with pytest.raises(nb6.NB6Error):
            nb6.nb6_create(0, **bad)


def test_neighbour_overflow_and_cap(ctx):
    nb6 = _nb6()
    cfg = config(1)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["all"][:200]
    load(ctx, cl)
    _, _, ref = oracle_ref(cl, idx)
    full = check_mode(ctx, cl, idx, "ff", "cap_full")
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                     1, cap=3)
    assert rc == nb6.NB6_WARN_NB_OVERFLOW
    np.testing.assert_array_equal(nnb, full[2])
    for q in range(len(idx)):
        k = min(3, nnb[q])
        np.testing.assert_array_equal(lst[q, :k], full[3][q, :k])
    np.testing.assert_array_equal(acc, full[0])
    acc0, jerk0, nnb0, _, rc0 = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                       1, cap=0)
    np.testing.assert_array_equal(nnb0, full[2])
    np.testing.assert_array_equal(acc0, full[0])


def test_device_mode_matches_host_mode(ctx):
    import torch
    nb6 = _nb6()
    cfg = config(1)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["all"]
    load(ctx, cl)
    acc_h, jerk_h, nnb_h, lst_h, _ = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx],
                                                            cl.dtr[idx], 1, 128)
    dev = torch.device("cuda:0")
    ni = len(idx)
    t_idx = torch.from_numpy(idx).to(dev)
    t_h2 = torch.from_numpy(cl.h2[idx].copy()).to(dev)
    t_dtr = torch.from_numpy(cl.dtr[idx].copy()).to(dev)
    acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    jerk = torch.empty_like(acc)
    nnb = torch.empty(ni, dtype=torch.int32, device=dev)
    lst = torch.empty((ni, 128), dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream()
    rc = nb6.nb6_regular_force(ctx, 0, ni, t_idx, t_h2, t_dtr, 1, acc, jerk, nnb, lst, 128,
                               nb6.NB6_MEM_DEVICE, s)
    nb6.check(ctx, rc)
    nb6.check(ctx, nb6.nb6_sync_status(ctx, s))
    np.testing.assert_array_equal(acc.cpu().numpy(), acc_h)
    np.testing.assert_array_equal(jerk.cpu().numpy(), jerk_h)
    np.testing.assert_array_equal(nnb.cpu().numpy(), nnb_h)
    l = lst.cpu().numpy()
    for q in range(ni):
        k = min(128, nnb_h[q])
        np.testing.assert_array_equal(l[q, :k], lst_h[q, :k])


def test_errors(ctx):
    import torch
    nb6 = _nb6()
    cfg = config(1)
    cl = cfg["cluster"]
    load(ctx, cl)
    idx = np.array([0, 5, 9], np.int32)
    h2 = cl.h2[idx].copy()
    dtr = cl.dtr[idx].copy()
    out = [np.empty((3, 3)), np.empty((3, 3)), np.empty(3, np.int32), np.empty((3, 8), np.int32)]
    bad = idx.copy()
    bad[1] = cl.n
    assert nb6.nb6_regular_force(ctx, 0, 3, bad, h2, dtr, 1, *out, 8) == nb6.NB6_ERR_ARG
    h2b = h2.copy()
    h2b[2] = 0.0
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2b, dtr, 1, *out, 8) == nb6.NB6_ERR_ARG
    # the criterion's time offset is forward: a negative or non-finite dtr is refused
    for bad_dtr in (-2.0 ** -8, np.nan, np.inf):
        dtrb = dtr.copy()
        dtrb[1] = bad_dtr
        assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtrb, 1, *out, 8) == nb6.NB6_ERR_ARG
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtr, 3, *out, 8) == nb6.NB6_ERR_ARG
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtr, 1, *out, -1) == nb6.NB6_ERR_ARG
    assert nb6.nb6_regular_force(ctx, 7, 3, idx, h2, dtr, 1, *out, 8) == nb6.NB6_ERR_STATE
    # FF predicted to a later block time -> the FP64 stream (still at the
    # earlier one) is refused; predicted to that time too, it is usable
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb + 2.0 ** -10, nb6.NB6_DX_FF))
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtr, 2, *out, 8) == nb6.NB6_ERR_STATE
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb + 2.0 ** -10, nb6.NB6_DX_FP64))
    usable = (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW)
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtr, 2, *out, 8) in usable
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtr, 1, *out, 8) in usable
    # a load invalidates the prediction
    load(ctx, cl)
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, 2, cl.m[:2], cl.x[:2], cl.v[:2], cl.a[:2],
                                          cl.jerk[:2], cl.t[:2], np.array([0, 1], np.int32)))
    assert nb6.nb6_regular_force(ctx, 0, 3, idx, h2, dtr, 1, *out, 8) == nb6.NB6_ERR_STATE
    # non-finite host state is refused
    xb = cl.x.copy()
    xb[4, 1] = np.nan
    assert nb6.nb6_load_particles(ctx, 1, cl.n, cl.m, xb, cl.v, cl.a, cl.jerk,
                                  cl.t) == nb6.NB6_ERR_ARG
    # device-side validation: bad index and bad h2 become NaN rows + status
    load(ctx, cl)
    dev = torch.device("cuda:0")
    t_idx = torch.tensor([0, cl.n + 5, 9], dtype=torch.int32, device=dev)
    t_h2 = torch.tensor([h2[0], h2[1], -1.0], dtype=torch.float64, device=dev)
    t_dtr = torch.tensor(dtr, dtype=torch.float64, device=dev)
    acc = torch.empty((3, 3), dtype=torch.float64, device=dev)
    jerk = torch.empty_like(acc)
    nnb = torch.empty(3, dtype=torch.int32, device=dev)
    lst = torch.empty((3, 8), dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream()
    nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, 3, t_idx, t_h2, t_dtr, 1, acc, jerk, nnb,
                                         lst, 8, nb6.NB6_MEM_DEVICE, s))
    assert nb6.nb6_sync_status(ctx, s) == nb6.NB6_ERR_DEVICE_INPUT
    assert nb6.nb6_sync_status(ctx, s) == nb6.NB6_OK  # cleared
    a = acc.cpu().numpy()
    assert np.all(np.isfinite(a[0])) and np.all(np.isnan(a[1])) and np.all(np.isnan(a[2]))
    assert list(nnb.cpu().numpy()[1:]) == [-1, -1]
    # a negative or NaN dtr found on the device: NaN rows, nnb = -1, status
    t_idx = torch.tensor(idx, dtype=torch.int32, device=dev)
    t_h2 = torch.tensor(h2, dtype=torch.float64, device=dev)
    t_dtr = torch.tensor([dtr[0], -dtr[1], np.nan], dtype=torch.float64, device=dev)
    nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, 3, t_idx, t_h2, t_dtr, 1, acc, jerk, nnb,
                                         lst, 8, nb6.NB6_MEM_DEVICE, s))
    assert nb6.nb6_sync_status(ctx, s) == nb6.NB6_ERR_DEVICE_INPUT
    a = acc.cpu().numpy()
    assert np.all(np.isfinite(a[0])) and np.all(np.isnan(a[1])) and np.all(np.isnan(a[2]))
    assert list(nnb.cpu().numpy()[1:]) == [-1, -1]


def test_empty_blocks(ctx):
    """n_i == 0 is a no-op for every block call, with NULL arrays, in both
    memory kinds; the context computes normally afterwards."""
    nb6 = _nb6()
    cl = make_cluster(512, 41, masses="equal", k_nb=16)
    load(ctx, cl)
    params = (0.02, 2.0 ** -20, 1.0, 0.5, 2.0)
    nulls = {name: None for name, _ in nb6.nb6_corr_block._fields_[2:]}
    for mk in (nb6.NB6_MEM_HOST, nb6.NB6_MEM_DEVICE):
        assert nb6.nb6_regular_force(ctx, 0, 0, None, None, None, MODES["ff"], None, None,
                                     None, None, 0, mk) == nb6.NB6_OK
        assert nb6.nb6_set_lists(ctx, 0, 0, None, None, None, 8, mk) == nb6.NB6_OK
        assert nb6.nb6_irregular_force(ctx, 0, cl.tb, 0, None, None, None, mk) == nb6.NB6_OK
        assert nb6.nb6_regular_correct(ctx, 0, 1.0, nulls, params, mk) == nb6.NB6_OK
    idx = np.arange(0, cl.n, 4, dtype=np.int32)
    check_mode(ctx, cl, idx, "ff", "after_empty_blocks")


def test_subset_update_then_predict(ctx):
    nb6 = _nb6()
    cfg = config(2, n=4096)
    cl = cfg["cluster"]
    load(ctx, cl)
    rng = np.random.Generator(np.random.PCG64(9))
    upd = np.sort(rng.choice(cl.n, 300, replace=False)).astype(np.int32)
    cl.x[upd] += rng.normal(0, 1e-3, (300, 3))
    cl.v[upd] *= 1.01
    cl.t[upd] = cl.tb - 2.0 ** -10
    nb6.check(ctx, nb6.nb6_load_particles(
        ctx, 0, len(upd), np.ascontiguousarray(cl.m[upd]), np.ascontiguousarray(cl.x[upd]),
        np.ascontiguousarray(cl.v[upd]), np.ascontiguousarray(cl.a[upd]),
        np.ascontiguousarray(cl.jerk[upd]), np.ascontiguousarray(cl.t[upd]), upd))
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, 0))
    idx = np.sort(rng.choice(cl.n, 512, replace=False)).astype(np.int32)
    check_mode(ctx, cl, idx, "fp64", "subset_update")


def test_repeat_calls_are_bitwise_identical(ctx):
    nb6 = _nb6()
    cfg = config(2)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["random1024"]
    load(ctx, cl)
    a = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx], 1, 256)
    b = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx], 1, 256)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("block,mode", [("all", "ff"), ("pow2_0", "ff"), ("pow2_4", "ff"),
                                        ("pow2_10", "ff"), ("pow2_14", "ff"),
                                        ("all", "fp64"), ("pow2_10", "fp64"),
                                        ("all", "fp32"), ("pow2_10", "fp32"),
                                        ("all", "local"), ("pow2_0", "local"),
                                        ("pow2_4", "local"), ("pow2_10", "local"),
                                        ("pow2_14", "local")])
def test_config3_full_size_sampled(ctx, block, mode):
    """N = 131072 with binaries, in the launch configuration the benchmark
    times; the oracle checks a sample of the active i, with each coordinate
    mode's bars."""
    nb6 = _nb6()
    cfg = config(3)
    cl = cfg["cluster"]
    idx = cfg["blocks"][block]
    load(ctx, cl)
    cap = 256
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                     MODES[mode], cap)
    rng = np.random.Generator(np.random.PCG64(5))
    samp = np.sort(rng.choice(len(idx), min(256, len(idx)), replace=False))
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    si = idx[samp]
    ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
    c = compare(acc[samp], jerk[samp], nnb[samp], lst[samp], cap, ref, cl.m, xp, vp, si,
                cl.h2[si], cl.dtr[si])
    s = c.summary()
    s["slices"] = nb6.nb6_last_slices(ctx)
    _record(f"C3_{block}_{mode}", s)
    assert c.incomplete == 0
    if mode == "fp32":
        assert c.list_mismatch <= max(1, len(samp) // 100), c.mismatches[:10]
    else:
        assert c.list_mismatch == 0 and c.nnb_mismatch == 0, c.mismatches[:10]
    tol = TOL_SCALED[mode]
    assert s["acc_scaled_max"] <= tol and s["jerk_scaled_max"] <= tol, s
    if TOL_REL[mode] is not None:
        assert s.get("acc_rel_max", 0.0) <= TOL_REL[mode], s
        assert s.get("jerk_rel_max", 0.0) <= TOL_REL[mode], s


def test_config3_two_i_per_lane_sampled():
    """The two-i-per-lane kernel on all 131072 particles of C3 (its plan at
    full size), sampled against the oracle with the FF bars."""
    nb6 = _nb6()
    c2 = nb6.nb6_create(0, ipl_hint=2)
    try:
        cfg = config(3)
        cl = cfg["cluster"]
        idx = cfg["blocks"]["all"]
        load(c2, cl)
        cap = 256
        acc, jerk, nnb, lst, rc = nb6.regular_force_host(c2, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                         MODES["ff"], cap)
        assert nb6.nb6_last_plan(c2)[0] == 2
        rng = np.random.Generator(np.random.PCG64(6))
        samp = np.sort(rng.choice(len(idx), 256, replace=False))
        xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
        si = idx[samp]
        ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
        c = compare(acc[samp], jerk[samp], nnb[samp], lst[samp], cap, ref, cl.m, xp, vp, si,
                    cl.h2[si], cl.dtr[si])
        s = c.summary()
        _record("C3_all_ff_ipl2", s)
        assert c.incomplete == 0 and c.list_mismatch == 0 and c.nnb_mismatch == 0
        assert s["acc_scaled_max"] <= 1e-6 and s["jerk_scaled_max"] <= 1e-6, s
        assert s.get("acc_rel_max", 0.0) <= 1e-6 and s.get("jerk_rel_max", 0.0) <= 1e-6, s
    finally:
        nb6.nb6_destroy(c2)


@pytest.mark.parametrize("mode", ["ff", "fp64", "fp32", "local"])
@pytest.mark.parametrize("block", ["random4096", "all"])
def test_config5_full_size_sampled(ctx, block, mode):
    """N = 2^20, ~100 neighbours, in every coordinate mode, in the launch
    configuration the benchmark times; the oracle checks 256 sampled i."""
    nb6 = _nb6()
    cfg = config(5)
    cl = cfg["cluster"]
    idx = cfg["blocks"][block]
    load(ctx, cl)
    cap = 256
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                     MODES[mode], cap)
    rng = np.random.Generator(np.random.PCG64(6))
    samp = np.sort(rng.choice(len(idx), 256, replace=False))
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    si = idx[samp]
    ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
    c = compare(acc[samp], jerk[samp], nnb[samp], lst[samp], cap, ref, cl.m, xp, vp, si,
                cl.h2[si], cl.dtr[si])
    s = c.summary()
    s["slices"] = nb6.nb6_last_slices(ctx)
    _record(f"C5_{block}_{mode}", s)
    del acc, jerk, nnb, lst
    assert c.incomplete == 0
    if mode != "fp32":
        assert c.list_mismatch == 0 and c.nnb_mismatch == 0, c.mismatches[:10]
    else:
        assert c.list_mismatch <= len(si) // 100, c.mismatches[:10]
    assert s["acc_scaled_max"] <= TOL_SCALED[mode] and s["jerk_scaled_max"] <= TOL_SCALED[mode], s
    if TOL_REL[mode] is not None:
        assert s.get("acc_rel_max", 0.0) <= TOL_REL[mode], s
        assert s.get("jerk_rel_max", 0.0) <= TOL_REL[mode], s


@pytest.mark.parametrize("mode", ["ff", "fp64", "fp32", "local"])
def test_potential(ctx, mode):
    """The optional regular potential (-sum m/r over the non-neighbours) against
    the oracle, on a one-lane-per-i block, a small lanes-per-i block and C3's
    binaries; asking for it leaves acc, jerk and the lists bit-identical."""
    nb6 = _nb6()
    tol = {"ff": 1e-6, "fp64": 1e-6, "fp32": 1e-5, "local": 1e-6}[mode]
    cases = [(config(2)["cluster"], config(2)["blocks"]["random1024"]),
             (config(2)["cluster"], config(2)["blocks"]["random1024"][:37])]
    if mode in ("ff", "local"):
        c3 = config(3)
        cases.append((c3["cluster"], c3["blocks"]["pow2_12"]))
    for cl, idx in cases:
        load(ctx, cl)
        a0, j0, n0, l0, _ = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                   MODES[mode], 256)
        a1, j1, n1, l1, _, pot = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                        MODES[mode], 256, with_pot=True)
        assert np.array_equal(a0, a1) and np.array_equal(j0, j1) and np.array_equal(n0, n1)
        for q in range(len(idx)):
            k = min(n0[q], 256)
            assert np.array_equal(l0[q, :k], l1[q, :k])
        rng = np.random.Generator(np.random.PCG64(13))
        samp = np.sort(rng.choice(len(idx), min(128, len(idx)), replace=False))
        xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
        si = idx[samp]
        ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
        ok = n0[samp] == ref.nnb  # boundary pairs move a term between the two sums
        rel = np.abs(pot[samp] - ref.pot) / np.abs(ref.pot)
        print(mode, len(idx), "pot rel err max %.3g" % rel[ok].max(), flush=True)
        assert ok.mean() > 0.98 and rel[ok].max() <= tol, rel[ok].max()


@pytest.mark.parametrize("mode", ["ff", "local"])
@pytest.mark.parametrize("n", [1024, 1500])
def test_everything_neighbour_long_lists(ctx, n, mode):
    """h -> infinity: every j is a neighbour.  N = 1024 fills the largest list
    exactly (1023 entries, sorted on the GPU); N = 1500 overflows it and the
    ordered overflow scan must return the first 1023 indices (in the local
    mode it visits the particles through their slots in the spatial order).
    Four i (64 lanes per i) and 300 i (32 lanes per i, and one lane per i)."""
    nb6 = _nb6()
    cl = make_cluster(n, 31, masses="equal", k_nb=8)
    load(ctx, cl)
    idx = np.array([0, 7, n // 2, n - 1], np.int32)
    cap = nb6.NB6_MAX_CAP
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, 1e30, cl.dtr[idx],
                                                     MODES[mode], cap)
    assert np.all(acc == 0.0) and np.all(jerk == 0.0)
    assert np.all(nnb == n - 1)
    assert rc == (nb6.NB6_OK if n - 1 <= cap else nb6.NB6_WARN_NB_OVERFLOW)
    for q, i in enumerate(idx):
        want = [j for j in range(n) if j != i][:cap]
        np.testing.assert_array_equal(lst[q, :min(cap, n - 1)], want)
    # 300 i: 32 lanes per i (a cluster this small), then one lane per i
    # (forced): every work item finds more neighbours per lane than the
    # lane's staged run holds, so full runs, the per-neighbour reservations
    # past them and the flushes between tiles all take part
    idx = np.sort(np.random.Generator(np.random.PCG64(5)).choice(n, 300, replace=False))
    idx = idx.astype(np.int32)
    one = nb6.nb6_create(0, jl_hint=1)
    try:
        load(one, cl)
        for c, lanes in ((ctx, 32), (one, 1)):
            acc, jerk, nnb, lst, rc = nb6.regular_force_host(c, 0, idx, 1e30, cl.dtr[idx],
                                                             MODES[mode], cap)
            assert nb6.nb6_last_plan(c)[1] == lanes
            assert np.all(acc == 0.0) and np.all(jerk == 0.0)
            assert np.all(nnb == n - 1)
            for q, i in enumerate(idx):
                want = np.delete(np.arange(n), i)[:cap]
                np.testing.assert_array_equal(lst[q, :min(cap, n - 1)], want)
    finally:
        nb6.nb6_destroy(one)
    with pytest.raises(Exception):
        nb6.regular_force_host(ctx, 0, idx, 1e30, cl.dtr[idx], MODES[mode], cap + 1)


@pytest.mark.parametrize("mode", ["ff", "fp64", "fp32", "local"])
def test_overflow_rescan_every_mode(ctx, mode):
    """A list capacity below the neighbour count: the finalize rebuilds such a
    list by an ordered rescan in the call's own coordinate mode, which must
    give the first cap entries of the full list and the true count."""
    nb6 = _nb6()
    cfg = config(1)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["all"][:300]
    load(ctx, cl)
    full = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx], MODES[mode], 256)
    assert full[4] == nb6.NB6_OK
    for cap in (1, 5):
        acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                         MODES[mode], cap)
        assert rc == nb6.NB6_WARN_NB_OVERFLOW
        assert np.any(full[2] > cap)
        np.testing.assert_array_equal(nnb, full[2])
        np.testing.assert_array_equal(acc, full[0])
        np.testing.assert_array_equal(jerk, full[1])
        for q in range(len(idx)):
            k = min(cap, nnb[q])
            np.testing.assert_array_equal(lst[q, :k], full[3][q, :k])


def test_counts_reset_between_calls(ctx):
    """The per-i neighbour counters are zeroed once and reset by every call's
    finalize: calls of growing and shrinking size, with overflowing and
    complete lists, on one context give the same bits as on fresh contexts."""
    nb6 = _nb6()
    cfg = config(1)
    cl = cfg["cluster"]
    order = cfg["blocks"]["all"]
    load(ctx, cl)
    plan = [(1, 64), (300, 2), (64, 64), (1024, 64), (5, 0), (1024, 3), (700, 64)]
    got = []
    for ni, cap in plan:
        idx = order[:ni]
        got.append(nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx], 1, cap))
    for (ni, cap), g in zip(plan, got):
        fresh = nb6.nb6_create(0)
        try:
            load(fresh, cl)
            idx = order[:ni]
            w = nb6.regular_force_host(fresh, 0, idx, cl.h2[idx], cl.dtr[idx], 1, cap)
        finally:
            nb6.nb6_destroy(fresh)
        for a, b in zip(g[:3], w[:3]):
            np.testing.assert_array_equal(a, b)
        for q in range(ni):  # slots past a row's count are not written
            k = min(cap, g[2][q])
            np.testing.assert_array_equal(g[3][q, :k], w[3][q, :k])
        assert g[4] == w[4]


def test_tiny_clusters_and_repeated_indices(ctx):
    """Degenerate inputs: a one-particle cluster (no j other than i: zero force,
    empty list), a two-body pair against its closed form, and an active block
    that names the same particle more than once (independent, identical
    rows)."""
    from workloads.clusters import Cluster
    nb6 = _nb6()
    z3 = np.zeros((1, 3))
    one = Cluster(m=np.array([0.5]), x=np.array([[0.3, -0.2, 0.1]]), v=np.array([[0.1, 0, 0]]),
                  a=z3, jerk=z3, t=np.zeros(1), tb=0.0, h2=np.array([0.01]),
                  dtr=np.array([0.0]))
    for mode in MODES.values():
        load(ctx, one)
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, one.tb, mode))
        acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, np.zeros(1, np.int32),
                                                         one.h2, one.dtr, mode, 4)
        assert rc == nb6.NB6_OK
        assert np.all(acc == 0.0) and np.all(jerk == 0.0) and nnb[0] == 0
    # two bodies 1.5 apart with radius 0.1: each feels the other's full force
    m = np.array([0.25, 0.75])
    x = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0]])
    v = np.array([[0.0, 0.1, 0.0], [0.0, -0.2, 0.05]])
    two = Cluster(m=m, x=x, v=v, a=np.zeros((2, 3)), jerk=np.zeros((2, 3)), t=np.zeros(2),
                  tb=0.0, h2=np.full(2, 0.01), dtr=np.zeros(2))
    load(ctx, two)
    R = x[1] - x[0]
    V = v[1] - v[0]
    r = np.linalg.norm(R)
    want_a = m[1] * R / r ** 3
    want_j = m[1] * (V / r ** 3 - 3.0 * np.dot(R, V) * R / r ** 5)
    for name, mode in MODES.items():
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, two.tb, mode))
        acc, jerk, nnb, lst, rc = nb6.regular_force_host(
            ctx, 0, np.array([0, 1], np.int32), two.h2, two.dtr, mode, 4)
        assert np.all(nnb == 0)
        tol = 1e-6 if name != "fp32" else 1e-5
        np.testing.assert_allclose(acc[0], want_a, rtol=tol, atol=tol * np.abs(want_a).max())
        np.testing.assert_allclose(jerk[0], want_j, rtol=tol, atol=tol * np.abs(want_j).max())
        np.testing.assert_allclose(m[0] * acc[0], -m[1] * acc[1], rtol=tol)
    # the same particle several times in one block
    cfg = config(1)
    cl = cfg["cluster"]
    load(ctx, cl)
    idx = np.array([5, 900, 5, 0, 900, 5, 1023], np.int32)
    xp, vp, ref = oracle_ref(cl, idx)
    acc, jerk, nnb, lst = check_mode(ctx, cl, idx, "ff", "repeated_indices", ref=(xp, vp, ref))
    for a_, b_ in ((0, 2), (0, 5), (1, 4)):
        np.testing.assert_array_equal(acc[a_], acc[b_])
        np.testing.assert_array_equal(jerk[a_], jerk[b_])
        assert nnb[a_] == nnb[b_]
        np.testing.assert_array_equal(lst[a_, :nnb[a_]], lst[b_, :nnb[b_]])


@pytest.mark.parametrize("mode", ["ff", "fp64", "fp32", "local"])
def test_two_i_per_lane(mode):
    """The two-i-per-lane force kernel (a context option; the default plan
    takes one): oracle parity on a ragged random block and a whole cluster,
    and the same bits as one i per lane under the same slicing."""
    nb6 = _nb6()
    cfg = config(2)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["random1024"][:1000]
    ref = oracle_ref(cl, idx)
    got = {}
    for ipl in (2, 1):
        # one lane per i forced: this block in this cluster would otherwise
        # take lanes per i
        c = nb6.nb6_create(0, ipl_hint=ipl, slice_hint=24, jl_hint=1 if ipl == 1 else 0)
        try:
            load(c, cl)
            got[ipl] = check_mode(c, cl, idx, mode, f"ipl{ipl}_C2_{mode}", ref=ref)
            assert nb6.nb6_last_plan(c)[0] == ipl
        finally:
            nb6.nb6_destroy(c)
    for a, b in zip(got[1][:3], got[2][:3]):
        np.testing.assert_array_equal(a, b)
    c = nb6.nb6_create(0, ipl_hint=2)
    try:
        cfg1 = config(1)
        cl1 = cfg1["cluster"]
        load(c, cl1)
        check_mode(c, cl1, cfg1["blocks"]["all"], mode, f"ipl2_C1_{mode}")
    finally:
        nb6.nb6_destroy(c)


def test_nonfinite_device_state_is_reported(ctx):
    """A non-finite coordinate loaded from device arrays (no host check) is
    caught by the predictor: nb6_sync_status reports NB6_ERR_DEVICE_INPUT
    once, and a clean reload makes the cluster usable again."""
    import torch
    nb6 = _nb6()
    cfg = config(1)
    cl = cfg["cluster"]
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    xb = cl.x.copy()
    xb[4, 1] = np.nan
    s = torch.cuda.current_stream()
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, cl.n, T(cl.m), T(xb), T(cl.v), T(cl.a),
                                          T(cl.jerk), T(cl.t), mem_kind=nb6.NB6_MEM_DEVICE,
                                          stream=s))
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, 0, s))
    assert nb6.nb6_sync_status(ctx, s) == nb6.NB6_ERR_DEVICE_INPUT
    assert nb6.nb6_sync_status(ctx, s) == nb6.NB6_OK
    load(ctx, cl)
    idx = cfg["blocks"]["all"][:64]
    check_mode(ctx, cl, idx, "ff", "reload_after_nonfinite")


def test_local_order_follows_the_state(ctx):
    """The local stream's spatial order is built from the stored state at a
    full load and rebuilt once subset updates have touched as many particles
    as the cluster holds.  Corrector-sized moves of a quarter of the cluster
    per step keep the bars while the order ages; the fourth update triggers
    the rebuild, after which the results are bit-identical to a fresh context
    that full-loads the same state."""
    import dataclasses
    nb6 = _nb6()
    base = config(2, n=4096)["cluster"]
    cl = dataclasses.replace(base, x=base.x.copy(), v=base.v.copy(), t=base.t.copy())
    load(ctx, cl)
    rng = np.random.Generator(np.random.PCG64(21))
    idx = np.sort(rng.choice(cl.n, 512, replace=False)).astype(np.int32)
    check_mode(ctx, cl, idx, "local", "order_fresh")
    perm = rng.permutation(cl.n)
    for step in range(4):
        upd = np.sort(perm[step * 1024:(step + 1) * 1024]).astype(np.int32)
        # the stored state of a block after its step: drifted by v dt
        cl.x[upd] += cl.v[upd] * 2.0 ** -7
        cl.t[upd] = cl.tb
        nb6.check(ctx, nb6.nb6_load_particles(
            ctx, 0, len(upd), np.ascontiguousarray(cl.m[upd]), np.ascontiguousarray(cl.x[upd]),
            np.ascontiguousarray(cl.v[upd]), np.ascontiguousarray(cl.a[upd]),
            np.ascontiguousarray(cl.jerk[upd]), np.ascontiguousarray(cl.t[upd]), upd))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, nb6.NB6_DX_LOCAL))
        got = check_mode(ctx, cl, idx, "local", f"order_step{step}")
    fresh = nb6.nb6_create(0)
    try:
        load(fresh, cl)
        want = nb6.regular_force_host(fresh, 0, idx, cl.h2[idx], cl.dtr[idx], MODES["local"],
                                      512)
    finally:
        nb6.nb6_destroy(fresh)
    for a, b in zip(got[:3], want[:3]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("mode", ["ff", "fp64", "fp32", "local"])
def test_momentum_conservation_c1(ctx, mode):
    """C1 with a uniform neighbour radius and dtr = 0: the partition is then
    symmetric (j lists i whenever i lists j), so the regular forces are
    pairwise antisymmetric and sum m_i acc_i and sum m_i jerk_i vanish in
    exact arithmetic.  On the GPU output both stay below 1e-6 of
    sum m_i |acc_i| (and of sum m_i |jerk_i|); the lists come out symmetric."""
    import dataclasses
    nb6 = _nb6()
    cfg = config(1)
    base = cfg["cluster"]
    h2 = float(np.median(base.h2))
    cl = dataclasses.replace(base, h2=np.full(base.n, h2), dtr=np.zeros(base.n))
    idx = cfg["blocks"]["all"]
    load(ctx, cl)
    cap = 512
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                     MODES[mode], cap)
    assert rc == nb6.NB6_OK
    nbrs = [set(lst[q, :nnb[q]].tolist()) for q in range(cl.n)]
    assert all(q in nbrs[j] for q in range(cl.n) for j in nbrs[q])
    m = cl.m[:, None]
    pa = np.linalg.norm((m * acc).sum(0)) / np.abs(m * np.linalg.norm(acc, axis=1)[:, None]).sum()
    pj = np.linalg.norm((m * jerk).sum(0)) / np.abs(m * np.linalg.norm(jerk, axis=1)[:, None]).sum()
    _record(f"momentum_C1_{mode}", {"acc": float(pa), "jerk": float(pj)})
    assert pa <= 1e-6 and pj <= 1e-6, (pa, pj)


@pytest.mark.parametrize("mode", ["ff", "local"])
def test_spatial_i_order_changes_no_bits(mode):
    """A block of at least 8192 particles that holds three quarters of its
    cluster runs in the cluster's spatial order of its particles; a context
    with NB6_OPT_CALLER_ORDER runs the same call in the caller's order.  Every
    output is the same bits (with repeated particles in the block, and with an
    index out of range, which both flag and both give a NaN row), and the
    results match the oracle on sampled rows."""
    import torch
    nb6 = _nb6()
    cl = make_cluster(10000, 41, masses="imf", k_nb=30)
    rng = np.random.Generator(np.random.PCG64(17))
    idx = rng.permutation(cl.n)[:9000]
    idx = np.concatenate([idx, idx[:300]])  # 300 particles twice
    rng.shuffle(idx)
    idx = idx.astype(np.int32)
    assert len(idx) >= 8192 and 4 * len(idx) >= 3 * cl.n
    cap = 128
    outs = []
    for flags in (0, nb6.NB6_OPT_CALLER_ORDER):
        c = nb6.nb6_create(0, flags=flags)
        try:
            load(c, cl)
            outs.append(nb6.regular_force_host(c, 0, idx, cl.h2[idx], cl.dtr[idx], MODES[mode],
                                               cap))
            assert nb6.nb6_last_plan(c)[1] == 1
        finally:
            nb6.nb6_destroy(c)
    (a0, j0, n0, l0, r0), (a1, j1, n1, l1, r1) = outs
    assert r0 == r1
    # with the potential: its sums through the i-order as well
    pots = []
    for flags in (0, nb6.NB6_OPT_CALLER_ORDER):
        c = nb6.nb6_create(0, flags=flags)
        try:
            load(c, cl)
            res_p = nb6.regular_force_host(c, 0, idx, cl.h2[idx], cl.dtr[idx], MODES[mode], cap,
                                           with_pot=True)
            np.testing.assert_array_equal(res_p[0], a0)
            pots.append(res_p[5])
        finally:
            nb6.nb6_destroy(c)
    np.testing.assert_array_equal(pots[0], pots[1])
    assert np.all(np.isfinite(pots[0])) and np.all(pots[0] < 0.0)
    np.testing.assert_array_equal(a0, a1)
    np.testing.assert_array_equal(j0, j1)
    np.testing.assert_array_equal(n0, n1)
    k = np.minimum(n0, cap)
    for q in range(len(idx)):
        np.testing.assert_array_equal(l0[q, :k[q]], l1[q, :k[q]])
    # repeated particles: identical rows
    first = {}
    for q, p in enumerate(idx):
        if p in first:
            np.testing.assert_array_equal(a0[q], a0[first[p]])
            assert n0[q] == n0[first[p]]
        else:
            first[p] = q
    samp = np.sort(rng.choice(len(idx), 256, replace=False))
    si = idx[samp]
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
    cmp_ = compare(a0[samp], j0[samp], n0[samp], l0[samp], cap, ref, cl.m, xp, vp, si,
                   cl.h2[si], cl.dtr[si])
    s = cmp_.summary()
    _record(f"iorder_{mode}", s)
    assert cmp_.list_mismatch == 0 and cmp_.nnb_mismatch == 0, s
    assert s["acc_scaled_max"] <= 1e-6 and s["jerk_scaled_max"] <= 1e-6, s
    # an index out of range (device arrays: no host check) in the block
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    bad = idx.copy()
    bad[4321] = cl.n
    st = torch.cuda.current_stream()
    res = []
    for flags in (0, nb6.NB6_OPT_CALLER_ORDER):
        c = nb6.nb6_create(0, flags=flags)
        try:
            load(c, cl)
            acc = torch.empty((len(bad), 3), dtype=torch.float64, device=dev)
            jerk = torch.empty_like(acc)
            nnb = torch.empty(len(bad), dtype=torch.int32, device=dev)
            lst = torch.empty((len(bad), cap), dtype=torch.int32, device=dev)
            h2 = cl.h2[np.minimum(bad, cl.n - 1)]
            dtr = cl.dtr[np.minimum(bad, cl.n - 1)]
            nb6.check(c, nb6.nb6_regular_force(c, 0, len(bad), T(bad, torch.int32), T(h2), T(dtr),
                                               MODES[mode], acc, jerk, nnb, lst, cap,
                                               nb6.NB6_MEM_DEVICE, st))
            assert nb6.nb6_sync_status(c, st) == nb6.NB6_ERR_DEVICE_INPUT
            res.append((acc.cpu().numpy(), nnb.cpu().numpy()))
        finally:
            nb6.nb6_destroy(c)
    assert np.all(np.isnan(res[0][0][4321])) and res[0][1][4321] == -1
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])
    ok = np.arange(len(bad)) != 4321
    np.testing.assert_array_equal(res[0][0][ok], a0[ok])
