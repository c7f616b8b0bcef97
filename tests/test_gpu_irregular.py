"""GPU tests of the irregular force over stored neighbour lists (section 3.3
step 4) through the C ABI: nb6_set_lists + nb6_irregular_force against the
FP64 oracle, the regular/irregular partition end to end, list storage
semantics and argument errors.

The kernel computes in FP64, so the bar is far below the regular force's:
per-particle errors scaled by the sum of term magnitudes <= 1e-10 (the only
differences are the rounding of the two predictors and of the sums).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import config, make_cluster  # noqa: E402

TOL = 1e-10


def _nb6():
    from paper_1205_1222_amd import nb6
    return nb6


@pytest.fixture(scope="module")
def ctx():
    nb6 = _nb6()
    c = nb6.nb6_create(0)
    yield c
    nb6.nb6_destroy(c)


def load(ctx, cl, cluster=0, predict=True):
    nb6 = _nb6()
    nb6.check(ctx, nb6.nb6_load_particles(ctx, cluster, cl.n, cl.m, cl.x, cl.v, cl.a,
                                          cl.jerk, cl.t))
    if predict:
        nb6.check(ctx, nb6.nb6_predict_j(ctx, cluster, cl.tb, 0))


def check_irr(acc, jerk, ref, name):
    ea = np.linalg.norm(acc - ref.acc, axis=1) / np.where(ref.sa > 0, ref.sa, 1.0)
    ej = np.linalg.norm(jerk - ref.jerk, axis=1) / np.where(ref.sj > 0, ref.sj, 1.0)
    print(name, "irregular scaled err acc %.3g jerk %.3g" % (ea.max(), ej.max()), flush=True)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(jerk))
    assert ea.max() <= TOL and ej.max() <= TOL, (name, ea.max(), ej.max())
    zero = ref.sa == 0
    assert np.all(acc[zero] == 0) and np.all(jerk[zero] == 0)


def regular_lists(ctx, cl, idx, cap=512):
    nb6 = _nb6()
    acc, jerk, nnb, lst, rc = nb6.regular_force_host(ctx, 0, idx, cl.h2[idx], cl.dtr[idx],
                                                     nb6.NB6_DX_FF, cap)
    assert rc == nb6.NB6_OK and nnb.max() <= cap
    return acc, jerk, nnb, lst


@pytest.mark.parametrize("cfg_id", [1, 2])
def test_irregular_matches_oracle(ctx, cfg_id):
    nb6 = _nb6()
    cfg = config(cfg_id)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["all" if cfg_id == 1 else "random1024"]
    load(ctx, cl)
    _, _, nnb, lst = regular_lists(ctx, cl, idx)
    nb6.set_lists_host(ctx, 0, idx, nnb, lst)
    acc, jerk, pot = nb6.irregular_force_host(ctx, 0, cl.tb, idx, with_pot=True)
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    lists = [lst[q, :nnb[q]] for q in range(len(idx))]
    ref = oracle.irregular_force(cl.m, xp, vp, idx, lists)
    check_irr(acc, jerk, ref, f"C{cfg_id}")
    has = ref.pot != 0
    assert np.all(pot[~has] == 0)
    assert np.max(np.abs(pot[has] - ref.pot[has]) / np.abs(ref.pot[has])) <= TOL
    acc0, jerk0 = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    assert np.array_equal(acc0, acc) and np.array_equal(jerk0, jerk)
    # another block time: the library predicts every needed particle itself
    tb2 = cl.tb + 2.0 ** -10
    acc2, jerk2 = nb6.irregular_force_host(ctx, 0, tb2, idx)
    xp2, vp2 = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, tb2)
    check_irr(acc2, jerk2, oracle.irregular_force(cl.m, xp2, vp2, idx, lists), f"C{cfg_id}_t2")
    assert not np.array_equal(acc, acc2)


def test_regular_plus_irregular_is_the_full_force(ctx):
    """Section 3.3: the regular force over non-neighbours plus the irregular
    force over the list is the force of every other particle."""
    nb6 = _nb6()
    cl = make_cluster(2048, 41, masses="imf", k_nb=40)
    idx = np.arange(0, cl.n, 2, dtype=np.int32)
    load(ctx, cl)
    racc, rjerk, nnb, lst = regular_lists(ctx, cl, idx)
    nb6.set_lists_host(ctx, 0, idx, nnb, lst)
    iacc, ijerk = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    full = oracle.regular_force(cl.m, xp, vp, idx, 1e-300, 0.0, lcap=4)
    ea = np.linalg.norm(racc + iacc - full.acc, axis=1) / full.sa
    ej = np.linalg.norm(rjerk + ijerk - full.jerk, axis=1) / full.sj
    print("partition scaled err", ea.max(), ej.max(), flush=True)
    assert ea.max() <= 1e-6 and ej.max() <= 1e-6


def test_potential_energy(ctx):
    """W = (1/2) sum m_i (phi_reg,i + phi_irr,i) over a whole cluster from the
    GPU's two potentials, against the oracle's full potential: the energy
    check of section 4 (it quotes 1e-8 for the GPU's potential; here the
    FP32 regular sum, compensated by the FP64 tile folds)."""
    nb6 = _nb6()
    cl = make_cluster(4096, 53, masses="imf", k_nb=40)
    idx = np.arange(cl.n, dtype=np.int32)
    load(ctx, cl)
    _, _, nnb, lst, _, preg = nb6.regular_force_host(ctx, 0, idx, cl.h2, cl.dtr,
                                                     nb6.NB6_DX_FF, 512, with_pot=True)
    assert nnb.max() <= 512
    nb6.set_lists_host(ctx, 0, idx, nnb, lst)
    _, _, pirr = nb6.irregular_force_host(ctx, 0, cl.tb, idx, with_pot=True)
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    full = oracle.regular_force(cl.m, xp, vp, idx, 1e-300, 0.0, lcap=4)
    w_gpu = 0.5 * np.sum(cl.m * (preg + pirr))
    w_ref = 0.5 * np.sum(cl.m * full.pot)
    print("W gpu %.15g oracle %.15g rel %.3g" % (w_gpu, w_ref, abs(w_gpu / w_ref - 1)), flush=True)
    assert abs(w_gpu / w_ref - 1.0) <= 1e-7
    per = np.abs(preg + pirr - full.pot) / np.abs(full.pot)
    assert per.max() <= 1e-6, per.max()


def test_config3_full_size_device_chain(ctx):
    """N = 131072 with binaries, all active: the regular force's device
    outputs go straight into nb6_set_lists, then the irregular force of all
    particles; a sample is checked against the oracle."""
    import torch
    nb6 = _nb6()
    cfg = config(3)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["all"]
    ni = len(idx)
    load(ctx, cl)
    dev = torch.device("cuda:0")
    cap = 256
    T = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    d_idx, d_h2, d_dtr = T(idx, torch.int32), T(cl.h2[idx]), T(cl.dtr[idx])
    racc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    rjerk = torch.empty_like(racc)
    nnb = torch.empty(ni, dtype=torch.int32, device=dev)
    lst = torch.empty((ni, cap), dtype=torch.int32, device=dev)
    iacc = torch.empty_like(racc)
    ijerk = torch.empty_like(racc)
    st = torch.cuda.current_stream()
    nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, ni, d_idx, d_h2, d_dtr, nb6.NB6_DX_FF, racc,
                                         rjerk, nnb, lst, cap, nb6.NB6_MEM_DEVICE, st))
    nb6.check(ctx, nb6.nb6_set_lists(ctx, 0, ni, d_idx, nnb, lst, cap, nb6.NB6_MEM_DEVICE, st))
    nb6.check(ctx, nb6.nb6_irregular_force(ctx, 0, cl.tb, ni, d_idx, iacc, ijerk,
                                           nb6.NB6_MEM_DEVICE, st))
    nb6.check(ctx, nb6.nb6_sync_status(ctx, st))
    nnb_h = nnb.cpu().numpy()
    assert nnb_h.max() <= cap
    rng = np.random.Generator(np.random.PCG64(8))
    samp = np.sort(rng.choice(ni, 512, replace=False))
    lst_h = lst.cpu().numpy()
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    lists = [lst_h[q, :nnb_h[q]] for q in samp]
    ref = oracle.irregular_force(cl.m, xp, vp, idx[samp], lists)
    check_irr(iacc.cpu().numpy()[samp], ijerk.cpu().numpy()[samp], ref, "C3_all")
    # the binaries' pairs are neighbours: their irregular force is large
    assert np.median(ref.sa) > 0


def test_config5_random_block(ctx):
    """N = 2^20, a block of 4096 random active particles (~100 neighbours
    each): lists from the regular force, stored, then the irregular force;
    a sample is checked against the oracle."""
    nb6 = _nb6()
    cfg = config(5)
    cl = cfg["cluster"]
    idx = cfg["blocks"]["random4096"]
    load(ctx, cl)
    _, _, nnb, lst = regular_lists(ctx, cl, idx, cap=512)
    nb6.set_lists_host(ctx, 0, idx, nnb, lst)
    acc, jerk = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    rng = np.random.Generator(np.random.PCG64(9))
    samp = np.sort(rng.choice(len(idx), 256, replace=False))
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    ref = oracle.irregular_force(cl.m, xp, vp, idx[samp], [lst[q, :nnb[q]] for q in samp])
    check_irr(acc[samp], jerk[samp], ref, "C5_random4096")
    assert np.median(nnb) > 50


def test_list_semantics(ctx):
    nb6 = _nb6()
    cl = make_cluster(500, 43, masses="imf", k_nb=10)
    load(ctx, cl, predict=False)
    n = cl.n
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.arange(0, n, 5, dtype=np.int32)
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    # never set: every list is empty
    acc, jerk = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    assert np.all(acc == 0) and np.all(jerk == 0)
    # unsorted lists with the particle itself and a repeated entry, cap 8
    lists = []
    for i in idx:
        others = rng.choice(np.delete(np.arange(n), i), 5, replace=False)
        lists.append(np.concatenate([others, [i], others[:1]]).astype(np.int32))
    rows = np.zeros((len(idx), 8), np.int32)
    for q, l in enumerate(lists):
        rows[q, :len(l)] = l
    nb6.set_lists_host(ctx, 0, idx, [len(l) for l in lists], rows)
    acc, jerk = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    check_irr(acc, jerk, oracle.irregular_force(cl.m, xp, vp, idx, lists), "semantics")
    # growing the rows keeps the stored lists; a repeated active i is fine
    other = np.array([1, 2, 3], np.int32)
    long_rows = np.tile(np.arange(100, 164, dtype=np.int32), (3, 1))
    nb6.set_lists_host(ctx, 0, other, [64, 10, 0], long_rows)
    both = np.concatenate([idx, other, idx[:2]]).astype(np.int32)
    all_lists = lists + [long_rows[0, :64], long_rows[1, :10], long_rows[2, :0]] + lists[:2]
    acc, jerk = nb6.irregular_force_host(ctx, 0, cl.tb, both)
    check_irr(acc, jerk, oracle.irregular_force(cl.m, xp, vp, both, all_lists), "grown")
    assert np.array_equal(acc[:2], acc[-2:])
    # repeat calls give the same bits
    acc2, jerk2 = nb6.irregular_force_host(ctx, 0, cl.tb, both)
    assert np.array_equal(acc, acc2) and np.array_equal(jerk, jerk2)
    # a full reload empties every list
    load(ctx, cl, predict=False)
    acc, _ = nb6.irregular_force_host(ctx, 0, cl.tb, both)
    assert np.all(acc == 0)


def test_errors(ctx):
    import torch
    nb6 = _nb6()
    cl = make_cluster(300, 47, masses="equal", k_nb=8)
    load(ctx, cl, predict=False)
    n = cl.n
    idx = np.array([0, 1], np.int32)
    rows = np.array([[2, 3], [4, 5]], np.int32)
    A = lambda *a: np.ascontiguousarray(np.array(*a), np.int32)  # noqa: E731

    def set_rc(i, k, r, cap=2):
        return nb6.nb6_set_lists(ctx, 0, len(i), A(i), A(k), A(r), cap)
    assert set_rc([0, n], [2, 2], rows) == nb6.NB6_ERR_ARG          # particle out of range
    assert set_rc([0, 0], [2, 2], rows) == nb6.NB6_ERR_ARG          # listed twice
    assert set_rc([0, 1], [3, 2], rows) == nb6.NB6_ERR_ARG          # count above cap
    assert set_rc([0, 1], [2, 2], [[2, n], [4, 5]]) == nb6.NB6_ERR_ARG  # entry out of range
    assert set_rc([0, 1], [2, 2], rows, cap=0) == nb6.NB6_ERR_ARG
    assert set_rc([0, 1], [2, 2], rows, cap=nb6.NB6_MAX_LIST_CAP + 1) == nb6.NB6_ERR_ARG
    assert nb6.nb6_set_lists(ctx, 9, 2, idx, A([2, 2]), rows, 2) == nb6.NB6_ERR_STATE
    acc = np.empty((2, 3))
    jerk = np.empty((2, 3))
    assert nb6.nb6_irregular_force(ctx, 0, cl.tb, 2, A([0, n]), acc, jerk) == nb6.NB6_ERR_ARG
    assert nb6.nb6_irregular_force(ctx, 0, float("nan"), 2, idx, acc, jerk) == nb6.NB6_ERR_ARG
    assert nb6.nb6_irregular_force(ctx, 3, cl.tb, 2, idx, acc, jerk) == nb6.NB6_ERR_STATE
    # DEVICE mode: an invalid entry is flagged and that list is stored empty
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    d_idx = torch.tensor([0, 1], dtype=torch.int32, device=dev)
    d_cnt = torch.tensor([2, 2], dtype=torch.int32, device=dev)
    d_rows = torch.tensor([[2, 3], [4, n + 7]], dtype=torch.int32, device=dev)
    nb6.check(ctx, nb6.nb6_set_lists(ctx, 0, 2, d_idx, d_cnt, d_rows, 2, nb6.NB6_MEM_DEVICE, st))
    assert nb6.nb6_sync_status(ctx, st) == nb6.NB6_ERR_DEVICE_INPUT
    acc, jerk = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    assert np.any(acc[0] != 0) and np.all(acc[1] == 0)
    # DEVICE mode: an out-of-range active particle gives a NaN row
    d_bad = torch.tensor([0, n], dtype=torch.int32, device=dev)
    out = torch.empty((2, 3), dtype=torch.float64, device=dev)
    out2 = torch.empty_like(out)
    nb6.check(ctx, nb6.nb6_irregular_force(ctx, 0, cl.tb, 2, d_bad, out, out2,
                                           nb6.NB6_MEM_DEVICE, st))
    assert nb6.nb6_sync_status(ctx, st) == nb6.NB6_ERR_DEVICE_INPUT
    o = out.cpu().numpy()
    assert np.all(np.isfinite(o[0])) and np.all(np.isnan(o[1]))


def test_large_host_lists_packed(ctx):
    """Lists above 1 MB go up packed from host arrays (rows cut to their
    counts, put back in place on the GPU): the irregular force over them
    equals the one over the same lists set from device arrays, and the
    oracle's; the regular call's host-array lists come back packed too and
    equal its device-array lists."""
    import torch
    nb6 = _nb6()
    cfg = config(2)
    cl = cfg["cluster"]
    idx = np.arange(cl.n, dtype=np.int32)[:12000]
    load(ctx, cl)
    cap = 256
    _, _, nnb, lst = regular_lists(ctx, cl, idx, cap=cap)
    assert len(idx) * cap * 4 > (1 << 20)
    d_idx = torch.from_numpy(idx).to("cuda:0")
    d_out = (torch.empty((len(idx), 3), dtype=torch.float64, device="cuda:0"),
             torch.empty((len(idx), 3), dtype=torch.float64, device="cuda:0"),
             torch.empty(len(idx), dtype=torch.int32, device="cuda:0"),
             torch.empty((len(idx), cap), dtype=torch.int32, device="cuda:0"))
    nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, len(idx), d_idx,
                                         torch.from_numpy(cl.h2[idx]).to("cuda:0"),
                                         torch.from_numpy(cl.dtr[idx]).to("cuda:0"),
                                         nb6.NB6_DX_FF, *d_out, cap, nb6.NB6_MEM_DEVICE))
    torch.cuda.synchronize()
    d_nnb = d_out[2].cpu().numpy()
    d_lst = d_out[3].cpu().numpy()
    np.testing.assert_array_equal(d_nnb, nnb)
    for q in range(len(idx)):
        np.testing.assert_array_equal(d_lst[q, :nnb[q]], lst[q, :nnb[q]])
    # lists set from host arrays (packed) and from device arrays
    nb6.set_lists_host(ctx, 0, idx, nnb, lst)
    acc_h, jerk_h = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    nb6.check(ctx, nb6.nb6_set_lists(ctx, 0, len(idx), d_idx, d_out[2], d_out[3], cap,
                                     nb6.NB6_MEM_DEVICE))
    torch.cuda.synchronize()
    nb6.check(ctx, nb6.nb6_sync_status(ctx))
    acc_d, jerk_d = nb6.irregular_force_host(ctx, 0, cl.tb, idx)
    np.testing.assert_array_equal(acc_h, acc_d)
    np.testing.assert_array_equal(jerk_h, jerk_d)
    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    sub = np.arange(0, len(idx), 97)
    ref = oracle.irregular_force(cl.m, xp, vp, idx[sub], [lst[q, :nnb[q]] for q in sub])
    check_irr(acc_h[sub], jerk_h[sub], ref, "packed_lists")
