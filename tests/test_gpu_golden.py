"""The hand-derived closed-form cases of tests/golden/closed_forms.json (two-
and three-body forces and jerks, the tie rules and the velocity criterion of
section 3.2, the potential) through the GPU path, in every coordinate mode,
against the hand-derived values themselves rather than the oracle; and
coincident distinct particles (neighbours of each other whatever their
radius, never a force term).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from workloads.clusters import Cluster  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
MODES = {"ff": 1, "fp64": 2, "fp32": 4, "local": 8}
# scaled by the sum of the terms' magnitudes: FP32 arithmetic per term
TOL = {"ff": 1e-6, "fp64": 1e-6, "fp32": 1e-5, "local": 1e-6}


def _nb6():
    from paper_1205_1222_amd import nb6
    return nb6


@pytest.fixture(scope="module")
def ctx():
    nb6 = _nb6()
    c = nb6.nb6_create(0)
    yield c
    nb6.nb6_destroy(c)


def _run(ctx, m, x, v, active, h2, dtr, mode, cap=8):
    nb6 = _nb6()
    n = len(m)
    z = np.zeros((n, 3))
    cl = Cluster(m=np.asarray(m, float), x=np.asarray(x, float), v=np.asarray(v, float),
                 a=z, jerk=z, t=np.zeros(n), tb=0.0, h2=np.ones(n), dtr=np.zeros(n))
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, cl.m, cl.x, cl.v, cl.a, cl.jerk, cl.t))
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, 0.0, MODES[mode]))
    return nb6.regular_force_host(ctx, 0, np.asarray(active, np.int32), np.asarray(h2, float),
                                  np.asarray(dtr, float), MODES[mode], cap, with_pot=True)


def _scales(m, x, v, i, neighbours):
    """Sums of the term magnitudes of i's acceleration, jerk and potential."""
    sa = sj = sp = 0.0
    for j in range(len(m)):
        if j == i or j in neighbours:
            continue
        R = np.subtract(x[j], x[i])
        V = np.subtract(v[j], v[i])
        r = np.linalg.norm(R)
        sa += m[j] / r ** 2
        sj += m[j] * (np.linalg.norm(V) / r ** 3 + 3 * abs(np.dot(R, V)) / r ** 4)
        sp += m[j] / r
    return sa, sj, sp


@pytest.mark.parametrize("mode", sorted(MODES))
def test_closed_form_cases(ctx, mode):
    cases = json.load(open(GOLDEN))["force_cases"]
    for case in cases:
        acc, jerk, nnb, lst, rc, pot = _run(ctx, case["m"], case["x"], case["v"], case["active"],
                                            case["h2"], case["dtr"], mode)
        name = f"{case['name']}/{mode}"
        assert rc == _nb6().NB6_OK, name
        for q, i in enumerate(case["active"]):
            want_list = sorted(case["lists"][q])
            assert nnb[q] == len(want_list), (name, q, nnb[q])
            assert sorted(lst[q, :nnb[q]].tolist()) == want_list, name
            sa, sj, sp = _scales(case["m"], case["x"], case["v"], i, set(want_list))
            ea = np.max(np.abs(acc[q] - case["acc"][q])) / max(sa, 1e-300)
            # a case whose jerk was not worked out by hand says "skip"
            ej = 0.0 if case["jerk"] == "skip" else \
                np.max(np.abs(jerk[q] - case["jerk"][q])) / max(sj, 1e-300)
            ep = abs(pot[q] - case["pot"][q]) / max(sp, 1e-300)
            print(name, q, "scaled errors %.2g %.2g %.2g" % (ea, ej, ep), flush=True)
            assert ea <= TOL[mode] and ej <= TOL[mode] and ep <= TOL[mode], (name, q, ea, ej, ep)


@pytest.mark.parametrize("mode", sorted(MODES))
def test_coincident_particles(ctx, mode):
    """Particles 0 and 1 share a position (and differ in velocity): with any
    positive radius each is the other's neighbour, and particle 2, at
    distance 2, gives the only force term."""
    m = [0.25, 0.5, 1.0]
    x = [[0.5, -0.25, 1.0], [0.5, -0.25, 1.0], [2.5, -0.25, 1.0]]
    v = [[0.0, 0.0, 0.0], [0.125, 0.0, 0.0], [0.0, 0.0, 0.0]]
    acc, jerk, nnb, lst, rc, pot = _run(ctx, m, x, v, [0, 1], [1e-6, 1e-6], [0.0, 0.0], mode)
    assert list(nnb) == [1, 1]
    assert lst[0, 0] == 1 and lst[1, 0] == 0
    for q in range(2):
        np.testing.assert_allclose(acc[q], [1.0 / 4.0, 0.0, 0.0], rtol=TOL[mode])
        np.testing.assert_allclose(pot[q], -0.5, rtol=TOL[mode])
    np.testing.assert_allclose(jerk[0], [0.0, 0.0, 0.0], atol=1e-12)
    # particle 1 moves along +x towards 2: V = -0.125 x_hat, R.V = -0.25,
    # jerk = m (V / r^3 - 3 (R.V) R / r^5) = (-1/64 + 3/64, 0, 0)
    np.testing.assert_allclose(jerk[1], [2.0 / 64.0, 0.0, 0.0], rtol=TOL[mode])
