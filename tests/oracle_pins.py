"""Pins for the FP64 oracle: checks against facts the paper and mathematics fix.

(The irregular-force pins at the end tie that function to the hand-derived
golden values, to the pinned regular force through the partition of section
3.3, to Newton's third law and to a finite-difference jerk.)

Each ``pin_*`` function takes the ctypes handle of an oracle build (``None``
for the default build) and raises ``AssertionError`` when the oracle
disagrees with:

* hand-derived closed forms (``tests/golden/closed_forms.json``);
* exact rational arithmetic on tiny random inputs (neighbour decisions and
  the Taylor predictor);
* Newton's third law (momentum conservation under a symmetric criterion);
* a central finite difference of the acceleration along straight-line drift
  (pins the jerk);
* the smooth mean field of a Plummer sphere (pins sign, mass and distance
  powers of the full sum);
* the limits h -> infinity (everything is a neighbour) and the triangle
  inequality for the force scales.

The same functions run against deliberately broken builds of the oracle in
``test_oracle_mutants.py``, which shows that each plausible slip fails at
least one pin.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np

import oracle
from workloads import make_cluster

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _close(a, b, tol):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return np.all(np.abs(a - b) <= tol * (1.0 + np.abs(b)))


# --------------------------------------------------------------------------
def pin_golden_forces(lib=None):
    cases = json.load(open(GOLDEN))["force_cases"]
    for c in cases:
        m = np.array(c["m"], float)
        xp = np.array(c["x"], float)
        vp = np.array(c["v"], float)
        r = oracle.regular_force(m, xp, vp, c["active"], c["h2"], c["dtr"],
                                 lcap=16, lib=lib)
        assert _close(r.acc, c["acc"], 1e-14), (c["name"], r.acc, c["acc"])
        if c["jerk"] != "skip":
            assert _close(r.jerk, c["jerk"], 1e-14), (c["name"], r.jerk, c["jerk"])
        assert _close(r.pot, c["pot"], 1e-14), (c["name"], r.pot, c["pot"])
        assert _close(r.sa, c["sa"], 1e-14), (c["name"], r.sa, c["sa"])
        assert _close(r.sj, c["sj"], 1e-14), (c["name"], r.sj, c["sj"])
        got = [list(map(int, l)) for l in r.lists]
        assert got == c["lists"], (c["name"], got, c["lists"])
        assert list(map(int, r.nnb)) == [len(l) for l in c["lists"]], c["name"]


def pin_pair_terms_golden(lib=None):
    """Per-pair terms on the hand-derived two-body cases (pair i=0, j=1)."""
    cases = {c["name"]: c for c in json.load(open(GOLDEN))["force_cases"]}
    for name in ("two_body_static", "two_body_transverse_velocity",
                 "two_body_radial_velocity", "velocity_criterion_off"):
        c = cases[name]
        rmin, dacc, djrk = oracle.pair_terms([0], [1], [c["dtr"][0]], c["m"], c["x"], c["v"],
                                             lib=lib)
        assert _close(dacc[0], c["acc"][0], 1e-14), (name, dacc)
        assert _close(djrk[0], c["jerk"][0], 1e-14), (name, djrk)
        r = np.linalg.norm(np.subtract(c["x"][1], c["x"][0]))
        assert abs(rmin[0] - r) <= 1e-15 * r, (name, rmin)
    # the velocity criterion's end point: |R + dt V| = |3 - 3| = 0
    c = cases["velocity_criterion_catches_approach"]
    rmin, _, _ = oracle.pair_terms([0], [1], [c["dtr"][0]], c["m"], c["x"], c["v"], lib=lib)
    assert rmin[0] == 0.0


def pin_golden_predict(lib=None):
    cases = json.load(open(GOLDEN))["predict_cases"]
    for c in cases:
        xp, vp = oracle.predict(c["x"], c["v"], c["a"], c["jerk"], c["t"],
                                c["tb"], lib=lib)
        assert _close(xp, c["xp"], 1e-15), (c["name"], xp)
        assert _close(vp, c["vp"], 1e-15), (c["name"], vp)


# --------------------------------------------------------------------------
def _tiny_inputs(seed, n=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1.0, 1.0, (n, 3))
    v = rng.normal(0.0, 1.0, (n, 3))
    m = rng.uniform(0.5, 2.0, n) / n
    h2 = rng.uniform(0.05, 0.6, n) ** 2
    dtr = 2.0 ** -rng.integers(1, 5, n).astype(float)
    return m, x, v, h2, dtr


def pin_exact_rational_lists(lib=None):
    """Neighbour sets against exact rational arithmetic on the FP64 inputs."""
    for seed in (1, 2, 3):
        m, x, v, h2, dtr = _tiny_inputs(seed)
        n = len(m)
        idx = np.arange(n)
        r = oracle.regular_force(m, x, v, idx, h2, dtr, lcap=n, lib=lib)
        X = [[Fraction(float(c)) for c in row] for row in x]
        V = [[Fraction(float(c)) for c in row] for row in v]
        n_checked = 0
        for i in range(n):
            H2 = Fraction(float(h2[i]))
            D = Fraction(float(dtr[i]))
            want, tie = [], set()
            for j in range(n):
                if j == i:
                    continue
                R = [X[j][k] - X[i][k] for k in range(3)]
                W = [V[j][k] - V[i][k] for k in range(3)]
                P = [R[k] + D * W[k] for k in range(3)]
                r2 = sum(c * c for c in R)
                p2 = sum(c * c for c in P)
                q = min(r2, p2)
                if abs(q - H2) <= H2 * Fraction(1, 10 ** 12):
                    tie.add(j)
                if q < H2:
                    want.append(j)
            got = list(map(int, r.lists[i]))
            diff = set(got) ^ set(want)
            assert diff <= tie, (seed, i, sorted(diff))
            assert got == sorted(got)
            n_checked += len(want)
        assert n_checked > 0


def pin_exact_rational_predict(lib=None):
    rng = np.random.Generator(np.random.PCG64(7))
    n = 12
    x, v, a, j = (rng.normal(0, 1, (n, 3)) for _ in range(4))
    t = rng.uniform(0.0, 1.0, n)
    tb = 1.0 + 2.0 ** -7
    xp, vp = oracle.predict(x, v, a, j, t, tb, lib=lib)
    for k in range(n):
        dt = Fraction(tb) - Fraction(float(t[k]))
        for c in range(3):
            X, Vv, A, J = (Fraction(float(q[k, c])) for q in (x, v, a, j))
            ex = X + Vv * dt + A * dt ** 2 / 2 + J * dt ** 3 / 6
            ev = Vv + A * dt + J * dt ** 2 / 2
            sx = abs(X) + abs(Vv * dt) + abs(A * dt ** 2) + abs(J * dt ** 3)
            sv = abs(Vv) + abs(A * dt) + abs(J * dt ** 2)
            assert abs(Fraction(float(xp[k, c])) - ex) <= Fraction(1, 10 ** 15) * sx
            assert abs(Fraction(float(vp[k, c])) - ev) <= Fraction(1, 10 ** 15) * sv


# --------------------------------------------------------------------------
def pin_momentum(lib=None):
    """Uniform h and dt_reg = 0 make the criterion symmetric: sum m a = 0."""
    for masses in ("equal", "imf"):
        cl = make_cluster(512, 99, masses=masses, stored_state=False, k_nb=8)
        n = cl.n
        idx = np.arange(n)
        r = oracle.regular_force(cl.m, cl.x, cl.v, idx, 0.15 ** 2, 0.0,
                                 lcap=n, lib=lib)
        assert r.nnb.sum() > n  # the criterion removed some pairs
        for q in (r.acc, r.jerk):
            tot = (cl.m[:, None] * q).sum(0)
            scale = (cl.m * np.linalg.norm(q, axis=1)).sum()
            assert np.all(np.abs(tot) <= 1e-13 * scale), (masses, tot, scale)


def pin_fd_jerk(lib=None):
    """Jerk = d(acc)/dt along straight-line drift, by central difference."""
    cl = make_cluster(256, 5, masses="imf", stored_state=False, k_nb=8)
    n = cl.n
    idx = np.arange(n)
    z = np.zeros((n, 3))
    base = oracle.regular_force(cl.m, cl.x, cl.v, idx, 1e-30, 0.0, lcap=4, lib=lib)
    d = 1e-6
    xp, _ = oracle.predict(cl.x, cl.v, z, z, np.zeros(n), d, lib=lib)
    xm, _ = oracle.predict(cl.x, cl.v, z, z, np.zeros(n), -d, lib=lib)
    ap = oracle.regular_force(cl.m, xp, cl.v, idx, 1e-30, 0.0, lcap=4, lib=lib).acc
    am = oracle.regular_force(cl.m, xm, cl.v, idx, 1e-30, 0.0, lcap=4, lib=lib).acc
    fd = (ap - am) / (2 * d)
    err = np.linalg.norm(fd - base.jerk, axis=1) / base.sj
    assert err.max() < 1e-6, err.max()


def pin_plummer_mean_field(lib=None):
    """The regular force of a Plummer sphere follows its smooth mean field.

    With a fixed exclusion radius h and no velocity term, the excluded ball
    around each particle is nearly uniform, and a uniform ball exerts no
    force at its own centre; so the regular acceleration follows the Plummer
    field a(r) = -r (r^2 + b^2)^-3/2 (b = 3 pi/16, G = M = 1); the density
    gradient across the ball adds its pull (2 pi/3) h^2 grad rho, which is
    subtracted from the expectation.  The regular jerk holds the neighbour set fixed, so it
    is the tidal tensor of the mass *outside* the ball applied to the
    particle's velocity, plus a zero-mean term from the field particles'
    motion.  The ball's own tidal tensor is -(4 pi/3) rho I, hence
        J = (T_plummer + (4 pi/3) rho(r) I) v,
        T_plummer = -I/s^3 + 3 x x^T / s^5,  s^2 = r^2 + b^2,
        (4 pi/3) rho(r) = b^-3 (1 + r^2/b^2)^-5/2.
    """
    cl = make_cluster(16384, 11, masses="equal", stored_state=False, k_nb=8)
    n = cl.n
    idx = np.arange(n)
    r = oracle.regular_force(cl.m, cl.x, cl.v, idx, 0.06 ** 2, 0.0, lcap=4096, lib=lib)
    b = 3.0 * np.pi / 16.0
    x, v = cl.x, cl.v
    s2 = (x * x).sum(1) + b * b
    rad = np.sqrt((x * x).sum(1))
    h = 0.06
    rho0 = 3.0 / (4.0 * np.pi * b ** 3)
    drho = -5.0 * rho0 * (rad / b ** 2) * (1.0 + rad ** 2 / b ** 2) ** -3.5
    a_mf = -x / s2[:, None] ** 1.5 - (2.0 * np.pi / 3.0) * h * h * (drho / rad)[:, None] * x
    tv = -v / s2[:, None] ** 1.5 + 3.0 * ((x * v).sum(1) / s2 ** 2.5)[:, None] * x
    ball = (1.0 / b ** 3) * (1.0 + rad ** 2 / b ** 2) ** -2.5
    j_mf = tv + ball[:, None] * v
    sel = rad < 3.0
    ca = (r.acc[sel] * a_mf[sel]).sum() / (a_mf[sel] ** 2).sum()
    cj = (r.jerk[sel] * j_mf[sel]).sum() / (j_mf[sel] ** 2).sum()
    assert abs(ca - 1.0) < 0.02, ca
    assert abs(cj - 1.0) < 0.05, cj
    # radial profile of the acceleration in equal-count bins
    edges = np.quantile(rad[sel], np.linspace(0, 1, 9))
    for lo, hi in zip(edges[:-1], edges[1:]):
        s = sel & (rad >= lo) & (rad < hi)
        ar = (r.acc[s] * x[s]).sum(1) / rad[s]
        am = (a_mf[s] * x[s]).sum(1) / rad[s]
        assert abs(ar.mean() / am.mean() - 1.0) < 0.03, (lo, hi, ar.mean(), am.mean())


# --------------------------------------------------------------------------
def pin_everything_neighbour(lib=None):
    m, x, v, h2, dtr = _tiny_inputs(4, n=24)
    n = len(m)
    r = oracle.regular_force(m, x, v, np.arange(n), 1e30, dtr, lcap=n, lib=lib)
    assert np.all(r.acc == 0.0) and np.all(r.jerk == 0.0)
    for i in range(n):
        assert list(map(int, r.lists[i])) == [j for j in range(n) if j != i]
    assert np.all(r.nnb == n - 1)


def pin_scales_and_truncation(lib=None):
    m, x, v, h2, dtr = _tiny_inputs(5, n=40)
    n = len(m)
    full = oracle.regular_force(m, x, v, np.arange(n), h2, dtr, lcap=n, lib=lib)
    assert np.all(np.linalg.norm(full.acc, axis=1) <= full.sa * (1 + 1e-14))
    assert np.all(np.linalg.norm(full.jerk, axis=1) <= full.sj * (1 + 1e-14))
    short = oracle.regular_force(m, x, v, np.arange(n), h2, dtr, lcap=2, lib=lib)
    assert np.array_equal(short.nnb, full.nnb)
    for i in range(n):
        assert np.array_equal(short.lists[i], full.lists[i][:2])
    assert np.array_equal(short.acc, full.acc)


# --------------------------------------------------------------------------
# Potential
# --------------------------------------------------------------------------
def pin_potential_gradient(lib=None):
    """The acceleration is minus the gradient of the potential at the
    particle: central differences of phi_i in each coordinate of x_i, the
    other particles fixed (no neighbours, so the sums cover every j)."""
    cl = make_cluster(300, 31, masses="imf", stored_state=False, k_nb=8)
    n = cl.n
    base = oracle.regular_force(cl.m, cl.x, cl.v, np.arange(n), 1e-300, 0.0, lcap=4, lib=lib)
    d = 1e-6
    for i in range(0, n, 37):
        g = np.zeros(3)
        for c in range(3):
            xp = cl.x.copy()
            xm = cl.x.copy()
            xp[i, c] += d
            xm[i, c] -= d
            pp = oracle.regular_force(cl.m, xp, cl.v, [i], 1e-300, 0.0, lcap=4, lib=lib).pot[0]
            pm = oracle.regular_force(cl.m, xm, cl.v, [i], 1e-300, 0.0, lcap=4, lib=lib).pot[0]
            g[c] = (pp - pm) / (2 * d)
        err = np.linalg.norm(-g - base.acc[i]) / base.sa[i]
        assert err < 1e-5, (i, err)


def pin_potential_plummer(lib=None):
    """The potential of a Plummer sphere sample follows -M (r^2 + b^2)^-1/2
    (G = M = 1, b = 3 pi/16); without the neighbour ball of radius h the
    regular potential lacks that ball's share, 2 pi rho h^2 for a uniform
    ball, which is added back here."""
    cl = make_cluster(16384, 11, masses="equal", stored_state=False, k_nb=8)
    n = cl.n
    idx = np.arange(0, n, 4)
    b = 3.0 * np.pi / 16.0
    x = cl.x[idx]
    rad = np.sqrt((x * x).sum(1))
    phi_mf = -1.0 / np.sqrt(rad ** 2 + b * b)
    full = oracle.regular_force(cl.m, cl.x, cl.v, idx, 1e-300, 0.0, lcap=4, lib=lib)
    h = 0.06
    reg = oracle.regular_force(cl.m, cl.x, cl.v, idx, h * h, 0.0, lcap=4096, lib=lib)
    rho = 3.0 / (4.0 * np.pi * b ** 3) * (1.0 + rad ** 2 / b ** 2) ** -2.5
    sel = rad < 3.0
    for got, expect in ((full.pot, phi_mf), (reg.pot, phi_mf + 2.0 * np.pi * rho * h * h)):
        edges = np.quantile(rad[sel], np.linspace(0, 1, 9))
        for lo, hi in zip(edges[:-1], edges[1:]):
            s_ = sel & (rad >= lo) & (rad < hi)
            assert abs(got[s_].mean() / expect[s_].mean() - 1.0) < 0.01, (lo, hi)
    # virial equilibrium in Henon units: W = (1/2) sum m phi = 2 E = -1/2
    allp = oracle.regular_force(cl.m, cl.x, cl.v, np.arange(n), 1e-300, 0.0, lcap=4, lib=lib)
    w = 0.5 * (cl.m * allp.pot).sum()
    assert abs(w + 0.5) < 0.02, w


# --------------------------------------------------------------------------
# Irregular force (section 3.3 step 4)
# --------------------------------------------------------------------------
def pin_irregular_golden(lib=None):
    """With every other particle listed, the irregular force is the whole sum:
    the hand-derived values of the golden cases that have no neighbours."""
    for c in json.load(open(GOLDEN))["force_cases"]:
        if any(c["lists"]):
            continue
        m = np.array(c["m"], float)
        xp = np.array(c["x"], float)
        vp = np.array(c["v"], float)
        n = len(m)
        act = list(c["active"])
        lists = [[j for j in range(n) if j != i] for i in act]
        r = oracle.irregular_force(m, xp, vp, act, lists, lib=lib)
        assert _close(r.acc, c["acc"], 1e-14), (c["name"], r.acc, c["acc"])
        if c["jerk"] != "skip":
            assert _close(r.jerk, c["jerk"], 1e-14), (c["name"], r.jerk, c["jerk"])
        assert _close(r.pot, c["pot"], 1e-14), (c["name"], r.pot, c["pot"])


def pin_irregular_complements_regular(lib=None):
    """Section 3.3 splits the force: regular over the non-neighbours plus
    irregular over the list L_i equals the regular force with no neighbour
    at all (h -> 0), for any radius and time-step."""
    cl = make_cluster(300, 17, masses="imf", stored_state=False, k_nb=12)
    n = cl.n
    idx = np.arange(0, n, 3)
    full = oracle.regular_force(cl.m, cl.x, cl.v, idx, 1e-300, 0.0, lcap=4, lib=lib)
    assert full.nnb.max() == 0
    for h2, dtr in ((cl.h2[idx], cl.dtr[idx]), (cl.h2[idx] * 4.0, 0.0)):
        reg = oracle.regular_force(cl.m, cl.x, cl.v, idx, h2, dtr, lcap=n, lib=lib)
        assert reg.nnb.sum() > len(idx)
        irr = oracle.irregular_force(cl.m, cl.x, cl.v, idx, reg.lists, lib=lib)
        for a, b, full_q, sc in ((reg.acc, irr.acc, full.acc, full.sa),
                                 (reg.jerk, irr.jerk, full.jerk, full.sj)):
            err = np.linalg.norm(a + b - full_q, axis=1) / sc
            assert err.max() < 1e-13, err.max()
        # the magnitude sums and the potential split the same way
        assert np.all(np.abs(reg.sa + irr.sa - full.sa) <= 1e-13 * full.sa)
        assert np.all(np.abs(reg.sj + irr.sj - full.sj) <= 1e-13 * full.sj)
        assert np.all(np.abs(reg.pot + irr.pot - full.pot) <= 1e-13 * np.abs(full.pot))


def pin_irregular_momentum(lib=None):
    """Symmetric lists (uniform h, dt_reg = 0, all active): sum m F_I = 0 and
    sum m dF_I/dt = 0 (Newton's third law within the neighbour spheres)."""
    cl = make_cluster(400, 23, masses="imf", stored_state=False, k_nb=10)
    n = cl.n
    idx = np.arange(n)
    reg = oracle.regular_force(cl.m, cl.x, cl.v, idx, 0.2 ** 2, 0.0, lcap=n, lib=lib)
    irr = oracle.irregular_force(cl.m, cl.x, cl.v, idx, reg.lists, lib=lib)
    for q in (irr.acc, irr.jerk):
        tot = (cl.m[:, None] * q).sum(0)
        scale = (cl.m * np.linalg.norm(q, axis=1)).sum()
        assert np.all(np.abs(tot) <= 1e-13 * scale), (tot, scale)


def pin_irregular_fd_jerk(lib=None):
    """dF_I/dt = d(F_I)/dt along straight-line drift with the lists held fixed."""
    cl = make_cluster(200, 29, masses="imf", stored_state=False, k_nb=20)
    n = cl.n
    idx = np.arange(n)
    z = np.zeros((n, 3))
    reg = oracle.regular_force(cl.m, cl.x, cl.v, idx, cl.h2, 0.0, lcap=n, lib=lib)
    base = oracle.irregular_force(cl.m, cl.x, cl.v, idx, reg.lists, lib=lib)
    d = 1e-7
    xp, _ = oracle.predict(cl.x, cl.v, z, z, np.zeros(n), d, lib=lib)
    xm, _ = oracle.predict(cl.x, cl.v, z, z, np.zeros(n), -d, lib=lib)
    ap = oracle.irregular_force(cl.m, xp, cl.v, idx, reg.lists, lib=lib).acc
    am = oracle.irregular_force(cl.m, xm, cl.v, idx, reg.lists, lib=lib).acc
    fd = (ap - am) / (2 * d)
    has = base.sj > 0
    assert has.sum() > n // 2
    err = np.linalg.norm(fd - base.jerk, axis=1)[has] / base.sj[has]
    assert err.max() < 1e-5, err.max()


def pin_irregular_list_semantics(lib=None):
    """Empty lists give zero; an entry equal to i adds nothing; the order of
    the entries does not matter; a repeated entry counts twice."""
    m, x, v, h2, dtr = _tiny_inputs(7, n=30)
    n = len(m)
    rng = np.random.default_rng(3)
    idx = np.arange(n)
    lists = [rng.choice([j for j in range(n) if j != i], 6, replace=False) for i in idx]
    base = oracle.irregular_force(m, x, v, idx, lists, lib=lib)
    assert np.all(base.sa > 0)
    empty = oracle.irregular_force(m, x, v, idx, [[] for _ in idx], lib=lib)
    assert np.all(empty.acc == 0) and np.all(empty.jerk == 0) and np.all(empty.sa == 0)
    with_self = [np.concatenate([[i], l]) for i, l in zip(idx, lists)]
    r = oracle.irregular_force(m, x, v, idx, with_self, lib=lib)
    assert np.array_equal(r.acc, base.acc) and np.array_equal(r.jerk, base.jerk)
    rev = oracle.irregular_force(m, x, v, idx, [l[::-1] for l in lists], lib=lib)
    assert _close(rev.acc, base.acc, 1e-15) and _close(rev.jerk, base.jerk, 1e-15)
    one = [l[:1] for l in lists]
    r1 = oracle.irregular_force(m, x, v, idx, one, lib=lib)
    r2 = oracle.irregular_force(m, x, v, idx, [np.concatenate([l, l]) for l in one], lib=lib)
    assert _close(r2.acc, 2.0 * r1.acc, 1e-15) and _close(r2.jerk, 2.0 * r1.jerk, 1e-15)


# --------------------------------------------------------------------------
# Regular corrector (section 3.3 step 7, section 3.6, equation 1)
# --------------------------------------------------------------------------
def _cubic_block(rng, n, h):
    """A regular force that is an exact cubic in time: returns the corrector
    inputs of one step of length h and the exact F2(t), F3."""
    c = rng.normal(size=(4, n, 3))
    c[3] *= 10.0
    f_old, fd_old = c[0], c[1]
    f_new = c[0] + c[1] * h + c[2] * h * h / 2.0 + c[3] * h ** 3 / 6.0
    fd_new = c[1] + c[2] * h + c[3] * h * h / 2.0
    return f_old, fd_old, f_new, fd_new, c[2] + c[3] * h, c[3]


def pin_corrector_hermite_cubic(lib=None):
    """Hermite interpolation is exact for a cubic force: F2 at the new time
    and F3 come back to rounding, and with no list change dF = F_new - F_old."""
    rng = np.random.default_rng(41)
    n, t, h = 64, 1.0, 2.0 ** -5
    f_old, fd_old, f_new, fd_new, f2, f3 = _cubic_block(rng, n, h)
    z = np.zeros((n, 3))
    g = rng.normal(size=(n, 3))
    r = oracle.regular_correct(t, np.full(n, t - h), f_old, fd_old, f_new, fd_new, g, z, g, z,
                               0.1, 40, 40, lib=lib)
    assert _close(r.df, f_new - f_old, 1e-15) and _close(r.dfd, fd_new - fd_old, 1e-15)
    assert np.max(np.abs(r.f2 - f2) / (1.0 + np.abs(f2))) < 1e-9
    assert np.max(np.abs(r.f3 - f3) / (1.0 + np.abs(f3))) < 1e-9


def pin_corrector_list_change(lib=None):
    """Section 3.6: a term that moves between the regular and the irregular
    force at the new time changes nothing -- the regular change is taken over
    a fixed neighbour set."""
    rng = np.random.default_rng(43)
    n, t, h = 64, 0.75, 2.0 ** -6
    f_old, fd_old, f_new, fd_new, _, _ = _cubic_block(rng, n, h)
    g_old, gd_old = rng.normal(size=(2, n, 3))
    x, xd = rng.normal(size=(2, n, 3))
    base = oracle.regular_correct(t, np.full(n, t - h), f_old, fd_old, f_new, fd_new,
                                  g_old, gd_old, g_old, gd_old, 0.1, 40, 40, lib=lib)
    moved = oracle.regular_correct(t, np.full(n, t - h), f_old, fd_old, f_new + x, fd_new + xd,
                                   g_old, gd_old, g_old - x, gd_old - xd, 0.1, 40, 40, lib=lib)
    # (rounding of the moved term, ~1e-16, reaches F3 amplified by 12 / h^3)
    for a, b, tol in ((base.df, moved.df, 1e-14), (base.dfd, moved.dfd, 1e-14),
                      (base.f2, moved.f2, 1e-8), (base.f3, moved.f3, 1e-8)):
        assert np.max(np.abs(a - b) / (1.0 + np.abs(a))) < tol
    # and the raw difference without the correction would not agree
    raw = oracle.regular_correct(t, np.full(n, t - h), f_old, fd_old, f_new + x, fd_new + xd,
                                 g_old, gd_old, g_old, gd_old, 0.1, 40, 40, lib=lib)
    assert np.max(np.abs(raw.f3 - base.f3)) > 1.0


def pin_corrector_step(lib=None):
    """The step criterion on a harmonic force F = A cos(w t) is sqrt(eta)/w;
    the step is the largest power of two below it, at most twice the last
    step, and dividing the block time."""
    eta = 0.02
    for w, h, t, expect in ((100.0, 2.0 ** -10, 1.0, 2.0 ** -10),      # criterion
                            (1.0, 2.0 ** -6, 1.0, 2.0 ** -5),          # doubling limit
                            (1.0, 2.0 ** -6, 3.0 * 2.0 ** -6, 2.0 ** -6),  # commensurate
                            (1.0e4, 2.0 ** -14, 1.0, 2.0 ** -16)):     # dt_min
        a = np.array([[0.3, -0.4, 1.2]])
        f = lambda s: a * np.cos(w * s)              # noqa: E731
        fd = lambda s: -a * w * np.sin(w * s)        # noqa: E731
        r = oracle.regular_correct(t, [t - h], f(t - h), fd(t - h), f(t), fd(t),
                                   np.zeros((1, 3)), np.zeros((1, 3)), np.zeros((1, 3)),
                                   np.zeros((1, 3)), 0.1, 40, 40, eta=eta,
                                   dt_min=2.0 ** -16, lib=lib)
        assert r.dt_new[0] == expect, (w, h, t, r.dt_new[0], expect)
    # the criterion itself, where the Hermite derivatives are accurate
    w, h, t = 3.0, 2.0 ** -14, 0.5
    a = np.array([[1.0, 2.0, -0.5]])
    r = oracle.regular_correct(t, [t - h], a * np.cos(w * (t - h)), -a * w * np.sin(w * (t - h)),
                               a * np.cos(w * t), -a * w * np.sin(w * t), np.zeros((1, 3)),
                               np.zeros((1, 3)), np.zeros((1, 3)), np.zeros((1, 3)),
                               0.1, 40, 40, eta=eta, dt_min=2.0 ** -30, lib=lib)
    f2_exact = -w * w * a * np.cos(w * t)
    assert np.max(np.abs(r.f2 - f2_exact)) < 1e-6 * w * w


def pin_corrector_radius(lib=None):
    """Equation (1): h_new = h_old (n_p / n)^(1/3), within the limits."""
    z = np.zeros((5, 3))
    h_old = np.array([0.1, 0.1, 0.2, 0.3, 0.4])
    nnb = np.array([50, 50, 8, 0, 27])
    n_p = np.array([50.0, 400.0, 1.0, 50.0, 64.0])
    r = oracle.regular_correct(1.0, np.full(5, 0.5), z, z, z, z, z, z, z, z, h_old, nnb, n_p,
                               f_lo=0.25, f_hi=1.5, lib=lib)
    expect = h_old * np.array([1.0, 1.5, 0.5, 1.5, 4.0 / 3.0])
    assert _close(r.h_new, expect, 1e-15), (r.h_new, expect)


ALL_PINS = [  # roughly cheapest first
    pin_golden_forces,
    pin_pair_terms_golden,
    pin_golden_predict,
    pin_everything_neighbour,
    pin_scales_and_truncation,
    pin_exact_rational_predict,
    pin_exact_rational_lists,
    pin_momentum,
    pin_fd_jerk,
    pin_plummer_mean_field,
    pin_corrector_hermite_cubic,
    pin_corrector_list_change,
    pin_corrector_step,
    pin_corrector_radius,
    pin_potential_gradient,
    pin_potential_plummer,
    pin_irregular_golden,
    pin_irregular_list_semantics,
    pin_irregular_complements_regular,
    pin_irregular_momentum,
    pin_irregular_fd_jerk,
]
