"""The seeded inputs follow their stated recipe (CPU): Plummer spheres in
Henon units, the power-law mass function, bound primordial binaries in
their separation range, neighbour radii holding about k neighbours, and
stored states on the block-step grid.  The generators hold none of the
method's arithmetic; these checks pin their statistics."""
import numpy as np
import pytest

from workloads import make_cluster


def _potential_energy(m, x, rows=512):
    w = 0.0
    for i0 in range(0, len(m), rows):
        d = x[i0:i0 + rows, None, :] - x[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        ii = np.arange(i0, min(i0 + rows, len(m)))
        r[np.arange(len(ii)), ii] = np.inf
        w -= 0.5 * (m[ii, None] * m[None, :] / r).sum()
    return w


def test_plummer_in_henon_units():
    cl = make_cluster(4096, 3, masses="equal", k_nb=32, stored_state=False)
    assert abs(cl.m.sum() - 1.0) < 1e-12
    assert np.abs((cl.m[:, None] * cl.x).sum(0)).max() < 1e-12     # c.m. at rest
    assert np.abs((cl.m[:, None] * cl.v).sum(0)).max() < 1e-12     # at the origin
    t = 0.5 * (cl.m * (cl.v ** 2).sum(1)).sum()
    w = _potential_energy(cl.m, cl.x)
    assert abs((t + w) + 0.25) < 0.02          # E = -1/4 (sampling noise ~1/sqrt(N))
    assert abs(2 * t / -w - 1.0) < 0.08        # virial equilibrium
    r = np.sqrt((cl.x ** 2).sum(1))
    # half-mass radius of the Henon-unit Plummer sphere: b / sqrt(2^(2/3) - 1) ~ 0.769
    assert abs(np.median(r) - 0.769) < 0.04


def test_power_law_masses():
    cl = make_cluster(16384, 5, masses="imf", m_lo=0.1, m_hi=10.0, k_nb=16,
                      stored_state=False)
    m = cl.m
    assert abs(m.sum() - 1.0) < 1e-12
    assert m.max() / m.min() <= 100.0 * (1 + 1e-12)
    # slope of dN/dm on log bins, fitted over the range
    edges = np.geomspace(m.min(), m.max(), 12)
    cnt, _ = np.histogram(m, edges)
    dm = np.diff(edges)
    mid = np.sqrt(edges[1:] * edges[:-1])
    ok = cnt > 20
    slope = np.polyfit(np.log(mid[ok]), np.log(cnt[ok] / dm[ok]), 1)[0]
    assert abs(slope + 2.35) < 0.12, slope


def test_primordial_binaries():
    cl = make_cluster(8192, 7, masses="imf", m_lo=0.1, m_hi=100.0, binary_fraction=0.1,
                      k_nb=50)
    pairs = cl.binaries
    assert len(pairs) == 8192 // 20
    assert len(np.unique(pairs)) == 2 * len(pairs)
    i, j = pairs[:, 0], pairs[:, 1]
    d = cl.x[j] - cl.x[i]
    r = np.sqrt((d * d).sum(1))
    dv = cl.v[j] - cl.v[i]
    mt = cl.m[i] + cl.m[j]
    energy = 0.5 * (dv * dv).sum(1) - mt / r          # per unit reduced mass
    assert np.all(energy < 0)                          # every pair bound
    sma = -mt / (2 * energy)
    assert sma.min() > 1e-4 * (1 - 1e-6) and sma.max() < 1e-2 * (1 + 1e-6)
    # log-uniform semi-major axes: about half below the geometric mean 1e-3
    assert 0.4 < np.mean(sma < 1e-3) < 0.6
    # the pairs' members are each other's neighbours (r far inside h)
    assert np.all(r * r < cl.h2[i]) and np.all(r * r < cl.h2[j])


@pytest.mark.parametrize("k", [16, 50])
def test_neighbour_radii_hold_about_k(k):
    cl = make_cluster(4096, 11, masses="equal", k_nb=k)
    from scipy.spatial import cKDTree
    tree = cKDTree(cl.x)
    counts = np.array([len(tree.query_ball_point(cl.x[q], np.sqrt(cl.h2[q]))) - 1
                       for q in range(0, cl.n, 7)])
    assert abs(counts.mean() - k) < 0.1 * k, counts.mean()


def test_stored_state_on_the_block_grid():
    cl = make_cluster(2048, 13, masses="imf", binary_fraction=0.1, k_nb=20)
    dt = cl.tb - cl.t
    assert np.all(dt >= 0)
    # each stored time is a multiple of its own step, within one step of tb
    steps = 2.0 ** -np.arange(3, 25)
    for q in range(0, cl.n, 5):
        ok = [(cl.t[q] / s == np.floor(cl.t[q] / s)) and (dt[q] < s) for s in steps]
        assert any(ok), q
    assert np.all((cl.dtr >= 2.0 ** -10) & (cl.dtr <= 2.0 ** -6))
