"""Seeded star-cluster generators (Plummer spheres, IMF masses, binaries).

Units are the standard N-body (Henon) units the paper's benchmarks use
(section 4): G = 1, total mass M = 1, total energy E = -1/4.  A Plummer
sphere then has scale length b = 3 pi / 16.

Recipes (the paper fixes only "isolated Plummer models in virial
equilibrium, equal masses, E = -0.25, M = 1"; everything else is a stated
choice of this generator):

* Plummer positions and velocities: inverse-CDF radius and von Neumann
  rejection for the speed (Aarseth, Henon & Wielen 1974), radii truncated at
  mass fraction 0.999, isotropic directions, then shifted to the c.m. frame.
* Masses: equal (1/N), or a power law dN/dm ~ m^-2.35 between m_lo and m_hi
  drawn by inverse CDF and normalised to total mass 1.
* Primordial binaries: a fraction of the Plummer points become pairs with
  log-uniform semi-major axis, thermal eccentricity (e = sqrt(u)), random
  orientation and uniform mean anomaly (Kepler's equation solved by Newton
  iteration).
* Stored state: the Plummer point is the state at its own time t_j; the
  stored acceleration and jerk are those of the smooth Plummer potential
  (they only feed the predictor, so any smooth field of the right size will
  do); time-steps are powers of two, and t_j is the last multiple of the
  step not after the block time.
* Neighbour radii: distance to the k-th nearest particle times a factor
  drawn from U(0.95, 1.05), so the boundary never sits exactly on a particle.
* Regular steps dt_reg = 2^-k with k uniform in {6, ..., 10}.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CONFIG_SEED_BASE = 12051222
B_HENON = 3.0 * np.pi / 16.0


@dataclass
class Cluster:
    m: np.ndarray          # [n] masses
    x: np.ndarray          # [n,3] stored positions at t
    v: np.ndarray          # [n,3] stored velocities
    a: np.ndarray          # [n,3] stored acceleration
    jerk: np.ndarray       # [n,3] stored jerk
    t: np.ndarray          # [n] time of the stored state
    tb: float              # block time the cluster is predicted to
    h2: np.ndarray         # [n] squared neighbour radius
    dtr: np.ndarray        # [n] regular time-step
    binaries: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))

    @property
    def n(self) -> int:
        return len(self.m)


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit_vectors(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def plummer(n: int, rng: np.random.Generator, mfrac_max: float = 0.999):
    """Positions and velocities of an n-point Plummer sphere, Henon units."""
    u = rng.uniform(0.0, mfrac_max, n)
    u = np.maximum(u, 1e-300)
    r = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)          # Plummer units (b = 1)
    x = r[:, None] * _unit_vectors(rng, n)
    # speed fraction q of the local escape speed, density q^2 (1-q^2)^3.5
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (1.0 + r * r) ** -0.25
    v = (q * vesc)[:, None] * _unit_vectors(rng, n)
    # Plummer units -> Henon units (E = -1/4): length x 3pi/16, speed / sqrt
    x *= B_HENON
    v /= np.sqrt(B_HENON)
    return x, v


def salpeter_masses(n, rng, m_lo, m_hi, alpha=2.35):
    """Power-law masses dN/dm ~ m^-alpha on [m_lo, m_hi], total mass 1."""
    u = rng.uniform(0.0, 1.0, n)
    p = 1.0 - alpha
    m = (m_lo ** p + u * (m_hi ** p - m_lo ** p)) ** (1.0 / p)
    return m / m.sum()


def _kepler_E(M, e):
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E = E - f / (1.0 - e * np.cos(E))
    return E


def _random_rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], 1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], 1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1),
    ], axis=1)


def add_binaries(m_pairs, x_cm, v_cm, rng, a_lo=1e-4, a_hi=1e-2):
    """Split c.m. points into Keplerian pairs.

    ``m_pairs`` is [nb, 2].  Returns positions and velocities [nb, 2, 3].
    """
    nb = len(x_cm)
    mtot = m_pairs.sum(axis=1)
    sma = np.exp(rng.uniform(np.log(a_lo), np.log(a_hi), nb))
    ecc = np.sqrt(rng.uniform(0.0, 1.0, nb))
    Mano = rng.uniform(0.0, 2.0 * np.pi, nb)
    E = _kepler_E(Mano, ecc)
    nmot = np.sqrt(mtot / sma ** 3)
    Edot = nmot / (1.0 - ecc * np.cos(E))
    sq = np.sqrt(1.0 - ecc * ecc)
    rel = np.stack([sma * (np.cos(E) - ecc), sma * sq * np.sin(E), np.zeros(nb)], 1)
    vrel = np.stack([-sma * np.sin(E) * Edot, sma * sq * np.cos(E) * Edot, np.zeros(nb)], 1)
    rot = _random_rotations(rng, nb)
    rel = np.einsum("nij,nj->ni", rot, rel)
    vrel = np.einsum("nij,nj->ni", rot, vrel)
    f1 = (m_pairs[:, 1] / mtot)[:, None]
    f2 = (m_pairs[:, 0] / mtot)[:, None]
    xs = np.stack([x_cm - f1 * rel, x_cm + f2 * rel], axis=1)
    vs = np.stack([v_cm - f1 * vrel, v_cm + f2 * vrel], axis=1)
    return xs, vs


def plummer_mean_field(x, v, b=B_HENON, mass=1.0):
    """Acceleration and its time derivative in the smooth Plummer potential."""
    s2 = (x * x).sum(1) + b * b
    s3 = s2 ** -1.5
    s5 = s2 ** -2.5
    xv = (x * v).sum(1)
    a = -mass * x * s3[:, None]
    j = -mass * (v * s3[:, None] - 3.0 * (xv * s5)[:, None] * x)
    return a, j


def neighbour_radii(x, k, rng, spread=0.05):
    """h_i = (distance to k-th nearest other particle) * U(1-spread, 1+spread)."""
    from scipy.spatial import cKDTree

    tree = cKDTree(x)
    d, _ = tree.query(x, k=[k + 1], workers=-1)
    d = d[:, 0]
    return d * rng.uniform(1.0 - spread, 1.0 + spread, len(x))


def regular_steps(n, rng, kmin=6, kmax=10):
    return 2.0 ** -rng.integers(kmin, kmax + 1, n).astype(np.float64)


def make_cluster(n, seed, *, masses="equal", m_lo=0.1, m_hi=10.0,
                 binary_fraction=0.0, k_nb=50, stored_state=True,
                 step_k=(3, 12)) -> Cluster:
    """A seeded cluster of exactly n stars, ready to be predicted to ``tb``."""
    rng = _rng(seed)
    n_pairs = int(n * binary_fraction) // 2
    n_sys = n - n_pairs
    xs, vs = plummer(n_sys, rng)
    if masses == "equal":
        m_all = np.full(n, 1.0 / n)
    else:
        m_all = salpeter_masses(n, rng, m_lo, m_hi)
    # systems [0, n_single) are single stars, the rest become pairs
    n_single = n_sys - n_pairs
    x = np.empty((n, 3))
    v = np.empty((n, 3))
    x[:n_single] = xs[:n_single]
    v[:n_single] = vs[:n_single]
    pairs = np.zeros((n_pairs, 2), np.int32)
    if n_pairs:
        mp = m_all[n_single:].reshape(n_pairs, 2)
        bx, bv = add_binaries(mp, xs[n_single:], vs[n_single:], rng)
        x[n_single:] = bx.reshape(-1, 3)
        v[n_single:] = bv.reshape(-1, 3)
        first = n_single + 2 * np.arange(n_pairs)
        pairs = np.stack([first, first + 1], 1).astype(np.int32)
    # shuffle so binaries are spread over the index range
    perm = rng.permutation(n)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    x, v, m_all = x[perm], v[perm], m_all[perm]
    pairs = inv[pairs].astype(np.int32)
    # c.m. frame
    M = m_all.sum()
    x -= (m_all[:, None] * x).sum(0) / M
    v -= (m_all[:, None] * v).sum(0) / M

    tb = 1.0 + float(2 * rng.integers(0, 2 ** 28) + 1) * 2.0 ** -30
    if stored_state:
        a, j = plummer_mean_field(x, v)
        dt_j = 2.0 ** -rng.integers(step_k[0], step_k[1] + 1, n).astype(np.float64)
        if n_pairs:
            dt_j[pairs.ravel()] = 2.0 ** -24
        t = np.floor(tb / dt_j) * dt_j
    else:
        a = np.zeros((n, 3))
        j = np.zeros((n, 3))
        t = np.full(n, tb)
    h = neighbour_radii(x, k_nb, rng)
    dtr = regular_steps(n, rng)
    return Cluster(m_all, x, v, a, j, t, tb, h * h, dtr, pairs)


# --------------------------------------------------------------------------
# The benchmark configurations
# --------------------------------------------------------------------------
_CONFIGS = {
    1: dict(n=1024, masses="equal", k_nb=32, stored_state=False),
    2: dict(n=16384, masses="imf", m_lo=0.1, m_hi=10.0, k_nb=50),
    3: dict(n=131072, masses="imf", m_lo=0.1, m_hi=100.0, binary_fraction=0.1, k_nb=50),
    5: dict(n=1048576, masses="equal", k_nb=100),
}

CONFIG_DESCRIPTION = {
    1: "Plummer N=1024, equal masses, all active, ~32 neighbours",
    2: "Plummer N=16384, IMF 0.1-10, stored state predicted to t_b, 1024 random active, ~50 neighbours",
    3: "Plummer N=131072, IMF 0.1-100, 10% binaries, stored state, power-of-2 blocks, ~50 neighbours",
    4: "serving trace: 64 Plummer clusters, N log-uniform 4096..65536",
    5: "Plummer N=1048576, equal masses, all active and 4096-active, ~100 neighbours",
}


def config(ci: int, seed: int | None = None, n: int | None = None) -> dict:
    """Cluster and active sets of benchmark configuration ``ci``.

    ``n`` overrides the particle number (for quick runs of the same recipe).
    Returns dict(cluster, blocks: {name: idx array}, seed, description).
    """
    if ci not in _CONFIGS:
        raise ValueError(f"no single-cluster configuration {ci}")
    seed = CONFIG_SEED_BASE + ci if seed is None else seed
    kw = dict(_CONFIGS[ci])
    if n is not None:
        kw["n"] = n
    N = kw.pop("n")
    cl = make_cluster(N, seed, **kw)
    rng = _rng(seed + 1000)
    blocks = {"all": np.arange(N, dtype=np.int32)}
    if ci == 2:
        blocks["random1024"] = np.sort(rng.choice(N, min(1024, N), replace=False)).astype(np.int32)
    if ci == 3:
        for k in range(0, 18):
            if 2 ** k <= N:
                blocks[f"pow2_{k}"] = np.sort(rng.choice(N, 2 ** k, replace=False)).astype(np.int32)
    if ci == 5:
        blocks["random4096"] = np.sort(rng.choice(N, min(4096, N), replace=False)).astype(np.int32)
        blocks["sample10000"] = np.sort(rng.choice(N, min(10000, N), replace=False)).astype(np.int32)
    return dict(cluster=cl, blocks=blocks, seed=seed,
                description=CONFIG_DESCRIPTION[ci])


def serving_trace(n_clusters=64, n_requests=20000, seed=None, n_lo=4096,
                  n_hi=65536, k_nb=50, build_clusters=True):
    """Clusters and a request list for the serving workload.

    Each request is (cluster id, active index array, block-time offset).  The
    arrival times are left to the caller (open-loop Poisson at a chosen rate).
    """
    seed = CONFIG_SEED_BASE + 4 if seed is None else seed
    rng = _rng(seed)
    sizes = np.round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_clusters))).astype(int)
    clusters = []
    if build_clusters:
        for c, nc in enumerate(sizes):
            clusters.append(make_cluster(int(nc), seed * 1000 + c, masses="equal", k_nb=k_nb))
    reqs = []
    for _ in range(n_requests):
        c = int(rng.integers(0, n_clusters))
        nc = int(sizes[c])
        kmax = int(np.floor(np.log2(nc)))
        k = int(rng.integers(4, kmax + 1))
        idx = np.sort(rng.choice(nc, 2 ** k, replace=False)).astype(np.int32)
        reqs.append((c, idx))
    return dict(sizes=sizes, clusters=clusters, requests=reqs, seed=seed)
