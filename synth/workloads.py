"""Synthetic tables and query sets shaped like the paper's workload.

The paper tunes OpenMC on a depleted-fuel reactor problem (hundreds of
nuclides, materials of very different sizes, particles in flight from 1e5 to
about 8e6; section 5.1 and Table 1).  No evaluated nuclear data is used here:
every table and query below is drawn from `synth.rng` with a fixed seed.

Recipes (base seed S = 240209222; substream t of S is `Stream(S, t)`):

* config 1 tables (substream 1): 20 nuclides x 2,000 points.  E[0] = 1e-5,
  E[-1] = 1.0, the 1,998 interior points log-uniform in (1e-5, 1), sorted
  (a nuclide whose draw has a tie or touches an end is redrawn).  Five
  channels per point, lognormal(0, 1).  4 materials, L ~ U{2..20} distinct
  nuclides each (a prefix of a random permutation, stored sorted by id),
  densities 1 - U in (0, 1].
* config 2 tables (substream 2): 355 nuclides x 11,303 points with
  E[p] = exp(ln 1e-5 + (p + d) h), h = ln(1e5) / 11,302, d ~ U(-0.45, 0.45)
  inside and d = 0 at both ends (ends set to exactly 1e-5 and 1.0).  Five
  lognormal channels.  12 materials: material 0 has 321 nuclides, material 1
  has 4, materials 2..11 have floor(exp(U(ln 4, ln 321))) nuclides.
* queries: E log-uniform on [1e-5, 1), m uniform over the materials.
  Config 1 uses substream 11 (100,000 queries), config 2 substream 12
  (10,000,000), config 3 substream 13 (config-1 tables, 10,000,000),
  config 4 batch i substream 14 + i.
* config 5 (substream 15): 2,000 requests of floor(exp(U(ln 1e3, ln 1e6)))
  lookups; each E is log-uniform with probability 0.7, else drawn from one of
  16 narrow Gaussian peaks N(c, (0.005 c)^2) whose centres are log-uniform
  (redrawn while outside [1e-5, 1)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .rng import Stream

BASE_SEED = 240209222
N_CHANNELS = 5
E_LO, E_HI = 1.0e-5, 1.0


@dataclass
class Tables:
    """Pointwise per-nuclide tables and material compositions (host arrays).

    energy[grid_offsets[k]:grid_offsets[k+1]] is nuclide k's strictly
    increasing grid; xs[p, c] is channel c at point p (point-major).
    Material m lists nuclides mat_nuclides[mat_offsets[m]:mat_offsets[m+1]]
    with densities mat_density over the same range.
    """
    grid_offsets: np.ndarray   # int64 [K+1]
    energy: np.ndarray         # float64 [P]
    xs: np.ndarray             # float64 [P, 5]
    mat_offsets: np.ndarray    # int32 [M+1]
    mat_nuclides: np.ndarray   # int32 [sum L]
    mat_density: np.ndarray    # float64 [sum L]

    @property
    def n_nuclides(self) -> int:
        return len(self.grid_offsets) - 1

    @property
    def n_materials(self) -> int:
        return len(self.mat_offsets) - 1

    def grid(self, k: int) -> np.ndarray:
        return self.energy[self.grid_offsets[k]:self.grid_offsets[k + 1]]

    def channels(self, k: int) -> np.ndarray:
        return self.xs[self.grid_offsets[k]:self.grid_offsets[k + 1]]

    def material(self, m: int):
        a, b = self.mat_offsets[m], self.mat_offsets[m + 1]
        return self.mat_nuclides[a:b], self.mat_density[a:b]

    def material_sizes(self) -> np.ndarray:
        return np.diff(self.mat_offsets).astype(np.int64)


@dataclass
class Queries:
    E: np.ndarray     # float64 [N]
    mat: np.ndarray   # int32 [N]

    def __len__(self):
        return len(self.E)


def mean_nuclides(t: Tables, q: Queries) -> float:
    """Mean number of nuclides per lookup over a query set."""
    if len(q) == 0:
        return 0.0
    return float(t.material_sizes()[q.mat].mean())


def _sorted_interior(s: Stream, n_inner: int, lo: float, hi: float) -> np.ndarray:
    """n_inner sorted log-uniform draws strictly inside (lo, hi), no ties."""
    while True:
        v = np.sort(s.log_uniform(n_inner, lo, hi))
        full = np.concatenate(([lo], v, [hi]))
        if np.all(np.diff(full) > 0):
            return v


def _materials(s: Stream, k: int, sizes) -> tuple:
    offs = [0]
    nucs, dens = [], []
    for L in sizes:
        ids = np.sort(s.permutation(k)[:L]).astype(np.int32)
        nucs.append(ids)
        dens.append(s.uniform_open0(int(L)))
        offs.append(offs[-1] + int(L))
    return (np.asarray(offs, dtype=np.int32), np.concatenate(nucs),
            np.concatenate(dens))


def random_tables(seed: int, n_nuclides: int, points, n_materials: int,
                  sizes=None, stream: int = 100) -> Tables:
    """Small log-uniform tables of the config-1 kind, for tests.

    `points` is one grid length for all nuclides or a list of lengths (>= 2);
    `sizes` the material sizes (default U{1..K}).
    """
    s = Stream(seed, stream)
    if np.isscalar(points):
        points = [int(points)] * n_nuclides
    grids = []
    for n in points:
        inner = _sorted_interior(s, n - 2, E_LO, E_HI) if n > 2 else np.empty(0)
        grids.append(np.concatenate(([E_LO], inner, [E_HI])))
    energy = np.concatenate(grids)
    offs = np.zeros(n_nuclides + 1, dtype=np.int64)
    offs[1:] = np.cumsum(points)
    xs = s.lognormal(len(energy) * N_CHANNELS).reshape(-1, N_CHANNELS)
    if sizes is None:
        sizes = s.integers(n_materials, 1, n_nuclides)
    mo, mn, md = _materials(s, n_nuclides, sizes)
    return Tables(offs, energy, xs, mo, mn, md)


def random_queries(seed: int, tables: Tables, n: int, stream: int = 200,
                   lo: float = E_LO, hi: float = E_HI) -> Queries:
    s = Stream(seed, stream)
    E = s.log_uniform(n, lo, hi)
    m = s.integers(n, 0, tables.n_materials - 1).astype(np.int32)
    return Queries(E, m)


def config1_tables(seed: int = BASE_SEED) -> Tables:
    s = Stream(seed, 1)
    K, n = 20, 2000
    grids = [np.concatenate(([E_LO], _sorted_interior(s, n - 2, E_LO, E_HI),
                             [E_HI])) for _ in range(K)]
    energy = np.concatenate(grids)
    offs = np.arange(K + 1, dtype=np.int64) * n
    xs = s.lognormal(K * n * N_CHANNELS).reshape(-1, N_CHANNELS)
    sizes = s.integers(4, 2, 20)
    mo, mn, md = _materials(s, K, sizes)
    return Tables(offs, energy, xs, mo, mn, md)


def config2_tables(seed: int = BASE_SEED, n_nuclides: int = 355,
                   n_points: int = 11303) -> Tables:
    s = Stream(seed, 2)
    K, n = n_nuclides, n_points
    h = np.log(E_HI / E_LO) / (n - 1)
    p = np.arange(n, dtype=np.float64)
    delta = s.uniform(K * n).reshape(K, n) * 0.9 - 0.45
    delta[:, 0] = 0.0
    delta[:, -1] = 0.0
    energy = np.exp(np.log(E_LO) + (p[None, :] + delta) * h)
    energy[:, 0] = E_LO
    energy[:, -1] = E_HI
    assert np.all(np.diff(energy, axis=1) > 0)
    energy = energy.reshape(-1)
    offs = np.arange(K + 1, dtype=np.int64) * n
    xs = s.lognormal(K * n * N_CHANNELS).reshape(-1, N_CHANNELS)
    big = min(321, K)
    small = min(4, K)
    rest = np.floor(np.exp(np.log(4.0) + s.uniform(10) *
                           (np.log(321.0) - np.log(4.0)))).astype(np.int64)
    sizes = [big, small] + [int(min(max(v, 1), K)) for v in rest]
    mo, mn, md = _materials(s, K, sizes)
    return Tables(offs, energy, xs, mo, mn, md)


def _queries(seed, stream, n, n_materials) -> Queries:
    s = Stream(seed, stream)
    E = s.log_uniform(n, E_LO, E_HI)
    m = s.integers(n, 0, n_materials - 1).astype(np.int32)
    return Queries(E, m)


def config1_queries(n: int = 100_000, seed: int = BASE_SEED) -> Queries:
    return _queries(seed, 11, n, 4)


def config2_queries(n: int = 10_000_000, seed: int = BASE_SEED) -> Queries:
    return _queries(seed, 12, n, 12)


def config3_queries(n: int = 10_000_000, seed: int = BASE_SEED) -> Queries:
    return _queries(seed, 13, n, 4)


def config4_queries(i: int, n: int, seed: int = BASE_SEED) -> Queries:
    return _queries(seed, 14 + i, n, 12)


def config5_requests(n_requests: int = 2000, n_materials: int = 12,
                     seed: int = BASE_SEED, lo: float = 1e3, hi: float = 1e6,
                     with_queries: bool = True):
    """Request sizes and (optionally) the concatenated queries of the stream.

    Returns (sizes int64 [R], Queries over sum(sizes) lookups or None).
    """
    s = Stream(seed, 15)
    sizes = np.floor(np.exp(np.log(lo) + s.uniform(n_requests) *
                            (np.log(hi) - np.log(lo)))).astype(np.int64)
    if not with_queries:
        return sizes, None
    centres = s.log_uniform(16, E_LO, E_HI)
    total = int(sizes.sum())
    m = s.integers(total, 0, n_materials - 1).astype(np.int32)
    E = s.log_uniform(total, E_LO, E_HI)
    peaked = s.uniform(total) >= 0.7
    q = s.integers(total, 0, 15)
    idx = np.nonzero(peaked)[0]
    c = centres[q[idx]]
    vals = c + 0.005 * c * s.normal(len(idx))
    bad = (vals < E_LO) | (vals >= E_HI)
    while np.any(bad):
        bi = np.nonzero(bad)[0]
        cb = c[bi]
        vals[bi] = cb + 0.005 * cb * s.normal(len(bi))
        bad = (vals < E_LO) | (vals >= E_HI)
    E[idx] = vals
    return sizes, Queries(E, m)
