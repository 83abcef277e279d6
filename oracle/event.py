"""Serial reference of the toy event loop around the lookup.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline).  It shares nothing with the HIP library.

What it computes: the outcome of every history of the event loop that
include/xs.h defines for xs_event_run.  The paper's application runs a
buffer of particles in flight through event kernels, refilling finished
slots from the source (section 5.1); because every random number of a
history depends only on (seed, history, collision), a history's outcome
does not depend on the buffer at all.  So this reference follows each
history on its own, from its source draw to its end:

  source:    E = 0.01 + 0.99 * v0,  m = min(floor(v1 * M), M - 1)
  collision c = 1, 2, ...:  S = the lookup of (E, m) (FP64 oracle, or its
             FP32 form widened to FP64), u = the three draws of collision c
             absorbed (fate 1)       if u0 * (S0 + S1) < 0.25 * S1
             else E' = E * (0.2 + 0.8 * u1)
                  cut off (fate 2)   if E' < e_cut
                  limit (fate 3)     if c == 2^18 - 1
                  else E = E'; if u2 < 0.2: m = min(floor((u2 * 5) * M), M - 1)

Draw i of collision c of history h is SplitMix64 (Steele, Lea & Flood
2014) at counter h * 2^20 + c * 4 + i: x = mix64(seed + (counter + 1) * G),
u = (x >> 11) * 2^-53.  The histories are advanced together, one collision
per step, only to call the lookup oracle on many queries at once; no
history ever reads another's state.
"""
from __future__ import annotations

import numpy as np

from . import lookup, lookup_f32

GAMMA = 0x9E3779B97F4A7C15
COLLISION_LIMIT = (1 << 18) - 1
_MASK = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64's output function on uint64 words."""
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def draw(seed: int, h: np.ndarray, c: np.ndarray, i: int) -> np.ndarray:
    """Uniform draws in [0, 1) for histories h at collisions c."""
    with np.errstate(over="ignore"):
        ctr = (h.astype(np.uint64) << np.uint64(20)) + \
              (c.astype(np.uint64) << np.uint64(2)) + np.uint64(i)
        x = mix64(np.uint64(seed & _MASK) + (ctr + np.uint64(1)) *
                  np.uint64(GAMMA))
    return (x >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def run_histories(tables, n_histories: int, seed: int, fp32: bool = False,
                  e_cut: float = 1e-5, threads: int = 1):
    """Returns (collisions int32, final energy float64, fate uint8), one
    entry per history."""
    M = tables.n_materials
    h = np.arange(n_histories, dtype=np.int64)
    zero = np.zeros(n_histories, dtype=np.int64)
    E = 0.01 + 0.99 * draw(seed, h, zero, 0)
    m = np.minimum((draw(seed, h, zero, 1) * M).astype(np.int64), M - 1)
    m = m.astype(np.int32)
    coll = np.zeros(n_histories, dtype=np.int32)
    e_end = np.zeros(n_histories, dtype=np.float64)
    fate = np.zeros(n_histories, dtype=np.uint8)
    live = np.arange(n_histories)
    c = 0
    while len(live):
        c += 1
        if fp32:
            S = lookup_f32(tables, E[live], m[live], threads=threads)
            S = S.astype(np.float64)
        else:
            S = lookup(tables, E[live], m[live], threads=threads)
        cc = np.full(len(live), c, dtype=np.int64)
        u0 = draw(seed, live, cc, 0)
        u1 = draw(seed, live, cc, 1)
        u2 = draw(seed, live, cc, 2)
        s0, s1 = S[:, 0], S[:, 1]
        absorbed = u0 * (s0 + s1) < 0.25 * s1
        e_new = E[live] * (0.2 + 0.8 * u1)
        cut = ~absorbed & (e_new < e_cut)
        limit = ~absorbed & ~cut & (c >= COLLISION_LIMIT)
        ends = absorbed | cut | limit
        idx = live[ends]
        coll[idx] = c
        e_end[idx] = np.where(absorbed[ends], E[idx], e_new[ends])
        fate[idx] = np.where(absorbed[ends], 1, np.where(cut[ends], 2, 3))
        go = live[~ends]
        E[go] = e_new[~ends]
        move = u2[~ends] < 0.2
        mv = go[move]
        m[mv] = np.minimum(((u2[~ends][move] * 5.0) * M).astype(np.int64),
                           M - 1).astype(np.int32)
        live = go
    return coll, e_end, fate
