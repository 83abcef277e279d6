"""Pins of the event-loop reference (oracle/event.py) against facts that do
not come from it: the published SplitMix64 sequence, the geometric law of
the number of collisions when the cross sections are constant, the energy
window a cut-off history must end in, and the source distribution."""
import numpy as np

import synth
from oracle import event

GAMMA = np.uint64(0x9E3779B97F4A7C15)


def const_tables(a: float, b: float, n_materials: int = 1):
    """One nuclide whose five channels are constant in energy; every
    material holds it with density 1."""
    energy = np.array([1e-5, 0.5, 1.0])
    xs = np.tile(np.array([a, b, 1.0, 1.0, 1.0]), (3, 1))
    return synth.Tables(np.array([0, 3], np.int64), energy, xs,
                        np.arange(n_materials + 1, dtype=np.int32),
                        np.zeros(n_materials, np.int32),
                        np.ones(n_materials))


def test_splitmix64_published_sequence():
    """SplitMix64 seeded with 0 starts e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f (Steele, Lea & Flood 2014; the widely reproduced
    reference sequence)."""
    with np.errstate(over="ignore"):
        got = [int(event.mix64(np.array([GAMMA * np.uint64(j)]))[0])
               for j in (1, 2, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # counter 0 of history 0, collision 0, draw 0 is that first word
    u = event.draw(0, np.array([0]), np.array([0]), 0)[0]
    assert u == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


def test_collisions_are_geometric_with_constant_cross_sections():
    """S0 = 3, S1 = 1: absorbed iff 4 u0 < 0.25, i.e. u0 < 1/16 — a
    geometric number of collisions with mean 16 (the cut-off is set out of
    reach)."""
    t = const_tables(3.0, 1.0)
    n = 20000
    coll, e_end, fate = event.run_histories(t, n, seed=11, e_cut=1e-300)
    assert np.all(fate == 1)
    mean = coll.mean()
    se = np.sqrt((1 - 1 / 16) * 16 ** 2 / n)
    assert abs(mean - 16.0) < 5 * se, mean
    # P(first collision absorbs) = 1/16
    p1 = np.mean(coll == 1)
    assert abs(p1 - 1 / 16) < 5 * np.sqrt(p1 * (1 - p1) / n)


def test_no_absorption_ends_in_the_cutoff_window():
    """S1 = 0 never absorbs: every history ends cut off, one collision after
    its energy was still >= e_cut, so e_cut * 0.2 <= E_end < e_cut."""
    t = const_tables(3.0, 0.0, n_materials=3)
    coll, e_end, fate = event.run_histories(t, 5000, seed=3, e_cut=1e-3)
    assert np.all(fate == 2)
    assert np.all(e_end < 1e-3) and np.all(e_end >= 0.2 * 1e-3)
    assert coll.min() >= 1


def test_source_is_uniform():
    """Source energies uniform on [0.01, 1) (mean 0.505) and materials
    uniform: the first collision sees them unchanged when it absorbs."""
    n = 40000
    h = np.arange(n)
    z = np.zeros(n, np.int64)
    E = 0.01 + 0.99 * event.draw(5, h, z, 0)
    assert E.min() >= 0.01 and E.max() < 1.0
    assert abs(E.mean() - 0.505) < 5 * 0.99 / np.sqrt(12 * n)
    M = 4
    m = np.minimum((event.draw(5, h, z, 1) * M).astype(int), M - 1)
    counts = np.bincount(m, minlength=M)
    assert np.all(np.abs(counts - n / M) < 5 * np.sqrt(n / M))


def test_energy_loss_law_by_walds_identity():
    """Each scattering multiplies E by 0.2 + 0.8 u, so ln(E0 / E_end) is a
    sum of N i.i.d. terms of mean mu = -1.25 * integral of ln x over
    [0.2, 1] = 1.25 * (0.8 + 0.2 ln 0.2); by Wald's identity
    E[ln(E0 / E_end)] = mu * E[N] exactly."""
    t = const_tables(3.0, 0.0)
    n = 5000
    seed = 21
    coll, e_end, fate = event.run_histories(t, n, seed=seed, e_cut=1e-3)
    h = np.arange(n)
    E0 = 0.01 + 0.99 * event.draw(seed, h, np.zeros(n, np.int64), 0)
    mu = 1.25 * (0.8 + 0.2 * np.log(0.2))
    ratio = np.mean(np.log(E0 / e_end)) / np.mean(coll)
    assert abs(ratio - mu) < 0.01, (ratio, mu)
