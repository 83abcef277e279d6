"""Pins: checks of the CPU oracle against facts it does not compute itself.

Each pin takes an oracle library handle (`oracle.load()` or a deliberately
broken build of the same source) and raises AssertionError when the oracle
disagrees with what the mathematics fixes.  The paper prints no worked
lookup (section 5.1 names the operation only), so the pins are:

* brute force: the bracket by counting equals bisection and
  numpy.searchsorted on every probe of tiny grids;
* closed forms: grid-point queries return the tabulated values exactly,
  clamped queries return the end values, affine data is reproduced within a
  few ulp, exact midpoints give the rounded mean;
* invariants: scaling all densities by 2^s scales the result exactly;
  splitting a material's list adds up within L ulp;
* exact arithmetic: rational evaluation of the definition bounds the
  rounding error; numpy.interp (a different formula) agrees within the same
  bound;
* the FP32 form stays within its error bound of the FP64 result, also on a
  sum of many equal terms where uncompensated FP32 summation fails;
* a hand-worked example (tests/golden/worked_example.txt), and one of the
  FP32 form with exact expected bits (tests/golden/worked_example_f32.txt).
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

import oracle
import synth

U64 = 2.0 ** -53
U32 = 2.0 ** -24
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _single_nuclide_materials(t: synth.Tables) -> synth.Tables:
    """Same nuclides, one material per nuclide with density 1.0."""
    K = t.n_nuclides
    return synth.Tables(t.grid_offsets, t.energy, t.xs,
                        np.arange(K + 1, dtype=np.int32),
                        np.arange(K, dtype=np.int32), np.ones(K))


def _probes(g: np.ndarray) -> np.ndarray:
    pts = list(g)
    pts += [np.nextafter(x, np.inf) for x in g]
    pts += [np.nextafter(x, -np.inf) for x in g]
    pts += list(0.5 * (g[1:] + g[:-1]))
    pts += [g[0] * 0.5, g[0] * 1e-3, g[-1] * 2.0, g[-1] * 1e6,
            np.nextafter(0.0, 1.0), 1e300]
    return np.asarray(pts, dtype=np.float64)


def pin_bracket_brute(lib):
    """count == bisect == clip(searchsorted(g, e, 'right') - 1, 0, n-2)."""
    s = synth.Stream(7, 1)
    for n in (2, 3, 4, 5, 8, 17, 64):
        grids = [np.arange(1, n + 1, dtype=np.float64),
                 np.sort(s.log_uniform(n, 1e-5, 1.0)),
                 np.cumsum(s.uniform_open0(n))]
        for g in grids:
            assert np.all(np.diff(g) > 0)
            for e in _probes(g):
                want = int(np.clip(np.searchsorted(g, e, side="right") - 1,
                                   0, n - 2))
                c = oracle.bracket_count(g, e, lib=lib)
                b = oracle.bracket_bisect(g, e, lib=lib)
                assert c == want, (n, e, c, want)
                assert b == want, (n, e, b, want)


def pin_lookup_index_brute(lib):
    """Indices reported by the lookup equal the counting definition."""
    t = synth.random_tables(11, 5, [2, 3, 9, 40, 200], 4)
    ts = _single_nuclide_materials(t)
    for k in range(t.n_nuclides):
        g = t.grid(k)
        E = _probes(g)
        m = np.full(len(E), k, dtype=np.int32)
        _, idx, _ = oracle.lookup(ts, E, m, with_index=True, lib=lib)
        _, idx_c, _ = oracle.lookup(ts, E, m, search="count", with_index=True,
                                    lib=lib)
        want = np.clip(np.searchsorted(g, E, side="right") - 1, 0, len(g) - 2)
        assert np.array_equal(idx, want)
        assert np.array_equal(idx_c, want)


def pin_grid_points_exact(lib):
    """At E = E_k[p] a one-nuclide, density-1 material returns X_k[p] exactly,
    for every p including the last one (f = 1, g = 0)."""
    t = synth.random_tables(12, 4, [2, 3, 17, 300], 2)
    ts = _single_nuclide_materials(t)
    for k in range(t.n_nuclides):
        g = t.grid(k)
        out = oracle.lookup(ts, g, np.full(len(g), k, np.int32), lib=lib)
        assert np.array_equal(out, t.channels(k)), k


def pin_clamp(lib):
    """Energies outside the grid take the end values exactly."""
    t = synth.random_tables(13, 3, [2, 5, 50], 2)
    ts = _single_nuclide_materials(t)
    for k in range(t.n_nuclides):
        g, X = t.grid(k), t.channels(k)
        E = np.array([g[0] * 0.5, np.nextafter(g[0], 0), g[0] * 1e-9,
                      g[-1] * 2.0, np.nextafter(g[-1], np.inf), 1e200])
        out = oracle.lookup(ts, E, np.full(len(E), k, np.int32), lib=lib)
        assert np.array_equal(out[:3], np.repeat(X[:1], 3, axis=0))
        assert np.array_equal(out[3:], np.repeat(X[-1:], 3, axis=0))


def _round_fraction(x: Fraction) -> float:
    return float(x)  # Fraction -> float rounds to nearest


def pin_affine(lib):
    """X_k[p][c] = a_c + b_c E_k[p] with a, b > 0 is reproduced between the
    nodes: |sigma(E) - (a + b E)| <= 10 u (a + b E)."""
    s = synth.Stream(14, 1)
    g = np.concatenate(([1e-5], np.sort(s.log_uniform(98, 1e-5, 1.0)), [1.0]))
    a = np.array([0.5, 1.0, 2.0, 3.0, 0.125])
    b = np.array([1.0, 7.0, 0.25, 100.0, 3.0])
    X = a[None, :] + b[None, :] * g[:, None]
    t = synth.Tables(np.array([0, len(g)], np.int64), g, X,
                     np.array([0, 1], np.int32), np.array([0], np.int32),
                     np.array([1.0]))
    E = s.log_uniform(2000, 1e-5, 1.0)
    out = oracle.lookup(t, E, np.zeros(len(E), np.int32), lib=lib)
    want = a[None, :] + b[None, :] * E[:, None]
    assert np.all(np.abs(out - want) <= 10 * U64 * want)


def pin_constant(lib):
    """Constant data c comes back within 3 ulp of c anywhere."""
    s = synth.Stream(15, 1)
    g = np.concatenate(([1e-5], np.sort(s.log_uniform(30, 1e-5, 1.0)), [1.0]))
    c = np.array([0.75, 1.0, 0.1, 3.3, 1e-3])
    X = np.repeat(c[None, :], len(g), axis=0)
    t = synth.Tables(np.array([0, len(g)], np.int64), g, X,
                     np.array([0, 1], np.int32), np.array([0], np.int32),
                     np.array([1.0]))
    E = s.log_uniform(3000, 1e-6, 2.0)
    out = oracle.lookup(t, E, np.zeros(len(E), np.int32), lib=lib)
    assert np.all(np.abs(out - c[None, :]) <= 3 * U64 * c[None, :])


def pin_midpoint(lib):
    """On an integer grid, E halfway between nodes gives f = 1/2 exactly and
    the channel equals the correctly rounded mean of the two nodes."""
    g = np.array([1.0, 2.0, 3.0, 5.0, 8.0, 13.0])
    s = synth.Stream(16, 1)
    X = s.lognormal(len(g) * 5).reshape(-1, 5)
    t = synth.Tables(np.array([0, len(g)], np.int64), g, X,
                     np.array([0, 1], np.int32), np.array([0], np.int32),
                     np.array([1.0]))
    E = 0.5 * (g[1:] + g[:-1])
    out = oracle.lookup(t, E, np.zeros(len(E), np.int32), lib=lib)
    for q in range(len(E)):
        for c in range(5):
            want = _round_fraction((Fraction(X[q, c]) + Fraction(X[q + 1, c]))
                                   / 2)
            assert out[q, c] == want, (q, c)


def pin_density_scaling(lib):
    """Scaling every density by 2^s scales every sum by 2^s, bit for bit."""
    t = synth.random_tables(17, 6, 40, 4)
    q = synth.random_queries(17, t, 3000)
    base = oracle.lookup(t, q.E, q.mat, lib=lib)
    for sh in (-8, -3, -1, 1, 2, 8):
        ts = synth.Tables(t.grid_offsets, t.energy, t.xs, t.mat_offsets,
                          t.mat_nuclides, t.mat_density * 2.0 ** sh)
        out = oracle.lookup(ts, q.E, q.mat, lib=lib)
        assert np.array_equal(out, base * 2.0 ** sh), sh


def pin_additivity(lib):
    """A material equals the sum of its list's prefix and suffix within L u
    (all terms are positive)."""
    t = synth.random_tables(18, 12, 60, 1, sizes=[12])
    nuc, rho = t.material(0)
    q = synth.random_queries(18, t, 2000)
    q.mat[:] = 0
    full = oracle.lookup(t, q.E, q.mat, lib=lib)
    for cut in (1, 5, 11):
        parts = synth.Tables(t.grid_offsets, t.energy, t.xs,
                             np.array([0, cut, len(nuc)], np.int32), nuc, rho)
        a = oracle.lookup(parts, q.E, np.zeros(len(q), np.int32), lib=lib)
        b = oracle.lookup(parts, q.E, np.ones(len(q), np.int32), lib=lib)
        assert np.all(np.abs(full - (a + b)) <= (len(nuc) + 1) * U64 * full)


def exact_lookup(t: synth.Tables, e: float, m: int):
    """The definition evaluated in exact rational arithmetic.

    Returns (S_exact [5] Fractions, conditioning [5] = sum rho |hi - lo|,
    bracket list)."""
    nuc, rho = t.material(m)
    S = [Fraction(0)] * 5
    cond = [0.0] * 5
    idx = []
    E = Fraction(e)
    for k, r in zip(nuc, rho):
        g = t.grid(int(k))
        X = t.channels(int(k))
        n = len(g)
        count = sum(1 for x in g if Fraction(x) <= E)
        i = min(max(count - 1, 0), n - 2)
        idx.append(i)
        Eh = min(max(E, Fraction(g[0])), Fraction(g[-1]))
        f = (Eh - Fraction(g[i])) / (Fraction(g[i + 1]) - Fraction(g[i]))
        for c in range(5):
            lo, hi = Fraction(X[i, c]), Fraction(X[i + 1, c])
            S[c] += Fraction(r) * ((1 - f) * lo + f * hi)
            cond[c] += float(r) * abs(float(X[i + 1, c]) - float(X[i, c]))
    return S, cond, idx


def pin_exact_rational(lib):
    """|S - S_exact| <= (L + 8) u S_exact + 4 u sum_j rho_j |hi_j - lo_j|,
    and the indices equal the exact brackets."""
    t = synth.random_tables(19, 5, [2, 3, 9, 20, 33], 3, sizes=[1, 3, 5])
    s = synth.Stream(19, 2)
    E = np.concatenate((s.log_uniform(150, 1e-5, 1.0),
                        t.grid(3)[::3], t.grid(2),
                        [1e-7, 3.0, 1.0, 1e-5]))
    m = s.integers(len(E), 0, 2).astype(np.int32)
    out, idx, off = oracle.lookup(t, E, m, with_index=True, lib=lib)
    for q in range(len(E)):
        S, cond, bi = exact_lookup(t, float(E[q]), int(m[q]))
        L = len(bi)
        assert list(idx[off[q]:off[q + 1]]) == bi, q
        for c in range(5):
            err = abs(Fraction(out[q, c]) - S[c])
            bound = (L + 8) * U64 * float(S[c]) + 4 * U64 * cond[c]
            assert float(err) <= bound, (q, c, float(err), bound)


def numpy_interp_sum(t: synth.Tables, E: np.ndarray, mat: np.ndarray):
    """sum_j rho_j numpy.interp(E, E_k, X_k[:, c]) per query, and the
    conditioning sum_j rho_j |X_k[i+1, c] - X_k[i, c]|."""
    out = np.zeros((len(E), 5))
    cond = np.zeros((len(E), 5))
    for m in range(t.n_materials):
        sel = np.nonzero(mat == m)[0]
        if len(sel) == 0:
            continue
        nuc, rho = t.material(m)
        for k, r in zip(nuc, rho):
            g, X = t.grid(int(k)), t.channels(int(k))
            i = np.clip(np.searchsorted(g, E[sel], side="right") - 1, 0,
                        len(g) - 2)
            for c in range(5):
                out[sel, c] += r * np.interp(E[sel], g, X[:, c])
                cond[sel, c] += r * np.abs(X[i + 1, c] - X[i, c])
    return out, cond


def pin_numpy_interp(lib, n: int = 100_000):
    """Config-1 tables and queries: the oracle agrees with a numpy.interp sum
    within (L + 8) u S + 4 u cond (+ the numpy side's own rounding)."""
    t = synth.config1_tables()
    q = synth.config1_queries(n)
    out = oracle.lookup(t, q.E, q.mat, lib=lib)
    ref, cond = numpy_interp_sum(t, q.E, q.mat)
    L = t.material_sizes()[q.mat][:, None]
    bound = 2 * ((L + 8) * U64 * ref + 4 * U64 * cond)
    assert np.all(np.abs(out - ref) <= bound)


def pin_f32_bound(lib, n: int = 100_000):
    """The FP32 form is within 9 u32 relative of the FP64 result, per
    channel (rounded tables 2u, f and g 2u, two products and an add 3u,
    density and its product 2u, compensated sum 2u; 9u32 ~ 5.4e-7)."""
    t = synth.config1_tables()
    q = synth.config1_queries(n)
    ref = oracle.lookup(t, q.E, q.mat, lib=lib)
    f32 = oracle.lookup_f32(t, q.E, q.mat, lib=lib).astype(np.float64)
    rel = np.abs(f32 - ref) / ref
    assert rel.max() <= 9 * U32, rel.max()


def pin_f32_many_terms(lib):
    """2,000 nuclides with equal data: uncompensated FP32 summation drifts
    by ~1e-5 here; the compensated sum must stay within 9 u32."""
    K = 2000
    g = np.tile(np.array([1e-5, 1.0]), K)
    X = np.full((2 * K, 5), 0.1)
    X[:, 1] = 0.3
    X[:, 2] = 1.0 / 3.0
    X[:, 3] = 0.7
    X[:, 4] = 1.1
    t = synth.Tables(np.arange(K + 1, dtype=np.int64) * 2, g, X,
                     np.array([0, K], np.int32), np.arange(K, dtype=np.int32),
                     np.full(K, 0.1))
    E = np.array([1e-5, 0.3, 0.77, 1.0])
    m = np.zeros(len(E), np.int32)
    ref = oracle.lookup(t, E, m, lib=lib)
    f32 = oracle.lookup_f32(t, E, m, lib=lib).astype(np.float64)
    assert np.all(np.abs(f32 - ref) <= 9 * U32 * ref)


def pin_f32_skewed_interval(lib):
    """One interval whose low end is 1e4 times its high end, queried close to
    the high end: g = 1 - f must be formed before rounding to FP32 (forming
    it in FP32 costs ~u32 * lo / hi relative)."""
    g = np.array([1e-5, 1.0])
    X = np.array([[1e4, 2e4, 5e3, 1e4, 3e4], [1.0, 1.5, 0.7, 1.0, 2.0]])
    t = synth.Tables(np.array([0, 2], np.int64), g, X,
                     np.array([0, 1], np.int32), np.array([0], np.int32),
                     np.array([1.0]))
    E = 1.0 - np.array([1e-4, 3e-5, 1.7e-5, 1e-3, 0.3333e-4])
    m = np.zeros(len(E), np.int32)
    ref = oracle.lookup(t, E, m, lib=lib)
    f32 = oracle.lookup_f32(t, E, m, lib=lib).astype(np.float64)
    assert np.all(np.abs(f32 - ref) <= 9 * U32 * ref)


def _num(v: str) -> float:
    """A decimal or hexadecimal (0x1.8p-1) floating-point literal."""
    return float.fromhex(v) if "0x" in v.lower() else float(v)


def read_worked_example(path: str = None):
    """Parse tests/golden/worked_example.txt (or another file of that
    format, such as worked_example_f32.txt)."""
    path = path or os.path.join(GOLDEN, "worked_example.txt")
    grids, xs, mats, queries = [], [], [], []
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        kind, *rest = line.split()
        if kind == "nuclide":
            grids.append([_num(v) for v in rest])
            xs.append([])
        elif kind == "point":
            xs[-1].append([_num(v) for v in rest])
        elif kind == "material":
            ids, dens = rest[0].split(","), rest[1].split(",")
            mats.append(([int(v) for v in ids], [_num(v) for v in dens]))
        elif kind == "query":
            e, m = _num(rest[0]), int(rest[1])
            idx = [int(v) for v in rest[2].split(",")]
            want = [_num(v) for v in rest[3:8]]
            queries.append((e, m, idx, want))
    offs = np.zeros(len(grids) + 1, np.int64)
    offs[1:] = np.cumsum([len(g) for g in grids])
    mo = np.zeros(len(mats) + 1, np.int32)
    mo[1:] = np.cumsum([len(a) for a, _ in mats])
    t = synth.Tables(offs, np.concatenate(grids), np.concatenate(xs),
                     mo, np.concatenate([a for a, _ in mats]).astype(np.int32),
                     np.concatenate([b for _, b in mats]))
    return t, queries


def pin_worked_example(lib):
    """The hand-worked example: indices and sums exactly as derived."""
    t, queries = read_worked_example()
    E = np.array([q[0] for q in queries])
    m = np.array([q[1] for q in queries], np.int32)
    out, idx, off = oracle.lookup(t, E, m, with_index=True, lib=lib)
    for r, (e, mm, want_idx, want) in enumerate(queries):
        assert list(idx[off[r]:off[r + 1]]) == want_idx, (e, mm)
        assert list(out[r]) == want, (e, mm, list(out[r]), want)


def pin_f32_worked_example(lib):
    """The hand-worked FP32 example (tests/golden/worked_example_f32.txt):
    dyadic tables whose channel values and densities carry bits beyond
    FP32's significand, so rounding X and rho to FP32 before the products,
    the ties to even and the Kahan compensation each show in the expected
    bits of the sums."""
    t, queries = read_worked_example(
        os.path.join(GOLDEN, "worked_example_f32.txt"))
    E = np.array([q[0] for q in queries])
    m = np.array([q[1] for q in queries], np.int32)
    got = oracle.lookup_f32(t, E, m, lib=lib)
    _, idx, off = oracle.lookup(t, E, m, with_index=True, lib=lib)
    for r, (e, mm, want_idx, want) in enumerate(queries):
        assert list(idx[off[r]:off[r + 1]]) == want_idx, (e, mm)
        w = np.array(want, dtype=np.float64)
        assert np.array_equal(w.astype(np.float32).astype(np.float64), w), \
            "an expected value is not an FP32 number"
        assert np.array_equal(got[r].view(np.uint32),
                              w.astype(np.float32).view(np.uint32)), \
            (e, mm, [float(x).hex() for x in got[r]],
             [float(x).hex() for x in w])


def pin_invalid_inputs(lib):
    """E not finite or not > 0, or m out of range: NaN outputs, index -1."""
    t = synth.random_tables(20, 3, 10, 2, sizes=[2, 3])
    E = np.array([np.nan, -1.0, 0.0, np.inf, 0.5, 0.5, 0.5])
    m = np.array([0, 1, 0, 1, 2, -1, 1], np.int32)
    out, idx, off = oracle.lookup(t, E, m, with_index=True, lib=lib)
    assert np.all(np.isnan(out[:6]))
    assert np.all(np.isfinite(out[6]))
    assert np.all(idx[off[0]:off[4]] == -1)
    assert off[5] == off[4] and off[6] == off[5]


ALL_PINS = [
    pin_bracket_brute, pin_lookup_index_brute, pin_grid_points_exact,
    pin_clamp, pin_affine, pin_constant, pin_midpoint, pin_density_scaling,
    pin_additivity, pin_exact_rational, pin_numpy_interp, pin_f32_bound,
    pin_f32_many_terms, pin_f32_skewed_interval, pin_worked_example,
    pin_f32_worked_example, pin_invalid_inputs,
]


def run_all(lib_path: str, quick: bool = True) -> list:
    """Run every pin against the library at lib_path; return failing names."""
    lib = oracle.load(lib_path)
    failed = []
    for pin in ALL_PINS:
        try:
            if quick and pin in (pin_numpy_interp, pin_f32_bound):
                pin(lib, n=20_000)
            else:
                pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    return failed
