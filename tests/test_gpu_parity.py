"""HIP lookup against the CPU oracle, through the C interface.

Bars (fixed here, from the requirements of the lookup):
  * brackets: bit-exact for every grid method;
  * FP64 sums: <= 1e-12 relative per channel, and in fact bit-identical
    (same operations in the same order, correctly rounded division, no fused
    multiply-add on either side);
  * FP32 form: bit-identical to the oracle's FP32 form and <= 2e-6 relative to
    the FP64 oracle per channel;
  * sort policy, threshold, block size and lookups per thread never change a
    single bit of the output.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

FP64_TOL = 1e-12
FP32_TOL = 2e-6
ALL_FLAGS = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype,
                                                       device="cuda:0")


def run(tables, E, m, **kw):
    prec = kw.pop("precision", xs.XS_FP64)
    p = xs.make_params(precision=prec, **kw)
    out = xs.xs_lookup_batch(tables, E, m, params=p)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def rel_err(got, ref):
    return np.abs(got.astype(np.float64) - ref) / np.abs(ref)


@pytest.fixture(scope="module")
def cfg1():
    t = synth.config1_tables()
    q = synth.config1_queries()
    say("cfg1: building tables (all structures, 4000 hash bins)")
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    ref = oracle.lookup(t, q.E, q.mat)
    ref32 = oracle.lookup_f32(t, q.E, q.mat)
    return dict(t=t, q=q, h=h, E=dev(q.E, torch.float64),
                m=dev(q.mat, torch.int32), ref=ref, ref32=ref32)


@pytest.mark.parametrize("grid", ["nuclide", "hash", "unionized"])
def test_cfg1_fp64_matches_oracle(cfg1, grid):
    say("cfg1 fp64", grid)
    out = run(cfg1["h"], cfg1["E"], cfg1["m"], grid=grid, sort="none",
              block_size=256, lookups_per_thread=1)
    assert rel_err(out, cfg1["ref"]).max() <= FP64_TOL
    assert np.array_equal(out, cfg1["ref"])


@pytest.mark.parametrize("grid", ["nuclide", "hash", "unionized"])
def test_cfg1_fp32_matches_oracle(cfg1, grid):
    say("cfg1 fp32", grid)
    out = run(cfg1["h"], cfg1["E"], cfg1["m"], precision=xs.XS_FP32, grid=grid,
              sort="material_energy", block_size=256, lookups_per_thread=2)
    assert out.dtype == np.float32
    err = rel_err(out, cfg1["ref"])
    say("fp32 rel err max per channel", err.max(axis=0), "mean", err.mean(axis=0))
    assert err.max() <= FP32_TOL
    assert np.array_equal(out, cfg1["ref32"])


@pytest.mark.parametrize("grid", ["nuclide", "hash", "unionized"])
def test_cfg1_indices_bit_exact(cfg1, grid):
    say("cfg1 indices", grid)
    t, q = cfg1["t"], cfg1["q"]
    _, idx_ref, off = oracle.lookup(t, q.E, q.mat, with_index=True)
    idx = xs.xs_lookup_indices(cfg1["h"], cfg1["E"], cfg1["m"],
                               dev(off, torch.int64), grid=grid)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), idx_ref)


KNOBS = [
    dict(sort="none", block_size=64, lookups_per_thread=1, unroll=1),
    dict(sort="none", block_size=512, lookups_per_thread=2, unroll=1),
    dict(sort="material", sort_threshold=0, block_size=128, lookups_per_thread=3),
    dict(sort="energy", sort_threshold=0, block_size=512, lookups_per_thread=4),
    dict(sort="material_energy", sort_threshold=0, block_size=256,
         lookups_per_thread=8),
    dict(sort="band_material", sort_threshold=0, block_size=256,
         lookups_per_thread=1, unroll=4),
    dict(sort="band_material", sort_threshold=0, block_size=256,
         lookups_per_thread=2, unroll=2),
    dict(sort="none", block_size=512, lookups_per_thread=1, unroll=2),
    dict(sort="material_energy", sort_threshold=xs.INT64_MAX, block_size=192,
         lookups_per_thread=5),
    dict(sort="band_material", sort_threshold=20000, block_size=64,
         lookups_per_thread=7),
    dict(sort="energy", sort_threshold=0, block_size=256, lookups_per_thread=2,
         unroll=4),
    dict(sort="band_material", sort_threshold=0, block_size=256,
         lookups_per_thread=1, unroll=1, lds_stage=1),
    dict(sort="none", block_size=128, lookups_per_thread=1, unroll=1,
         lds_stage=1),
    dict(sort="material_energy", sort_threshold=0, block_size=1024,
         lookups_per_thread=1, unroll=1, lds_stage=1),
    dict(sort="band_material", sort_threshold=0, block_size=128,
         lookups_per_thread=2, unroll=1, lds_stage=1),
    dict(sort="none", block_size=512, lookups_per_thread=2, unroll=1,
         lds_stage=1),
    dict(sort="band_material", sort_threshold=0, block_size=64,
         lookups_per_thread=1, unroll=1, lds_stage=2),
    dict(sort="material_energy", sort_threshold=0, block_size=256,
         lookups_per_thread=2, unroll=1, lds_stage=2),
    dict(sort="band_material", sort_threshold=0, block_size=128,
         lookups_per_thread=1, unroll=1, lds_stage=3),
    dict(sort="none", block_size=1024, lookups_per_thread=1, unroll=1,
         lds_stage=3),
    dict(sort="band_material", sort_threshold=0, block_size=512,
         lookups_per_thread=2, unroll=1, lds_stage=3),
    dict(sort="none", block_size=256, lookups_per_thread=1, unroll=1,
         lds_stage=0, wave_per_lookup=1),
    dict(sort="band_material", sort_threshold=0, block_size=64,
         lookups_per_thread=1, unroll=1, lds_stage=0, wave_per_lookup=1),
]


@pytest.mark.parametrize("precision", [xs.XS_FP64, xs.XS_FP32])
@pytest.mark.parametrize("grid", ["nuclide", "hash", "unionized"])
def test_knobs_never_change_bits(cfg1, grid, precision):
    say("knobs", grid, precision)
    ref = cfg1["ref"] if precision == xs.XS_FP64 else cfg1["ref32"]
    for k in KNOBS:
        out = run(cfg1["h"], cfg1["E"], cfg1["m"], precision=precision,
                  grid=grid, **k)
        assert np.array_equal(out, ref), k


def test_default_params(cfg1):
    out = xs.xs_lookup_batch(cfg1["h"], cfg1["E"], cfg1["m"])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), cfg1["ref"])
    # one query per lane or more: banded sort, LDS-staged windows (wider
    # ones for sparser batches), union grid when built
    for n, shape in ((300000, 3), (2000000, 2), (10000000, 1)):
        p = xs.xs_resolve_params(cfg1["h"], n)
        assert p.grid == xs.XS_GRID_UNIONIZED and p.block_size == 128
        assert p.sort == xs.XS_SORT_BAND_MATERIAL and p.unroll == 1
        assert p.lds_stage == shape and p.wave_per_lookup == 0
        assert p.sort_threshold == 20000 and p.lookups_per_thread == 1
    # explicit fields that exclude staging keep one lane per query unstaged
    for kw in (dict(lookups_per_thread=4), dict(unroll=2),
               dict(wave_per_lookup=1, block_size=128)):
        p = xs.xs_resolve_params(cfg1["h"], 300000, xs.make_params(**kw))
        assert p.lds_stage == 0, kw
    out = xs.xs_lookup_batch(cfg1["h"], cfg1["E"], cfg1["m"],
                             params=xs.make_params(lookups_per_thread=4))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), cfg1["ref"])
    # fewer queries than lanes on the chip: one wave per query, unsorted
    p = xs.xs_resolve_params(cfg1["h"], 100000)
    assert p.grid == xs.XS_GRID_UNIONIZED and p.block_size == 128
    assert p.sort == xs.XS_SORT_NONE and p.wave_per_lookup == 1
    assert p.unroll == 1 and p.lookups_per_thread == 1
    # explicit fields that exclude it keep one lane per query
    for kw in (dict(lookups_per_thread=2), dict(block_size=512),
               dict(unroll=2), dict(lds_stage=1)):
        p = xs.xs_resolve_params(cfg1["h"], 100000, xs.make_params(**kw))
        assert p.wave_per_lookup == 0, kw


def test_edge_queries(cfg1):
    """Grid points of every nuclide, their neighbours, out-of-range energies,
    invalid energies and materials."""
    t = cfg1["t"]
    pts = []
    for k in range(t.n_nuclides):
        g = t.grid(k)
        pts += [g, np.nextafter(g, 0), np.nextafter(g, np.inf)]
    E = np.concatenate(pts + [np.array([1e-9, 1e-6, 2.0, 1e30])])
    m = np.arange(len(E), dtype=np.int32) % t.n_materials
    E2 = np.concatenate([E, [np.nan, -1.0, 0.0, np.inf, 0.5, 0.5]])
    m2 = np.concatenate([m, np.array([0, 1, 2, 3, 4, -1], np.int32)])
    ref = oracle.lookup(t, E2, m2)
    ref32 = oracle.lookup_f32(t, E2, m2)
    # every launch shape: the LDS-staged kernel's block edges then fall on
    # grid points, below the lowest and above the highest union-grid energy
    for grid in ("nuclide", "hash", "unionized"):
        for k in KNOBS:
            out = run(cfg1["h"], dev(E2, torch.float64), dev(m2, torch.int32),
                      grid=grid, **k)
            np.testing.assert_array_equal(out, ref)
            out = run(cfg1["h"], dev(E2, torch.float64), dev(m2, torch.int32),
                      precision=xs.XS_FP32, grid=grid, **k)
            np.testing.assert_array_equal(out, ref32)
    assert np.all(np.isnan(ref[-6:]))


@pytest.mark.parametrize("shape", [dict(lookups_per_thread=1, block_size=128,
                                         lds_stage=1),
                                    dict(lookups_per_thread=2, block_size=64,
                                         lds_stage=3)])
@pytest.mark.parametrize("invalid", [0.0, 0.05])
def test_staged_blocks_of_several_materials(cfg1, shape, invalid):
    """Sorted, LDS-staged batches: a block that straddles two groups of the
    sort key (or holds invalid queries) takes the per-lane walk instead of
    the staged one; with 5 % invalid queries spread over the batch most
    blocks are of that kind.  Every valid query matches the oracle, every
    invalid one is NaN, in both precisions and every grid."""
    say("mixed blocks", shape, invalid)
    t, q = cfg1["t"], cfg1["q"]
    E = q.E.copy()
    m = q.mat.copy()
    bad = np.zeros(len(E), bool)
    if invalid:
        pick = synth.Stream(41, 2).uniform(len(E)) < invalid
        bad = pick
        E[pick & (np.arange(len(E)) % 2 == 0)] = -1.0
        m[pick & (np.arange(len(E)) % 2 == 1)] = t.n_materials
    ref = oracle.lookup(t, E, m)
    ref32 = oracle.lookup_f32(t, E, m)
    Ed, md = dev(E, torch.float64), dev(m, torch.int32)
    for grid in ("unionized", "nuclide", "hash"):
        for sort in ("band_material", "material_energy"):
            for prec, want in ((xs.XS_FP64, ref), (xs.XS_FP32, ref32)):
                out = run(cfg1["h"], Ed, md, precision=prec, grid=grid,
                          sort=sort, sort_threshold=0, unroll=1, **shape)
                np.testing.assert_array_equal(out, want)
    assert np.isnan(ref[bad]).all() and not np.isnan(ref[~bad]).any()


def test_empty_and_tiny(cfg1):
    h = cfg1["h"]
    E = cfg1["E"][:0]
    m = cfg1["m"][:0]
    out = xs.xs_lookup_batch(h, E, m)
    assert out.shape == (0, 5)
    for n in (1, 2, 63, 65, 257, 4097):
        out = run(h, cfg1["E"][:n], cfg1["m"][:n], sort="material_energy",
                  sort_threshold=0, lookups_per_thread=3, block_size=64)
        assert np.array_equal(out, cfg1["ref"][:n]), n


def test_degenerate_tables():
    """Two-point nuclides, one-nuclide materials, one hash bin, one material."""
    t = synth.random_tables(31, 6, [2, 2, 3, 50, 2, 700], 5,
                            sizes=[1, 6, 2, 1, 3])
    q = synth.random_queries(31, t, 50_001, lo=1e-6, hi=3.0)
    ref = oracle.lookup(t, q.E, q.mat)
    ref32 = oracle.lookup_f32(t, q.E, q.mat)
    E, m = dev(q.E, torch.float64), dev(q.mat, torch.int32)
    for bins in (1, 100, 4000, 100000):
        h = xs.xs_create_tables(t, ALL_FLAGS, bins)
        for grid in ("nuclide", "hash", "unionized"):
            out = run(h, E, m, grid=grid, sort="material_energy", sort_threshold=0)
            assert np.array_equal(out, ref), (bins, grid)
            out = run(h, E, m, precision=xs.XS_FP32, grid=grid, sort="none")
            assert np.array_equal(out, ref32), (bins, grid)
        h.close()
    one = synth.random_tables(32, 3, 40, 1, sizes=[3])
    q1 = synth.random_queries(32, one, 1000)
    h = xs.xs_create_tables(one, ALL_FLAGS, 64)
    out = run(h, dev(q1.E, torch.float64), dev(q1.mat, torch.int32),
              sort="material_energy", sort_threshold=0)
    assert np.array_equal(out, oracle.lookup(one, q1.E, q1.mat))


@pytest.mark.parametrize("bins", [1, 100, 4000, 8192, 100000])
def test_hash_bins_indices(cfg1, bins):
    t, q = cfg1["t"], cfg1["q"]
    _, idx_ref, off = oracle.lookup(t, q.E[:20000], q.mat[:20000], with_index=True)
    h = xs.xs_create_tables(t, xs.XS_BUILD_HASH, bins)
    idx = xs.xs_lookup_indices(h, cfg1["E"][:20000], cfg1["m"][:20000],
                               dev(off, torch.int64), grid="hash")
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    h.close()


def test_union_bin_edges(cfg1):
    """Energies at and next to every edge of the logarithmic bins over the
    union grid (about 32 union points per bin), where the rounding of log
    decides the bin: brackets and sums stay the oracle's in every kernel
    that searches the union grid per lookup."""
    say("union bin edges")
    t = cfg1["t"]
    u = np.unique(t.energy)
    U = xs.xs_table_info(cfg1["h"])["union_size"]
    assert U == len(u)
    UB = max(1, min(U // 32, 1 << 20))
    uln = np.log(u[0])
    step = (np.log(u[-1]) - uln) / UB
    edges = np.exp(uln + np.arange(UB + 1) * step)
    E = np.concatenate([edges, np.nextafter(edges, 0), np.nextafter(edges, np.inf),
                        u[::7], np.nextafter(u[::7], 0)])
    E = E[(E > 0) & np.isfinite(E)]
    m = (np.arange(len(E)) % t.n_materials).astype(np.int32)
    ref, idx_ref, off = oracle.lookup(t, E, m, with_index=True)
    Ed, md = dev(E, torch.float64), dev(m, torch.int32)
    idx = xs.xs_lookup_indices(cfg1["h"], Ed, md, dev(off, torch.int64),
                               grid="unionized")
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    for k in (dict(sort="none", lookups_per_thread=1, unroll=2),
              dict(sort="none", lookups_per_thread=1, unroll=1, lds_stage=0,
                   wave_per_lookup=1, block_size=128)):
        out = run(cfg1["h"], Ed, md, grid="unionized", **k)
        assert np.array_equal(out, ref), k


@pytest.mark.parametrize("queue", [xs.XS_QUEUE_COMPACT, xs.XS_QUEUE_PREDICATED])
@pytest.mark.parametrize("sort", ["none", "material_energy", "band_material"])
@pytest.mark.parametrize("frac", [0.3, 0.0, 1.0])
def test_active_mask(cfg1, queue, sort, frac):
    """Inactive slots keep their sentinel; active ones match the oracle.
    A compacted queue, or a sorted one whose inactive lookups go last,
    serves only its active head (a device-side count, or block ranges of
    the groups without the inactive flag): none, some or all active, in
    the per-lane, LDS-staged and one-wave-per-lookup kernels."""
    n = len(cfg1["q"])
    s = synth.Stream(33, 1)
    act = (s.uniform(n) < frac).astype(np.uint8)
    sentinel = -7.25
    for prec, ref in ((xs.XS_FP64, cfg1["ref"]), (xs.XS_FP32, cfg1["ref32"])):
        dt = torch.float64 if prec == xs.XS_FP64 else torch.float32
        for shape in (dict(lookups_per_thread=2),
                      dict(grid="unionized", lookups_per_thread=1, unroll=1,
                           lds_stage=1, block_size=128),
                      dict(grid="unionized", lookups_per_thread=1, unroll=1,
                           lds_stage=3, block_size=64),
                      dict(grid="unionized", lookups_per_thread=1, unroll=1,
                           wave_per_lookup=1, block_size=128)):
            out = torch.full((n, 5), sentinel, dtype=dt, device="cuda:0")
            p = xs.make_params(precision=prec, sort=sort, sort_threshold=0,
                               queue=queue, **shape)
            xs.xs_lookup_active(cfg1["h"], cfg1["E"], cfg1["m"],
                                dev(act, torch.uint8), out, params=p)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            a = act.astype(bool)
            assert np.all(o[~a] == sentinel), shape
            assert np.array_equal(o[a], ref[a]), shape


def test_errors_from_device_calls(cfg1):
    h = cfg1["h"]
    with pytest.raises(xs.XsError) as e:
        xs.xs_lookup_batch(h, cfg1["E"], cfg1["m"],
                           params=xs.make_params(block_size=100))
    assert e.value.status == xs.XS_EINVAL
    for bad in (dict(block_size=1024, lookups_per_thread=5),
                dict(block_size=1024, lookups_per_thread=2, unroll=2),
                dict(lookups_per_thread=3, unroll=2), dict(unroll=3),
                dict(sort=5), dict(grid=3), dict(lds_stage=4),
                dict(lds_stage=-2),
                dict(lds_stage=1, lookups_per_thread=3),
                dict(lds_stage=1, lookups_per_thread=2, block_size=1024),
                dict(lds_stage=1, unroll=2), dict(wave_per_lookup=2),
                dict(wave_per_lookup=1, block_size=512, unroll=1),
                dict(wave_per_lookup=1, lookups_per_thread=2, unroll=1),
                dict(wave_per_lookup=1, unroll=2),
                dict(wave_per_lookup=1, lds_stage=1, unroll=1)):
        with pytest.raises(xs.XsError) as e:
            xs.xs_lookup_batch(h, cfg1["E"], cfg1["m"],
                               params=xs.make_params(**bad))
        assert e.value.status == xs.XS_EINVAL, bad
    small = xs.xs_create_tables(cfg1["t"], 0, 0)
    for p in (xs.make_params(grid="hash"), xs.make_params(grid="unionized"),
              xs.make_params(precision=xs.XS_FP32, grid="nuclide")):
        with pytest.raises(xs.XsError) as e:
            xs.xs_lookup_batch(small, cfg1["E"], cfg1["m"], params=p)
        assert e.value.status == xs.XS_ENOTBUILT
    # too small a workspace
    p = xs.make_params(sort="material_energy", sort_threshold=0)
    need = xs.xs_workspace_size(h, 1000, p)
    assert need > 0
    ws = torch.empty(need // 2, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(xs.XsError) as e:
        xs.xs_lookup_batch(h, cfg1["E"][:1000], cfg1["m"][:1000], params=p,
                           workspace=(ws, ws.data_ptr(), need // 2))
    assert e.value.status == xs.XS_EWORKSPACE
    small.close()


def test_union_by_material(cfg1):
    """The by-material union index gives the same brackets and bits."""
    t, q = cfg1["t"], cfg1["q"]
    h = xs.xs_create_tables(t, ALL_FLAGS | xs.XS_BUILD_UNION_BY_MATERIAL, 4000)
    info = xs.xs_table_info(h)
    assert info["bytes_union"] == info["union_size"] * (8 + 4 * len(t.mat_nuclides))
    _, idx_ref, off = oracle.lookup(t, q.E, q.mat, with_index=True)
    idx = xs.xs_lookup_indices(h, cfg1["E"], cfg1["m"], dev(off, torch.int64),
                               grid="unionized")
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    for k in KNOBS:
        out = run(h, cfg1["E"], cfg1["m"], grid="unionized", **k)
        assert np.array_equal(out, cfg1["ref"]), k
        out = run(h, cfg1["E"], cfg1["m"], precision=xs.XS_FP32,
                  grid="unionized", **k)
        assert np.array_equal(out, cfg1["ref32"]), k
    h.close()


def test_table_info(cfg1):
    info = xs.xs_table_info(cfg1["h"])
    t = cfg1["t"]
    assert info["n_nuclides"] == 20 and info["n_materials"] == 4
    assert info["n_points"] == len(t.energy)
    assert info["union_size"] == len(np.unique(t.energy))
    assert info["n_hash_bins"] == 4000
    assert info["e_min"] == 1e-5 and info["e_max"] == 1.0


def test_profile_counts(cfg1):
    h = cfg1["h"]
    xs.xs_profile_begin(h)
    for _ in range(3):
        xs.xs_lookup_batch(h, cfg1["E"], cfg1["m"],
                           params=xs.make_params(sort="material_energy",
                                                 sort_threshold=0))
    prof = xs.xs_profile_end(h)
    assert prof["calls"] == 3 and prof["sorted_calls"] == 3
    assert prof["lookups"] == 3 * len(cfg1["q"])
    assert prof["ms_lookup"] > 0 and prof["ms_sort"] > 0
    assert prof["ms_total"] >= prof["ms_lookup"]


@pytest.mark.parametrize("union_by_material", [False, True])
def test_lds_staging_groups(union_by_material):
    """LDS staging on materials longer than one staging group (70 and 33
    nuclides) with windows that fit (small blocks) and windows that do not
    (large blocks, per-lane search for that nuclide): identical bits to the
    oracle for every grid method, both precisions and all three stage
    shapes."""
    say("lds groups", union_by_material)
    t = synth.random_tables(17, 80, 500, 3, sizes=[70, 33, 5])
    q = synth.random_queries(17, t, 60_000)
    flags = ALL_FLAGS | (xs.XS_BUILD_UNION_BY_MATERIAL if union_by_material
                         else 0)
    h = xs.xs_create_tables(t, flags, 1000)
    try:
        ref = oracle.lookup(t, q.E, q.mat)
        ref32 = oracle.lookup_f32(t, q.E, q.mat)
        E, m = dev(q.E, torch.float64), dev(q.mat, torch.int32)
        grids = ("unionized",) if union_by_material else (
            "nuclide", "hash", "unionized")
        for grid in grids:
            for bs, lpt, sort in ((64, 1, "band_material"),
                                  (256, 1, "material_energy"),
                                  (1024, 1, "band_material"), (128, 1, "none"),
                                  (64, 2, "band_material"),
                                  (512, 2, "material_energy")):
                for prec, r in ((xs.XS_FP64, ref), (xs.XS_FP32, ref32)):
                    for shape in (1, 2, 3):
                        out = run(h, E, m, precision=prec, grid=grid,
                                  sort=sort, sort_threshold=0, block_size=bs,
                                  lookups_per_thread=lpt, unroll=1,
                                  lds_stage=shape)
                        assert np.array_equal(out, r), (grid, bs, lpt, sort,
                                                        prec, shape)
    finally:
        h.close()


def test_concurrent_streams_share_tables(cfg1):
    """Several streams using one table handle at once, each with its own
    workspace (sorted batches), give the oracle's bits."""
    say("concurrent streams")
    h, E, m = cfg1["h"], cfg1["E"], cfg1["m"]
    n = E.numel()
    k = 4
    parts = [(i * n // k, (i + 1) * n // k) for i in range(k)]
    streams = [torch.cuda.Stream() for _ in range(k)]
    for prec, ref in ((xs.XS_FP64, cfg1["ref"]), (xs.XS_FP32, cfg1["ref32"])):
        p = xs.make_params(prec, grid="hash", sort="band_material",
                           sort_threshold=0, block_size=256,
                           lookups_per_thread=1, unroll=2)
        dt = torch.float64 if prec == xs.XS_FP64 else torch.float32
        out = torch.full((n, 5), -1.0, dtype=dt, device="cuda:0")
        wss = [xs._workspace(xs.xs_workspace_size(h, b - a, p), E.device)
               for a, b in parts]
        cur = torch.cuda.current_stream()
        for rep in range(3):
            for s in streams:
                s.wait_stream(cur)
            for s, (a, b), w in zip(streams, parts, wss):
                with torch.cuda.stream(s):
                    xs.xs_lookup_batch(h, E[a:b], m[a:b], out=out[a:b],
                                       params=p, workspace=w, stream=s)
            for s in streams:
                cur.wait_stream(s)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), (prec, rep)


@pytest.mark.parametrize("golden", ["worked_example.txt",
                                    "worked_example_f32.txt"])
def test_worked_examples_exact(golden):
    """The hand-worked examples (tests/golden/) through every grid method and
    kernel family: the FP64 file's sums in FP64, the FP32 file's exact bits
    in the FP32 form, and every bracket as derived."""
    import os
    from tests import pins
    t, queries = pins.read_worked_example(
        os.path.join(pins.GOLDEN, golden))
    prec = xs.XS_FP32 if golden.endswith("_f32.txt") else xs.XS_FP64
    # every query repeated so blocks of every kernel fill up
    reps = 300
    E1 = np.array([q[0] for q in queries])
    m1 = np.array([q[1] for q in queries], np.int32)
    E_np, m_np = np.tile(E1, reps), np.tile(m1, reps)
    want = np.tile(np.array([q[3] for q in queries]), (reps, 1))
    E, m = dev(E_np, torch.float64), dev(m_np, torch.int32)
    h = xs.xs_create_tables(t, ALL_FLAGS, 7)
    try:
        shapes = [dict(sort="none", block_size=256, lookups_per_thread=1,
                       unroll=1),
                  dict(sort="material_energy", sort_threshold=0,
                       block_size=128, lookups_per_thread=2, unroll=2),
                  dict(sort="band_material", sort_threshold=0, block_size=128,
                       lookups_per_thread=1, unroll=1, lds_stage=1),
                  dict(sort="band_material", sort_threshold=0, block_size=64,
                       lookups_per_thread=1, unroll=1, lds_stage=3),
                  dict(sort="none", block_size=128, lookups_per_thread=1,
                       unroll=1, lds_stage=0, wave_per_lookup=1)]
        for grid in ("nuclide", "hash", "unionized"):
            for k in shapes:
                out = run(h, E, m, precision=prec, grid=grid, **k)
                if prec == xs.XS_FP32:
                    ok = np.array_equal(out.view(np.uint32),
                                        want.astype(np.float32).view(np.uint32))
                else:
                    ok = np.array_equal(out, want)
                assert ok, (golden, grid, k)
            off = oracle.index_offsets(t, m_np)
            idx = xs.xs_lookup_indices(h, E, m, dev(off, torch.int64),
                                       grid=grid)
            torch.cuda.synchronize()
            want_idx = np.concatenate([q[2] for q in queries] * reps)
            assert np.array_equal(idx.cpu().numpy(), want_idx), (golden, grid)
    finally:
        h.close()


@pytest.mark.parametrize("grid", ["unionized", "nuclide", "hash"])
def test_wave_kernel_reads_record_pairs(cfg1, grid):
    """With XS_BUILD_FP32_PAIRS the one-wave-per-lookup kernel of the FP32
    form reads each bracket as one aligned 64-byte pair (union and bisection
    grids; the hash grid keeps its three-record window): same bits as the
    oracle's FP32 form and as the kernel on a handle without pairs, sorted
    and unsorted; the pairs add 64 bytes per grid point."""
    say("pairs", grid)
    t = cfg1["t"]
    h = xs.xs_create_tables(t, ALL_FLAGS | xs.XS_BUILD_FP32_PAIRS, 4000)
    try:
        info, base = xs.xs_table_info(h), xs.xs_table_info(cfg1["h"])
        assert info["bytes_fp32"] == base["bytes_fp32"] + 64 * info["n_points"]
        for sort in ("none", "energy"):
            p = xs.make_params(xs.XS_FP32, grid=grid, sort=sort,
                               sort_threshold=0, block_size=256,
                               lookups_per_thread=1, unroll=1, lds_stage=0,
                               wave_per_lookup=1)
            out = xs.xs_lookup_batch(h, cfg1["E"], cfg1["m"], params=p)
            plain = xs.xs_lookup_batch(cfg1["h"], cfg1["E"], cfg1["m"],
                                       params=p)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, cfg1["ref32"]), sort
            assert np.array_equal(got, plain.cpu().numpy()), sort
    finally:
        h.close()


def test_wave_union_search_dense_and_sparse_bins():
    """The wave kernel's union search reads one logarithmic bin's points at
    once; a bin holding 64 points or more, and energies that the rounding of
    log puts in a neighbouring bin, take the whole-grid search instead.  A
    table with a dense cluster (2,000 points within 0.1 % of 1e-3) and long
    empty stretches exercises both; every form returns the oracle's bits."""
    import synth
    say("wave union dense bins")
    t = synth.random_tables(17, 6, [300, 40, 2000, 7, 120, 2], 5,
                            sizes=[6, 1, 3, 4, 2])
    k = 2  # the third nuclide: 2,000 points packed near 1e-3
    a, b = t.grid_offsets[k], t.grid_offsets[k + 1]
    e = np.array(t.energy, dtype=np.float64)
    e[a] = 1e-5
    e[b - 1] = 1.0
    e[a + 1:b - 1] = 1e-3 * (1.0 + np.linspace(0.0, 1e-3, b - a - 2))
    t = synth.Tables(t.grid_offsets, e, t.xs, t.mat_offsets, t.mat_nuclides,
                     t.mat_density)
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    try:
        u = np.unique(e)
        near = np.concatenate([e[a:b:37], np.nextafter(e[a:b:37], 0),
                               np.nextafter(e[a:b:37], np.inf),
                               u[::5], np.nextafter(u[::5], 0)])
        q = synth.random_queries(18, t, 30_000)
        E = np.concatenate([q.E, near[(near > 0) & np.isfinite(near)]])
        m = (np.arange(len(E)) % t.n_materials).astype(np.int32)
        ref = oracle.lookup(t, E, m)
        ref32 = oracle.lookup_f32(t, E, m)
        Ed, md = dev(E, torch.float64), dev(m, torch.int32)
        for prec, want in ((xs.XS_FP64, ref), (xs.XS_FP32, ref32)):
            for bs in (64, 256):
                out = run(h, Ed, md, precision=prec, grid="unionized",
                          sort="none", block_size=bs, lookups_per_thread=1,
                          unroll=1, lds_stage=0, wave_per_lookup=1)
                assert np.array_equal(out, want), (prec, bs)
    finally:
        h.close()


def test_fraction_division_on_adversarial_spacings():
    """The fraction's correctly rounded division (seeded, in the FP32 form,
    by the reciprocal the FP32 records carry) on spacings whose mantissas
    are all ones, exact powers of two, one ulp above them, and ratios of
    odd integers, queried at sixteenths of every interval, at its ends and
    their neighbours: every kernel returns the oracle's bits in both
    forms."""
    import synth
    say("division on adversarial spacings")
    steps = np.array([np.ldexp(2.0 - 2.0 ** -52, -21), 2.0 ** -20,
                      np.ldexp(1.0 + 2.0 ** -52, -20), 3.0 * 2.0 ** -21,
                      np.ldexp(1.0 - 2.0 ** -53, -19), 7.0 / 3.0 * 2.0 ** -20,
                      np.ldexp(1.5, -22), np.ldexp(1.9999999999999996, -18)])
    grids = []
    for k, start in enumerate((1e-3, 0.25, 0.5 - 2.0 ** -30)):
        d = np.roll(steps, k)
        e = start + np.concatenate(([0.0], np.cumsum(np.tile(d, 150))))
        grids.append(e)
    offs = np.zeros(4, dtype=np.int64)
    offs[1:] = np.cumsum([len(g) for g in grids])
    energy = np.concatenate(grids)
    assert all(np.all(np.diff(g) > 0) for g in grids)
    s = synth.Stream(19, 1)
    xsv = s.lognormal(len(energy) * 5).reshape(-1, 5)
    t = synth.Tables(offs, energy, xsv, np.array([0, 3, 4, 6], np.int32),
                     np.array([0, 1, 2, 1, 2, 0], np.int32),
                     np.array([1.0, 0.5, 0.25, 1.0, 0.75, 0.125]))
    h = xs.xs_create_tables(t, ALL_FLAGS, 1000)
    try:
        E = []
        for g in grids:
            lo, hi = g[:-1], g[1:]
            for j in range(17):
                E.append(lo + (hi - lo) * (j / 16.0))
            E += [np.nextafter(lo, np.inf), np.nextafter(hi, 0)]
        E = np.concatenate(E)
        m = (np.arange(len(E)) % 3).astype(np.int32)
        ref, ref32 = oracle.lookup(t, E, m), oracle.lookup_f32(t, E, m)
        Ed, md = dev(E, torch.float64), dev(m, torch.int32)
        shapes = [dict(sort="none", lookups_per_thread=1, unroll=1),
                  dict(sort="band_material", sort_threshold=0, block_size=128,
                       lookups_per_thread=1, unroll=1, lds_stage=1),
                  dict(sort="band_material", sort_threshold=0, block_size=64,
                       lookups_per_thread=2, unroll=1, lds_stage=3),
                  dict(sort="none", block_size=64, lookups_per_thread=1,
                       unroll=1, lds_stage=0, wave_per_lookup=1)]
        for prec, want in ((xs.XS_FP64, ref), (xs.XS_FP32, ref32)):
            for grid in ("nuclide", "hash", "unionized"):
                for k in shapes:
                    out = run(h, Ed, md, precision=prec, grid=grid, **k)
                    assert np.array_equal(out, want), (prec, grid, k)
    finally:
        h.close()
