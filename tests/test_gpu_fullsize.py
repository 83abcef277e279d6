"""Full-size synthetic workload (355 nuclides x 11,303 points, 12 materials,
10M lookups) in the launch shapes the benchmark times.

The oracle computes every one of the 10M lookups (FP64 and the FP32 form, on
the host's cores); the GPU outputs are compared with it element by element:
the plain FP64 lookup and the benchmark's tuned path (unionized grid indexed
by material, banded sort, LDS staging in each stage shape at 128 and 256
lanes) over the whole batch, and the brackets of every (lookup, nuclide)
pair of the batch for all three grid methods, in 1M-lookup chunks, and
half-active masked batches (compacted, sorted and predicated).  Other
launch shapes are checked through properties that hold at any size: every
grid method, sort policy and launch shape gives bit-identical sums within
one precision.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

N = 10_000_000
SAMPLES = 20_000
CHUNK = 1_000_000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


@pytest.fixture(scope="module")
def full():
    say("full size: generating tables and 10M queries")
    t = synth.config2_tables()
    q = synth.config2_queries(N)
    # the benchmark's build: the union index stored per material
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL)
    say("full size: building tables (hash 8192 bins, union grid by material)")
    h = xs.xs_create_tables(t, flags, 8192)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    s = synth.Stream(41, 1)
    pick = np.unique(np.concatenate([
        s.integers(SAMPLES, 0, N - 1), np.arange(64), np.arange(N - 64, N)]))
    th = host_threads()
    say(f"full size: oracle over all {N} lookups on {th} threads")
    ref_all = oracle.lookup(t, q.E, q.mat, threads=th)
    ref32_all = oracle.lookup_f32(t, q.E, q.mat, threads=th)
    yield dict(t=t, q=q, h=h, E=E, m=m, pick=pick, ref=ref_all[pick],
               ref32=ref32_all[pick], ref_all=ref_all, ref32_all=ref32_all)
    h.close()


def run(f, n=N, **kw):
    p = xs.make_params(**kw)
    out = xs.xs_lookup_batch(f["h"], f["E"][:n], f["m"][:n], params=p)
    torch.cuda.synchronize()
    return out


PLAIN = dict(precision=xs.XS_FP64, grid="nuclide", sort="none", block_size=256,
             lookups_per_thread=1)


def test_plain_fp64_whole_batch(full):
    say("plain fp64 full size, every lookup against the oracle")
    out = run(full, **PLAIN).cpu().numpy()
    ref = full["ref_all"]
    rel = np.abs(out - ref) / ref
    say("plain fp64 max rel per channel", rel.max(axis=0))
    assert rel.max() <= 1e-12
    assert np.array_equal(out, ref)
    assert np.all(np.isfinite(out)) and np.all(out > 0)
    full["out64"] = torch.from_numpy(out)


# Every shape the tuner returns at 10M lookups on these tables: union grid
# (by material), banded sort, LDS staging in each stage shape, 128- and
# 256-lane blocks, one or two lookups per lane.
BENCH_SHAPES = [dict(lds_stage=s, block_size=b, lookups_per_thread=l)
                for s in (1, 2, 3) for b in (128, 256) for l in (1, 2)]


@pytest.mark.parametrize("shape", BENCH_SHAPES,
                         ids=[f"stage{k['lds_stage']}-b{k['block_size']}-"
                              f"lpt{k['lookups_per_thread']}"
                              for k in BENCH_SHAPES])
def test_tuned_path_whole_batch(full, shape):
    say("tuned path, every lookup against the oracle", shape)
    out = run(full, precision=xs.XS_FP32, grid="unionized",
              sort="band_material", sort_threshold=0, unroll=1,
              **shape).cpu().numpy()
    bad = np.count_nonzero(out.view(np.uint32) !=
                           full["ref32_all"].view(np.uint32))
    assert bad == 0, (shape, bad)
    ref = full["ref_all"]
    rel = np.abs(out.astype(np.float64) - ref) / ref
    say("  max rel per channel", rel.max(axis=0), "mean", rel.mean(axis=0))
    assert rel.max() <= 2e-6


# Masked batches at full size: half of the slots active.  A compacted queue,
# or a sorted one whose inactive lookups go last, is served through its
# active head (device-side count, or block ranges of the unflagged groups)
# dealt over all XCDs.
MASKED_SHAPES = [dict(lds_stage=1, block_size=128, sort="band_material",
                      queue=xs.XS_QUEUE_COMPACT),
                 dict(lds_stage=3, block_size=128, sort="band_material",
                      queue=xs.XS_QUEUE_COMPACT),
                 dict(lds_stage=1, block_size=128, sort="none",
                      queue=xs.XS_QUEUE_COMPACT),
                 dict(lds_stage=0, block_size=256, sort="none",
                      queue=xs.XS_QUEUE_COMPACT),
                 dict(lds_stage=0, block_size=256, sort="none",
                      queue=xs.XS_QUEUE_PREDICATED)]


@pytest.mark.parametrize("shape", MASKED_SHAPES,
                         ids=[f"stage{k['lds_stage']}-{k['sort']}-q{k['queue']}"
                              for k in MASKED_SHAPES])
def test_masked_half_active_whole_batch(full, shape):
    say("masked full size, half active", shape)
    act = (synth.Stream(43, 1).uniform(N) < 0.5).astype(np.uint8)
    sentinel = -3.5
    out = torch.full((N, 5), sentinel, dtype=torch.float32, device="cuda:0")
    p = xs.make_params(precision=xs.XS_FP32, grid="unionized",
                       sort_threshold=0, lookups_per_thread=1, unroll=1,
                       **shape)
    xs.xs_lookup_active(full["h"], full["E"], full["m"],
                        torch.from_numpy(act).to("cuda:0"), out, params=p)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    a = act.astype(bool)
    assert np.all(o[~a] == sentinel), shape
    bad = np.count_nonzero(o[a].view(np.uint32) !=
                           full["ref32_all"][a].view(np.uint32))
    assert bad == 0, (shape, bad)


@pytest.mark.parametrize("grid", ["nuclide", "hash", "unionized"])
@pytest.mark.parametrize("sort", ["none", "material", "energy", "material_energy",
                                  "band_material"])
def test_fp64_grids_and_sorts_identical(full, grid, sort):
    say("fp64 full size", grid, sort)
    if "out64" not in full:
        pytest.skip("plain run failed")
    out = run(full, precision=xs.XS_FP64, grid=grid, sort=sort,
              sort_threshold=0, block_size=256, lookups_per_thread=2)
    assert torch.equal(out.cpu(), full["out64"])


@pytest.mark.parametrize("grid", ["nuclide", "hash", "unionized"])
def test_fp32_samples_and_bound(full, grid):
    say("fp32 full size", grid)
    out = run(full, precision=xs.XS_FP32, grid=grid, sort="material_energy",
              sort_threshold=20000, block_size=256, lookups_per_thread=2)
    o = out.cpu().numpy()
    assert np.array_equal(o, full["ref32_all"])
    if "out64" in full:
        ref = full["out64"].numpy()
        rel = np.abs(o.astype(np.float64) - ref) / ref
        say("fp32 rel err per channel max", rel.max(axis=0), "mean",
            rel.mean(axis=0))
        assert rel.max() <= 2e-6
    for k in (dict(sort="none", block_size=1024, lookups_per_thread=1),
              dict(sort="material", sort_threshold=0, block_size=512,
                   lookups_per_thread=4),
              dict(sort="band_material", sort_threshold=0, block_size=256,
                   lookups_per_thread=1, unroll=4),
              dict(sort="band_material", sort_threshold=0, block_size=512,
                   lookups_per_thread=2, unroll=2),
              dict(sort="band_material", sort_threshold=0, block_size=256,
                   lookups_per_thread=1, unroll=1, lds_stage=1),
              dict(sort="band_material", sort_threshold=0, block_size=128,
                   lookups_per_thread=2, unroll=1, lds_stage=1),
              dict(sort="band_material", sort_threshold=0, block_size=128,
                   lookups_per_thread=1, unroll=1, lds_stage=2),
              dict(sort="band_material", sort_threshold=0, block_size=256,
                   lookups_per_thread=2, unroll=1, lds_stage=3)):
        o2 = run(full, precision=xs.XS_FP32, grid=grid, **k).cpu().numpy()
        assert np.array_equal(o2, o), k
    full["out32_" + grid] = o


@pytest.mark.parametrize("n", [100_000, 1_000_000])
def test_sparser_prefixes_in_every_kernel(full, n):
    """The first n lookups of the batch are sparser in energy per material,
    so wider stage shapes and one wave per lookup are the tuned choices
    there: every kernel gives the bits of the same lookups in the full
    batch."""
    say("prefix", n)
    if "out32_unionized" not in full:
        pytest.skip("full FP32 run failed")
    ref = full["out32_unionized"][:n]
    for k in (dict(sort="band_material", sort_threshold=0, block_size=64,
                   lookups_per_thread=1, unroll=1, lds_stage=s)
              for s in (1, 2, 3)):
        o = run(full, n=n, precision=xs.XS_FP32, grid="unionized", **k)
        assert np.array_equal(o.cpu().numpy(), ref), (n, k)
    for grid in ("unionized", "hash", "nuclide"):
        for srt in ("none", "band_material"):
            o = run(full, n=n, precision=xs.XS_FP32, grid=grid, sort=srt,
                    sort_threshold=0, block_size=128, lookups_per_thread=1,
                    unroll=1, lds_stage=0, wave_per_lookup=1)
            assert np.array_equal(o.cpu().numpy(), ref), (n, grid, srt)
    # untuned defaults at this size
    o = xs.xs_lookup_batch(full["h"], full["E"][:n], full["m"][:n],
                           params=xs.xs_params_default(xs.XS_FP32))
    torch.cuda.synchronize()
    assert np.array_equal(o.cpu().numpy(), ref)


def test_union_index_by_nuclide_full(full):
    """The [U][K] union index (5.7 GB here) instead of the per-material one:
    identical bits."""
    if "out64" not in full:
        pytest.skip("plain run failed")
    say("union index [U][K], full size")
    h = xs.xs_create_tables(full["t"], xs.XS_BUILD_FP32 | xs.XS_BUILD_UNIONIZED,
                            0)
    try:
        for k in (dict(sort="band_material", sort_threshold=0, lookups_per_thread=1,
                       unroll=4),
                  dict(sort="none", lookups_per_thread=2, unroll=1)):
            p = xs.make_params(xs.XS_FP64, grid="unionized", block_size=256, **k)
            out = xs.xs_lookup_batch(h, full["E"], full["m"], params=p)
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), full["out64"]), k
        p = xs.make_params(xs.XS_FP32, grid="unionized", sort="band_material",
                           sort_threshold=0, block_size=256, lookups_per_thread=1,
                           unroll=2)
        o = xs.xs_lookup_batch(h, full["E"], full["m"], params=p).cpu().numpy()
        assert np.array_equal(o[full["pick"]], full["ref32"])
    finally:
        h.close()


def test_ragged_batch(full):
    n = N - 9
    say("ragged", n)
    out = run(full, n=n, precision=xs.XS_FP64, grid="hash",
              sort="material_energy", sort_threshold=0, block_size=192,
              lookups_per_thread=3)
    if "out64" in full:
        assert torch.equal(out.cpu(), full["out64"][:n])


def test_indices_whole_batch(full):
    """The brackets of every (lookup, nuclide) pair of the 10M batch, from
    each grid method, against the oracle's, in 1M-lookup chunks."""
    t, q = full["t"], full["q"]
    th = host_threads()
    for a in range(0, N, CHUNK):
        b = min(N, a + CHUNK)
        say("indices", a, b)
        _, idx_ref, off = oracle.lookup(t, q.E[a:b], q.mat[a:b],
                                        with_index=True, threads=th)
        offd = torch.from_numpy(off).to("cuda:0")
        for grid in ("nuclide", "hash", "unionized"):
            got = xs.xs_lookup_indices(full["h"], full["E"][a:b],
                                       full["m"][a:b], offd, grid=grid)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), idx_ref), (a, grid)
            del got


@pytest.mark.parametrize("grid,prec", [("unionized", xs.XS_FP64),
                                       ("hash", xs.XS_FP32)])
def test_requests_full(full, grid, prec):
    """Uneven requests over the full-size tables in one launch: FP64 equals
    the plain batch bit for bit, the FP32 form equals the oracle's samples."""
    if "out64" not in full:
        pytest.skip("plain run failed")
    s = synth.Stream(43, 1)
    sizes = np.floor(np.exp(np.log(1e3) + s.uniform(60) *
                            (np.log(3e5) - np.log(1e3)))).astype(np.int64)
    sizes[7] = 0
    say("requests full size", grid, prec, int(sizes.sum()), "lookups")
    dt = torch.float64 if prec == xs.XS_FP64 else torch.float32
    starts = np.concatenate(([0], np.cumsum(sizes)))
    reqs = [(full["E"][a:b], full["m"][a:b],
             torch.empty((b - a, 5), dtype=dt, device="cuda:0"))
            for a, b in zip(starts[:-1], starts[1:])]
    p = xs.make_params(prec, grid=grid, unroll=2)
    batch = xs.xs_lookup_requests(full["h"], reqs, params=p)
    stats, makespan = xs.xs_requests_stats(batch)
    assert makespan > 0 and [st["n"] for st in stats] == list(sizes)
    got = torch.cat([o for _, _, o in reqs]).cpu().numpy()
    end = int(starts[-1])
    if prec == xs.XS_FP64:
        assert np.array_equal(got, full["out64"][:end].numpy())
    else:
        sel = full["pick"] < end
        assert sel.sum() > 100
        assert np.array_equal(got[full["pick"][sel]], full["ref32"][sel])


def test_largest_batch(full):
    """n = 2^31 - 1, the largest batch the interface takes (positions and the
    permutation are int32): the full-size queries' first 2^20 repeated 2,048
    times and cut one short.  Every repeat of the base chunk must give the
    base chunk's bits (a property at any size), the base chunk must match the
    oracle's samples, and both a sorted LDS-staged and an unsorted launch
    shape must agree."""
    if "out64" not in full:
        pytest.skip("plain run failed")
    c = 1 << 20
    n = (1 << 31) - 1
    say("largest batch", n)
    E = full["E"][:c].repeat(2048)[:n]
    m = full["m"][:c].repeat(2048)[:n]
    base = full["out64"][:c].to(device="cuda:0", dtype=torch.float64)
    pick = full["pick"][full["pick"] < c]
    for kw in (dict(grid="unionized", sort="band_material", sort_threshold=0,
                    block_size=128, lookups_per_thread=1, unroll=1,
                    lds_stage=1),
               dict(grid="hash", sort="none", block_size=256,
                    lookups_per_thread=1, unroll=2)):
        say("largest batch", kw)
        p = xs.make_params(xs.XS_FP32, **kw)
        out = xs.xs_lookup_batch(full["h"], E, m, params=p)
        torch.cuda.synchronize()
        first = out[:c]
        got = first.cpu().numpy()
        assert np.array_equal(got[pick], full["ref32"][:len(pick)]), kw
        full_chunks = out[:2047 * c].view(2047, c, 5)
        assert torch.equal(full_chunks, first.unsqueeze(0).expand(2047, c, 5)), kw
        assert torch.equal(out[2047 * c:], first[:c - 1]), kw
        rel = (first.double() - base).abs() / base
        assert float(rel.max()) <= 2e-6
        del out, first, full_chunks
        torch.cuda.empty_cache()
