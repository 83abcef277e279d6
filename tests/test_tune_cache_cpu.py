"""The tuned-parameter file without a device (the paper's performance
database, section 3): entries keyed by device, table checksum, precision,
entry point and batch-size class survive a round trip, replace each other
by key only, ignore lines that do not parse, are written atomically (no
temporary file left behind), and bad keys or paths are refused.  The search
that fills it is the mock-evaluator search of test_tune_cpu."""
import math
import os

import pytest

from paper_2402_09222_amd import xs

INT64_MAX = (1 << 63) - 1
DEV = "AMD Instinct MI355X|gfx950:sramecc+:xnack-|256CU"


def params(**kw):
    base = dict(precision=xs.XS_FP32, grid=xs.XS_GRID_HASH,
                sort=xs.XS_SORT_BAND_MATERIAL, block_size=128,
                lookups_per_thread=1, lds_stage=1, sort_threshold=20000,
                queue=xs.XS_QUEUE_COMPACT, unroll=1, wave_per_lookup=0,
                hash_bins=8192)
    base.update(kw)
    return xs.make_params(**base)


def same(a, b):
    return a.as_dict() == b.as_dict()


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not os.path.exists(xs.LIB_PATH):
        from paper_2402_09222_amd import build
        build.build()
    return xs.load_library()


def test_round_trip_and_missing(tmp_path):
    path = str(tmp_path / "tuned.txt")
    k = xs.make_tune_key(DEV, 0x0123456789ABCDEF, xs.XS_FP32, False, 1_000_000)
    assert k.size_class == 19
    assert xs.xs_tune_cache_get(path, k) is None  # no file yet
    p = params()
    xs.xs_tune_cache_put(path, k, p, 1.25)
    got = xs.xs_tune_cache_get(path, k)
    assert got is not None and same(got[0], p) and got[1] == 1.25
    # the never-sort threshold and an unsorted entry round-trip exactly
    k2 = xs.make_tune_key(DEV, 0x0123456789ABCDEF, xs.XS_FP32, False, 100_000)
    p2 = params(sort=xs.XS_SORT_NONE, sort_threshold=INT64_MAX,
                grid=xs.XS_GRID_UNIONIZED, hash_bins=0, wave_per_lookup=1,
                lds_stage=0)
    xs.xs_tune_cache_put(path, k2, p2, 0.2)
    assert same(xs.xs_tune_cache_get(path, k2)[0], p2)
    assert same(xs.xs_tune_cache_get(path, k)[0], p)
    # any other field of the key misses
    for other in (
            xs.make_tune_key(DEV + "x", 0x0123456789ABCDEF, 1, False, 1_000_000),
            xs.make_tune_key(DEV, 0x0123456789ABCDEE, 1, False, 1_000_000),
            xs.make_tune_key(DEV, 0x0123456789ABCDEF, 0, False, 1_000_000),
            xs.make_tune_key(DEV, 0x0123456789ABCDEF, 1, True, 1_000_000),
            xs.make_tune_key(DEV, 0x0123456789ABCDEF, 1, False, 2_000_000)):
        assert xs.xs_tune_cache_get(path, other) is None
    # a size of the same class hits
    same_class = xs.make_tune_key(DEV, 0x0123456789ABCDEF, 1, False, 600_000)
    assert same(xs.xs_tune_cache_get(path, same_class)[0], p)


def test_replace_by_key_and_atomic_rewrite(tmp_path):
    path = str(tmp_path / "tuned.txt")
    keys = [xs.make_tune_key(DEV, 77, xs.XS_FP64, a, n)
            for a in (False, True) for n in (1e5, 1e6, 8e6)]
    for i, k in enumerate(keys):
        xs.xs_tune_cache_put(path, k, params(precision=xs.XS_FP64,
                                             block_size=64 * (i + 1)), i)
    newer = params(precision=xs.XS_FP64, block_size=1024, queue=1)
    xs.xs_tune_cache_put(path, keys[2], newer, 9.5)
    lines = [l for l in open(path).read().splitlines() if not l.startswith("#")]
    assert len(lines) == len(keys)  # replaced, not appended
    for i, k in enumerate(keys):
        p, ms = xs.xs_tune_cache_get(path, k)
        if i == 2:
            assert same(p, newer) and ms == 9.5
        else:
            assert p.block_size == 64 * (i + 1) and ms == i
    assert os.listdir(tmp_path) == ["tuned.txt"]  # no temporary file left


def test_unparsable_lines_are_ignored(tmp_path):
    path = str(tmp_path / "tuned.txt")
    k = xs.make_tune_key(DEV, 5, xs.XS_FP32, False, 4_000_000)
    p = params()
    xs.xs_tune_cache_put(path, k, p, 1.0)
    good = [l for l in open(path).read().splitlines() if not l.startswith("#")]
    junk = [
        "# a comment",
        "",
        "garbage",
        good[0].rsplit("\t", 1)[0] + "\tnan",          # bad time
        good[0].replace("\t0000000000000005", "\t5"),  # short checksum
        "\t".join(good[0].split("\t")[:6]),            # missing field
        good[0].replace(" 8192\t", " 8192 7\t"),      # eleven parameters
        good[0].replace(f"\t{k.size_class}\t", "\t99\t"),  # class out of range
    ]
    with open(path, "w") as f:
        f.write("\n".join(junk) + "\n")
    assert xs.xs_tune_cache_get(path, k) is None
    with open(path, "a") as f:
        f.write(good[0] + "\n")
    got = xs.xs_tune_cache_get(path, k)
    assert same(got[0], p) and got[1] == 1.0


def test_put_refuses_bad_keys_and_paths(tmp_path):
    path = str(tmp_path / "tuned.txt")
    p = params()
    bad_keys = [
        xs.make_tune_key("dev\twith tab", 1, xs.XS_FP32, False, 10),
        xs.make_tune_key("", 1, xs.XS_FP32, False, 10),
        xs.make_tune_key(DEV, 1, xs.XS_FP64, False, 10),  # precision differs
    ]
    for k in bad_keys:
        with pytest.raises(xs.XsError) as e:
            xs.xs_tune_cache_put(path, k, p, 1.0)
        assert e.value.status == xs.XS_EINVAL
    k = xs.make_tune_key(DEV, 1, xs.XS_FP32, False, 10)
    for ms in (math.nan, math.inf, -1.0):
        with pytest.raises(xs.XsError):
            xs.xs_tune_cache_put(path, k, p, ms)
    with pytest.raises(xs.XsError) as e:
        xs.xs_tune_cache_put(str(tmp_path / "no" / "such" / "dir.txt"), k, p, 1.0)
    assert e.value.status == xs.XS_EINVAL and "cannot write" in str(e.value)
    assert not os.path.exists(path)


def test_search_winners_per_size_through_the_cache(tmp_path):
    """The paper's particles-in-flight list, each size tuned by the forest
    search on a mock clock whose best hash grid and threshold depend on n,
    stored and read back; the stored winners keep their conditional
    parameters' fixed values."""
    path = str(tmp_path / "tuned.txt")
    sizes = [100_000, 500_000, 1_000_000, 2_000_000, 4_000_000, 8_000_000]
    bins = [4000, 8192, 32768]

    def clock(n):
        def f(p):
            c = {0: 4.0, 1: 1.0, 2: 1.5}[p.grid]
            if p.grid == 1:  # more bins pay at larger n in this mock
                want = 4000 if n < 1e6 else (8192 if n < 4e6 else 32768)
                c *= 1.0 if p.hash_bins == want else 1.4
            if p.sort != 0:
                c *= 1.0 if (n >= p.sort_threshold) == (n >= 1e6) else 1.5
            c *= 1.0 + 0.1 * abs(p.block_size.bit_length() - 8)
            return c
        return f

    for n in sizes:
        cfg = xs.xs_tune_config_default(strategy=1, max_evals=64, seed=3,
                                        timeout_factor=0.0, hash_bins=bins,
                                        precision=xs.XS_FP32)
        r = xs.xs_tune_search(7, cfg, lambda p, cut, n=n: clock(n)(p))
        k = xs.make_tune_key(DEV, 42, xs.XS_FP32, False, n)
        xs.xs_tune_cache_put(path, k, r.best, r.best_ms)
    for n in sizes:
        p, ms = xs.xs_tune_cache_get(path, xs.make_tune_key(
            DEV, 42, xs.XS_FP32, False, n))
        assert ms == pytest.approx(clock(n)(p), rel=1e-5)
        if p.grid != 1:
            assert p.hash_bins == 0
        if p.sort == 0:
            assert p.sort_threshold == INT64_MAX
        assert p.queue == xs.XS_QUEUE_COMPACT
