"""The device tuner (xs_tune) end to end: its first evaluation is the
untuned default for the batch size, the winner is never slower than it,
later calls with automatic fields run the winner, and the results stay the
oracle's bits whatever it picked."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

ALL_FLAGS = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED
KEYS = ("grid", "sort", "block_size", "lookups_per_thread", "unroll",
        "lds_stage", "wave_per_lookup")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype,
                                                       device="cuda:0")


def choice(p):
    return tuple(getattr(p, k) for k in KEYS)


@pytest.fixture(scope="module")
def env():
    t = synth.config1_tables()
    q = synth.config1_queries()
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    yield dict(t=t, q=q, h=h, ref={xs.XS_FP64: oracle.lookup(t, q.E, q.mat),
                                   xs.XS_FP32: oracle.lookup_f32(t, q.E, q.mat)})
    h.close()


@pytest.mark.parametrize("prec", [xs.XS_FP64, xs.XS_FP32])
@pytest.mark.parametrize("n", [20_000, 100_000])
def test_tune_baseline_winner_and_reuse(env, prec, n):
    say("tune", prec, n)
    h, q = env["h"], env["q"]
    E, m = dev(q.E[:n], torch.float64), dev(q.mat[:n], torch.int32)
    xs.xs_set_tuned(h, 1, None)  # forget earlier tuning
    default = xs.xs_resolve_params(h, n, xs.xs_params_default(prec))
    cfg = xs.xs_tune_config_default(precision=prec, max_evals=16, reps=2)
    r = xs.xs_tune(h, E, m, cfg)
    say("baseline", r.baseline.as_dict(), r.baseline_ms, "best",
        r.best.as_dict(), r.best_ms, "evals", r.evaluated)
    assert choice(r.baseline) == choice(default)
    assert r.best_ms <= r.baseline_ms
    assert 1 <= r.evaluated <= 16 and 1 <= r.best_eval <= r.evaluated
    # later automatic calls of this size class run the winner
    assert choice(xs.xs_resolve_params(h, n, xs.xs_params_default(prec))) == \
        choice(r.best)
    out = xs.xs_lookup_batch(h, E, m, params=xs.xs_params_default(prec))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), env["ref"][prec][:n])
    xs.xs_set_tuned(h, 1, None)
    assert choice(xs.xs_resolve_params(h, n, xs.xs_params_default(prec))) == \
        choice(default)


BINS = (4000, 8192, 32768)


@pytest.fixture(scope="module")
def multi():
    """config-1 tables with three hash grids (the paper's default bin count
    and two more), and a second handle over the same data."""
    t = synth.config1_tables()
    q = synth.config1_queries()
    h = xs.xs_create_tables(t, ALL_FLAGS, BINS[0], extra_hash_bins=BINS[1:])
    yield dict(t=t, q=q, h=h,
               ref={xs.XS_FP64: oracle.lookup(t, q.E, q.mat),
                    xs.XS_FP32: oracle.lookup_f32(t, q.E, q.mat)})
    h.close()


def test_every_hash_grid_matches_oracle(multi):
    say("hash grids", BINS)
    h, q = multi["h"], multi["q"]
    info = xs.xs_table_info(h)
    assert info["n_hash_grids"] == 3 and info["hash_bins"] == list(BINS)
    assert info["n_hash_bins"] == BINS[0]
    E, m = dev(q.E, torch.float64), dev(q.mat, torch.int32)
    for prec in (xs.XS_FP64, xs.XS_FP32):
        for b in BINS:
            for sort in ("none", "band_material"):
                p = xs.make_params(prec, grid="hash", hash_bins=b, sort=sort,
                                   sort_threshold=0)
                assert xs.xs_resolve_params(h, len(q.E), p).hash_bins == b
                out = xs.xs_lookup_batch(h, E, m, params=p)
                torch.cuda.synchronize()
                assert np.array_equal(out.cpu().numpy(), multi["ref"][prec]), \
                    (prec, b, sort)
    # automatic bins resolve to the default grid; other grids carry 0
    assert xs.xs_resolve_params(h, 1000, xs.make_params(
        xs.XS_FP64, grid="hash")).hash_bins == BINS[0]
    assert xs.xs_resolve_params(h, 1000, xs.make_params(
        xs.XS_FP64, grid="unionized", hash_bins=8192)).hash_bins == 0
    with pytest.raises(xs.XsError) as e:
        xs.xs_resolve_params(h, 1000, xs.make_params(
            xs.XS_FP64, grid="hash", hash_bins=5000))
    assert e.value.status == xs.XS_ENOTBUILT


def test_checksum_keys_the_table_data(multi):
    t = multi["t"]
    a = xs.xs_table_info(multi["h"])["checksum"]
    h2 = xs.xs_create_tables(t, ALL_FLAGS, BINS[0], extra_hash_bins=BINS[1:])
    assert xs.xs_table_info(h2)["checksum"] == a
    h2.close()
    h3 = xs.xs_create_tables(t, ALL_FLAGS, BINS[0], extra_hash_bins=BINS[1:2])
    assert xs.xs_table_info(h3)["checksum"] != a
    h3.close()
    t2 = synth.config1_tables()
    t2.xs[7, 3] = np.nextafter(t2.xs[7, 3], np.inf)
    h4 = xs.xs_create_tables(t2, ALL_FLAGS, BINS[0], extra_hash_bins=BINS[1:])
    assert xs.xs_table_info(h4)["checksum"] != a
    h4.close()


def test_tune_sizes_through_the_cache(multi, tmp_path):
    """The N list is tuned once and written to the cache; a second handle
    over the same tables resolves every size from the file without running
    anything, and its automatic lookups then run the cached winners and
    return the oracle's bits."""
    say("tune sizes with cache")
    h, q = multi["h"], multi["q"]
    path = str(tmp_path / "tuned.txt")
    sizes = [20_000, 50_000, 100_000]
    E, m = dev(q.E, torch.float64), dev(q.mat, torch.int32)
    xs.xs_set_tuned(h, 1, None)
    cfg = xs.xs_tune_config_default(precision=xs.XS_FP32, max_evals=24, reps=2)
    res = xs.xs_tune(h, E, m, cfg, sizes=sizes, cache_path=path)
    assert [r.n for r in res] == sizes
    for r in res:
        say("tuned", r.n, r.best.as_dict(), r.best_ms, "evals", r.evaluated,
            "measured", r.measured)
        assert r.from_cache == 0 and 1 <= r.measured <= r.evaluated <= 24
        assert r.best_ms <= r.baseline_ms
        if r.best.grid == xs.XS_GRID_HASH:
            assert r.best.hash_bins in BINS
        else:
            assert r.best.hash_bins == 0
        if r.best.sort == xs.XS_SORT_NONE:
            assert r.best.sort_threshold == xs.INT64_MAX
        else:
            assert r.best.sort_threshold in (0, 20000, xs.INT64_MAX)
    lines = [l for l in open(path).read().splitlines() if not l.startswith("#")]
    assert len(lines) == len(sizes)

    h2 = xs.xs_create_tables(multi["t"], ALL_FLAGS, BINS[0],
                             extra_hash_bins=BINS[1:])
    try:
        again = xs.xs_tune(h2, E, m, cfg, sizes=sizes, cache_path=path)
        for r0, r in zip(res, again):
            assert r.from_cache == 1 and r.evaluated == 0 and r.measured == 0
            assert choice(r.best) == choice(r0.best)
            assert r.best.hash_bins == r0.best.hash_bins
            assert r.best.sort_threshold == r0.best.sort_threshold
        for n, r0 in zip(sizes, res):
            got = xs.xs_resolve_params(h2, n, xs.xs_params_default(xs.XS_FP32))
            assert choice(got) == choice(r0.best)
            out = xs.xs_lookup_batch(h2, E[:n], m[:n])  # NULL parameters: FP64
            out32 = xs.xs_lookup_batch(h2, E[:n], m[:n],
                                       params=xs.xs_params_default(xs.XS_FP32))
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(),
                                  multi["ref"][xs.XS_FP64][:n])
            assert np.array_equal(out32.cpu().numpy(),
                                  multi["ref"][xs.XS_FP32][:n])
    finally:
        h2.close()
    # a third handle loads the file directly (a serving process at start-up)
    h3 = xs.xs_create_tables(multi["t"], ALL_FLAGS, BINS[0],
                             extra_hash_bins=BINS[1:])
    try:
        assert xs.xs_tune_load(h3, path) == len(sizes)
        for n, r0 in zip(sizes, res):
            got = xs.xs_resolve_params(h3, n, xs.xs_params_default(xs.XS_FP32))
            assert choice(got) == choice(r0.best)
        assert xs.xs_tune_load(h3, str(tmp_path / "missing.txt")) == 0
    finally:
        h3.close()
    # other tables (another checksum) load nothing from it
    h4 = xs.xs_create_tables(multi["t"], ALL_FLAGS, BINS[0])
    try:
        assert xs.xs_tune_load(h4, path) == 0
    finally:
        h4.close()


def test_tune_active_with_queue_mode(multi):
    """xs_lookup_active tuned with the queue mode in the space: the winner is
    recorded for xs_lookup_active only, and active slots get the oracle's
    bits while inactive rows stay untouched."""
    say("tune active")
    h, q = multi["h"], multi["q"]
    n = 60_000
    E, m = dev(q.E[:n], torch.float64), dev(q.mat[:n], torch.int32)
    act_np = (np.arange(n) % 3 != 1).astype(np.uint8)
    act = dev(act_np, torch.uint8)
    xs.xs_set_tuned(h, 1, None)
    batch_before = xs.xs_resolve_params(h, n, xs.xs_params_default(xs.XS_FP64))
    cfg = xs.xs_tune_config_default(precision=xs.XS_FP64, max_evals=24, reps=2)
    r = xs.xs_tune(h, E, m, cfg, active=act)
    say("active winner", r.best.as_dict(), r.best_ms)
    assert r.best.queue in (xs.XS_QUEUE_COMPACT, xs.XS_QUEUE_PREDICATED)
    # the batch entry point is unaffected
    after = xs.xs_resolve_params(h, n, xs.xs_params_default(xs.XS_FP64))
    assert choice(after) == choice(batch_before)
    out = torch.full((n, 5), -5.0, dtype=torch.float64, device="cuda:0")
    xs.xs_lookup_active(h, E, m, act, out, params=xs.xs_params_default(xs.XS_FP64))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    on = act_np == 1
    assert np.array_equal(got[on], multi["ref"][xs.XS_FP64][:n][on])
    assert np.all(got[~on] == -5.0)
    xs.xs_set_tuned(h, 1, None)
