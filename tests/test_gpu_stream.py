"""Persistent-kernel request streams against the oracle: every request's
output is bit-identical to the oracle's (FP64 and the FP32 form), across
grid methods, uneven sizes (empty, sub-tile, tile edges, many tiles) and
repeated graph replays with eager work in between."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

ALL_FLAGS = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED
SIZES = [0, 1, 63, 1023, 1024, 1025, 4999, 30000, 63000]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    t = synth.config1_tables()
    q = synth.config1_queries(sum(SIZES))
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    ref = oracle.lookup(t, q.E, q.mat)
    ref32 = oracle.lookup_f32(t, q.E, q.mat)
    yield dict(t=t, q=q, h=h, E=E, m=m, ref=ref, ref32=ref32)
    h.close()


def batch(env, sizes, prec):
    dt = torch.float64 if prec == xs.XS_FP64 else torch.float32
    reqs, spans, a = [], [], 0
    for n in sizes:
        out = torch.full((n, 5), -3.0, dtype=dt, device="cuda:0")
        reqs.append((env["E"][a:a + n], env["m"][a:a + n], out))
        spans.append((a, a + n))
        a += n
    return reqs, spans


@pytest.mark.parametrize("prec", [xs.XS_FP64, xs.XS_FP32])
@pytest.mark.parametrize("grid,unroll", [("nuclide", 1), ("hash", 2),
                                         ("unionized", 4), ("hash", 1)])
def test_stream_matches_oracle(env, grid, unroll, prec):
    say("stream", grid, unroll, prec)
    p = xs.make_params(prec, grid=grid, unroll=unroll)
    st = xs.xs_stream_create(env["h"], p, max_requests=64)
    rp = xs.xs_stream_params(st)
    assert rp.grid == xs.GRIDS[grid] and rp.unroll == unroll
    ref = env["ref"] if prec == xs.XS_FP64 else env["ref32"]
    for rnd in range(3):  # graph replays, eager work in between
        sizes = SIZES if rnd != 1 else SIZES[::-1][:5]
        reqs, spans = batch(env, sizes, prec)
        xs.xs_stream_submit(st, reqs)
        stats, makespan = xs.xs_stream_wait(st)
        assert len(stats) == len(sizes)
        for (E, m, out), (a, b), s in zip(reqs, spans, stats):
            assert s["n"] == b - a
            assert np.array_equal(out.cpu().numpy(), ref[a:b]), (rnd, a, b)
            if b > a:
                assert 0 <= s["start_us"] <= s["end_us"] <= makespan + 1e-6
            else:
                assert s["latency_us"] == 0
        eager = xs.xs_lookup_batch(env["h"], env["E"][:5000], env["m"][:5000],
                                   params=xs.make_params(prec, grid=grid))
        torch.cuda.synchronize()
        assert np.array_equal(eager.cpu().numpy(), ref[:5000])
    st.close()


def test_stream_errors(env):
    st = xs.xs_stream_create(env["h"], xs.make_params(xs.XS_FP64), max_requests=4)
    reqs, _ = batch(env, [10, 20], xs.XS_FP64)
    with pytest.raises(xs.XsError):
        xs.xs_stream_wait(st)  # nothing in flight
    xs.xs_stream_submit(st, reqs)
    with pytest.raises(xs.XsError) as e:
        xs.xs_stream_submit(st, reqs)  # previous batch not waited for
    assert e.value.status == xs.XS_EINVAL
    xs.xs_stream_wait(st)
    too_many, _ = batch(env, [1] * 5, xs.XS_FP64)
    with pytest.raises(xs.XsError):
        xs.xs_stream_submit(st, too_many)
    st.close()
    with pytest.raises(xs.XsError):
        xs.xs_stream_create(env["h"], None, max_requests=0)


def check_batch(env, reqs, spans, stats, makespan, prec):
    ref = env["ref"] if prec == xs.XS_FP64 else env["ref32"]
    assert len(stats) == len(spans)
    for (E, m, out), (a, b), s in zip(reqs, spans, stats):
        assert s["n"] == b - a
        assert np.array_equal(out.cpu().numpy(), ref[a:b]), (a, b)
        if b > a:
            assert 0 <= s["start_us"] <= s["end_us"] <= makespan + 1e-6
        else:
            assert s["latency_us"] == 0


@pytest.mark.parametrize("prec", [xs.XS_FP64, xs.XS_FP32])
@pytest.mark.parametrize("grid", ["unionized", "hash", "nuclide"])
def test_sorted_stream_matches_oracle(env, grid, prec):
    """A stream whose parameters sort every batch runs the batch-sorted
    pipeline captured into its graph: every request equals the oracle, every
    request ends after the last one started (all are gathered, sorted and
    looked up together), across replays of larger and smaller batches than
    before (buffers grow, the graph is updated or rebuilt) with eager work in
    between."""
    say("sorted stream", grid, prec)
    p = xs.make_params(prec, grid=grid, sort="band_material", sort_threshold=0)
    st = xs.xs_stream_create(env["h"], p, max_requests=64)
    rounds = [[1023, 4999, 30000], SIZES, SIZES[::-1][:5], SIZES]
    for rnd, sizes in enumerate(rounds):
        reqs, spans = batch(env, sizes, prec)
        xs.xs_stream_submit(st, reqs)
        stats, makespan = xs.xs_stream_wait(st)
        check_batch(env, reqs, spans, stats, makespan, prec)
        live = [s for s in stats if s["n"] > 0]
        assert min(s["end_us"] for s in live) >= max(s["start_us"] for s in live)
        eager = xs.xs_lookup_batch(env["h"], env["E"][:5000], env["m"][:5000],
                                   params=xs.make_params(prec, grid=grid))
        torch.cuda.synchronize()
        ref = env["ref"] if prec == xs.XS_FP64 else env["ref32"]
        assert np.array_equal(eager.cpu().numpy(), ref[:5000]), rnd
    st.close()


def test_stream_switches_between_modes(env):
    """With a sort threshold of 50,000 lookups, batches below it run the
    persistent kernel and batches above it the sorted pipeline, in any order
    on one stream; with debug mode on every batch runs the persistent kernel
    (the sorted pipeline's lookup cannot be captured while it synchronises).
    Every request equals the oracle."""
    say("stream modes")
    prec = xs.XS_FP32
    p = xs.make_params(prec, grid="unionized", sort="band_material",
                       sort_threshold=50000, block_size=128)
    st = xs.xs_stream_create(env["h"], p, max_requests=64)
    small = [1, 63, 1023, 1025, 4999, 30000]          # 37,111 lookups
    large = SIZES                                      # 101,135 lookups
    for sizes in (small, large, small, large, large, small):
        reqs, spans = batch(env, sizes, prec)
        xs.xs_stream_submit(st, reqs)
        stats, makespan = xs.xs_stream_wait(st)
        check_batch(env, reqs, spans, stats, makespan, prec)
    xs.xs_set_debug(env["h"], True)
    try:
        reqs, spans = batch(env, large, prec)
        xs.xs_stream_submit(st, reqs)
        stats, makespan = xs.xs_stream_wait(st)
        check_batch(env, reqs, spans, stats, makespan, prec)
    finally:
        xs.xs_set_debug(env["h"], False)
    st.close()
