"""Debug mode (xs_set_debug): invalid queries turn into XS_EINVAL with their
count and first position while the results are still written (NaN rows,
-1 indices); inactive slots are not checked; results are bit-identical with
debug mode on and off; the hash-grid counters move only where a hash search
leaves its fast window, and never exceed the searches made."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

ALL_FLAGS = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype,
                                                       device="cuda:0")


@pytest.fixture(scope="module")
def env():
    t = synth.config1_tables()
    q = synth.config1_queries()
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    yield dict(t=t, q=q, h=h)
    xs.xs_set_debug(h, False)
    h.close()


def test_debug_off_by_default_and_bits_unchanged(env):
    say("debug bits")
    h, q = env["h"], env["q"]
    assert xs.xs_debug_counters(h) == dict(on=0, calls=0, invalid_queries=0,
                                           hash_bin_scans=0,
                                           hash_full_searches=0)
    E, m = dev(q.E, torch.float64), dev(q.mat, torch.int32)
    outs = {}
    for on in (False, True):
        xs.xs_set_debug(h, on)
        for grid in ("nuclide", "hash", "unionized"):
            p = xs.make_params(xs.XS_FP64, grid=grid, sort="band_material",
                               sort_threshold=0)
            outs[(on, grid)] = xs.xs_lookup_batch(h, E, m, params=p).cpu().numpy()
    ref = oracle.lookup(env["t"], q.E, q.mat)
    for k, v in outs.items():
        assert np.array_equal(v, ref), k
    c = xs.xs_debug_counters(h)
    assert c["on"] == 1 and c["calls"] == 3 and c["invalid_queries"] == 0
    pairs = int(np.diff(env["t"].mat_offsets)[q.mat].sum())
    assert 0 <= c["hash_full_searches"] <= c["hash_bin_scans"] <= pairs
    xs.xs_set_debug(h, False)
    assert xs.xs_debug_counters(h)["on"] == 0


def test_invalid_queries_fail_with_count_and_position(env):
    say("debug invalid")
    h, t = env["h"], env["t"]
    M = t.n_materials
    E = np.array([0.5, np.nan, 0.25, -1.0, 0.5, 0.0, np.inf, 0.125, 0.5])
    m = np.array([0, 1, 2, 0, -1, 1, 2, 3, M], np.int32)
    bad = ~(np.isfinite(E) & (E > 0) & (m >= 0) & (m < M))
    Ed, md = dev(E, torch.float64), dev(m, torch.int32)
    ref = oracle.lookup(t, E, m)
    xs.xs_set_debug(h, True)
    try:
        for grid in ("nuclide", "hash", "unionized"):
            out = torch.zeros((len(E), 5), dtype=torch.float64, device="cuda:0")
            with pytest.raises(xs.XsError) as e:
                xs.xs_lookup_batch(h, Ed, md, out=out,
                                   params=xs.make_params(grid=grid))
            assert e.value.status == xs.XS_EINVAL
            msg = str(e.value)
            assert f"{int(bad.sum())} of {len(E)}" in msg, msg
            assert f"first at {int(np.argmax(bad))}" in msg, msg
            got = out.cpu().numpy()
            assert np.array_equal(got, ref, equal_nan=True), grid
            assert np.all(np.isnan(got[bad]))
        c = xs.xs_debug_counters(h)
        assert c["calls"] == 3 and c["invalid_queries"] == 3 * int(bad.sum())
        # inactive invalid slots are not checked
        act = dev((~bad).astype(np.uint8), torch.uint8)
        out = torch.zeros((len(E), 5), dtype=torch.float64, device="cuda:0")
        xs.xs_lookup_active(h, Ed, md, act, out)
        got = out.cpu().numpy()
        assert np.array_equal(got[~bad], ref[~bad])
        # the validation path reports the same queries
        sizes = np.where((m >= 0) & (m < M),
                         np.diff(t.mat_offsets)[np.clip(m, 0, M - 1)], 0)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        with pytest.raises(xs.XsError) as e:
            xs.xs_lookup_indices(h, Ed, md, dev(off, torch.int64),
                                 grid="hash")
        assert e.value.status == xs.XS_EINVAL
    finally:
        xs.xs_set_debug(h, False)
    # off again: invalid queries are NaN rows without an error
    out = xs.xs_lookup_batch(h, Ed, md)
    assert np.array_equal(out.cpu().numpy(), ref, equal_nan=True)


def test_hash_counters_track_the_bin_width(env):
    """One hash bin per table: the fast window (two intervals from the bin's
    bracket) misses for most queries, so the scan counter grows with the
    lookups; with 4,000 bins far fewer searches leave the fast window."""
    say("debug hash counters")
    t, q = env["t"], env["q"]
    E, m = dev(q.E, torch.float64), dev(q.mat, torch.int32)
    pairs = int(np.diff(t.mat_offsets)[q.mat].sum())
    ref = oracle.lookup(t, q.E, q.mat)
    scans = {}
    for bins in (1, 4000):
        h = xs.xs_create_tables(t, xs.XS_BUILD_HASH, bins)
        try:
            xs.xs_set_debug(h, True)
            p = xs.make_params(grid="hash", sort="none")
            out = xs.xs_lookup_batch(h, E, m, params=p).cpu().numpy()
            assert np.array_equal(out, ref), bins
            c = xs.xs_debug_counters(h)
            assert c["calls"] == 1
            assert c["hash_full_searches"] <= c["hash_bin_scans"] <= pairs
            scans[bins] = c["hash_bin_scans"]
        finally:
            h.close()
    say("hash bin scans", scans, "pairs", pairs)
    assert scans[1] > pairs // 2
    assert scans[4000] < scans[1] // 10


def test_set_debug_errors(env):
    with pytest.raises(xs.XsError) as e:
        xs.load_library()
        st = xs.load_library().xs_set_debug(env["h"].handle, 2)
        xs._check(st, "xs_set_debug")
    assert e.value.status == xs.XS_EINVAL
