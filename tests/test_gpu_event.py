"""The toy event loop (xs_event_run) against its serial reference: every
history's collision count, final energy and fate are bit-identical to
oracle/event.py, for FP64 and the FP32 form, every grid method, queued and
queueless lookups, sorted and unsorted queues, and buffers smaller than,
not a multiple of, and larger than the number of histories."""
import sys

import numpy as np
import pytest

import synth
from oracle import event as event_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

ALL_FLAGS = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED
H = 3000
SEED = 99


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    t = synth.config1_tables()
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    ref = {False: event_oracle.run_histories(t, H, SEED, fp32=False),
           True: event_oracle.run_histories(t, H, SEED, fp32=True)}
    yield dict(t=t, h=h, ref=ref)
    h.close()


CASES = [
    (xs.XS_FP64, dict(grid="hash", queue=xs.XS_QUEUE_COMPACT, sort="none"), 256),
    (xs.XS_FP64, dict(grid="unionized", queue=xs.XS_QUEUE_PREDICATED,
                      sort="band_material", sort_threshold=0), 1000),
    (xs.XS_FP64, dict(grid="nuclide", queue=xs.XS_QUEUE_COMPACT,
                      sort="material_energy", sort_threshold=0), 5000),
    (xs.XS_FP32, dict(grid="hash", queue=xs.XS_QUEUE_PREDICATED, sort="none",
                      unroll=2), 777),
    (xs.XS_FP32, dict(grid="unionized", queue=xs.XS_QUEUE_COMPACT,
                      sort="band_material", sort_threshold=0,
                      lookups_per_thread=1, unroll=1, lds_stage=1,
                      block_size=128), 2048),
]


@pytest.mark.parametrize("prec,kw,slots", CASES)
def test_event_loop_matches_reference(env, prec, kw, slots):
    say("event", prec, kw, slots)
    p = xs.make_params(prec, **kw)
    res, tal = xs.xs_event_run(env["h"], slots, H, SEED, params=p,
                               check_every=4)
    coll, e_end, fate = env["ref"][prec == xs.XS_FP32]
    assert res["histories"] == H
    assert np.array_equal(tal["fate"].cpu().numpy(), fate)
    assert np.array_equal(tal["collisions"].cpu().numpy(), coll)
    assert np.array_equal(tal["energy"].cpu().numpy(), e_end)
    # one lookup per collision
    assert res["lookups"] == int(coll.sum())
    assert res["iterations"] >= coll.max()


def test_event_loop_limits_and_errors(env):
    say("event errors")
    p = xs.make_params(xs.XS_FP64, grid="hash")
    with pytest.raises(xs.XsError) as e:
        xs.xs_event_run(env["h"], 64, H, SEED, params=p, max_iterations=3,
                        check_every=1)
    assert e.value.status == xs.XS_ETIMEOUT
    for bad in (dict(e_cut=0.0), dict(check_every=0),
                dict(max_iterations=0)):
        with pytest.raises(xs.XsError) as e:
            xs.xs_event_run(env["h"], 64, 10, SEED, params=p, **bad)
        assert e.value.status == xs.XS_EINVAL, bad
    res, _ = xs.xs_event_run(env["h"], 64, 0, SEED, params=p)
    assert res == {"iterations": 0, "lookups": 0, "histories": 0}
