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
