"""xs_lookup_batch_noalloc (sort scratch in the library's fixed device array)
against xs_lookup_batch with a caller workspace: bit-identical outputs on
two calls in a row, the second smaller, for sorted and unsorted launch
shapes in both precisions; the sorted-size limit; outputs also equal the
oracle's."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402

ALL_FLAGS = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED
N1, N2 = 120_001, 37_777  # several radix tiles, ragged tails


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    t = synth.config1_tables()
    q = synth.config1_queries(N1)
    h = xs.xs_create_tables(t, ALL_FLAGS, 4000)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    ref = oracle.lookup(t, q.E, q.mat)
    ref32 = oracle.lookup_f32(t, q.E, q.mat)
    yield dict(h=h, E=E, m=m, ref=ref, ref32=ref32)
    h.close()


SHAPES = [
    dict(grid="nuclide", sort="material_energy", sort_threshold=0),
    dict(grid="hash", sort="band_material", sort_threshold=0),
    dict(grid="unionized", sort="band_material", sort_threshold=0,
         block_size=128, lookups_per_thread=1, unroll=1, lds_stage=1),
    dict(grid="unionized", sort="energy", sort_threshold=0),
    dict(grid="hash", sort="none"),
]


@pytest.mark.parametrize("prec", [xs.XS_FP64, xs.XS_FP32])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_noalloc_matches_batch(env, shape, prec):
    kw = SHAPES[shape]
    say("noalloc", kw, prec)
    p = xs.make_params(prec, **kw)
    ref = env["ref"] if prec == xs.XS_FP64 else env["ref32"]
    dt = torch.float64 if prec == xs.XS_FP64 else torch.float32
    for n in (N1, N2):  # the second call is smaller: stale scratch must not leak
        want = xs.xs_lookup_batch(env["h"], env["E"][:n], env["m"][:n],
                                  params=p)
        out = torch.full((n, 5), -7.0, dtype=dt, device="cuda:0")
        xs.xs_lookup_batch_noalloc(env["h"], env["E"][:n], env["m"][:n],
                                   out=out, params=p)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want.cpu().numpy()), (kw, n)
        assert np.array_equal(got, ref[:n]), (kw, n)


def test_noalloc_empty_and_limit(env):
    say("noalloc limits")
    p = xs.make_params(xs.XS_FP32, grid="hash", sort="band_material",
                       sort_threshold=0)
    e0 = env["E"][:0]
    m0 = env["m"][:0]
    out = xs.xs_lookup_batch_noalloc(env["h"], e0, m0, params=p)
    assert out.shape == (0, 5)
    # One more sorted lookup than the scratch holds is refused on the host
    # before anything is enqueued (the tensors are valid either way).
    big = xs.XS_NOALLOC_MAX_SORTED + 1
    E = torch.full((big,), 0.5, dtype=torch.float64, device="cuda:0")
    m = torch.zeros(big, dtype=torch.int32, device="cuda:0")
    with pytest.raises(xs.XsError) as ei:
        xs.xs_lookup_batch_noalloc(env["h"], E, m, params=p)
    assert ei.value.status == xs.XS_EWORKSPACE
    assert "at most 8323456 sorted lookups" in str(ei.value)
    # The largest sorted batch fills the scratch exactly and still matches
    # xs_lookup_batch.
    n = xs.XS_NOALLOC_MAX_SORTED
    q = synth.config1_queries(n)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    got = xs.xs_lookup_batch_noalloc(env["h"], E, m, params=p)
    want = xs.xs_lookup_batch(env["h"], E, m, params=p)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    # Unsorted batches need no scratch, so the limit does not apply.
    pn = xs.make_params(xs.XS_FP32, grid="hash", sort="none")
    big_n = n + 1000
    q = synth.config1_queries(big_n)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    got = xs.xs_lookup_batch_noalloc(env["h"], E, m, params=pn)
    want = xs.xs_lookup_batch(env["h"], E, m, params=pn)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
