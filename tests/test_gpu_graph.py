"""Lookups captured in a HIP graph (torch.cuda.CUDAGraph on ROCm): the
whole xs_lookup_batch sequence (sort passes and lookup kernel) records into
a graph, and every replay — with other device work and synchronisations in
between — gives the eager result bit for bit, which equals the oracle's."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec,kw", [
    (xs.XS_FP64, dict(grid="hash", sort="band_material", sort_threshold=0,
                      block_size=256, lookups_per_thread=1, unroll=2)),
    (xs.XS_FP32, dict(grid="unionized", sort="band_material",
                      sort_threshold=0, block_size=128, lookups_per_thread=1,
                      unroll=1, lds_stage=1)),
    (xs.XS_FP32, dict(grid="nuclide", sort="none", block_size=256,
                      lookups_per_thread=2, unroll=1)),
])
def test_graph_replays_match_eager_and_oracle(prec, kw):
    say("graph", prec, kw)
    t = synth.config1_tables()
    q = synth.config1_queries(50_000)
    h = xs.xs_create_tables(t, xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH |
                            xs.XS_BUILD_UNIONIZED, 4000)
    try:
        ref = (oracle.lookup(t, q.E, q.mat) if prec == xs.XS_FP64
               else oracle.lookup_f32(t, q.E, q.mat))
        E = torch.from_numpy(q.E).to("cuda:0")
        m = torch.from_numpy(q.mat).to("cuda:0")
        p = xs.make_params(prec, **kw)
        dt = torch.float64 if prec == xs.XS_FP64 else torch.float32
        out = torch.zeros((len(q), 5), dtype=dt, device="cuda:0")
        ws = xs._workspace(xs.xs_workspace_size(h, len(q), p), E.device)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up off the default stream
            xs.xs_lookup_batch(h, E, m, out=out, params=p, workspace=ws)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        eager = out.clone()
        assert np.array_equal(eager.cpu().numpy(), ref)
        g = torch.cuda.CUDAGraph()
        out.zero_()
        with torch.cuda.graph(g):
            xs.xs_lookup_batch(h, E, m, out=out, params=p, workspace=ws)
        for rep in range(3):
            out.fill_(-1.0)
            x = torch.randn(1 << 18, device="cuda:0")  # other work between
            assert torch.isfinite(x.sum())
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), rep
        del g
    finally:
        h.close()
