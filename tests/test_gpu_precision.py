"""FP32 form on 10M lookups of the config-1 tables (the precision
configuration): per-channel max and mean relative error against the FP64
oracle, printed and bounded by 2e-6; every lookup bit-identical to the
oracle's FP32 form."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2402_09222_amd import xs  # noqa: E402


def test_fp32_error_statistics_10m():
    t = synth.config1_tables()
    q = synth.config3_queries(10_000_000)
    print("config 3: oracle FP64 and FP32 forms on 10M lookups", flush=True)
    ref = oracle.lookup(t, q.E, q.mat, threads=16)
    ref32 = oracle.lookup_f32(t, q.E, q.mat, threads=16)
    h = xs.xs_create_tables(t, xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH |
                            xs.XS_BUILD_UNIONIZED, 4000)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    stats = {}
    for grid in ("nuclide", "hash", "unionized"):
        p = xs.make_params(xs.XS_FP32, grid=grid, sort="band_material",
                           sort_threshold=0, block_size=256,
                           lookups_per_thread=1, unroll=2)
        out = xs.xs_lookup_batch(h, E, m, params=p).cpu().numpy()
        assert np.array_equal(out, ref32), grid
        rel = np.abs(out.astype(np.float64) - ref) / ref
        stats[grid] = {"max": rel.max(axis=0).tolist(),
                       "mean": rel.mean(axis=0).tolist()}
        print(grid, json.dumps(stats[grid]), flush=True)
        assert rel.max() <= 2e-6
    h.close()
    d = os.environ.get("XS_STATS_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "fp32_error_config3.json"), "w") as f:
            json.dump(stats, f, indent=1)
