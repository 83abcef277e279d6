"""Throughput of the batched macroscopic cross-section lookup on one MI355X.

One step = one call of xs_lookup_batch over the whole batch (queue sort, when
the parameters ask for it, plus the lookup kernel), inputs resident in HBM.
The workload is the full-size synthetic table set: 355 nuclides x 11,303
grid points, 12 materials of 4 to 321 nuclides, 10,000,000 lookups with
log-uniform energies and uniform materials (see synth.workloads).

Two forms are timed for the headline: the plain FP64 lookup (per-nuclide
bisection, no sort, 256-lane blocks, one lookup per lane) and the FP32 form
with parameters chosen by the library's tuner; `value` is the latter.  The
FP64 form tuned the same way is timed beside them (`tuned_fp64`), so the
FP32 form's gain over plain FP64 splits into method and precision.  Each
step is one batch sorted and looked up, start to end, on one stream; the
same steps alternating over two streams (one step's sort overlapping the
previous step's lookup, as a serving loop would run them) are timed beside
it (`tuned_fp32.two_streams`, outside `value`).  The JSON line carries
the dominant kernel's roofline (algorithmic flops or bytes per launch /
average kernel time from HIP events on the launch stream, against the
vendor peaks, with the issue ceiling and the demand and measured HBM
figures beside it), the serial CPU oracle's rate (best of 5, on one thread
and on every thread of the process's CPU share) and the comparison of both
timed outputs with the oracle on every lookup of the batch; the run exits
with status 1 if either differs beyond its bar.  After the timed steps (and
outside `value`), `extras` carries the particles-in-flight sweep (1e5 to
8e6 lookups, the FP32 form tuned per size over the launch shapes and the
paper's tunables) and the uneven request stream (the graph-launched
request stream in both modes against per-request launches, p50/p99 latency)
in brief, each checked against the oracle on samples (--no-extras skips them).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# Vendor vector peaks (TFLOP/s): FP32 157.3 and FP64 78.6.  They count a
# fused multiply-add as two flops and, for FP32, packed two-wide issue.
VENDOR_PEAK_TFLOPS = {0: 78.6, 1: 157.3}
# The issue ceiling of the lookup's own arithmetic: 256 compute units x 64
# lanes x 2.4 GHz = 39.3e12 operations/s.  The lookup's products and sums
# must round separately (no fused multiply-add) and packed FP32 code
# generation is off, so each of its operations takes one lane-issue.
ISSUE_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
METRIC = ("macro-XS lookups/s (FP64 plain vs FP32 autotuned) + % HBM "
          "roofline, 1 MI355X")
# Parity bars: FP64 relative error per channel, FP32 form against FP64.
TOL_FP64 = 1e-12
TOL_FP32 = 2e-6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_lookup(precision: int, nbar: float) -> float:
    """Algorithmic bytes one lookup must move.

    FP64: energy + material in (12), five sums out (40), and per nuclide the
    bracketing pair of points (2 x (8 energy + 5 x 8 channels) = 96) plus its
    material entry (4 id + 8 density).  FP32 form: 12 in, 20 out, per nuclide
    2 x (8 + 5 x 4) = 56 plus 8 (id + FP32 density)."""
    if precision == 0:
        return 52.0 + 108.0 * nbar
    return 32.0 + 64.0 * nbar


def flops_per_pair(precision: int) -> float:
    """Algorithmic floating-point operations per (lookup, nuclide): 3
    subtractions, 1 division, 10 multiplications and 5 additions to
    interpolate, 5 multiplications and 5 additions to accumulate (29); the
    FP32 form adds 15 for the Kahan compensation (44)."""
    return 29.0 if precision == 0 else 44.0


def roofline(n: int, nbar: float, precision: int, kernel_ms: float,
             traffic) -> dict:
    """Roofline of one lookup kernel from its average launch time.

    `achieved` is always algorithmic work per launch / kernel time.  The
    ALU view reports the algorithmic flops against the vendor peak of the
    precision (the primary fraction) and against the issue ceiling of
    non-fused, non-packed operations.  The HBM view reports the algorithmic
    bytes as *demand* (above 1 means the demand is served from caches) and,
    when counters were taken, the measured HBM traffic.  The bound is the
    ALU one when its issue fraction exceeds the memory fraction (measured
    traffic, else the demand when it is at most 1)."""
    sec = kernel_ms * 1e-3
    B = bytes_per_lookup(precision, nbar)
    demand = n * B / sec / 1e9
    F = flops_per_pair(precision)
    alu_ach = n * nbar * F / sec / 1e12
    vendor = VENDOR_PEAK_TFLOPS[precision]
    hbm = {"peak": HBM_PEAK_GBS, "unit": "GB/s",
           "demand_bytes_per_lookup": B, "demand_gbs": demand,
           "demand_frac": demand / HBM_PEAK_GBS,
           "demand_note": "algorithmic bytes / kernel time; above 1 the "
                          "demand is served from caches, not HBM"}
    alu = {"unit": "TFLOP/s", "flops_per_pair": F, "pairs": n * nbar,
           "achieved": alu_ach, "vendor_peak": vendor,
           "vendor_frac": alu_ach / vendor,
           "issue_peak": ISSUE_PEAK_TFLOPS,
           "issue_frac": alu_ach / ISSUE_PEAK_TFLOPS,
           "issue_note": "one non-fused, non-packed operation per lane and "
                         "cycle on 256 CUs at 2.4 GHz"}
    if traffic is not None:
        hbm["measured_bytes_per_launch"] = traffic
        hbm["measured_gbs"] = traffic / sec / 1e9
        hbm["measured_frac"] = hbm["measured_gbs"] / HBM_PEAK_GBS
        mem_frac = hbm["measured_frac"]
    else:
        mem_frac = hbm["demand_frac"] if hbm["demand_frac"] <= 1.0 else 0.0
    if alu["issue_frac"] >= mem_frac:
        out = {"bound": "alu", "achieved": alu_ach, "peak": vendor,
               "unit": "TFLOP/s", "frac": alu_ach / vendor}
    else:
        out = {"bound": "hbm", "achieved": demand, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": demand / HBM_PEAK_GBS}
    out.update({"traffic": traffic, "kernel_ms": kernel_ms, "hbm": hbm,
                "alu": alu})
    return out


def lookup_sources_hash() -> str:
    """Hash of the lookup kernels' code (comments and blank space removed,
    so a comment edit does not orphan measured counters)."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_09222_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith("xs_lookup") or f == "xs_internal.h":
            text = open(os.path.join(csrc, f)).read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def kernel_name(p, pairs: bool = False) -> str:
    """The lookup kernel a resolved parameter set launches, as rocprofv3
    names it (template arguments: grid, precision, LPT[, U or stage shape];
    for one wave per lookup: grid, precision and whether it reads the FP32
    record pairs, which it does when the tables hold them)."""
    if getattr(p, "wave_per_lookup", 0) == 1:
        use = bool(pairs and p.precision == 1 and p.grid != 1)
        return (f"k_lookup_wave<{p.grid}, {p.precision}, "
                f"{'true' if use else 'false'}>")
    if p.lds_stage:
        return (f"k_lookup_lds<{p.grid}, {p.precision}, {p.lookups_per_thread}, "
                f"{p.lds_stage}>")
    return (f"k_lookup<{p.grid}, {p.precision}, {p.lookups_per_thread}, "
            f"{p.unroll}>")


def measured_traffic(kernel: str, block: int, n: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none for this kernel, block size and
    batch, or it was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "lookup_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        entries = json.load(open(path)).get("entries", [])
    except (OSError, ValueError, AttributeError):
        return None
    for rec in entries:
        if (rec.get("kernel") == kernel and rec.get("block_size") == block
                and rec.get("n_lookups") == n
                and rec.get("source_hash") == lookup_sources_hash()):
            return rec.get("hbm_bytes_per_launch")
    return None


def prewarm(fn, seconds: float) -> dict:
    """Untimed steps for about `seconds` before the warm-up steps.  After
    the tuner (or table creation) the first ~25 steps of a fresh output and
    workspace run up to 10 % slower than the sustained rate (measured per
    group of 20 calls: 1.32 ms of lookup kernel in the first group, 1.19 from
    the second on), more than five warm-up steps absorb; these bring the
    device to the state a serving loop runs in.  Reported in the line."""
    import torch
    if seconds <= 0:
        return {"seconds": 0.0, "steps": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while True:
        for _ in range(10):  # back to back, as in the timed steps
            fn()
        k += 10
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            break
    return {"seconds": round(time.perf_counter() - t0, 3), "steps": k}


def time_steps(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def kernel_time(xs, h, fn, calls: int) -> dict:
    import torch
    torch.cuda.synchronize()
    xs.xs_profile_begin(h)
    for _ in range(calls):
        fn()
    prof = xs.xs_profile_end(h)
    c = max(prof["calls"], 1)
    return {"ms_lookup": prof["ms_lookup"] / c, "ms_sort": prof["ms_sort"] / c,
            "ms_total": prof["ms_total"] / c, "calls": prof["calls"]}


def host_cpus() -> dict:
    """The host's CPUs as this process sees them: `nproc` (all online CPUs),
    `affinity` (the CPUs this process may run on), `quota` (the cgroup CPU
    quota in CPUs, None when unlimited or unreadable), `threads` (what the
    CPU baseline uses: the affinity set, capped by the quota) and the CPU
    model name."""
    nproc = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = nproc
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(period)
    except (OSError, ValueError):
        try:
            q = int(open("/sys/fs/cgroup/cpu/cpu.cfs_quota_us").read())
            period = int(open("/sys/fs/cgroup/cpu/cpu.cfs_period_us").read())
            if q > 0:
                quota = q / period
        except (OSError, ValueError):
            pass
    threads = aff
    if quota is not None:
        threads = max(1, min(threads, int(quota)))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": nproc, "affinity": aff, "quota": quota,
            "threads": threads, "model": model}


def cpu_baseline(tables, q, seconds: float):
    """The serial oracle as it stands (gcc -O2), timed best of 5 on one
    thread and on every thread the process may use (each thread runs the
    unmodified serial routine on a contiguous slice).  Samples are the
    first lookups of the batch, sized so the ten runs take about `seconds`.
    Returns (baseline dict, the oracle's FP64 output when the all-thread
    sample was the whole batch, else None)."""
    import oracle
    ot = oracle.OracleTables(tables)
    host = host_cpus()
    T = host["threads"]
    probe = min(len(q), 4000)
    t0 = time.perf_counter()
    oracle.lookup(ot, q.E[:probe], q.mat[:probe])
    rate1 = probe / max(time.perf_counter() - t0, 1e-9)

    def best_of(n, threads, reps=5):
        times, out = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            out = oracle.lookup(ot, q.E[:n], q.mat[:n], threads=threads)
            times.append(time.perf_counter() - t0)
        return n / min(times), n / float(np.median(times)), out

    # about 70 % of the budget to the all-thread runs, 30 % to one thread
    n_all = int(min(len(q), max(probe, rate1 * T * 0.7 * seconds / 5)))
    n_one = int(min(len(q), max(probe, rate1 * 0.3 * seconds / 5)))
    best_all, med_all, out_all = best_of(n_all, T)
    best_one, med_one, _ = best_of(n_one, 1)
    base = {"value": best_all, "unit": "lookups/s", "cores": T,
            "kind": "oracle",
            "sample": f"first {n_all} of the {len(q)} lookups, serial oracle "
                      f"(gcc -O2) on {T} threads, each a contiguous slice; "
                      f"best of 5 (median {med_all:.4g}/s)",
            "single_thread": {"value": best_one, "median": med_one,
                              "sample": f"first {n_one} lookups, best of 5"},
            "host": host}
    return base, (out_all if n_all == len(q) else None)


def _rel_stats(got, ref):
    """Per-channel max and mean of |got - ref| / ref (ref > 0)."""
    rel = np.abs(got.astype(np.float64) - ref) / ref
    return ([float(x) for x in rel.max(axis=0)],
            [float(x) for x in rel.mean(axis=0)])


def parity_fp64(got, ref) -> dict:
    """The FP64 lookup against the FP64 oracle: per-channel relative error
    (bar 1e-12) and how many values are bit-identical."""
    mx, mean = _rel_stats(got, ref)
    same = int(np.count_nonzero(got == ref))
    return {"max_rel": mx, "mean_rel": mean, "bit_identical": same,
            "values": int(got.size), "bar": TOL_FP64,
            "ok": bool(max(mx) <= TOL_FP64)}


def parity_fp32(got, ref32, ref64) -> dict:
    """The FP32 form against the oracle's FP32 form (bit for bit) and
    against the FP64 oracle (per-channel relative error, bar 2e-6)."""
    mx, mean = _rel_stats(got, ref64)
    bad = int(np.count_nonzero(got.view(np.uint32) != ref32.view(np.uint32)))
    return {"max_rel": mx, "mean_rel": mean, "mismatches_vs_fp32_form": bad,
            "values": int(got.size), "bar": TOL_FP32,
            "ok": bool(bad == 0 and max(mx) <= TOL_FP32)}


def launch_key(p, n):
    """What decides the kernels a call with parameters p runs for n lookups:
    the threshold only says whether the sort runs, the hash-bin count only
    matters under the hash grid."""
    sorted_ = p.sort != 0 and n >= p.sort_threshold
    return (p.grid, p.hash_bins if p.grid == 1 else 0,
            p.sort if sorted_ else 0, p.block_size, p.lookups_per_thread,
            p.unroll, p.lds_stage, p.wave_per_lookup)


# Hash grids built next to the default one for the particles-in-flight sweep
# and the tuner study (paper Table 1: 100 to 100k bins, default 4,000).
EXTRA_HASH_BINS = (4000, 32768)


def _pctl(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(round(q * (len(v) - 1))))] if v else 0.0


IN_FLIGHT = (100_000, 500_000, 1_000_000, 2_000_000, 4_000_000, 8_000_000)


def in_flight_row(args, torch, synth, xs, h, t, i, n, full=True):
    """One batch size of the particles-in-flight sweep (config 4): the FP32
    form tuned for this size (forest search over the launch shapes and the
    paper's tunables: hash-bin count, sort threshold), timed, and checked
    against the oracle's FP32 form on 20,000 sampled lookups (bit for bit);
    plain FP64 beside it.  `full` adds the captured-graph replay and every
    sort policy at the tuned launch shape."""
    import oracle
    q = synth.config4_queries(i, n)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    nbar = synth.mean_nuclides(t, q)
    ws = xs._workspace(xs.xs_workspace_size(h, n, xs.make_params(
        sort="band_material", sort_threshold=0)), E.device)
    outs = {0: torch.empty((n, 5), device="cuda:0", dtype=torch.float64),
            1: torch.empty((n, 5), device="cuda:0", dtype=torch.float32)}
    steps = args.steps if full else max(3, args.steps // 2)

    def rate(p):
        sec = time_steps(lambda: xs.xs_lookup_batch(
            h, E, m, out=outs[p.precision], params=p, workspace=ws),
            steps, args.warmup)
        return n / sec

    cfg = xs.xs_tune_config_default(precision=xs.XS_FP32,
                                    max_evals=args.tune_evals, reps=3)
    r = xs.xs_tune(h, E, m, cfg, workspace=ws, sizes=[n],
                   cache_path=args.tune_cache)[0]
    best = xs.xs_resolve_params(h, n, r.best)
    row = {"n": n, "mean_nuclides": nbar, "tuned": best.as_dict(),
           "tuned_lookups_per_s": rate(best),
           "tuned_hash_bins": best.hash_bins,
           "tuned_sort_threshold": best.sort_threshold,
           "tuner": {"evaluated": r.evaluated, "measured": r.measured,
                     "cut": r.cut, "best_eval": r.best_eval,
                     "space_size": r.space_size,
                     "from_cache": r.from_cache}}
    pick = np.unique(synth.Stream(43, i).integers(20_000, 0, n - 1))
    got = outs[1].cpu().numpy()[pick]
    ref32 = oracle.lookup_f32(t, q.E[pick], q.mat[pick],
                              threads=host_cpus()["threads"])
    row["tuned_equals_oracle_on_sample"] = bool(np.array_equal(got, ref32))
    plain = xs.make_params(xs.XS_FP64, grid="nuclide", sort="none",
                           block_size=256, lookups_per_thread=1, unroll=1,
                           lds_stage=0, sort_threshold=xs.INT64_MAX)
    row["plain_fp64_lookups_per_s"] = rate(plain)
    if full:
        def graph_rate(p):
            """The same call captured once in a HIP graph and replayed."""
            out = outs[p.precision]
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                xs.xs_lookup_batch(h, E, m, out=out, params=p, workspace=ws)
            torch.cuda.current_stream().wait_stream(side)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                xs.xs_lookup_batch(h, E, m, out=out, params=p, workspace=ws)
            sec = time_steps(g.replay, args.steps, args.warmup)
            del g
            return n / sec
        row["tuned_graph_lookups_per_s"] = graph_rate(best)
        for name, sp in xs.SORTS.items():
            p = xs.xs_params()
            p.precision, p.grid, p.sort = best.precision, best.grid, sp
            p.block_size, p.lookups_per_thread = best.block_size, best.lookups_per_thread
            p.unroll, p.lds_stage, p.queue = best.unroll, best.lds_stage, best.queue
            p.wave_per_lookup = best.wave_per_lookup
            p.hash_bins = best.hash_bins
            p.sort_threshold = 0 if sp else xs.INT64_MAX
            row[f"fp32_sort_{name}_lookups_per_s"] = rate(p)
    log(f"n={n}: tuned {row['tuned_lookups_per_s']:.4g}/s "
        f"({best.as_dict()}), plain FP64 {row['plain_fp64_lookups_per_s']:.4g}/s")
    return row


def sweep_in_flight(args, torch, synth, xs):
    """Config 4: batches of 1e5 ... 8e6 lookups on the full-size tables, with
    hash grids of 4,000, 8,192 and 32,768 bins; per batch size the FP32 form
    is tuned and timed, eagerly and as one captured HIP graph replayed, beside
    the plain FP64 lookup and the FP32 form under each sort policy at the
    tuned launch shape.  One JSON line per batch size."""
    t = synth.config2_tables()
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL |
             xs.XS_BUILD_FP32_PAIRS)
    extra = [b for b in EXTRA_HASH_BINS if b != args.bins]
    h = xs.xs_create_tables(t, flags, args.bins, extra_hash_bins=extra)
    ok = True
    for i, n in enumerate(IN_FLIGHT):
        row = in_flight_row(args, torch, synth, xs, h, t, i, n, full=True)
        ok = ok and row["tuned_equals_oracle_on_sample"]
        print(json.dumps(row), flush=True)
    h.close()
    return 0 if ok else 1


def request_stream(args, torch, synth, xs):
    """Config 5: an uneven stream of requests (sizes log-uniform in
    [1e3, 1e6], energies 70 % log-uniform and 30 % from narrow peaks) served
    by a request stream (xs_stream_*, one graph launch for the whole batch:
    the sorted pipeline captured into the graph, and the persistent kernel
    over LDS-sorted tiles), by one xs_lookup_requests call (batch-sorted: one
    gathered, sorted queue; tile-sorted: one launch, tiles sorted in LDS),
    and by one xs_lookup_batch launch per request with parameters tuned per
    size class.  A request's latency in the one-launch forms runs from its
    first tile's start to its last tile's end (device wall clock); per
    launch it is the HIP event time of its call.  Every form's output is
    compared with the per-request launches' bit for bit, and those with the
    oracle's FP32 form on 200,000 sampled lookups."""
    t = synth.config2_tables()
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL |
             xs.XS_BUILD_FP32_PAIRS)
    h = xs.xs_create_tables(t, flags, args.bins)
    line, ok = request_stream_line(
        args, torch, synth, xs, h, t, args.stream_requests,
        (1_000, 10_000, 100_000, 1_000_000, 10_000_000))
    print(json.dumps(line), flush=True)
    h.close()
    if not ok:
        log("PARITY FAILURE in the request-stream forms")
        return 1
    return 0


def request_stream_line(args, torch, synth, xs, h, t, n_requests,
                        tune_classes):
    """The request-stream measurements on handle h (see request_stream):
    the first n_requests requests of the stream; the FP32 form is tuned for
    each size in tune_classes first (classes tuned earlier on h are
    reused).  Returns (JSON-ready dict, every parity check passed)."""
    log("generating the request stream")
    sizes, q = synth.config5_requests(n_requests)
    total = int(sizes.sum())
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    out = torch.empty((total, 5), device="cuda:0", dtype=torch.float32)
    offs = np.concatenate(([0], np.cumsum(sizes)))
    log(f"{len(sizes)} requests, {total} lookups")

    # Tune the FP32 form per size class on slices of the stream.
    for n in tune_classes:
        if n > total:
            continue
        cfg = xs.xs_tune_config_default(precision=xs.XS_FP32,
                                        max_evals=args.tune_evals, reps=3)
        r = xs.xs_tune(h, E[:n], m[:n], cfg)
        log(f"tuned class {n}: {r.best.as_dict()} {r.best_ms:.3f} ms")
    reqs = [(E[a:b], m[a:b], out[a:b]) for a, b in zip(offs[:-1], offs[1:])]

    # Per-request launches, HIP events around each call.
    ws = xs._workspace(xs.xs_workspace_size(h, int(sizes.max()),
                       xs.make_params(xs.XS_FP32, sort="band_material",
                                      sort_threshold=0)), E.device)
    p_auto = xs.xs_params_default(xs.XS_FP32)
    st = torch.cuda.current_stream()
    best_launch = None
    for rep in range(max(1, args.steps // 5) + 1):
        evs = [(torch.cuda.Event(enable_timing=True),
                torch.cuda.Event(enable_timing=True)) for _ in reqs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (e0, e1), (Er, mr, orr) in zip(evs, reqs):
            e0.record(st)
            xs.xs_lookup_batch(h, Er, mr, out=orr, params=p_auto, workspace=ws)
            e1.record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = [a.elapsed_time(b) * 1e3 for a, b in evs]
        if rep > 0 and (best_launch is None or wall < best_launch["wall_s"]):
            best_launch = {"wall_s": wall, "lookups_per_s": total / wall,
                           "p50_us": _pctl(lat, 0.5), "p99_us": _pctl(lat, 0.99)}
    # The whole batch in one call: batch-sorted (automatic parameters, a
    # sort policy) and tile-sorted (no global sort).
    def one_call(params):
        batch = None
        best = None
        for rep in range(max(1, args.steps // 5) + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            batch = xs.xs_lookup_requests(h, reqs, params=params, batch=batch)
            stats, makespan = xs.xs_requests_stats(batch)
            wall = time.perf_counter() - t0
            lat = [r["latency_us"] for r in stats]
            if rep > 0 and (best is None or wall < best["wall_s"]):
                best = {"wall_s": wall, "lookups_per_s": total / wall,
                        "device_makespan_us": makespan,
                        "p50_us": _pctl(lat, 0.5), "p99_us": _pctl(lat, 0.99)}
        return best

    def snapshot():
        torch.cuda.synchronize()
        return out.cpu().numpy()

    out_launch = snapshot()  # the per-request launches' results
    p_batch = xs.xs_resolve_params(h, total, p_auto)
    p_tile = xs.xs_params_default(xs.XS_FP32)
    p_tile.sort = xs.XS_SORT_NONE
    p_tile = xs.xs_resolve_params(h, total, p_tile)
    out.fill_(-1.0)
    res_batch = one_call(p_batch)
    same = {"one_call_batch_sorted": bool(np.array_equal(snapshot(), out_launch))}
    out.fill_(-1.0)
    res_tile = one_call(p_tile)
    same["one_call_tile_sorted"] = bool(np.array_equal(snapshot(), out_launch))

    # Request streams: one graph launch per batch of requests, with the
    # automatic parameters (the batch sorts: gather, sort, lookup and
    # scatter captured into the stream's graph) and without a sort (the
    # persistent kernel over LDS-sorted tiles).
    def run_stream(params):
        stream = xs.xs_stream_create(h, params, max_requests=len(reqs))
        out.fill_(-1.0)
        res = None
        for rep in range(max(1, args.steps // 5) + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs.xs_stream_submit(stream, reqs)
            stats, makespan = xs.xs_stream_wait(stream)
            wall = time.perf_counter() - t0
            lat = [r["latency_us"] for r in stats]
            if rep > 0 and (res is None or wall < res["wall_s"]):
                res = {"wall_s": wall, "lookups_per_s": total / wall,
                       "device_makespan_us": makespan,
                       "device_lookups_per_s": total / (makespan * 1e-6),
                       "p50_us": _pctl(lat, 0.5), "p99_us": _pctl(lat, 0.99)}
        p_stream = xs.xs_stream_params(stream)
        stream.close()
        return res, p_stream

    res_stream, _ = run_stream(p_auto)
    same["graph_stream_sorted"] = bool(np.array_equal(snapshot(), out_launch))
    p_unsorted = xs.xs_params_default(xs.XS_FP32)
    p_unsorted.sort = xs.XS_SORT_NONE
    res_persist, p_stream = run_stream(p_unsorted)
    same["graph_stream_persistent"] = bool(np.array_equal(snapshot(),
                                                          out_launch))

    # The per-request launches against the oracle's FP32 form on a sample.
    import oracle
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(total, size=min(total, 200_000), replace=False))
    ref32 = oracle.lookup_f32(t, q.E[pick], q.mat[pick],
                              threads=host_cpus()["threads"])
    oracle_ok = bool(np.array_equal(out_launch[pick], ref32))
    line = {"config": "uneven request stream", "requests": len(reqs),
            "lookups": total, "per_request_launches": best_launch,
            "graph_stream_sorted": res_stream,
            "graph_stream_persistent": res_persist,
            "one_call_batch_sorted": res_batch,
            "one_call_tile_sorted": res_tile,
            "batch_params": p_batch.as_dict(),
            "tile_params": p_tile.as_dict(),
            "persistent_params": p_stream.as_dict(),
            "bit_identical_to_per_request_launches": same,
            "per_request_launches_equal_oracle_on_sample": oracle_ok}
    return line, bool(oracle_ok and all(same.values()))


def tuner_study(args, torch, synth, xs):
    """The paper's search against exhaustive search on the tuning space
    (grid method x sort x block x lookups/lane x nuclides in flight x LDS
    stage shape x wave per lookup, FP32 form) for one batch of the full-size
    workload.  Every
    configuration is timed once (best of 3 after 1 warm-up, HIP events);
    then the forest search (LCB, kappa 1.96) and uniform random search are
    replayed on that measured table over many seeds, so both see identical
    costs.  Reports how close each gets to the optimum and after how many
    evaluations it first lands within 5 % of it."""
    t = synth.config2_tables()
    n = args.study_n
    q = synth.config4_queries(5, n) if n <= 8_000_000 else synth.config2_queries(n)
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL |
             xs.XS_BUILD_FP32_PAIRS)
    extra = [b for b in EXTRA_HASH_BINS if b != args.bins]
    bins = [args.bins] + extra
    h = xs.xs_create_tables(t, flags, args.bins, extra_hash_bins=extra)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    out = torch.empty((n, 5), device="cuda:0", dtype=torch.float32)
    ws = xs._workspace(xs.xs_workspace_size(h, n, xs.make_params(
        xs.XS_FP32, sort="band_material", sort_threshold=0)), E.device)
    st = torch.cuda.current_stream()
    ev = (torch.cuda.Event(enable_timing=True),
          torch.cuda.Event(enable_timing=True))
    keyf = ("grid", "hash_bins", "sort", "block_size", "lookups_per_thread",
            "unroll", "lds_stage", "wave_per_lookup")
    table = {}  # launch key -> best of 3 (configurations that launch the
                # same kernels at this n are timed once)

    def measure(p, cutoff):
        k = launch_key(p, n)
        if k in table:
            return table[k]
        xs.xs_lookup_batch(h, E, m, out=out, params=p, workspace=ws)
        best = float("inf")
        for _ in range(3):
            ev[0].record(st)
            xs.xs_lookup_batch(h, E, m, out=out, params=p, workspace=ws)
            ev[1].record(st)
            ev[1].synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]))
        table[k] = best
        if len(table) % 100 == 0:
            log(f"  {len(table)} configurations timed")
        return best

    log(f"tuner study: exhaustive timing of the space at n={n}")
    t0 = time.perf_counter()
    ex = xs.xs_tune_search(7, xs.xs_tune_config_default(
        precision=xs.XS_FP32, strategy=xs.XS_TUNE_EXHAUSTIVE,
        timeout_factor=0.0, hash_bins=bins, confirm=0), measure)
    wall = time.perf_counter() - t0
    opt = ex.best_ms
    log(f"exhaustive: {ex.space_size} configurations in {wall:.1f} s, "
        f"optimum {opt:.3f} ms {ex.best.as_dict()}")

    if args.study_table:
        with open(args.study_table, "w") as fh:
            json.dump({"n_lookups": n, "keys": list(keyf),
                       "rows": [list(k) + [v] for k, v in table.items()]}, fh)

    def replay(p, cutoff):
        return table[launch_key(p, n)]

    evals = args.tune_evals
    forest = []
    for seed in range(args.study_seeds):
        trace = []

        def rec(p, cutoff):
            v = replay(p, cutoff)
            trace.append(v)
            return v
        r = xs.xs_tune_search(7, xs.xs_tune_config_default(
            precision=xs.XS_FP32, strategy=xs.XS_TUNE_FOREST,
            max_evals=evals, seed=seed, hash_bins=bins, confirm=0), rec)
        run_best = np.minimum.accumulate(trace)
        hit = np.nonzero(run_best <= 1.05 * opt)[0]
        forest.append((r.best_ms / opt, int(hit[0]) + 1 if len(hit) else None))
    # every configuration of the space, each at its launch's time
    allc = []
    xs.xs_tune_search(7, xs.xs_tune_config_default(
        precision=xs.XS_FP32, strategy=xs.XS_TUNE_EXHAUSTIVE,
        timeout_factor=0.0, hash_bins=bins, confirm=0),
        lambda p, cutoff: allc.append(replay(p, cutoff)) or allc[-1])
    allv = np.array(allc)
    costs = np.sort(allv)
    rng = np.random.default_rng(7)
    rand = []
    for seed in range(args.study_seeds):
        pick = allv[rng.choice(len(allv), evals, replace=False)]
        run_best = np.minimum.accumulate(pick)
        hit = np.nonzero(run_best <= 1.05 * opt)[0]
        rand.append((run_best[-1] / opt, int(hit[0]) + 1 if len(hit) else None))

    def summary(rows):
        ratio = [r for r, _ in rows]
        hits = [e for _, e in rows if e is not None]
        return {"mean_best_over_opt": float(np.mean(ratio)),
                "max_best_over_opt": float(np.max(ratio)),
                "runs_within_5pct": len(hits),
                "median_evals_to_5pct": (float(np.median(hits)) if hits
                                         else None)}
    line = {"study": "tuner", "n_lookups": n, "space_size": ex.space_size,
            "distinct_launches": len(table), "hash_bins": bins,
            "evals_per_search": evals, "seeds": args.study_seeds,
            "exhaustive": {"best_ms": opt, "best": ex.best.as_dict(),
                           "wall_s": wall,
                           "configs_within_5pct": int(np.sum(costs <= 1.05 * opt)),
                           "median_ms": float(np.median(costs))},
            "forest_lcb": summary(forest), "random": summary(rand)}
    print(json.dumps(line), flush=True)
    h.close()
    return 0


def energy_study(args, torch, synth, xs):
    """Run time, energy and energy-delay product of the full-size lookup
    (the paper's three objectives, section 7).  The FP32 form is tuned three
    times with the forest search, once per objective, each evaluation
    taking the board power over >= 0.25 s of back-to-back batches (between
    two steps of the energy accumulator) times the batch's run time; the
    three winners and the plain FP64 form are then measured over >= 1 s."""
    from paper_2402_09222_amd.energy import EnergyMeter, measure
    meter = EnergyMeter(0)
    t = synth.config2_tables()
    q = synth.config2_queries(args.n)
    n = len(q)
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL |
             xs.XS_BUILD_FP32_PAIRS)
    h = xs.xs_create_tables(t, flags, args.bins)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    outs = {0: torch.empty((n, 5), device="cuda:0", dtype=torch.float64),
            1: torch.empty((n, 5), device="cuda:0", dtype=torch.float32)}
    ws = xs._workspace(xs.xs_workspace_size(h, n, xs.make_params(
        xs.XS_FP32, sort="band_material", sort_threshold=0)), E.device)

    def call(p):
        return lambda: xs.xs_lookup_batch(h, E, m, out=outs[p.precision],
                                          params=p, workspace=ws)

    objective = {"time_ms": lambda s, j: s * 1e3,
                 "energy_j": lambda s, j: j,
                 "edp_js": lambda s, j: j * s}
    winners = {}
    for name, f in objective.items():
        log(f"energy study: tuning for {name}")

        done = [0]

        def evaluate(p, cutoff, f=f, done=done):
            sec, joule, _ = measure(call(p), meter, min_seconds=0.25)
            done[0] += 1
            if done[0] % 16 == 0:
                log(f"  {done[0]} configurations measured")
            return f(sec, joule)
        r = xs.xs_tune_search(7, xs.xs_tune_config_default(
            precision=xs.XS_FP32, strategy=xs.XS_TUNE_FOREST,
            max_evals=args.tune_evals, seed=1), evaluate)
        winners[name] = r.best
    plain = xs.make_params(xs.XS_FP64, grid="nuclide", sort="none",
                           block_size=256, lookups_per_thread=1, unroll=1,
                           lds_stage=0, sort_threshold=xs.INT64_MAX)
    rows = {}
    for label, p in [("plain_fp64", plain)] + [(f"fp32_best_{k}", v)
                                               for k, v in winners.items()]:
        p = xs.xs_resolve_params(h, n, p)
        sec, joule, _ = measure(call(p), meter, min_seconds=1.0)
        rows[label] = {"params": p.as_dict(), "ms": sec * 1e3,
                       "window": dict(measure.last),
                       "joules": joule, "watts": joule / sec,
                       "nj_per_lookup": joule / n * 1e9,
                       "edp_js": joule * sec,
                       "lookups_per_s": n / sec}
        log(f"{label}: {sec*1e3:.3f} ms, {joule:.4f} J, {joule/sec:.0f} W")
    print(json.dumps({"study": "energy", "n_lookups": n, "forms": rows}),
          flush=True)
    meter.close()
    h.close()
    return 0


def stream_study(args, torch, synth, xs):
    """One batch split over k concurrent streams sharing one table handle
    (the paper's several MPI ranks per GPU, section 5.1) against one launch
    of the whole batch with the same parameters.  Each stream gets a
    contiguous share of the 10M lookups, its own workspace and output, and
    its own sort; the time is the wall time of the whole batch."""
    t = synth.config2_tables()
    q = synth.config2_queries(args.n)
    n = len(q)
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL |
             xs.XS_BUILD_FP32_PAIRS)
    h = xs.xs_create_tables(t, flags, args.bins)
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    out = torch.empty((n, 5), device="cuda:0", dtype=torch.float32)
    cfg = xs.xs_tune_config_default(precision=xs.XS_FP32,
                                    max_evals=args.tune_evals, reps=3)
    xs.xs_tune(h, E, m, cfg)
    rows = []
    for k in (1, 2, 4, 8):
        parts = [(i * n // k, (i + 1) * n // k) for i in range(k)]
        p = xs.xs_resolve_params(h, parts[0][1] - parts[0][0],
                                 xs.xs_params_default(xs.XS_FP32))
        streams = [torch.cuda.Stream() for _ in range(k)]
        wss = [xs._workspace(xs.xs_workspace_size(h, b - a, p), E.device)
               for a, b in parts]

        def step():
            cur = torch.cuda.current_stream()
            for s in streams:
                s.wait_stream(cur)
            for s, (a, b), w in zip(streams, parts, wss):
                with torch.cuda.stream(s):
                    xs.xs_lookup_batch(h, E[a:b], m[a:b], out=out[a:b],
                                       params=p, workspace=w, stream=s)
            for s in streams:
                cur.wait_stream(s)
        sec = time_steps(step, args.steps, args.warmup)
        rows.append({"streams": k, "params": p.as_dict(), "ms": sec * 1e3,
                     "lookups_per_s": n / sec})
        log(f"{k} streams: {sec*1e3:.3f} ms, {n/sec:.4g} lookups/s")
    print(json.dumps({"study": "concurrent streams", "n_lookups": n,
                      "rows": rows}), flush=True)
    h.close()
    return 0


def event_study(args, torch, synth, xs):
    """The toy event loop (xs_event_run) on the full-size tables: 2M
    histories through buffers of 2.5e5 and 1e6 particles in flight, queued
    (compaction) against queueless (predicated) lookups, sorted (banded,
    threshold 20,000) against unsorted, FP32 form with the tuned grid
    method.  Histories/s is the paper's figure of merit (particles/s)."""
    t = synth.config2_tables()
    flags = (xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_UNIONIZED |
             xs.XS_BUILD_UNION_BY_MATERIAL |
             xs.XS_BUILD_FP32_PAIRS)
    h = xs.xs_create_tables(t, flags, args.bins)
    H = args.event_histories
    rows = []
    for slots in (250_000, 1_000_000):
        q = synth.config4_queries(2, slots)
        E = torch.from_numpy(q.E).to("cuda:0")
        m = torch.from_numpy(q.mat).to("cuda:0")
        xs.xs_tune(h, E, m, xs.xs_tune_config_default(
            precision=xs.XS_FP32, max_evals=args.tune_evals, reps=3))
        tuned = xs.xs_resolve_params(h, slots, xs.xs_params_default(xs.XS_FP32))
        for queue in (xs.XS_QUEUE_COMPACT, xs.XS_QUEUE_PREDICATED):
            for sort in ("none", "band_material"):
                p = xs.make_params(xs.XS_FP32, grid=tuned.grid, sort=sort,
                                   sort_threshold=20000, queue=queue,
                                   block_size=tuned.block_size,
                                   lookups_per_thread=tuned.lookups_per_thread,
                                   unroll=tuned.unroll,
                                   lds_stage=tuned.lds_stage)
                best = None
                for rep in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res, _ = xs.xs_event_run(h, slots, H, 1000 + rep, params=p)
                    torch.cuda.synchronize()
                    sec = time.perf_counter() - t0
                    if best is None or sec < best[0]:
                        best = (sec, res)
                sec, res = best
                row = {"slots": slots,
                       "queue": "queued" if queue == 0 else "queueless",
                       "sort": sort, "params": p.as_dict(), "s": sec,
                       "histories_per_s": H / sec,
                       "lookups_per_s": res["lookups"] / sec,
                       "iterations": res["iterations"],
                       "lookups": res["lookups"]}
                rows.append(row)
                log(f"slots {slots} {row['queue']} {sort}: "
                    f"{row['histories_per_s']:.4g} histories/s, "
                    f"{row['lookups_per_s']:.4g} lookups/s, "
                    f"{res['iterations']} iterations")
    print(json.dumps({"study": "event loop", "histories": H, "rows": rows}),
          flush=True)
    h.close()
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--bins", type=int, default=8192)
    ap.add_argument("--cpu-seconds", type=float, default=25.0,
                    help="budget of the CPU baseline's ten timed runs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--prewarm-s", type=float, default=0.2,
                    help="untimed steps for this long before the warm-up "
                         "steps of each timed form (0: none)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip comparing the timed outputs with the oracle")
    ap.add_argument("--no-union", action="store_true",
                    help="skip the 5.7 GB unionized index table")
    ap.add_argument("--params", type=str, default=None,
                    help="JSON dict of FP32 params instead of tuning")
    ap.add_argument("--tune-evals", type=int, default=96,
                    help="evaluation budget of the forest-surrogate tuner")
    ap.add_argument("--tune-cache", type=str, default=None,
                    help="tuned-parameter file read before and written after "
                    "tuning (--config 4)")
    ap.add_argument("--tune-strategy", choices=["forest", "exhaustive"],
                    default="forest")
    ap.add_argument("--only", choices=["plain", "tuned"], default=None,
                    help="time one form only (for profiling runs)")
    ap.add_argument("--config", type=int, choices=[2, 4, 5], default=2,
                    help="2: the headline line (default); 4: particles-in-"
                         "flight sweep; 5: uneven request stream")
    ap.add_argument("--stream-requests", type=int, default=2000)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the brief particles-in-flight sweep and request "
                    "stream that follow the timed steps")
    ap.add_argument("--extras-requests", type=int, default=100,
                    help="requests of the stream in the extras")
    ap.add_argument("--tuner-study", action="store_true",
                    help="exhaustive vs forest vs random search on the "
                         "tuning space (evaluations to the optimum)")
    ap.add_argument("--study-n", type=int, default=4_000_000)
    ap.add_argument("--study-seeds", type=int, default=20)
    ap.add_argument("--study-table", type=str, default=None,
                    help="also write every measured configuration here")
    ap.add_argument("--event", action="store_true",
                    help="toy event loop: histories/s, queued vs queueless, "
                         "sorted vs unsorted")
    ap.add_argument("--event-histories", type=int, default=2_000_000)
    ap.add_argument("--streams", action="store_true",
                    help="one batch split over 1, 2, 4, 8 concurrent streams")
    ap.add_argument("--energy", action="store_true",
                    help="run time / energy / EDP of the lookup and tuning "
                         "for each objective (board energy accumulator)")
    ap.add_argument("--gather-probe", action="store_true",
                    help="the achievable rate of random 32-128-byte reads "
                    "(paper_2402_09222_amd/probes/gather_probe.hip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain device copy of 2 GiB and exit (the "
                         "achievable-bandwidth figure and the reference for "
                         "scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not "
              "supported by this single-GPU build", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2402_09222_amd import xs

    if args.gather_probe:
        import subprocess
        exe = os.path.join(ROOT, "paper_2402_09222_amd", "gather_probe")
        if not os.path.exists(exe):
            raise RuntimeError(f"{exe} is missing: run __graft_entry__.build()")
        for mib in (128, 512):
            r = subprocess.run([exe, str(max(args.steps, 3)), str(mib)],
                               capture_output=True, text=True, timeout=120)
            if r.returncode != 0:
                log(r.stderr)
                return 1
            print(r.stdout.strip(), flush=True)
        return 0

    if args.copy_probe:
        nbytes = 2 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        sec = time_steps(lambda: dst.copy_(src), args.steps, args.warmup)
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "ms": sec * 1e3,
                          "gbs_read_plus_write": 2 * nbytes / sec / 1e9}),
              flush=True)
        return 0

    if args.event:
        return event_study(args, torch, synth, xs)
    if args.streams:
        return stream_study(args, torch, synth, xs)
    if args.energy:
        return energy_study(args, torch, synth, xs)
    if args.tuner_study:
        return tuner_study(args, torch, synth, xs)
    if args.config == 4:
        return sweep_in_flight(args, torch, synth, xs)
    if args.config == 5:
        return request_stream(args, torch, synth, xs)

    log("generating config-2 tables and queries")
    t = synth.config2_tables()
    q = synth.config2_queries(args.n)
    nbar = synth.mean_nuclides(t, q)
    flags = xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH | xs.XS_BUILD_FP32_PAIRS
    if not args.no_union:
        flags |= xs.XS_BUILD_UNIONIZED | xs.XS_BUILD_UNION_BY_MATERIAL
    extra = [b for b in EXTRA_HASH_BINS if b != args.bins]
    t0 = time.perf_counter()
    h = xs.xs_create_tables(t, flags, args.bins, extra_hash_bins=extra)
    build_s = time.perf_counter() - t0
    info = xs.xs_table_info(h)
    log(f"tables built in {build_s:.2f} s; mean nuclides per lookup {nbar:.2f}")
    E = torch.from_numpy(q.E).to("cuda:0")
    m = torch.from_numpy(q.mat).to("cuda:0")
    n = len(q)

    def runner(params):
        out = torch.empty((n, 5), device="cuda:0",
                          dtype=torch.float64 if params.precision == 0
                          else torch.float32)
        nb = xs.xs_workspace_size(h, n, params)
        ws = xs._workspace(nb, E.device)

        def fn():
            xs.xs_lookup_batch(h, E, m, out=out, params=params, workspace=ws)
        return fn, out

    def two_streams(params, serial_out):
        """The same steps issued alternately on two streams, each with its
        own workspace and output (a serving loop's double buffering): one
        step's sort overlaps the previous step's lookup.  Outside `value`;
        both outputs must equal the serial step's."""
        sts = [torch.cuda.Stream(), torch.cuda.Stream()]
        nb = xs.xs_workspace_size(h, n, params)
        wss = [xs._workspace(nb, E.device) for _ in sts]
        outs = [torch.empty((n, 5), device="cuda:0", dtype=torch.float32)
                for _ in sts]
        k = [0]

        def fn():
            j = k[0] % 2
            k[0] += 1
            xs.xs_lookup_batch(h, E, m, out=outs[j], params=params,
                               workspace=wss[j], stream=sts[j])
        torch.cuda.synchronize()
        sec = time_steps(fn, args.steps, args.warmup)
        same = all(np.array_equal(o.cpu().numpy(), serial_out) for o in outs)
        return {"value": n / sec, "ms_per_step": sec * 1e3, "streams": 2,
                "equal_to_serial_steps": bool(same)}

    def measure(params):
        params = xs.xs_resolve_params(h, n, params)
        fn, out = runner(params)
        pre = prewarm(fn, args.prewarm_s)
        sec = time_steps(fn, args.steps, args.warmup)
        kt = kernel_time(xs, h, fn, max(args.steps, 3))
        kname = kernel_name(params, pairs=bool(
            xs.xs_table_info(h)["build_flags"] & xs.XS_BUILD_FP32_PAIRS))
        traffic = measured_traffic(kname, params.block_size, n)
        rl = roofline(n, nbar, params.precision, kt["ms_lookup"], traffic)
        rl["kernel"] = kname
        torch.cuda.synchronize()
        return {
            "value": n / sec, "ms_per_step": sec * 1e3,
            "params": params.as_dict(), "kernel_ms": kt, "roofline": rl,
            "prewarm": pre,
        }, out.cpu().numpy()

    plain = tuned = None
    out_plain = out_tuned = None
    if args.only in (None, "plain"):
        p_plain = xs.make_params(xs.XS_FP64, grid="nuclide", sort="none",
                                 block_size=256, lookups_per_thread=1,
                                 unroll=1, lds_stage=0,
                                 sort_threshold=xs.INT64_MAX,
                                 queue=xs.XS_QUEUE_COMPACT)
        log("timing plain FP64")
        plain, out_plain = measure(p_plain)
        log(f"plain FP64: {plain['value']:.4g} lookups/s, "
            f"{plain['ms_per_step']:.3f} ms/step")
    tune_report = None
    if args.only in (None, "tuned"):
        if args.params:
            p32 = xs.make_params(xs.XS_FP32, **json.loads(args.params))
        else:
            cfg = xs.xs_tune_config_default(
                precision=xs.XS_FP32,
                strategy=(xs.XS_TUNE_FOREST if args.tune_strategy == "forest"
                          else xs.XS_TUNE_EXHAUSTIVE),
                max_evals=args.tune_evals, reps=3, warmup=1)
            log(f"tuning the FP32 form ({args.tune_strategy}, "
                f"{args.tune_evals} evaluations)")
            t0 = time.perf_counter()
            r = xs.xs_tune(h, E, m, cfg)
            tune_report = r.as_dict()
            tune_report["tune_s"] = time.perf_counter() - t0
            log(f"tuned in {tune_report['tune_s']:.1f} s: best {r.best_ms:.3f} "
                f"ms at evaluation {r.best_eval}/{r.evaluated}, baseline "
                f"{r.baseline_ms:.3f} ms, {r.cut} cut")
            # the tuned entry is recorded in the handle: resolve it as a
            # caller passing automatic parameters would
            p32 = xs.xs_resolve_params(h, n, xs.xs_params_default(xs.XS_FP32))
        log("timing FP32 form with", p32.as_dict())
        tuned, out_tuned = measure(p32)
        tuned["tuner"] = tune_report
        log(f"FP32 tuned: {tuned['value']:.4g} lookups/s, "
            f"{tuned['ms_per_step']:.3f} ms/step")
        if args.only is None:
            tuned["two_streams"] = two_streams(
                xs.xs_resolve_params(h, n, p32), out_tuned)
            log(f"FP32 tuned, steps alternating over two streams: "
                f"{tuned['two_streams']['value']:.4g} lookups/s")

    # The FP64 form tuned the same way: what the sort, the union index and
    # LDS staging give without the narrower data, so the FP32 form's gain
    # over plain FP64 splits into method and precision.
    tuned64 = out_tuned64 = None
    if args.only is None and not args.params:
        cfg = xs.xs_tune_config_default(precision=xs.XS_FP64,
                                        max_evals=args.tune_evals, reps=3,
                                        warmup=1)
        log("tuning the FP64 form")
        r = xs.xs_tune(h, E, m, cfg)
        p64 = xs.xs_resolve_params(h, n, xs.xs_params_default(xs.XS_FP64))
        tuned64, out_tuned64 = measure(p64)
        tuned64["tuner"] = {k: v for k, v in r.as_dict().items()
                            if k not in ("best", "baseline")}
        log(f"FP64 tuned: {tuned64['value']:.4g} lookups/s, "
            f"{tuned64['ms_per_step']:.3f} ms/step")

    head = tuned or plain
    cpu = None
    ref64 = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        cpu, ref64 = cpu_baseline(t, q, args.cpu_seconds)
        log(f"CPU oracle: {cpu['value']:.4g} lookups/s on {cpu['cores']} "
            f"threads, {cpu['single_thread']['value']:.4g} on one "
            f"({cpu['host']['model']}, nproc {cpu['host']['nproc']})")

    # The timed outputs against the oracle on every lookup of the batch.
    parity = None
    if not args.no_check:
        import oracle
        threads = host_cpus()["threads"]
        log("checking the timed outputs against the oracle")
        if ref64 is None:
            ref64 = oracle.lookup(t, q.E, q.mat, threads=threads)
        parity = {}
        if out_plain is not None:
            parity["plain_fp64"] = parity_fp64(out_plain, ref64)
        if out_tuned is not None:
            ref32 = oracle.lookup_f32(t, q.E, q.mat, threads=threads)
            parity["tuned_fp32"] = parity_fp32(out_tuned, ref32, ref64)
        if out_tuned64 is not None:
            parity["tuned_fp64"] = parity_fp64(out_tuned64, ref64)
        for k, v in parity.items():
            log(f"parity {k}: ok={v['ok']} max rel per channel "
                + " ".join(f"{x:.3g}" for x in v["max_rel"]))

    # The particles-in-flight sweep and the request stream in brief, after
    # the timed steps (they do not enter `value`).
    extras = None
    extras_ok = True
    if not args.no_extras and args.only is None and not args.params:
        extras = {"in_flight": []}
        log("extras: particles-in-flight sweep")
        for i, nn in enumerate(IN_FLIGHT):
            row = in_flight_row(args, torch, synth, xs, h, t, i, nn,
                                full=False)
            extras_ok = extras_ok and row["tuned_equals_oracle_on_sample"]
            extras["in_flight"].append(row)
        log(f"extras: request stream ({args.extras_requests} requests)")
        st_line, st_ok = request_stream_line(
            args, torch, synth, xs, h, t, args.extras_requests,
            (1_000, 10_000))
        extras["request_stream"] = st_line
        extras_ok = extras_ok and st_ok

    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if tuned else "f64",
        "data": "synthetic",
        "config": {
            "workload": ("synthetic full-size tables: 355 nuclides x 11,303 "
                         "points, 12 materials (4-321 nuclides), "
                         f"{n} lookups, E log-uniform, m uniform"),
            "n_lookups": n, "mean_nuclides": nbar,
            "hash_bins": info["hash_bins"], "union_size": info["union_size"],
            "table_build_s": build_s,
        },
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "parity": parity,
        "plain_fp64": plain,
        "tuned_fp32": tuned,
        "tuned_fp64": tuned64,
    }
    if plain and tuned:
        line["fp32_tuned_over_fp64_plain"] = tuned["value"] / plain["value"]
    if tuned64 and tuned:
        line["fp32_tuned_over_fp64_tuned"] = tuned["value"] / tuned64["value"]
    if tuned64 and plain:
        line["fp64_tuned_over_fp64_plain"] = tuned64["value"] / plain["value"]
    if extras is not None:
        line["extras"] = extras
    print(json.dumps(line), flush=True)
    h.close()
    if parity is not None and not all(v["ok"] for v in parity.values()):
        log("PARITY FAILURE: the timed outputs differ from the oracle")
        return 1
    if not extras_ok:
        log("PARITY FAILURE in the extras (in-flight sweep or request stream)")
        return 1
    if tuned and "two_streams" in tuned and \
            not tuned["two_streams"]["equal_to_serial_steps"]:
        log("PARITY FAILURE: two-stream steps differ from the serial steps")
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
