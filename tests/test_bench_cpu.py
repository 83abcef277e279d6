"""bench.py's host-side pieces, without a device: the refusal of more than
one GPU, the algorithmic byte and flop counts, the roofline's choice of
ceiling and the kernel names the counter summaries are keyed by."""
import pytest

import bench


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_counts():
    # FP64: 12 in + 40 out, 96 per bracket pair + 12 per material entry
    assert bench.bytes_per_lookup(0, 1.0) == 52 + 108
    # FP32 form: 12 in + 20 out, 56 + 8 per nuclide
    assert bench.bytes_per_lookup(1, 2.0) == 32 + 128
    assert bench.flops_per_pair(0) == 29 and bench.flops_per_pair(1) == 44


def test_roofline_picks_the_binding_ceiling():
    n, nbar = 10_000_000, 65.0
    # cache-served (demand above the HBM peak, modest measured traffic): ALU,
    # reported against the vendor FP32 peak, the issue ceiling beside it
    r = bench.roofline(n, nbar, 1, 1.5, 3.7e9)
    flops = n * nbar * 44 / 1.5e-3 / 1e12
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(flops)
    assert r["peak"] == pytest.approx(157.3)
    assert r["frac"] == pytest.approx(flops / 157.3)
    assert r["alu"]["issue_peak"] == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert r["alu"]["issue_frac"] == pytest.approx(flops / r["alu"]["issue_peak"])
    assert r["hbm"]["demand_frac"] > 1.0 and r["hbm"]["measured_frac"] < 0.5
    assert r["hbm"]["measured_gbs"] == pytest.approx(3.7e9 / 1.5e-3 / 1e9)
    assert r["traffic"] == 3.7e9
    # traffic-bound: the HBM ceiling, achieved = algorithmic bytes / time
    r = bench.roofline(n, nbar, 0, 60.0, 4.3e11)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(n * (52 + 108 * nbar) / 60e-3 / 1e9 / 8000)
    assert r["alu"]["vendor_peak"] == pytest.approx(78.6)
    # without counters, a demand above the peak cannot be the bound
    assert bench.roofline(n, nbar, 1, 1.5, None)["bound"] == "alu"


def test_parity_summary():
    import numpy as np
    ref = np.array([[1.0, 2.0, 3.0, 4.0, 5.0]] * 4)
    got = ref.copy()
    r = bench.parity_fp64(got, ref)
    assert r["ok"] and r["bit_identical"] == 20 and r["max_rel"] == [0.0] * 5
    got[2, 3] = 4.0 * (1 + 4e-12)
    r = bench.parity_fp64(got, ref)
    assert not r["ok"] and r["max_rel"][3] == pytest.approx(4e-12, rel=1e-3)
    ref32 = ref.astype(np.float32)
    r = bench.parity_fp32(ref32.copy(), ref32, ref)
    assert r["ok"] and r["mismatches_vs_fp32_form"] == 0
    bad = ref32.copy()
    bad[0, 0] = np.nextafter(np.float32(1.0), np.float32(2.0))
    r = bench.parity_fp32(bad, ref32, ref)
    assert not r["ok"] and r["mismatches_vs_fp32_form"] == 1
    assert r["max_rel"][0] < 2e-6  # within the bar, but not the form's bits


def test_host_cpu_description():
    d = bench.host_cpus()
    assert d["threads"] >= 1 and d["nproc"] >= 1
    assert d["threads"] <= d["affinity"] <= d["nproc"]
    assert isinstance(d["model"], str)


def test_kernel_names_and_traffic_keys():
    from paper_2402_09222_amd import xs
    p = xs.make_params(xs.XS_FP32, grid=2, lookups_per_thread=1, unroll=1,
                       lds_stage=1)
    assert bench.kernel_name(p) == "k_lookup_lds<2, 1, 1, 1>"
    p = xs.make_params(xs.XS_FP32, grid=2, lookups_per_thread=2, unroll=1,
                       lds_stage=3)
    assert bench.kernel_name(p) == "k_lookup_lds<2, 1, 2, 3>"
    p = xs.make_params(xs.XS_FP64, grid=0, lookups_per_thread=1, unroll=2,
                       lds_stage=0)
    assert bench.kernel_name(p) == "k_lookup<0, 0, 1, 2>"
    p = xs.make_params(xs.XS_FP32, grid=1, lookups_per_thread=1, unroll=1,
                       lds_stage=0, wave_per_lookup=1)
    assert bench.kernel_name(p) == "k_lookup_wave<1, 1, false>"
    assert bench.kernel_name(p, pairs=True) == "k_lookup_wave<1, 1, false>"
    p.grid = 2
    assert bench.kernel_name(p, pairs=True) == "k_lookup_wave<2, 1, true>"
    p.precision = 0
    assert bench.kernel_name(p, pairs=True) == "k_lookup_wave<2, 0, false>"
    assert bench.measured_traffic("no such kernel", 128, 10) is None
