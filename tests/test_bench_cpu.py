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
    # cache-served (demand above the HBM peak, modest measured traffic): ALU
    r = bench.roofline(n, nbar, 1, 1.5, 3.7e9)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(n * nbar * 44 / 1.5e-3 / 1e12)
    assert r["peak"] == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert r["hbm"]["frac"] > 1.0 and r["hbm"]["measured_frac"] < 0.5
    # traffic-bound: the HBM ceiling
    r = bench.roofline(n, nbar, 0, 60.0, 4.3e11)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(n * (52 + 108 * nbar) / 60e-3 / 1e9 / 8000)
    # without counters, a demand above the peak cannot be the bound
    assert bench.roofline(n, nbar, 1, 1.5, None)["bound"] == "alu"


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
    assert bench.kernel_name(p) == "k_lookup_wave<1, 1>"
    assert bench.measured_traffic("no such kernel", 128, 10) is None
