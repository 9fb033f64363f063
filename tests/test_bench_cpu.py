"""CPU: the bench line's roofline accounting for the environment update."""

import bench


def _tm(flops, ms, launches=2):
    return {"env_flops": flops, "env_ms": ms, "env_launches": launches}


def test_env_roofline_peaks_and_fractions():
    # complex128 on FP64 matrix cores, complex64 on FP32 ones
    r = bench.env_roofline(_tm(5.9e11, 10.0), "c128")
    assert r["peak"] == 78.6 and abs(r["achieved"] - 59.0) < 1e-9 and abs(r["frac"] - 59.0 / 78.6) < 1e-12
    r = bench.env_roofline(_tm(1.1e12, 10.0), "c64")
    assert r["peak"] == 157.3 and abs(r["achieved"] - 110.0) < 1e-9
    # split precisions: bf16/f16 matrix cores, three 16-bit products per real multiply
    for p in ("split_f16", "split_bf16"):
        r = bench.env_roofline(_tm(1.46e12, 10.0), p)
        assert r["peak"] == 2500.0
        assert abs(r["algorithmic_tflops"] - 146.0) < 1e-9
        assert abs(r["achieved"] - 3 * 146.0) < 1e-9 and abs(r["frac"] - 438.0 / 2500.0) < 1e-12
    # per-launch figures
    r = bench.env_roofline(_tm(1e12, 4.0, launches=4), "c128")
    assert r["flops_per_launch"] == 2.5e11 and r["avg_launch_ms"] == 1.0 and r["launches"] == 4
    assert bench.env_roofline(_tm(1e12, 0.0), "c128")["achieved"] == 0.0


def test_traffic_recorded_for_every_precision():
    for p in ("c128", "c64", "split_f16", "split_bf16"):
        r = bench.env_roofline(_tm(1e12, 10.0), p)
        assert r["traffic"] is not None and r["traffic"] > 0
