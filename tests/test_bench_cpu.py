"""Host logic of bench.py: the roofline object's choice of bound and its figures."""
import pytest

import bench

N = 2 ** 20 + 1


def _rec(kernel, flops):
    return {"kernels": {kernel: {"n_states": N, "flops_fp64_per_state": flops,
                                 "hbm_bytes": 123456789}}}


def test_below_the_ridge_is_priced_against_hbm():
    # 30 FP64 scalars per state (240 B) and 500 flops: 2.1 flop/B, under the
    # 78.6 TFLOP/s / 8 TB/s ridge
    kern = {"filter_up": (1, 0.05), "traj_down_adjoint": (1, 0.08)}
    r = bench.roofline_for(kern, _rec("traj_down_adjoint", 500.0), True, N, 4, 2, 8, "f64")
    assert r["kernel"] == "traj_down_adjoint"
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    algo = bench.kernel_bytes(4, 2, 8, "traj_down_adjoint") * N
    assert algo == 240 * N
    assert r["achieved"] == pytest.approx(algo / 0.08e-3 / 1e9, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["traffic"] == 123456789
    assert r["intensity_flop_per_byte"] == pytest.approx(500 / 240, abs=0.01)


def test_above_the_ridge_is_priced_against_the_fp64_roof():
    # the filter up-sweep reads 2 scalars per state: far above the ridge
    kern = {"filter_up": (1, 0.066), "fused_down": (1, 0.06)}
    r = bench.roofline_for(kern, _rec("filter_up", 950.0), True, N, 4, 2, 8, "f64")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(950.0 * N / 0.066e-3 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, rel=1e-3)


def test_stale_or_missing_counters():
    kern = {"filter_up": (1, 0.066), "traj_down_adjoint": (1, 0.08)}
    r = bench.roofline_for(kern, _rec("traj_down_adjoint", 500.0), False, N, 4, 2, 8, "f64")
    assert r["traffic"] is None and r["counters_current"] is False
    r = bench.roofline_for(kern, None, False, N, 4, 2, 8, "f64")
    assert r["bound"] == "hbm" and r["traffic"] is None
    # a flop count taken on another problem size is not used
    rec = _rec("traj_down_adjoint", 500.0)
    rec["kernels"]["traj_down_adjoint"]["n_states"] = N - 1
    r = bench.roofline_for(kern, rec, True, N, 4, 2, 8, "f64")
    assert r["bound"] == "hbm" and r["traffic"] is None and "flops_per_state" not in r


def test_counts_taken_at_another_schedule_are_not_used():
    kern = {"filter_up": (1, 0.066), "fused_down": (1, 0.06)}
    rec = _rec("filter_up", 950.0)
    rec["states_per_lane"] = 16
    r = bench.roofline_for(kern, rec, True, N, 4, 2, 8, "f64", 16)
    assert r["bound"] == "alu" and r["traffic"] == 123456789 and "counters_schedule" not in r
    r = bench.roofline_for(kern, rec, True, N, 4, 2, 8, "f64", 32)
    assert r["bound"] == "hbm" and r["traffic"] is None
    assert r["counters_schedule"] == {"profiled": 16, "measured": 32}
