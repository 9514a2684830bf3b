"""Host-side checks of bench.py's roofline model for the fused split forms (no
GPU): the slot counts per entry, the matrix-core time share and which bound is
reported, against hand-computed values."""
import math

import pytest

import bench

GAUSS = (1.0, 0.15, 0.5, 0.4)      # the ensemble's Gaussian Mexican hat
NPAD = 65536


def test_far_form_slots_per_entry():
    # far entry: one exp2 (4 slots) and the split by shift and subtraction (3)
    assert bench.fused_slots_per_w(0, 0, far=True) == 7.0
    # near entry: (rho t) / rho, two exp2, a multiply-add, the split
    assert bench.fused_slots_per_w(0, 0, far=False) == 13.0
    # without far blocks, the norm expansion leaves the 6 r^2 slots to the matrix
    # cores: Gaussian eval 7 + 2 * 4 + 1 = 16, minus 6, plus the dot-product split 2
    assert bench.eval_slots(0, 0) == 16.0
    assert bench.fused_slots_per_w(0, 0, norm=True) == 12.0
    assert bench.fused_slots_per_w(0, 0, norm=False) == 18.0


def test_norm_path_bound_and_kernel_name():
    assert bench.fused_norm_path(0, GAUSS, 0, 1.0)               # unit-size surface
    assert not bench.fused_norm_path(0, GAUSS, 0, 2.0)           # sig^2 max|x|^2 = 128 > 96
    assert not bench.fused_norm_path(1, GAUSS, 0, 1.0)           # exponential kernel: differences


def test_far_form_reports_matrix_core_time_share():
    avg_s, far = 1.65e-3, 0.75
    r = bench.ensemble_roofline("otf_bf16x3", NPAD, 0, GAUSS, avg_s, 1.0, far)
    w = float(NPAD) ** 2
    share = w * (384.0 / 2.5e15 + 8.0 / 157.3e12) / avg_s
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["kernel"] == "k_mfma_otf<bf16,0,2,8>"
    assert math.isclose(r["frac"], share, rel_tol=1e-12)
    assert math.isclose(r["achieved"], share * 2500.0, rel_tol=1e-12)
    assert math.isclose(r["mfma_time_frac"], share, rel_tol=1e-12)
    spw = 0.25 * 13.0 + 0.75 * 7.0
    assert math.isclose(r["slots_per_w"], spw, rel_tol=1e-12)
    assert math.isclose(r["alu_frac"], w * spw / avg_s / bench.VALU_LANES_PER_S, rel_tol=1e-12)
    assert r["alu_frac"] < r["frac"]


@pytest.mark.parametrize("avg_s", [1e-3, 1e-2])
def test_fp16_fused_form_is_vector_bound(avg_s):
    # FP16 takes the differences (no FP32 products for t): 18 + 2 = 20 slots per entry
    r = bench.ensemble_roofline("otf_fp16x3", NPAD, 0, GAUSS, avg_s, 1.0, 0.75)
    assert r["kernel"] == "k_mfma_otf<fp16,0,2,4>"
    assert r["slots_per_w"] == 20.0 and r["far_block_fraction"] == 0.0
    w = float(NPAD) ** 2
    assert math.isclose(r["mfma_time_frac"], w * 384.0 / 2.5e15 / avg_s, rel_tol=1e-12)
    assert r["bound"] == ("alu" if r["alu_frac"] >= r["mfma_time_frac"] else "mfma")
