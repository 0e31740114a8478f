"""CPU tests of bench.py's roofline choice and of its one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

NAMES = ("lq", "sytrd", "tri_eig", "ormtr", "gemm")


def _stats(**per):
    kms = {k: 0.0 for k in NAMES}
    kfl, kby, kn = dict(kms), dict(kms), {k: 0 for k in NAMES}
    for k, (ms, fl, by, n) in per.items():
        kms[k], kfl[k], kby[k], kn[k] = ms, fl, by, n
    return kms, kfl, kby, kn


def test_memory_bound_kernel_goes_under_the_hbm_roof():
    # 512 tridiagonalisations of 512 x 512 in 16 ms: 4m^3/3 flops and the
    # one-stage stream of ~200 MB per matrix -> ~0.9 flop/B, below the ridge
    m, nb = 512, 512
    fl, by = 4.0 / 3.0 * m ** 3 * nb, 200.7e6 * nb
    r = bench.roofline_of(*_stats(sytrd=(16.0, fl, by, 1), lq=(10.0, 1e12, 1e9, 1)))
    assert r["_class"] == "sytrd" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["peak"] == bench.HBM_PEAK_GBS
    assert r["achieved"] == pytest.approx(by / 16e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    assert r["intensity_flop_per_byte"] < r["ridge_flop_per_byte"]
    assert r["achieved_tflops"] == pytest.approx(fl / 16e-3 / 1e12, rel=1e-3)


def test_compute_bound_kernel_goes_under_its_unit_peak():
    # a GEMM at 200 flop/B sits above the FP64 ridge: MFMA roof in TFLOP/s
    r = bench.roofline_of(*_stats(gemm=(20.0, 2e12, 1e10, 4), sytrd=(5.0, 1e11, 1e11, 1)))
    assert r["_class"] == "gemm" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["peak"] == pytest.approx(bench.FP64_MFMA_PEAK_TFLOPS)
    assert r["achieved"] == pytest.approx(2e12 / 20e-3 / 1e12, rel=1e-3)
    assert r["algorithmic_bytes_per_launch"] == int(1e10 / 4)
    # a vector-ALU class above the ridge is priced against the ALU peak
    r = bench.roofline_of(*_stats(sytrd=(20.0, 2e12, 1e10, 4)))
    assert r["bound"] == "alu" and r["peak"] == pytest.approx(bench.FP64_VALU_PEAK_TFLOPS, rel=1e-3)


def test_classes_without_flops_are_not_dominant():
    # the eigensolver reports no flops: the longest class with flops is chosen
    r = bench.roofline_of(*_stats(tri_eig=(50.0, 0.0, 1e9, 1), ormtr=(10.0, 1e11, 1e9, 1)))
    assert r["_class"] == "ormtr"


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""
