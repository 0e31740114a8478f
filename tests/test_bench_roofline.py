"""CPU tests of bench.py's roofline choice and of its one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

NAMES = ("lq", "sytrd", "tri_eig", "ormtr", "gemm", "sb2st", "q2")


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
    r = bench.roofline_of(*_stats(sb2st=(20.0, 2e12, 1e10, 4)))
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


def test_model_flops_reproduce_the_flop_model_of_the_scope():
    # LAPACK-formula model of one compressed H|psi> at L = 20, N = 80, D = 256:
    # 110.1 GFLOP per layer-compression (QR 21.3, absorb L 13.0, SVD 69.4,
    # absorb S V^T 6.4), 8.51 PFLOP per H|psi> over 51,600 layer- and 25,640
    # add-compressions
    import bench
    n = 40
    chi = [min(2 ** j, 2 ** (n - j), 256) for j in range(n + 1)]
    doubled = [1] + [2 * x for x in chi[1:-1]] + [1]
    assert abs(bench.model_compress_flops(doubled, 256) / 1e9 - 110.13) < 0.01
    assert abs(bench.model_flops_per_H(20, 80, 256) / 1e15 - 8.507) < 0.001
    # an untruncated compression of a 4-site MPS by hand: bonds (1, 2, 4, 2, 1)
    # LQ: site 3 (2 x 2 -> 2*(2*2*4 - 2*8/3)), site 2 (4 x 4), site 1 (2 x 8)
    fl = bench.model_compress_flops([1, 2, 4, 2, 1], 16)
    assert fl > 0


def test_one_stage_sytrd_stream_bytes():
    import bench
    # m = 4: trailing sizes 3, 2 (columns 0, 1): 6 + 3 entries, no second panel
    assert bench.one_stage_sytrd_bytes(4) == 8.0 * (6 + 3)
    assert abs(bench.one_stage_sytrd_bytes(512) / 1e6 - 200.74) < 0.01


def test_tridiagonalisation_at_the_method_bytes_is_compute_bound():
    # the method's bytes of a 512 x 512 tridiagonalisation (m^2 + 3m doubles)
    # against 4m^3/3 flops: ~85 flop/B, above the ridge, so the band
    # reduction (FP64 MFMA) is measured against the FP64 matrix peak in TFLOP/s
    m, nb = 512, 512
    fl, by = 4.0 / 3.0 * m ** 3 * nb, 8.0 * (m * m + 3 * m) * nb
    r = bench.roofline_of(*_stats(sytrd=(16.0, fl, by, 1), lq=(10.0, 1e12, 1e9, 1)))
    assert r["_class"] == "sytrd" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["peak"] == pytest.approx(bench.FP64_MFMA_PEAK_TFLOPS, rel=1e-3)
    assert r["frac"] == pytest.approx(fl / 16e-3 / 1e12 / bench.FP64_MFMA_PEAK_TFLOPS, rel=1e-3)


def test_two_stage_band_reduction_stream_bytes():
    # m = 34: panel 0 (rows 16..33: 18 x 16 panel, product over a 2 x 2
    # tile triangle), then the update of A[16:, 16:] (2 x 2 tiles), then
    # panel 1 has 2 rows (rows 32, 33): product over 1 tile, update of
    # A[32:, 32:] (1 tile); the loop ends at c0 = 48
    el = (2 * 16 * 18 + 3 * 256) + (2 * 3 * 256) + (2 * 16 * 2 + 1 * 256) + (2 * 1 * 256)
    assert bench.two_stage_sy2sb_bytes(34) == 8.0 * el
    # 512 x 512: ~8x less than the one-stage stream
    assert bench.two_stage_sy2sb_bytes(512) < bench.one_stage_sytrd_bytes(512) / 5
