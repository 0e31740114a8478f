"""GPU test of the allocation-free overlap (mps_overlap_noalloc) through the
C ABI: same value as mps_overlap on two calls in a row, the second with a
smaller input, and a rejected bond beyond the scratch's limit.  Collected
last (file name), so that it also runs after every other GPU test."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import mps as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_12708_amd as p
    return p


def _noalloc(thck, a, b):
    import torch
    lib = thck.load_library()
    fn = lib.mps_overlap_noalloc
    from paper_2409_12708_amd import thck as T
    fn.argtypes = [C.POINTER(T.ThcMps), C.POINTER(T.ThcMps), C.c_void_p, C.c_void_p]
    fn.restype = C.c_int
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    ad, bd = a.desc(), b.desc()
    st = fn(C.byref(ad), C.byref(bd), C.c_void_p(out.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


def test_noalloc_overlap_matches_mps_overlap(thck):
    import torch
    rng = np.random.default_rng(90)
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), 10, 2)
    ctx = thck.Context(t, chi, zeta)
    for n, Da, Db in ((20, 256, 128), (8, 8, 4)):  # second call smaller
        a = thck.DeviceMPS.from_sites(synth.random_mps_tensors(rng, n, Da))
        b = thck.DeviceMPS.from_sites(synth.random_mps_tensors(rng, n, Db))
        ref = ctx.overlap(a, b)
        st, out = _noalloc(thck, a, b)
        assert st == 0
        torch.cuda.synchronize()
        got = float(out.cpu()[0])
        print(f"noalloc overlap n={n} D={Da}/{Db}: {got:.16e} vs mps_overlap {ref:.16e}")
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))
        if n == 8:  # small enough for the dense oracle
            dense = M.to_dense(a.to_sites()) @ M.to_dense(b.to_sites())
            assert abs(got - dense) <= 1e-13 * max(1.0, abs(dense))


def test_noalloc_overlap_rejects_bond_above_limit(thck):
    rng = np.random.default_rng(91)
    a = thck.DeviceMPS.from_sites(synth.random_mps_tensors(rng, 20, 600))
    st, out = _noalloc(thck, a, a)
    assert st == -6  # THC_ECAPACITY, nothing launched
    assert np.isnan(float(out.cpu()[0]))
