"""GPU tests of the C ABI's argument checks and of edge-sized problems.

Every rejected call must return its status without touching the GPU state
the next call sees; the edge sizes (two sites, THC rank one, sums with odd
counts at several tree levels) are checked against dense FP64 references.
"""
import numpy as np
import pytest

import synth
from oracle import fermion as F
from oracle import mps as M
from oracle import thc as TH

pytestmark = pytest.mark.gpu

EINVAL, ENONFINITE, ECAPACITY = -1, -4, -6


@pytest.fixture(scope="module")
def thck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_12708_amd as p
    return p


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _norm_mps(rng, n, D):
    psi = synth.random_mps_tensors(rng, n, D)
    return M.scale(psi, 1.0 / M.norm(psi))


def _status(fn):
    import paper_2409_12708_amd as p
    with pytest.raises(p.ThcError) as ei:
        fn()
    return ei.value.status


def test_rejected_arguments(thck):
    rng = np.random.default_rng(60)
    n = 8
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    psi = thck.DeviceMPS.from_sites(_norm_mps(rng, n, 4))
    # bond dimension beyond the kernels' limit, unknown precision
    assert _status(lambda: ctx.apply_H(psi, D=300)) == EINVAL
    assert _status(lambda: ctx.apply_H(psi, D=8, prec=7)) == EINVAL
    import ctypes as C
    o = thck.make_opts(8)
    # output smaller than thc_mps_capacity
    small = thck.DeviceMPS(n, 16)
    sd = small.desc()
    pd = psi.desc()
    assert ctx.lib.mps_compress(ctx.h, C.byref(pd), C.byref(sd), C.byref(o), None, None) == ECAPACITY
    # output aliasing the input
    big = thck.DeviceMPS.from_sites(_norm_mps(rng, n, 4), capacity_elems=thck.capacity(n, 8))
    bd = big.desc()
    assert ctx.lib.mps_compress(ctx.h, C.byref(bd), C.byref(bd), C.byref(o), None, None) == EINVAL
    # non-finite coefficient of a sum
    assert _status(lambda: ctx.sum_compress([1.0, float("nan")], [psi, psi], D=8)) == ENONFINITE
    # the context still works after the rejected calls
    ref = M.to_dense(psi.to_sites())
    got = M.to_dense(ctx.compress(psi, D=8).to_sites())
    assert _rel(got, ref) < 1e-12


def test_two_sites_rank_one(thck):
    # L = 1 spatial orbital (two spin-orbital sites), THC rank 1
    t, chi, zeta = synth.thc_factors(np.random.default_rng(61), 1, 1)
    rng = np.random.default_rng(62)
    psi = _norm_mps(rng, 2, 4)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.apply_H(thck.DeviceMPS.from_sites(psi), D=4)
    ref = F.apply_H_dense(M.to_dense(psi), t, TH.thc_v(chi, zeta))
    assert _rel(M.to_dense(out.to_sites()), ref) < 1e-12


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8, 9])
def test_sum_tree_counts(thck, k):
    # k terms: odd counts at one or more tree levels, so carried nodes and
    # nodes left in the truncation sweep's form (second members of pairs)
    # both reach later sums; untruncated, the result is the exact sum
    rng = np.random.default_rng(70 + k)
    n = 8
    terms = [_norm_mps(rng, n, 2) for _ in range(k)]
    coeffs = list(rng.standard_normal(k))
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    # compress each term first: library-made inputs carry their canonical form
    dev = [ctx.compress(thck.DeviceMPS.from_sites(x), D=16) for x in terms]
    out = ctx.sum_compress(coeffs, dev, D=16)
    ref = sum(c * M.to_dense(x) for c, x in zip(coeffs, terms))
    err = _rel(M.to_dense(out.to_sites()), ref)
    print(f"sum of {k}: rel err {err:.3e}, output form {out.canonical}")
    assert err < 1e-12
    assert out.canonical
    assert M.right_canonical_error(out.to_sites()) < 1e-12
