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


@pytest.mark.parametrize("c", [1e-100, 1e100])
def test_compress_extreme_scale(thck, c):
    # the Gram matrices reach 1e+-200 and their column norms square again:
    # the tridiagonalisation's scaled-norm branch and the eigensolver's
    # normalisation by ||T|| carry the untruncated result through exactly
    rng = np.random.default_rng(80)
    n = 8
    psi = M.scale(_norm_mps(rng, n, 8), c)
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    out = ctx.compress(thck.DeviceMPS.from_sites(psi), D=16)
    ref = M.to_dense(psi)
    assert _rel(M.to_dense(out.to_sites()), ref) < 1e-12


def _rainbow(n):
    """Bell pairs between sites j and n-1-j: the middle bond carries 2^(n/2)
    equal Schmidt values.  Site j < n/2 appends its bit to the bond index,
    site j >= n/2 removes the last appended bit (the pairs nest)."""
    h = n // 2
    sites = []
    for j in range(n):
        if j < h:
            l, r = 2 ** j, 2 ** (j + 1)
            A = np.zeros((l, 2, r))
            for L in range(l):
                for s in range(2):
                    A[L, s, 2 * L + s] = 1.0
        else:
            l, r = 2 ** (n - j), 2 ** (n - j - 1)
            A = np.zeros((l, 2, r))
            for R in range(r):
                for s in range(2):
                    A[2 * R + s, s, R] = 1.0
        sites.append(A)
    return M.scale(sites, 2.0 ** (-h / 2))


@pytest.mark.parametrize("flags", [0, 1])
def test_compress_degenerate_spectrum(thck, flags):
    # 64 equal Schmidt values at the middle bond: one eigenvalue cluster
    # larger than the eigensolver's 32-member cap
    n = 12
    psi = _rainbow(n)
    sv = M.schmidt_values(psi)[n // 2 - 1]
    assert np.allclose(sv[:64], 0.125) and len(sv) == 64
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), n // 2, 2)
    ctx = thck.Context(t, chi, zeta)
    ref = M.to_dense(psi)
    full = ctx.compress(thck.DeviceMPS.from_sites(psi), D=64, flags=flags)
    assert _rel(M.to_dense(full.to_sites()), ref) < 1e-12
    # truncated inside the cluster: the kept subspace is not unique, but the
    # result is the orthogonal projection of psi onto it, with half the norm^2
    half = M.to_dense(ctx.compress(thck.DeviceMPS.from_sites(psi), D=32, flags=flags).to_sites())
    assert abs(np.dot(half, ref) - np.dot(half, half)) < 1e-12
    assert abs(np.dot(half, half) - 0.5) < 1e-12


def test_zero_state_compresses_to_zero(thck):
    # the zero MPS (every site zero, bonds as a random state's): compression
    # and H application return the zero state, finite, with the oracle's
    # bond-1 rule (k = max(1, ...) when s_1 = 0)
    rng = np.random.default_rng(61)
    n = 8
    t, chi, zeta = synth.thc_factors(np.random.default_rng(1), n // 2, 3)
    ctx = thck.Context(t, chi, zeta)
    zero = [np.zeros_like(a) for a in synth.random_mps_tensors(rng, n, 8)]
    dz = thck.DeviceMPS.from_sites(zero)
    out = ctx.compress(dz, D=8)
    ref = M.compress(zero, 8)
    got = out.to_sites()
    assert all(np.isfinite(a).all() for a in got)
    assert not M.to_dense(got).any()
    assert out.bond_list() == M.bonds(ref)
    h = ctx.apply_H(dz, D=8)
    assert not M.to_dense(h.to_sites()).any()


def test_evolve_with_graphs_matches_eager(thck):
    # the time step's compression batches replayed from captured HIP graphs
    # give the eager results bit for bit (two steps: the second replays the
    # graphs the first captured)
    rng = np.random.default_rng(62)
    t, chi, zeta = synth.thc_factors(rng, 3, 4)
    psi = _norm_mps(rng, 6, 4)
    ctx = thck.Context(t, chi, zeta)
    res = []
    for flags in (0, thck.FLAG_GRAPHS):
        (out,), dims = thck.evolve([(ctx, thck.DeviceMPS.from_sites(psi), None, 4, {"flags": flags})], K=4,
                                   delta=0.05, n_steps=2)
        res.append([np.concatenate([a.reshape(-1) for a in p.to_sites()]) for p in out])
    for a, b in zip(*res):
        assert a.shape == b.shape and np.array_equal(a, b)
