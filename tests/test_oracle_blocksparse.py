"""Pins of the block-sparse (N, 2 S_z) compression oracle against the dense
path: the states carry their quantum numbers exactly, the block factorisations
give the dense spectra, and the compressed state (and every bond's kept
Schmidt values) equals ``mps.compress`` of the same state wherever the cut
falls in a gap of the spectrum (Fig. 3, with the label bookkeeping of an
abelian-symmetric MPS).
"""
import numpy as np
import pytest

from oracle import blocksparse as B
from oracle import fermion as F
from oracle import mps as M


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _sector_weight_outside(vec, n_sites, n_elec, two_sz):
    N = F.number_operator_dense(n_sites)
    S = F.sz_dense(n_sites)
    bad = (N != n_elec) | (S != two_sz)
    return float(np.linalg.norm(vec[bad]))


@pytest.mark.parametrize("n_sites,n_elec,two_sz", [(6, 3, 1), (8, 4, 0), (8, 3, -1), (10, 5, 1)])
def test_random_state_lies_in_its_sector(n_sites, n_elec, two_sz):
    rng = np.random.default_rng(n_sites * 10 + n_elec)
    bs = B.random_mps(rng, n_sites, n_elec, two_sz, D=4)
    v = B.to_dense(bs)
    assert np.linalg.norm(v) > 0.0
    assert _sector_weight_outside(v, n_sites, n_elec, two_sz) == 0.0


def test_occupation_state_and_labels():
    occ = [1, 1, 0, 1, 0, 0]
    bs = B.from_occupation(occ)
    v = B.to_dense(bs)
    idx = int("".join(str(x) for x in occ), 2)  # site 0 most significant
    assert v[idx] == 1.0 and np.count_nonzero(v) == 1
    # last bond label: N = 3, 2 S_z = (up: sites 0, 2, 4) - (down: 1, 3, 5) = 1 - 2
    assert list(bs.bonds[-1]) == [(3, -1)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_right_canonical_form_keeps_the_state(seed):
    rng = np.random.default_rng(100 + seed)
    bs = B.random_mps(rng, 8, 4, 0, D=5)
    rc = B.right_canonicalize(bs)
    assert _rel(B.to_dense(rc), B.to_dense(bs)) < 1e-13
    assert M.right_canonical_error(B.to_mps(rc)) < 1e-13


def test_block_spectra_are_the_dense_spectra():
    # the union of the blocks' singular values at every bond is the dense
    # bond spectrum: the site matrices are block-diagonal in the labels
    rng = np.random.default_rng(7)
    bs = B.random_mps(rng, 10, 5, 1, D=6)
    rec_b, rec_d = [], []
    B.svd_sweep(B.right_canonicalize(bs), D=10 ** 9, eps=0.0, record=rec_b)
    M.svd_sweep(M.right_canonicalize(B.to_mps(bs)), D=10 ** 9, eps=0.0, record=rec_d)
    for sb, sd in zip(rec_b, rec_d):
        nz = sd[sd > 1e-12 * sd[0]]
        assert sb.size >= nz.size
        assert np.allclose(sb[:nz.size], nz, rtol=1e-11, atol=0.0)
        assert np.all(sb[nz.size:] <= 1e-12 * sd[0])


def _gapped(rec, D):
    # the cut at every bond falls in a gap (no near-tie between the last kept
    # and the first dropped value), so the truncation is unique
    for s in rec:
        k = M.truncation_rank(s, D)
        if k < s.size and s[k - 1] - s[k] < 1e-6 * s[0]:
            return False
    return True


@pytest.mark.parametrize("seed,D", [(0, 3), (1, 4), (2, 6), (3, 2)])
def test_truncated_compression_equals_the_dense_path(seed, D):
    rng = np.random.default_rng(200 + seed)
    bs = B.random_mps(rng, 10, 5, 1, D=6)
    dense = B.to_mps(bs)
    rec = []
    want = M.compress(dense, D, record=rec)
    if not _gapped(rec, D):
        pytest.skip("a near-tie at a cut: the truncation is not unique")
    got_b = B.compress(bs, D)
    got = B.to_mps(got_b)
    assert _rel(M.to_dense(got), M.to_dense(want)) < 1e-11
    # the kept Schmidt values per bond, and every bond within D
    assert all(sum(b.values()) <= D for b in got_b.bonds)
    for sb, sd in zip(M.schmidt_values(got), M.schmidt_values(want)):
        k = min(sb.size, sd.size)
        assert np.allclose(sb[:k], sd[:k], rtol=1e-9, atol=1e-13 * sd[0])
    # the output is left-canonical up to the last site, block by block
    assert M.left_canonical_error(got) < 1e-12
    # and stays in the sector
    assert _sector_weight_outside(M.to_dense(got), 10, 5, 1) < 1e-14 * np.linalg.norm(M.to_dense(got))


def test_untruncated_compression_is_exact():
    rng = np.random.default_rng(9)
    bs = B.random_mps(rng, 8, 4, 0, D=4)
    out = B.compress(bs, D=10 ** 6)
    assert _rel(B.to_dense(out), B.to_dense(bs)) < 1e-12


def test_direct_sum_equals_the_dense_sum():
    rng = np.random.default_rng(11)
    a = B.random_mps(rng, 8, 4, 0, D=3)
    b = B.random_mps(rng, 8, 4, 0, D=2)
    c = B.from_occupation([1, 1, 0, 0, 1, 1, 0, 0])
    s = B.direct_sum([(0.7, a), (-1.3, b), (2.0, c)])
    want = 0.7 * B.to_dense(a) - 1.3 * B.to_dense(b) + 2.0 * B.to_dense(c)
    assert _rel(B.to_dense(s), want) < 1e-13
    # interior sectors add their dimensions
    for j in range(1, 8):
        for q, d in s.bonds[j].items():
            assert d == a.bonds[j].get(q, 0) + b.bonds[j].get(q, 0) + c.bonds[j].get(q, 0)
    # and the sum compresses as the dense sum does (gapped cut)
    rec = []
    want_c = M.compress(M.direct_sum([(0.7, B.to_mps(a)), (-1.3, B.to_mps(b)), (2.0, B.to_mps(c))]), 3, record=rec)
    if _gapped(rec, 3):
        assert _rel(B.to_dense(B.compress(s, 3)), M.to_dense(want_c)) < 1e-11


def test_block_svd_costs_less_than_dense():
    # the saving the block form is for: at half filling the bond matrices
    # split into several sectors, and the factorisation cost falls accordingly
    rng = np.random.default_rng(13)
    bs = B.random_mps(rng, 12, 6, 0, D=8, dims=lambda j, q: 8)
    blk, dense = B.svd_flops(bs)
    assert blk < 0.5 * dense
