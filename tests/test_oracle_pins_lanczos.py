"""Pins of the oracle's Lanczos eigensolves, its truncation rule and its
streamed tree (Sec. 2.2, eq. Krylov_H, eq. reortho, eq. eff_H; Fig. 3;
Sec. 4.5, Fig. 11).

Each check sets the oracle routine against something built independently:
a closed-form spectrum, the Rayleigh-Ritz projection of a dense matrix on an
orthonormal basis obtained by QR of the Krylov matrix, a hand-made spectrum
around the cutoff, or the level-by-level tree of ``sum_tree``.
"""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as OH
from oracle import lanczos as OL
from oracle import mps as M


def _sym(rng, n):
    a = rng.standard_normal((n, n))
    return a + a.T


def _textbook_lanczos(A, v, m):
    """Three-term Lanczos with full re-orthogonalisation: alpha, beta."""
    V = [v / np.linalg.norm(v)]
    alpha, beta = [], []
    for i in range(m):
        w = A @ V[i]
        alpha.append(V[i] @ w)
        for u in V:
            w = w - (u @ w) * u
        for u in V:  # second pass
            w = w - (u @ w) * u
        if i + 1 < m:
            b = np.linalg.norm(w)
            beta.append(b)
            V.append(w / b)
    return np.array(alpha), np.array(beta)


# ---------------------------------------------------------------------------
# ritz_tridiagonal
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m", [2, 5, 12])
def test_ritz_tridiagonal_kac_closed_form(m):
    # Sylvester-Kac matrix: zero diagonal, off-diagonal sqrt(k (m - k)),
    # spectrum -(m-1), -(m-3), ..., m-1.  The off-diagonal varies along the
    # matrix, so a beta shifted by one index changes the spectrum.
    beta = [np.sqrt(k * (m - k)) for k in range(1, m)]
    shift = 0.75
    got = OL.ritz_tridiagonal([shift] * m, beta)
    ref = shift + np.arange(-(m - 1), m, 2, dtype=float)
    assert np.allclose(got, ref, atol=1e-12 * m, rtol=0)


def test_ritz_tridiagonal_equals_krylov_projection():
    # Lanczos tridiagonal of a dense symmetric A == Rayleigh-Ritz values of A
    # on the Krylov space span{v, Av, ..., A^(m-1) v} (orthonormal basis by QR)
    rng = np.random.default_rng(3)
    n, m = 40, 7
    A = _sym(rng, n)
    v = rng.standard_normal(n)
    alpha, beta = _textbook_lanczos(A, v, m)
    K = np.stack([np.linalg.matrix_power(A, k) @ v for k in range(m)], axis=1)
    Q, _ = np.linalg.qr(K)
    ref = np.linalg.eigvalsh(Q.T @ A @ Q)
    got = OL.ritz_tridiagonal(alpha, beta)
    assert np.allclose(got, ref, atol=1e-9 * np.abs(ref).max(), rtol=0)
    # a beta taken one index late is caught
    bad = OL.ritz_tridiagonal(alpha, list(beta[1:]) + [beta[0]])
    assert not np.allclose(bad, ref, atol=1e-6 * np.abs(ref).max(), rtol=0)


# ---------------------------------------------------------------------------
# ritz_generalized: Cholesky branch and canonical orthogonalisation branch
# ---------------------------------------------------------------------------

def _projected(A, vecs):
    Q, _ = np.linalg.qr(np.stack(vecs, axis=1))
    return np.linalg.eigvalsh(Q.T @ A @ Q)


def test_ritz_generalized_nonorthogonal_basis_cholesky_branch():
    rng = np.random.default_rng(4)
    n = 12
    A = _sym(rng, n)
    B = [rng.standard_normal(n) for _ in range(4)]
    V = np.stack(B, axis=1)
    S, Hm = V.T @ V, V.T @ A @ V
    assert np.linalg.eigvalsh(S)[0] > OL.S_EIG_FLOOR
    got = OL.ritz_generalized(Hm, S)
    ref = _projected(A, B)
    assert got.shape == (4,)
    assert np.allclose(got, ref, atol=1e-11 * np.abs(ref).max(), rtol=0)


def test_ritz_generalized_repeated_vector_canonical_branch():
    # a basis with a repeated vector has an exactly singular S: the
    # canonical orthogonalisation drops that direction and returns the
    # Rayleigh-Ritz values on the span of the distinct vectors
    rng = np.random.default_rng(5)
    n = 10
    A = _sym(rng, n)
    b0, b1 = rng.standard_normal(n), rng.standard_normal(n)
    V = np.stack([b0, b1, b1], axis=1)
    S, Hm = V.T @ V, V.T @ A @ V
    assert np.linalg.eigvalsh(S)[0] < OL.S_EIG_FLOOR
    got = OL.ritz_generalized(Hm, S)
    ref = _projected(A, [b0, b1])
    assert got.shape == (2,)
    assert np.allclose(got, ref, atol=1e-10 * np.abs(ref).max(), rtol=0)


def test_ritz_generalized_symmetrises_M():
    # M_ij = <v_i|w_j> need not be symmetric after truncation: only its
    # symmetric part enters (reading A13)
    rng = np.random.default_rng(6)
    A = _sym(rng, 6)
    K = rng.standard_normal((6, 6))
    got = OL.ritz_generalized(A + (K - K.T), np.eye(6))
    ref = np.linalg.eigvalsh(A)
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max(), rtol=0)


# ---------------------------------------------------------------------------
# truncation_rank: k = max(1, min(D, #{s_i > eps s_1}))  (reading A5)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1.0, 1e-20, 1e+20])
def test_truncation_rank_straddles_relative_cutoff(scale):
    eps = M.CUTOFF
    s = scale * np.array([1.0, 0.5, 3e-14, 1.001e-14, 1.0 * eps, 0.999e-14, 1e-15, 0.0])
    # kept: 1, 0.5, 3e-14, 1.001e-14 (strictly above eps s_1); eps s_1 itself is dropped
    assert M.truncation_rank(s, D=100) == 4
    assert M.truncation_rank(s, D=3) == 3
    assert M.truncation_rank(s, D=1) == 1


def test_truncation_rank_degenerate_inputs():
    assert M.truncation_rank(np.zeros(5), D=4) == 1
    assert M.truncation_rank(np.array([]), D=4) == 1
    assert M.truncation_rank(np.array([2.0]), D=4) == 1
    assert M.truncation_rank(np.full(6, 0.3), D=4) == 4


def test_svd_sweep_applies_the_cutoff_per_bond():
    # a 6-site state whose middle Schmidt spectrum is (1, 1e-10, 1e-13,
    # 1e-15): the last value falls under the relative cutoff 1e-14
    rng = np.random.default_rng(7)
    u, _ = np.linalg.qr(rng.standard_normal((8, 4)))
    v, _ = np.linalg.qr(rng.standard_normal((8, 4)))
    mat = u @ np.diag([1.0, 1e-10, 1e-13, 1e-15]) @ v.T  # (sites 0-2) x (sites 3-5)
    assert M.bonds(M.compress(_mps_from_matrix(mat), D=64))[3] == 3
    # the same state scaled by 1e-30: the cutoff is relative to s_1
    assert M.bonds(M.compress(_mps_from_matrix(1e-30 * mat), D=64))[3] == 3
    # a looser cutoff drops 1e-13 as well; D caps the count
    assert M.bonds(M.compress(_mps_from_matrix(mat), D=64, eps=1e-12))[3] == 2
    assert M.bonds(M.compress(_mps_from_matrix(mat), D=1))[3] == 1


def _mps_from_matrix(mat):
    """Exact 6-site MPS of the 64-vector vec(mat) (C order), via SVDs."""
    vec = mat.reshape(-1)
    sites, rest, l = [], vec.reshape(1, -1), 1
    for _ in range(5):
        rest = rest.reshape(l * 2, -1)
        u, s, vt = np.linalg.svd(rest, full_matrices=False)
        sites.append(u.reshape(l, 2, -1))
        l = u.shape[1]
        rest = s[:, None] * vt
    sites.append(rest.reshape(l, 2, 1))
    return sites


# ---------------------------------------------------------------------------
# StreamTree and apply_H_mapped: the pairs of sum_tree / apply_H
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", list(range(1, 20)) + [31, 32, 33])
def test_stream_tree_equals_level_tree(k):
    rng = np.random.default_rng(100 + k)
    leaves = [synth.random_mps_tensors(rng, 6, 4) for _ in range(k)]
    ref = OH.sum_tree(leaves, D=3)
    tr = OH.StreamTree(D=3)
    for x in leaves:
        tr.push(x)
    got = tr.finish()
    assert M.bonds(got) == M.bonds(ref)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_stream_tree_accepts_complete_subtrees():
    rng = np.random.default_rng(200)
    leaves = [synth.random_mps_tensors(rng, 6, 4) for _ in range(11)]
    ref = OH.sum_tree(leaves, D=3)
    tr = OH.StreamTree(D=3)
    sub = OH.sum_tree(leaves[:8], D=3)  # complete subtree of 8 leaves, level 3
    tr.push(sub, 3)
    for x in leaves[8:]:
        tr.push(x)
    got = tr.finish()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("window", [1, 4, 16])
def test_apply_H_mapped_equals_apply_H(window):
    rng = np.random.default_rng(300)
    L, N = 3, 3
    t, chi, zeta = synth.thc_factors(rng, L, N)
    psi = synth.random_mps_tensors(rng, 2 * L, 8)
    ref = OH.apply_H(psi, t, chi, zeta, D=4, mode="tree")
    got = OH.apply_H_mapped(psi, t, chi, zeta, D=4, window=window)
    assert M.bonds(got) == M.bonds(ref)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_thin_svd_both_drivers_reconstruct():
    # the SVD step of Fig. 3 through either LAPACK driver: a = u s vt with
    # orthonormal factors and s the square roots of the eigenvalues of a^T a
    import scipy.linalg
    rng = np.random.default_rng(8)
    a = rng.standard_normal((12, 5)) @ rng.standard_normal((5, 9))  # rank 5
    for u, s, vt in (M.thin_svd(a), scipy.linalg.svd(a, full_matrices=False, lapack_driver="gesvd")):
        assert np.allclose(u @ np.diag(s) @ vt, a, atol=1e-13 * np.abs(a).max(), rtol=0)
        assert np.allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-14, rtol=0)
        ev = np.sort(np.linalg.eigvalsh(a.T @ a))[::-1]
        assert np.allclose(s[:5], np.sqrt(ev[:5]), rtol=1e-12, atol=0)
        assert np.all(s[5:] < 1e-13 * s[0])


def test_hartree_fock_krylov_vectors_have_degenerate_schmidt_pairs():
    # spin-free H and a closed-shell start: the Krylov vectors are spin-flip
    # symmetric, so at bonds between spatial orbitals (even bond index) the
    # Schmidt values come in exactly degenerate pairs; a truncation cut can
    # fall inside such a pair, where the truncated state is not unique
    # (reading A6)
    from oracle import lanczos as OL
    L, N = 4, 8
    t, chi, zeta = synth.thc_factors(np.random.default_rng(0), L, N)
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(L, 4))
    st = OL.KrylovState(hf, 2)
    OL.krylov_step(st, t, chi, zeta, D=64)
    sv = M.schmidt_values(st.v[1])
    pairs = 0
    for bond, s in enumerate(sv, start=1):
        s = s[s > 1e-12 * s[0]]
        ties = int(np.sum(np.abs(np.diff(s)) < 1e-10 * s[0]))
        if bond % 2 == 0:
            pairs += ties
    assert pairs >= 3
