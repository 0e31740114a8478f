"""Pins of the oracle's Ritz vectors, restarted Lanczos and excited-state
runs (Sec. 2.2: restarting recovers convergence lost to truncation; a start
vector orthogonal to the lower eigenstates yields the excited ones, as the
paper does from a Hartree-Fock single excitation, Sec. 4.1).

References built independently: the generalised eigenproblem's defining
relations, textbook dense restarted Lanczos, and exact diagonalisation of
the dense Fock-space H of eq. (1) in a particle-number / S_z sector.
"""
import numpy as np
import pytest

import synth
from oracle import fermion as F
from oracle import lanczos as OL
from oracle import mps as M
from oracle import thc as TH


def _dense_to_mps(vec, n):
    sites, rest, l = [], vec.reshape(1, -1), 1
    for _ in range(n - 1):
        rest = rest.reshape(l * 2, -1)
        u, s, vt = np.linalg.svd(rest, full_matrices=False)
        sites.append(u.reshape(l, 2, -1))
        l = u.shape[1]
        rest = s[:, None] * vt
    sites.append(rest.reshape(l, 2, 1))
    return sites


def _case(L=3, N=4, seed=16):
    t, chi, zeta = synth.thc_factors(np.random.default_rng(seed), L, N)
    H = F.hamiltonian_sparse(t, TH.thc_v(chi, zeta))
    return t, chi, zeta, H


@pytest.mark.parametrize("singular", [False, True])
def test_ritz_pairs_solve_the_generalised_problem(singular):
    # H_sym X = S X diag(w), X^T S X = I: the defining relations of the Ritz
    # pairs in a non-orthogonal basis (rows of V), with or without a repeated
    # basis vector
    rng = np.random.default_rng(40)
    n = 9
    A = rng.standard_normal((n, n))
    A = A + A.T
    B = [rng.standard_normal(n) for _ in range(4)]
    if singular:
        B.append(B[1].copy())
    V = np.stack(B, axis=1)
    S, Hm = V.T @ V, V.T @ A @ V
    w, X = OL.ritz_pairs(Hm, S)
    assert np.allclose(X.T @ S @ X, np.eye(X.shape[1]), atol=1e-10)
    assert np.allclose(Hm @ X, S @ X @ np.diag(w), atol=1e-9 * np.abs(w).max())
    assert np.allclose(w, OL.ritz_generalized(Hm, S), atol=1e-12 * np.abs(w).max())
    # the Ritz vectors V X are orthonormal Ritz vectors of A on span(V)
    R = V @ X
    assert np.allclose(R.T @ A @ R, np.diag(w), atol=1e-9 * np.abs(w).max())


def test_restarted_mps_lanczos_matches_dense():
    # untruncated (D above every Schmidt rank of 6 sites): the MPS run with
    # restarts from the lowest Ritz vector equals the dense run
    t, chi, zeta, H = _case()
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(3, 2))
    K, restarts = 3, 2
    dense = OL.dense_lanczos_restarted(lambda x: H @ x, M.to_dense(hf), K, restarts)
    st = OL.KrylovState(hf, K)
    got = []
    for r in range(restarts + 1):
        for _ in range(K):
            rg, _, _ = OL.krylov_step(st, t, chi, zeta, D=64)
            got.append(rg)
        if r < restarts:
            st = OL.restart(st, 0, D=64)
    assert len(got) == len(dense)
    for a, b in zip(got, dense):
        assert np.allclose(a, b, atol=1e-10, rtol=0)


def test_restart_improves_on_the_first_cycle():
    # the restarted runs keep lowering the lowest Ritz value towards the
    # sector's ground energy
    t, chi, zeta, H = _case()
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(3, 2))
    nn, sz = F.number_operator_dense(6), F.sz_dense(6)
    sec = np.where((nn == 2) & (sz == 0))[0]
    e0 = np.linalg.eigvalsh(H.toarray()[np.ix_(sec, sec)])[0]
    st = OL.KrylovState(hf, 2)
    lowest = []
    for r in range(4):
        for _ in range(2):
            rg, _, _ = OL.krylov_step(st, t, chi, zeta, D=64)
        lowest.append(rg[0])
        st = OL.restart(st, 0, D=64)
    assert all(b <= a + 1e-12 for a, b in zip(lowest, lowest[1:]))
    assert lowest[-1] - e0 < lowest[0] - e0
    assert lowest[-1] >= e0 - 1e-10


def test_excited_state_from_a_start_orthogonal_to_the_ground_state():
    # start: the Hartree-Fock single excitation with the exact ground state
    # of its sector projected out; the Krylov space then holds no ground
    # state component and the lowest Ritz value converges to E_1
    L = 3
    t, chi, zeta, H = _case(L=L)
    n = 2 * L
    nn, sz = F.number_operator_dense(n), F.sz_dense(n)
    sec = np.where((nn == 2) & (sz == 0))[0]
    Hs = H.toarray()[np.ix_(sec, sec)]
    ev, U = np.linalg.eigh(Hs)
    g = np.zeros(2 ** n)
    g[sec] = U[:, 0]
    phi = M.to_dense(synth.occupation_mps_tensors(synth.single_excitation_occupation(L, 2, 0)))
    phi = phi - (g @ phi) * g
    st = OL.KrylovState(_dense_to_mps(phi, n), 8)
    for _ in range(8):
        rg, _, b = OL.krylov_step(st, t, chi, zeta, D=64)
        if b < 1e-10:
            break
    assert abs(rg[0] - ev[1]) < 1e-8 * max(1.0, abs(ev[1]))
    assert rg[0] > ev[0] + 1e-6


def test_single_excitation_occupation():
    occ = synth.single_excitation_occupation(4, 4, spin=1)
    # orbitals 0 doubly occupied, orbital 1 up only, orbital 2 down only
    assert occ == [1, 1, 1, 0, 0, 1, 0, 0]
    with pytest.raises(ValueError):
        synth.single_excitation_occupation(2, 4)
