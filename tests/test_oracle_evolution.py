"""Pins of the oracle's Krylov time evolution (Sec. 2.2: psi(t + delta) =
sum_i a_i v_i with a(delta) = exp(-i delta H~) a(0); App. A error bound).

References built independently of ``oracle.evolution``: scipy's matrix
exponential of the dense Fock-space H of eq. (1) (``oracle.fermion``), the
Galerkin projection onto an orthonormalised span computed with a QR, the
closed form exp(-i E delta) psi of an eigenstate, the O(delta^K) order of a
K-vector Krylov step, and the Hochbruck-Lubich bound printed in App. A.
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import evolution as EV
from oracle import fermion as F
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


def _case(L, N, seed):
    rng = np.random.default_rng(seed)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    H = F.hamiltonian_sparse(t, TH.thc_v(chi, zeta)).toarray()
    return rng, t, chi, zeta, H


def _dense_hfun(H):
    n = int(np.log2(H.shape[0]))

    def h(x):
        return _dense_to_mps(H @ M.to_dense(x), n)
    return h


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --- the small problem ------------------------------------------------------

@pytest.mark.parametrize("singular", [False, True])
def test_coefficients_are_the_galerkin_exponential(singular):
    # basis B (columns, non-orthogonal, complex), A Hermitian: B a(delta) must
    # equal Q expm(-i delta Q^H A Q) Q^H b_0 with Q an orthonormal basis of
    # span(B) from a QR (rank-revealing for the singular case)
    rng = np.random.default_rng(3)
    n, m, delta = 12, 5, 0.37
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A + A.conj().T
    B = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    if singular:
        B[:, 3] = B[:, 1] + 2.0 * B[:, 0]
    S = B.conj().T @ B
    Mm = B.conj().T @ A @ B
    a = EV.evolution_coefficients(Mm, S, delta)
    Q, R, piv = scipy.linalg.qr(B, mode="economic", pivoting=True)
    r = int(np.sum(np.abs(np.diag(R)) > 1e-10 * abs(R[0, 0])))
    Q = Q[:, :r]
    want = Q @ scipy.linalg.expm(-1j * delta * (Q.conj().T @ A @ Q)) @ (Q.conj().T @ B[:, 0])
    assert _rel(B @ a, want) < 1e-12


def test_coefficients_orthonormal_basis_is_expm():
    rng = np.random.default_rng(4)
    m = 7
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = A + A.conj().T
    a = EV.evolution_coefficients(A, np.eye(m, dtype=complex), 0.8)
    assert np.allclose(a, scipy.linalg.expm(-0.8j * A)[:, 0], atol=1e-13)


def test_split_terms_order_and_skips():
    x = (["r0"], None)
    y = (["r1"], ["i1"])
    re, im = EV.split_terms([2.0 + 0.0j, 1.0 - 3.0j], [x, y])
    assert [c for c, _ in re] == [2.0, 1.0, 3.0]
    assert [p for _, p in re] == [["r0"], ["r1"], ["i1"]]
    assert [c for c, _ in im] == [1.0, -3.0]
    assert [p for _, p in im] == [["i1"], ["r1"]]


# --- whole steps against the dense exponential --------------------------------

@pytest.mark.parametrize("exact_H", [True, False])
def test_step_exhausting_the_krylov_space_is_exact(exact_H):
    # L = 2 (4 sites, 16 states): 16 Krylov vectors span every invariant
    # subspace the start vector touches, so the step is the exact exponential
    rng, t, chi, zeta, H = _case(2, 3, 11)
    psi = synth.random_mps_tensors(rng, 4, 4)
    psi = M.scale(psi, 1.0 / M.norm(psi))
    Hfun = _dense_hfun(H) if exact_H else None
    info = {}
    out = EV.evolve_step((psi, None), t, chi, zeta, 4, 16, 0.3, Hfun=Hfun, info=info)
    want = scipy.linalg.expm(-0.3j * H) @ M.to_dense(psi)
    assert info["m"] <= 16
    assert _rel(EV.to_dense_complex(out), want) < 1e-11
    assert abs(EV.cnorm(out) - 1.0) < 1e-12


def test_two_steps_through_a_complex_state():
    # the second step starts from a state with both parts present
    rng, t, chi, zeta, H = _case(2, 3, 12)
    psi = synth.random_mps_tensors(rng, 4, 4)
    out, dims = EV.evolve((psi, None), t, chi, zeta, 4, 16, 0.25, 2)
    assert out[0] is not None and out[1] is not None
    want = scipy.linalg.expm(-0.5j * H) @ M.to_dense(psi)
    assert _rel(EV.to_dense_complex(out), want) < 1e-11


def test_eigenstate_only_gains_a_phase():
    # an eigenvector of H: the Krylov space is one-dimensional (breakdown at
    # the first step) and psi(delta) = exp(-i E delta) psi
    rng, t, chi, zeta, H = _case(3, 4, 13)
    w, U = np.linalg.eigh(H)
    vec = U[:, 5]
    psi = _dense_to_mps(vec, 6)
    info = {}
    out = EV.evolve_step((psi, None), t, chi, zeta, 64, 6, 0.7, Hfun=_dense_hfun(H), info=info)
    assert info["m"] == 1
    assert _rel(EV.to_dense_complex(out), np.exp(-0.7j * w[5]) * vec) < 1e-12


def test_step_error_is_order_delta_to_the_K():
    # one step with K Krylov vectors errs by O(delta^K) (Sec. 2.2): halving
    # delta divides the error by ~2^K
    rng, t, chi, zeta, H = _case(3, 4, 14)
    v = rng.standard_normal(64)
    psi = _dense_to_mps(v / np.linalg.norm(v), 6)
    K = 3
    errs = []
    for delta in (0.004, 0.002):
        out = EV.evolve_step((psi, None), t, chi, zeta, 64, K, delta, Hfun=_dense_hfun(H))
        want = scipy.linalg.expm(-1j * delta * H) @ M.to_dense(psi)
        errs.append(np.linalg.norm(EV.to_dense_complex(out) - want))
    ratio = errs[0] / errs[1]
    assert 2 ** K * 0.8 < ratio < 2 ** K * 1.25, (errs, ratio)


def _hochbruck_lubich(Nk, Wd):
    # eq. error_bond of App. A
    if np.sqrt(Wd) <= Nk <= Wd / 2:
        return 10.0 * np.exp(-4.0 * Nk * Nk / (5.0 * Wd))
    if Nk >= Wd / 2:
        return 10.0 / (Wd / 4.0) * np.exp(-Wd / 4.0) * (np.e * Wd / (4.0 * Nk)) ** Nk
    return np.inf


@pytest.mark.parametrize("K,Wd", [(4, 0.2), (5, 0.5), (8, 1.0)])
def test_step_error_within_the_appendix_bound(K, Wd):
    rng, t, chi, zeta, H = _case(3, 4, 15)
    w = np.linalg.eigvalsh(H)
    W = w[-1] - w[0]
    delta = Wd / W
    v = rng.standard_normal(64)
    psi = _dense_to_mps(v / np.linalg.norm(v), 6)
    out = EV.evolve_step((psi, None), t, chi, zeta, 64, K, delta, Hfun=_dense_hfun(H))
    want = scipy.linalg.expm(-1j * delta * H) @ M.to_dense(psi)
    err = np.linalg.norm(EV.to_dense_complex(out) - want)
    assert err <= _hochbruck_lubich(K, Wd), (err, _hochbruck_lubich(K, Wd))


def test_truncated_evolution_keeps_number_and_spin_sectors():
    # H conserves N and S_z (eq. 1): starting in a sector, the evolved state
    # has no weight outside it, truncated or not (to the rounding of the
    # ~10^3 compressions of the two steps, each dropping values below 1e-14 s_1)
    L = 3
    rng = np.random.default_rng(17)
    t, chi, zeta = synth.thc_factors(rng, L, 4)
    occ = synth.single_excitation_occupation(L, 2)
    psi = synth.occupation_mps_tensors(occ)
    out, _ = EV.evolve((psi, None), t, chi, zeta, 3, 4, 0.1, 2)
    vec = EV.to_dense_complex(out)
    n = 2 * L
    Nd = F.number_operator_dense(n)
    Szd = F.sz_dense(n)
    n0 = sum(occ)
    sz0 = sum(occ[0::2]) - sum(occ[1::2])
    outside = (np.abs(Nd - n0) > 1e-9) | (np.abs(Szd - sz0) > 1e-9)
    assert np.linalg.norm(vec[outside]) < 1e-10 * np.linalg.norm(vec)
