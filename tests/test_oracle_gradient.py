"""Pins of the oracle's gradient of E = <psi|H_THC|psi> w.r.t. chi and zeta
(THC-factor fitting, Sec. 2.3; G-term structure, Sec. 3.1): central finite
differences of the energy, a dense two-body density matrix, the dense H of
eq. (1), and the MPS route against the dense route."""
import numpy as np
import pytest

import synth
from oracle import fermion as F
from oracle import gradient as OG
from oracle import mps as M
from oracle import thc as TH


def _state(L, D, seed):
    rng = np.random.default_rng(seed)
    psi = synth.random_mps_tensors(rng, 2 * L, D)
    return M.scale(psi, 1.0 / M.norm(psi))


def test_transition_1rdm_mps_matches_dense():
    L = 4
    bra, ket = _state(L, 4, 1), _state(L, 8, 2)
    g = OG.transition_1rdm_mps(bra, ket)
    b, k = M.to_dense(bra), M.to_dense(ket)
    n = 2 * L
    ref = np.array([[b @ F.apply_a(F.apply_a(k, j, n), i, n, dag=True) for j in range(n)] for i in range(n)])
    assert np.allclose(g, ref, atol=1e-13, rtol=0)


def test_energy_routes_match_eq1():
    L, N = 4, 5
    t, chi, zeta = synth.thc_factors(np.random.default_rng(3), L, N)
    psi = _state(L, 8, 4)
    vec = M.to_dense(psi)
    ref = vec @ F.apply_H_dense(vec, t, TH.thc_v(chi, zeta))  # eq. (1) with v from eq. thc
    assert abs(OG.energy_dense(vec, t, chi, zeta) - ref) < 1e-12 * abs(ref)
    assert abs(OG.energy_mps(psi, t, chi, zeta) - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("symmetric", [True, False])
def test_gradient_dense_matches_central_differences(symmetric):
    L, N = 3, 4
    rng = np.random.default_rng(5)
    t, chi, zeta = synth.thc_factors(rng, L, N)
    if not symmetric:
        zeta = zeta + 0.3 * rng.standard_normal((N, N))
    vec = M.to_dense(_state(L, 8, 6))
    dchi, dzeta = OG.gradient_dense(vec, chi, zeta)
    h = 1e-6
    fd_chi = np.zeros_like(chi)
    for p in range(L):
        for k in range(N):
            cp, cm = chi.copy(), chi.copy()
            cp[p, k] += h
            cm[p, k] -= h
            fd_chi[p, k] = (OG.energy_dense(vec, t, cp, zeta) - OG.energy_dense(vec, t, cm, zeta)) / (2 * h)
    fd_zeta = np.zeros_like(zeta)
    for a in range(N):
        for b in range(N):
            zp, zm = zeta.copy(), zeta.copy()
            zp[a, b] += h
            zm[a, b] -= h
            fd_zeta[a, b] = (OG.energy_dense(vec, t, chi, zp) - OG.energy_dense(vec, t, chi, zm)) / (2 * h)
    scale = max(np.abs(dchi).max(), np.abs(dzeta).max())
    assert np.allclose(dchi, fd_chi, atol=1e-7 * scale, rtol=0)
    assert np.allclose(dzeta, fd_zeta, atol=1e-7 * scale, rtol=0)
    # a dropped factor 2 or a missing transpose would fail
    assert not np.allclose(0.5 * dchi, fd_chi, atol=1e-3 * scale, rtol=0)


def test_zeta_gradient_from_dense_two_body_density():
    # dE/dzeta_{mu nu} = 1/2 sum_pqrs chi_p^mu chi_q^mu chi_r^nu chi_s^nu <E_pq E_rs>
    L, N = 3, 3
    t, chi, zeta = synth.thc_factors(np.random.default_rng(7), L, N)
    vec = M.to_dense(_state(L, 8, 8))
    G2 = np.zeros((L, L, L, L))
    for r in range(L):
        for s in range(L):
            w = F.apply_E(vec, r, s, L)
            for p in range(L):
                for q in range(L):
                    G2[p, q, r, s] = vec @ F.apply_E(w, p, q, L)
    ref = 0.5 * np.einsum("pm,qm,rn,sn,pqrs->mn", chi, chi, chi, chi, G2)
    _, dzeta = OG.gradient_dense(vec, chi, zeta)
    assert np.allclose(dzeta, ref, atol=1e-12 * np.abs(ref).max(), rtol=0)


def test_gradient_mps_matches_dense():
    L, N = 4, 4
    t, chi, zeta = synth.thc_factors(np.random.default_rng(9), L, N)
    psi = _state(L, 8, 10)
    dc_m, dz_m = OG.gradient_mps(psi, chi, zeta)
    dc_d, dz_d = OG.gradient_dense(M.to_dense(psi), chi, zeta)
    s = max(np.abs(dc_d).max(), np.abs(dz_d).max())
    assert np.allclose(dc_m, dc_d, atol=1e-12 * s, rtol=0)
    assert np.allclose(dz_m, dz_d, atol=1e-12 * s, rtol=0)
