"""GPU parity of the restarted Lanczos run, the Ritz vectors and an
excited-state run (Sec. 2.2; Sec. 4.1 runs the first excited state from an
excited start vector and restarts the iteration) against the FP64 oracle and
exact diagonalisation of the dense H of eq. (1) in its sector.
"""
import numpy as np
import pytest

import synth
from oracle import fermion as F
from oracle import lanczos as OL
from oracle import mps as M
from oracle import thc as TH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_12708_amd as p
    return p


def _dense_to_mps(vec, n):
    sites, rest, l = [], vec.reshape(1, -1), 1
    for _ in range(n - 1):
        rest = rest.reshape(l * 2, -1)
        u, s, vt = np.linalg.svd(rest, full_matrices=False)
        keep = max(1, int(np.count_nonzero(s > 1e-15 * s[0])))
        u, s, vt = u[:, :keep], s[:keep], vt[:keep]
        sites.append(u.reshape(l, 2, -1))
        l = u.shape[1]
        rest = s[:, None] * vt
    sites.append(rest.reshape(l, 2, 1))
    return sites


def _sector_spectrum(t, chi, zeta, L, n_up, n_dn):
    H = F.hamiltonian_sparse(t, TH.thc_v(chi, zeta)).toarray()
    n = 2 * L
    idx = np.arange(2 ** n)
    bits = (idx[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1  # site 0 most significant
    up, dn = bits[:, 0::2].sum(1), bits[:, 1::2].sum(1)
    sec = np.where((up == n_up) & (dn == n_dn))[0]
    ev, U = np.linalg.eigh(H[np.ix_(sec, sec)])
    return ev, U, sec


@pytest.mark.parametrize("D", [8, 4])
def test_restarted_lanczos_matches_oracle(thck, D):
    # L = 3: D = 8 is exact (largest Schmidt rank of 6 sites), D = 4 truncates
    L, N, K = 3, 4, 3
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(L, 2))
    ctx = thck.Context(t, chi, zeta)
    kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), K, D=D)
    st = OL.KrylovState(hf, K)
    tol = 1e-10 if D == 8 else 1e-8
    for cycle in range(3):
        for i in range(K):
            rg, rt, b = OL.krylov_step(st, t, chi, zeta, D=D)
            g, tt, bb = kr.step()
            print(f"restart D={D} cycle {cycle} step {i}: lowest Ritz {g[0]:.12f} vs {rg[0]:.12f}")
            assert np.allclose(g, rg, atol=tol, rtol=0), (cycle, i, g, rg)
        # the Ritz vector of the lowest value, then the restart from it
        ref_vec = M.to_dense(OL.ritz_vector(st, 0, D))
        got_vec = M.to_dense(kr.ritz_vector(0).to_sites())
        sign = np.sign(ref_vec @ got_vec)
        assert np.linalg.norm(sign * got_vec - ref_vec) < tol * 10 * np.linalg.norm(ref_vec)
        st = OL.restart(st, 0, D=D)
        kr.restart(0)
    kr.close()


def test_excited_state_from_orthogonal_start(thck):
    # the single excitation of the Hartree-Fock state with the exact ground
    # state of its sector projected out: the lowest Ritz value converges to
    # E_1 of the sector, on the GPU as in the oracle
    L, N = 3, 4
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    n = 2 * L
    ev, U, sec = _sector_spectrum(t, chi, zeta, L, 1, 1)
    g = np.zeros(2 ** n)
    g[sec] = U[:, 0]
    phi = M.to_dense(synth.occupation_mps_tensors(synth.single_excitation_occupation(L, 2, 0)))
    phi = phi - (g @ phi) * g
    start = _dense_to_mps(phi, n)
    K = 8
    ctx = thck.Context(t, chi, zeta)
    kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(start), K, D=8)
    st = OL.KrylovState(start, K)
    for i in range(K):
        rg, _, b = OL.krylov_step(st, t, chi, zeta, D=8)
        gv, _, bb = kr.step()
        assert abs(gv[0] - rg[0]) < 1e-10
        if b < 1e-10:
            break
    print(f"excited state: GPU {gv[0]:.12f}, oracle {rg[0]:.12f}, E1 {ev[1]:.12f}, E0 {ev[0]:.12f}")
    assert abs(gv[0] - ev[1]) < 1e-8 * max(1.0, abs(ev[1]))
    kr.close()


def test_ritz_index_out_of_range_is_rejected(thck):
    L, N = 3, 4
    t, chi, zeta = synth.thc_factors(np.random.default_rng(16), L, N)
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(L, 2))
    ctx = thck.Context(t, chi, zeta)
    kr = thck.Krylov(ctx, thck.DeviceMPS.from_sites(hf), 3, D=8)
    with pytest.raises(thck.ThcError):
        kr.ritz_vector(0)  # no step taken yet
    kr.step()
    with pytest.raises(thck.ThcError):
        kr.ritz_vector(1)  # one basis vector: only index 0
    kr.ritz_vector(0)
    kr.close()
